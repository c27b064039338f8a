// pq_mfma.hip -- fused PQ scoring by decoding into MFMA operands.
//
// The same scores as the table kernel (Sec. 4.2-4.3: by the ADC identity,
// sum_m T[i, m, c_jm] = q_i . concat_m C[m, c_jm]), computed the other way
// round: instead of a per-query table, the workgroup keeps the codebook
// itself in LDS (M x K x dsub FP16, 64 KiB at d = 128) and each wave
// rebuilds a 16-token document tile from it straight into the A operand of
// v_mfma_f32_16x16x32_f16: lane (r, g) of k-step c needs the 8 values
// c*32 + g*8 .. +8 of token r, which sit inside one centroid (dsub >= 8), so
// one ds_read_b128 fetches them. The decoded tile is then contracted with
// the query tokens held in VGPRs (B operand), several queries per wave, so
// one decode serves NQB x 16 query tokens. Running maxima stay in VGPRs; rows
// past a document's end are clamped to its last token; at the document's
// end two xor-shuffles finish the max over rows and four sum a query's
// tokens. FP16 products are exact and accumulate in FP32.
//
// Work item = (doc chunk, group of queries). Without candidate lists a group
// holds NQB / BPQ queries (BPQ = 16-column blocks per query, from the
// query-length bound); with candidate lists a group is one query.
#include "device_common.h"
#include "kernels.h"

namespace {

template <int M>
struct PqCodes;
template <>
struct PqCodes<4> {
  typedef uint32_t type;
  __device__ static uint32_t word(type v, int) { return v; }
};
template <>
struct PqCodes<8> {
  typedef uint2 type;
  __device__ static uint32_t word(type v, int w) { return w == 0 ? v.x : v.y; }
};
template <>
struct PqCodes<16> {
  typedef uint4 type;
  __device__ static uint32_t word(type v, int w) {
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
  }
};

template <int M, int DSUB, int NQB, int NW>
__global__ __launch_bounds__(NW * 64) void pq_mfma_kernel(PqParams P) {
  extern __shared__ u32x4 cb_lds[];  // codebooks [M][K][DSUB] FP16
  constexpr int DIM = M * DSUB;
  constexpr int NKS = DIM / 32;  // k-steps of 32
  typedef typename PqCodes<M>::type cvec;
  const int lane = lane_id();
  const int r = lane & 15, g = lane >> 4;
  const int wave = uniform(threadIdx.x >> 6);
  const int K = P.K;
  const int bpq = P.bpq;            // 16-column blocks per query
  const int gsz = P.group;          // queries per group
  const int64_t n_groups = (P.n_q + gsz - 1) / gsz;

  const int64_t item = blockIdx.x;
  const int64_t grp = item % n_groups;
  const int64_t chunk = item / n_groups;
  const int64_t a0 = grp * gsz;

  // doc (or candidate position) range of this item
  int64_t p0, p1;
  if (P.cand_off == nullptr) {
    p0 = (P.n_docs * chunk) / P.n_chunks;
    p1 = (P.n_docs * (chunk + 1)) / P.n_chunks;
  } else {
    const int64_t c0 = P.cand_off[a0], c1 = P.cand_off[a0 + 1];
    p0 = c0 + ((c1 - c0) * chunk) / P.n_chunks;
    p1 = c0 + ((c1 - c0) * (chunk + 1)) / P.n_chunks;
  }
  if (p0 >= p1) return;  // uniform for the whole workgroup

  // ---- codebooks into LDS (16-byte copies) ----
  {
    const int n16 = M * K * DSUB * 2 / 16;
    const u32x4* src = (const u32x4*)P.codebooks;
    for (int e = threadIdx.x; e < n16; e += NW * 64) cb_lds[e] = src[e];
  }

  // ---- query operand registers: block nb = query a0 + nb / bpq, rows
  // (nb % bpq) * 16 + r of that query (zero past its end) ----
  f16x8 qb[NQB][NKS];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) {
    const int64_t a = a0 + nb / bpq;
    int nq = 0;
    int64_t q0 = 0;
    if (a < P.n_q && nb / bpq < gsz) {
      q0 = P.q_off[a];
      nq = (int)(P.q_off[a + 1] - q0);
    }
    const int t = (nb % bpq) * 16 + r;
    const bool live = t < nq;
    const _Float16* qrow = (const _Float16*)P.q_tok + (q0 + (live ? t : 0)) * DIM + g * 8;
#pragma unroll
    for (int c = 0; c < NKS; ++c) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (live) v = *(const u32x4*)(qrow + c * 32);
      qb[nb][c] = __builtin_bit_cast(f16x8, v);
    }
  }
  // per query of the group (bit gq): exists, has tokens, exceeds its bound
  uint32_t valid_m = 0, nonempty_m = 0, poison_m = 0;
#pragma unroll
  for (int gq = 0; gq < NQB; ++gq) {
    const int64_t a = a0 + gq;
    if (gq < gsz && a < P.n_q) {
      const int nq = (int)(P.q_off[a + 1] - P.q_off[a]);
      valid_m |= 1u << gq;
      if (nq > 0) nonempty_m |= 1u << gq;
      if (nq > bpq * 16) poison_m |= 1u << gq;
    }
  }
  __syncthreads();

  // per-lane decode constants of k-step c: subspace m = (c*32 + g*8) / DSUB,
  // offset o inside the centroid; the 32/DSUB subspaces of one k-step lie in
  // one 4-byte word of the code vector
  int lbase[NKS], lsh[NKS];
#pragma unroll
  for (int c = 0; c < NKS; ++c) {
    const int kk = c * 32 + g * 8;
    const int m = kk / DSUB, o = kk % DSUB;
    lbase[c] = (m * K * DSUB + o) * 2;
    lsh[c] = 8 * (m & 3);
  }
  const char* cbl = (const char*)cb_lds;

  // ---- cursor over (document, 16-row tile) steps of this wave's documents
  // p0 + wave, p0 + wave + NW, ...; offsets by scalar loads one doc ahead ----
  const bool has_cand = P.cand_off != nullptr;
  auto doc_of = [&](int64_t pp) -> int64_t {
    return has_cand ? (int64_t)sload_i32(P.cand_ids, pp) : pp;
  };
  int64_t cp = p0 + wave;
  int64_t ct0 = 0, nx_s = 0, nx_e = 0;
  int cnd = 0, ctile = 0;
  if (cp < p1) {
    const int64_t b0 = doc_of(cp);
    ct0 = sload_i64(P.d_off, b0);
    cnd = (int)(sload_i64(P.d_off, b0 + 1) - ct0);
    if (cp + NW < p1) {
      const int64_t b1 = doc_of(cp + NW);
      nx_s = sload_i64(P.d_off, b1);
      nx_e = sload_i64(P.d_off, b1 + 1);
    }
  }
  auto next_doc = [&]() {
    cp += NW;
    ctile = 0;
    ct0 = nx_s;
    cnd = (int)(nx_e - nx_s);
    if (cp + NW < p1) {
      const int64_t b1 = doc_of(cp + NW);
      nx_s = sload_i64(P.d_off, b1);
      nx_e = sload_i64(P.d_off, b1 + 1);
    }
  };
  constexpr int F_VALID = 1, F_EMPTY = 2, F_DLAST = 4;
  const cvec* codes = (const cvec*)P.codes;
  const cvec* const zero = (const cvec*)zero_row_ptr();
  // every refill issues exactly one code load (a zero row when idle)
  auto fill = [&](cvec& cv, int& fl, int64_t& pp) {
    const cvec* src = zero;
    int f = 0;
    pp = cp;
    if (cp < p1) {
      if (cnd == 0) {
        f = F_VALID | F_EMPTY;
      } else {
        const int row = ctile * 16 + r;
        src = codes + ct0 + (row < cnd ? row : cnd - 1);
        f = F_VALID | ((ctile + 1) * 16 >= cnd ? F_DLAST : 0);
      }
    }
    cv = *src;
    fl = f;
    if (cp < p1) {
      if (cnd == 0 || (ctile + 1) * 16 >= cnd)
        next_doc();
      else
        ++ctile;
    }
  };

  auto store = [&](int64_t pp, int gq, float v) {
    // query longer than its bound: NaN (as a bit pattern; this file assumes
    // no NaN arithmetic)
    if ((poison_m >> gq) & 1u) v = __builtin_bit_cast(float, 0x7fc00000u);
    P.scores[has_cand ? pp : (a0 + gq) * P.n_docs + pp] = v;
  };

  float mx[NQB];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) mx[nb] = -__builtin_inff();

  auto consume = [&](const cvec& cv, int fl, int64_t pp) {
    if (!(fl & F_VALID)) return;
    if (fl & F_EMPTY) {
      if (lane == 0) {
        for (int gq = 0; gq < NQB; ++gq)
          if ((valid_m >> gq) & 1u) store(pp, gq, ((nonempty_m >> gq) & 1u) ? -__builtin_inff() : 0.f);
      }
      return;
    }
    f16x8 av[NKS];
#pragma unroll
    for (int c = 0; c < NKS; ++c) {
      const uint32_t code =
          __builtin_amdgcn_ubfe(PqCodes<M>::word(cv, (c * 32 / DSUB) >> 2), lsh[c], 8);
      av[c] = __builtin_bit_cast(f16x8, *(const u32x4*)(cbl + lbase[c] + code * (DSUB * 2)));
    }
    // k-step outer, query block inner: NQB independent accumulation chains
    // keep the matrix pipe busy between dependent MFMAs
    f32x4 acc[NQB];
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NKS; ++c)
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[c], qb[nb][c], acc[nb], 0, 0, 0);
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb)
      mx[nb] = fmaxf(mx[nb], fmaxf(fmaxf(acc[nb].x, acc[nb].y), fmaxf(acc[nb].z, acc[nb].w)));
    if (fl & F_DLAST) {
      float qsum = 0.f;
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb) {
        const float v = max_rows4(mx[nb]);
        qsum += v;
        mx[nb] = -__builtin_inff();
        if ((nb + 1) % bpq == 0) {
          const int gq = nb / bpq;
          float t = qsum;
          t = row_sum16(t);
          if (lane == 0 && ((valid_m >> gq) & 1u)) store(pp, gq, t);
          qsum = 0.f;
        }
      }
    }
  };

  // four ring slots, written out so each keeps its own registers
  cvec r0, r1, r2, r3;
  int f0, f1, f2, f3;
  int64_t q0p, q1p, q2p, q3p;
  fill(r0, f0, q0p);
  fill(r1, f1, q1p);
  fill(r2, f2, q2p);
  fill(r3, f3, q3p);
  if (f0 & F_VALID) {
    while (true) {
      consume(r0, f0, q0p);
      fill(r0, f0, q0p);
      consume(r1, f1, q1p);
      fill(r1, f1, q1p);
      consume(r2, f2, q2p);
      fill(r2, f2, q2p);
      consume(r3, f3, q3p);
      fill(r3, f3, q3p);
      if (!(f0 & F_VALID)) break;
    }
  }
}

template <int M, int DSUB, int NQB>
hipError_t launch_mfma_t(const PqParams& P, size_t lds, hipStream_t s) {
  constexpr int NW = 8;
  auto k = pq_mfma_kernel<M, DSUB, NQB, NW>;
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t n_groups = (P.n_q + P.group - 1) / P.group;
  const int64_t items = n_groups * P.n_chunks;
  hipLaunchKernelGGL(k, dim3((unsigned)items), dim3(NW * 64), lds, s, P);
  return hipGetLastError();
}

template <int M, int DSUB>
hipError_t launch_mfma_nqb(const PqParams& P, size_t lds, hipStream_t s) {
  constexpr int NKS = M * DSUB / 32;
  switch (P.nqb) {
    case 1: return launch_mfma_t<M, DSUB, 1>(P, lds, s);
    case 2: return launch_mfma_t<M, DSUB, 2>(P, lds, s);
    case 4:
      if constexpr (NKS <= 8) return launch_mfma_t<M, DSUB, 4>(P, lds, s);
      return hipErrorInvalidValue;
    default:
      if constexpr (NKS <= 4) return launch_mfma_t<M, DSUB, 8>(P, lds, s);
      return hipErrorInvalidValue;
  }
}

template <int M>
hipError_t launch_mfma_dsub(const PqParams& P, size_t lds, hipStream_t s) {
  switch (P.dsub) {
    case 8: return launch_mfma_nqb<M, 8>(P, lds, s);
    case 16: return launch_mfma_nqb<M, 16>(P, lds, s);
    default: return launch_mfma_nqb<M, 32>(P, lds, s);
  }
}

}  // namespace

hipError_t launch_pq_mfma(const PqParams& P, size_t lds, hipStream_t s) {
  switch (P.M) {
    case 4: return launch_mfma_dsub<4>(P, lds, s);
    case 8: return launch_mfma_dsub<8>(P, lds, s);
    default: return launch_mfma_dsub<16>(P, lds, s);
  }
}
