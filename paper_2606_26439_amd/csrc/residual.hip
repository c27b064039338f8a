// residual.hip -- MaxSim over residual-compressed documents.
//
// A document token is stored as a centroid id plus a residual quantized per
// dimension to NBITS bits (the compressed form of the PLAID/WARP indexes the
// paper compares with and plugs into): x_jk = C[id_j, k] + w[code_jk]. The
// score is Eq. (1) on these vectors, computed through the split
//   q_i . x_j = q_i . C[id_j] + q_i . r_j.
// The first term does not depend on the document, so one small MFMA kernel
// tabulates P[c, i] = C[c] . q_i for every centroid c and query token i (FP32,
// in the caller's workspace). The fused kernel then reads each document
// token's id (4 B) and packed residual (dim * NBITS / 8 B) once from HBM,
// seeds the accumulator of a 16-token tile with the gathered P entries,
// decodes the residual codes into FP16 through a byte-indexed table in LDS,
// and adds q_i . r_j with v_mfma_f32_16x16x32_f16 before the running max over
// tokens and the sum over query tokens. Decoded vectors are never written.
//
// Column order. Lane (r, g) of a k-step holds 8 consecutive columns of its
// row; here lane group g owns the contiguous quarter [g * dim/4, (g+1) * dim/4)
// of the dimensions and k-step s takes columns g * dim/4 + 8 s .. + 7. The
// query operand uses the same order, so every product pairs equal columns,
// and a lane's residual codes for all k-steps are one contiguous
// dim * NBITS / 32-byte piece of the packed row.
#include "device_common.h"
#include "kernels.h"

namespace {

// P[c, j] = C[c] . q_j over all centroids c and all query tokens j of the
// batch (row length n_qtok). One wave per 16 centroids; 4 waves per group.
template <int NKS>
__global__ __launch_bounds__(256) void centroid_table_kernel(ResParams P) {
  constexpr int DIM = NKS * 32;
  const int lane = lane_id();
  const int r = lane & 15, g = lane >> 4;
  const int64_t c0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const int64_t n_c = P.n_centroids;
  if (c0 >= n_c) return;  // uniform per wave
  const int64_t cr = c0 + r < n_c ? c0 + r : n_c - 1;
  const _Float16* crow = (const _Float16*)P.centroids + cr * DIM + g * (DIM / 4);
  f16x8 a[NKS];
#pragma unroll
  for (int s = 0; s < NKS; ++s) a[s] = *(const f16x8*)(crow + 8 * s);
  const int64_t nqt = P.n_qtok;
  for (int64_t j0 = 0; j0 < nqt; j0 += 16) {
    const int64_t j = j0 + r;
    const bool live = j < nqt;
    const _Float16* qrow = (const _Float16*)P.q_tok + (live ? j : 0) * DIM + g * (DIM / 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (live) v = *(const u32x4*)(qrow + 8 * s);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[s], __builtin_bit_cast(f16x8, v), acc, 0, 0,
                                                   0);
    }
    // lane holds centroids c0 + 4g + v, query token j
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = c0 + 4 * g + v;
      if (live && c < n_c) P.table[c * nqt + j] = acc[v];
    }
  }
}

// Residual bytes of one lane for one token, as 32-bit words.
template <int RB>
struct ResWords {
  static constexpr int N = RB < 4 ? 1 : RB / 4;
  uint32_t w[N];
  __device__ void load(const uint8_t* p) {
    if constexpr (RB == 2) {
      w[0] = *(const uint16_t*)p;
    } else if constexpr (RB == 4) {
      w[0] = *(const uint32_t*)p;
    } else if constexpr (RB == 8) {
      const uint2 v = *(const uint2*)p;
      w[0] = v.x;
      w[1] = v.y;
    } else {
#pragma unroll
      for (int h = 0; h < RB / 16; ++h) {
        const u32x4 v = *(const u32x4*)(p + 16 * h);
        w[4 * h] = v.x;
        w[4 * h + 1] = v.y;
        w[4 * h + 2] = v.z;
        w[4 * h + 3] = v.w;
      }
    }
  }
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = 0;
  }
  // byte j of the lane's piece, times `scale` (a power of two: the LUT entry size)
  __device__ uint32_t byte_offset(int j, int scale_log2) const {
    return __builtin_amdgcn_ubfe(w[j >> 2], 8 * (j & 3), 8) << scale_log2;
  }
};

template <int NBITS, int NKS, int NQB, int NW>
__global__ __launch_bounds__(NW * 64) void residual_maxsim_kernel(ResParams P) {
  constexpr int DIM = NKS * 32;
  constexpr int RB = NKS * NBITS;  // residual bytes per lane per token
  constexpr int ROWB = 4 * RB;     // bytes per packed token row
  constexpr int FPB = 8 / NBITS;   // fields per byte
  constexpr int EB = 2 * FPB;      // LUT entry bytes (FPB FP16 values)
  constexpr int EB_LOG2 = EB == 16 ? 4 : (EB == 8 ? 3 : 2);
  __shared__ __attribute__((aligned(16))) _Float16 lut[256 * FPB];

  const int lane = lane_id();
  const int r = lane & 15, g = lane >> 4;
  const int wave = uniform(threadIdx.x >> 6);
  const int64_t a = blockIdx.x % P.n_q;
  const int64_t chunk = blockIdx.x / P.n_q;

  int64_t p0, p1;
  if (P.cand_off == nullptr) {
    p0 = (P.n_docs * chunk) / P.n_chunks;
    p1 = (P.n_docs * (chunk + 1)) / P.n_chunks;
  } else {
    const int64_t c0 = P.cand_off[a], c1 = P.cand_off[a + 1];
    p0 = c0 + ((c1 - c0) * chunk) / P.n_chunks;
    p1 = c0 + ((c1 - c0) * (chunk + 1)) / P.n_chunks;
  }
  if (p0 >= p1) return;  // uniform for the whole workgroup

  // LUT: entry b holds the residual values of the FPB fields of byte b,
  // lowest field first (fields fill a byte from its least significant bit)
  for (int e = threadIdx.x; e < 256 * FPB; e += NW * 64) {
    const int b = e / FPB, f = e % FPB;
    lut[e] = ((const _Float16*)P.weights)[(b >> (f * NBITS)) & ((1 << NBITS) - 1)];
  }

  // query operand: block nb holds tokens nb*16 + r of query a (zero past its end)
  const int64_t qa0 = P.q_off[a];
  const int nq = (int)(P.q_off[a + 1] - qa0);
  f16x8 qb[NQB][NKS];
  int64_t qcol[NQB];  // table column of this lane's query token per block
  bool qlive[NQB];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) {
    const int t = nb * 16 + r;
    qlive[nb] = t < nq;
    qcol[nb] = qa0 + (qlive[nb] ? t : 0);
    const _Float16* qrow = (const _Float16*)P.q_tok + qcol[nb] * DIM + g * (DIM / 4);
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (qlive[nb]) v = *(const u32x4*)(qrow + 8 * s);
      qb[nb][s] = __builtin_bit_cast(f16x8, v);
    }
  }
  const bool poison = nq > NQB * 16;
  __syncthreads();

  // ---- cursor over (document, 16-row tile) steps of this wave's documents
  // p0 + wave, p0 + wave + NW, ... (offsets by scalar loads, one doc ahead)
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
  constexpr int F_VALID = 1, F_EMPTY = 2, F_DLAST = 4, F_TOK = 8;
  struct Tile {
    int64_t pp, tok0;
    int rows, flags;
  };
  auto next_tile = [&]() -> Tile {
    Tile t{cp, 0, 1, 0};
    if (cp < p1) {
      if (cnd == 0) {
        t.flags = F_VALID | F_EMPTY;
      } else {
        t.tok0 = ct0 + (int64_t)ctile * 16;
        t.rows = cnd - ctile * 16 < 16 ? cnd - ctile * 16 : 16;
        t.flags = F_VALID | F_TOK | ((ctile + 1) * 16 >= cnd ? F_DLAST : 0);
      }
      if (cnd == 0 || (ctile + 1) * 16 >= cnd) {
        cp += NW;
        ctile = 0;
        ct0 = nx_s;
        cnd = (int)(nx_e - nx_s);
        if (cp + NW < p1) {
          const int64_t b1 = doc_of(cp + NW);
          nx_s = sload_i64(P.d_off, b1);
          nx_e = sload_i64(P.d_off, b1 + 1);
        }
      } else {
        ++ctile;
      }
    }
    return t;
  };

  const uint32_t max_c = (uint32_t)(P.n_centroids - 1);
  // centroid ids of accumulator rows 4g .. 4g+3 (clamped to the tile's rows;
  // an id outside the table is clamped too, so a bad id cannot read outside it)
  auto load_ids = [&](const Tile& t, uint32_t (&id)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) id[v] = 0;
    if (t.flags & F_TOK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * g + v < t.rows ? 4 * g + v : t.rows - 1;
        const uint32_t c = (uint32_t)P.ids[t.tok0 + row];
        id[v] = c < max_c ? c : max_c;
      }
    }
  };
  auto load_rest = [&](const Tile& t, const uint32_t (&id)[4], ResWords<RB>& rw,
                       f32x4 (&pv)[NQB]) {
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) pv[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    rw.zero();
    if (t.flags & F_TOK) {
      const int row = r < t.rows ? r : t.rows - 1;
      rw.load(P.residuals + (t.tok0 + row) * ROWB + g * RB);
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb)
        if (qlive[nb]) {
#pragma unroll
          for (int v = 0; v < 4; ++v) pv[nb][v] = P.table[(int64_t)id[v] * P.n_qtok + qcol[nb]];
        }
    }
  };

  auto store = [&](int64_t pp, float v) {
    if (poison) v = __builtin_bit_cast(float, 0x7fc00000u);
    P.scores[has_cand ? pp : a * P.n_docs + pp] = v;
  };

  float mx[NQB];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) mx[nb] = -__builtin_inff();
  const char* lutb = (const char*)lut;

  auto consume = [&](const Tile& t, const ResWords<RB>& rw, const f32x4 (&pv)[NQB]) {
    if (t.flags & F_EMPTY) {
      if (lane == 0) store(t.pp, nq > 0 ? -__builtin_inff() : 0.f);
      return;
    }
    f32x4 acc[NQB];
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) acc[nb] = pv[nb];
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      // bytes s*NBITS .. s*NBITS + NBITS - 1 of the lane's piece decode to
      // the 8 residual values of k-step s
      u32x4 av;
      if constexpr (NBITS == 1) {
        av = *(const u32x4*)(lutb + rw.byte_offset(s, EB_LOG2));
      } else if constexpr (NBITS == 2) {
        const uint2 lo = *(const uint2*)(lutb + rw.byte_offset(2 * s, EB_LOG2));
        const uint2 hi = *(const uint2*)(lutb + rw.byte_offset(2 * s + 1, EB_LOG2));
        av = u32x4{lo.x, lo.y, hi.x, hi.y};
      } else {
        av = u32x4{*(const uint32_t*)(lutb + rw.byte_offset(4 * s, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 1, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 2, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 3, EB_LOG2))};
      }
      const f16x8 ah = __builtin_bit_cast(f16x8, av);
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, qb[nb][s], acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb)
      mx[nb] = fmaxf(mx[nb], fmaxf(fmaxf(acc[nb].x, acc[nb].y), fmaxf(acc[nb].z, acc[nb].w)));
    if (t.flags & F_DLAST) {
      float qsum = 0.f;
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb) {
        float v = mx[nb];
        v = fmaxf(v, xor_shfl(v, 16));
        v = fmaxf(v, xor_shfl(v, 32));
        qsum += v;
        mx[nb] = -__builtin_inff();
      }
      qsum += xor_shfl(qsum, 8);
      qsum += xor_shfl(qsum, 4);
      qsum += xor_shfl(qsum, 2);
      qsum += xor_shfl(qsum, 1);
      if (lane == 0) store(t.pp, qsum);
    }
  };

  // Software pipeline: ids two tiles ahead, residual codes and table entries
  // one tile ahead (their addresses need the ids), compute on the current.
  Tile ta = next_tile();
  uint32_t ia[4];
  load_ids(ta, ia);
  Tile tb = next_tile();
  uint32_t ib[4];
  load_ids(tb, ib);
  ResWords<RB> ra;
  f32x4 pa[NQB];
  load_rest(ta, ia, ra, pa);
  while (ta.flags & F_VALID) {
    const Tile tc = next_tile();
    uint32_t ic[4];
    load_ids(tc, ic);
    ResWords<RB> rb;
    f32x4 pb[NQB];
    load_rest(tb, ib, rb, pb);
    consume(ta, ra, pa);
    ta = tb;
    tb = tc;
    ra = rb;
#pragma unroll
    for (int v = 0; v < 4; ++v) ib[v] = ic[v];
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) pa[nb] = pb[nb];
  }
}

template <int NKS>
hipError_t launch_table_t(const ResParams& P, hipStream_t s) {
  const int64_t waves = (P.n_centroids + 15) / 16;
  hipLaunchKernelGGL(centroid_table_kernel<NKS>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                     s, P);
  return hipGetLastError();
}

template <int NBITS, int NKS, int NQB>
hipError_t launch_score_t(const ResParams& P, hipStream_t s) {
  constexpr int NW = 4;
  hipLaunchKernelGGL((residual_maxsim_kernel<NBITS, NKS, NQB, NW>),
                     dim3((unsigned)(P.n_q * P.n_chunks)), dim3(NW * 64), 0, s, P);
  return hipGetLastError();
}

template <int NBITS, int NKS>
hipError_t launch_score_nqb(const ResParams& P, hipStream_t s) {
  switch (P.nqb) {
    case 1: return launch_score_t<NBITS, NKS, 1>(P, s);
    case 2: return launch_score_t<NBITS, NKS, 2>(P, s);
    default: return launch_score_t<NBITS, NKS, 4>(P, s);
  }
}

template <int NBITS>
hipError_t launch_score_dim(const ResParams& P, hipStream_t s) {
  switch (P.dim) {
    case 64: return launch_score_nqb<NBITS, 2>(P, s);
    case 128: return launch_score_nqb<NBITS, 4>(P, s);
    default: return launch_score_nqb<NBITS, 8>(P, s);
  }
}

}  // namespace

hipError_t launch_residual(const ResParams& P, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (P.n_qtok > 0) {
    switch (P.dim) {
      case 64: e = launch_table_t<2>(P, s); break;
      case 128: e = launch_table_t<4>(P, s); break;
      default: e = launch_table_t<8>(P, s); break;
    }
    if (e != hipSuccess) return e;
  }
  switch (P.nbits) {
    case 1: return launch_score_dim<1>(P, s);
    case 2: return launch_score_dim<2>(P, s);
    default: return launch_score_dim<4>(P, s);
  }
}
