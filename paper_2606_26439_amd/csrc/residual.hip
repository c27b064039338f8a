// residual.hip -- MaxSim over residual-compressed documents.
//
// A document token is stored as a centroid id plus a residual quantized per
// dimension to NBITS bits (the compressed form of the PLAID/WARP indexes the
// paper compares with and plugs into): x_jk = C[id_j, k] + w[code_jk]. The
// score is Eq. (1) on these vectors, computed through the split
//   q_i . x_j = q_i . C[id_j] + q_i . r_j.
// The first term does not depend on the document, so one small MFMA kernel
// tabulates P[c, (a, t)] = C[c] . q_t of query a for every centroid c (FP32,
// in the caller's workspace; each query owns QW = 16 * NQB columns, NQB the
// 16-token blocks of the longest query rounded up to a power of two, zero
// past its last token). The fused kernel then reads each
// document token's id (4 B) and packed residual (dim * NBITS / 8 B) once from
// HBM, decodes the residual codes into FP16 through a byte-indexed table in
// LDS, and computes q_t . r_j with v_mfma_f32_16x16x32_f16 whose accumulator
// starts from the gathered table entries; the running max over tokens and the
// sum over query tokens follow. Decoded vectors are never written.
//
// Operand layout. The MFMA's rows are query tokens and its columns document
// tokens, so lane (r, g) of the accumulator holds document row r of the tile
// against query tokens 16 nb + 4g .. 16 nb + 4g + 3 of query block nb: the
// table entries it needs are consecutive in the centroid's table row and
// arrive in one 16-byte load per block. The sum over query tokens runs per
// row position over the blocks in order, then over the positions in a fixed
// tree, so a query scores the same bits whatever block count its batch uses
// (extra blocks add exact zeros at the end). In the k dimension lane group g
// owns the contiguous quarter [g * dim/4, (g+1) * dim/4) of the dimensions
// and k-step s takes columns g * dim/4 + 8 s .. + 7 of both operands, so a
// lane's residual codes for all k-steps are one contiguous dim * NBITS / 32-byte
// piece of the packed row.
#include <map>
#include <mutex>

#include "device_common.h"
#include "kernels.h"

namespace {

// P[c, a * QW + t] = C[c] . q_t of query a (t < its length), 0 for t up to
// QW. One wave per 16 centroids and every 16-column block of every query;
// 4 waves per group.
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
  const int64_t ncols = P.n_cols;
  const int bpq = P.nqb;
  for (int64_t blk = 0; blk < P.n_q * bpq; ++blk) {
    const int64_t qa = blk / bpq;
    const int t = (int)(blk % bpq) * 16 + r;
    const int64_t q0 = sload_i64(P.q_off, qa);
    const bool live = t < (int)(sload_i64(P.q_off, qa + 1) - q0);
    const _Float16* qrow = (const _Float16*)P.q_tok + (live ? q0 + t : 0) * DIM + g * (DIM / 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (live) v = *(const u32x4*)(qrow + 8 * s);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[s], __builtin_bit_cast(f16x8, v), acc, 0, 0,
                                                   0);
    }
    // lane holds centroids c0 + 4g + v, column blk * 16 + r
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t c = c0 + 4 * g + v;
      if (c < n_c) P.table[c * ncols + blk * 16 + r] = acc[v];
    }
  }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Residual bytes of one lane for one token, as 32-bit words.
template <int RB>
struct ResWords {
  static constexpr int N = RB < 4 ? 1 : RB / 4;
  uint32_t w[N];
  __device__ void load(const uint8_t* p) {
    if constexpr (RB == 2) {
      w[0] = __builtin_nontemporal_load((const uint16_t*)p);
    } else if constexpr (RB == 4) {
      w[0] = __builtin_nontemporal_load((const uint32_t*)p);
    } else if constexpr (RB == 8) {
      const u32x2 v = __builtin_nontemporal_load((const u32x2*)p);
      w[0] = v.x;
      w[1] = v.y;
    } else {
#pragma unroll
      for (int h = 0; h < RB / 16; ++h) {
        const u32x4 v = __builtin_nontemporal_load((const u32x4*)(p + 16 * h));
        w[4 * h] = v.x;
        w[4 * h + 1] = v.y;
        w[4 * h + 2] = v.z;
        w[4 * h + 3] = v.w;
      }
    }
  }
  // byte j of the lane's piece shifted left by scale_log2 (a byte offset into
  // the LUT, whose entries are 2^scale_log2 bytes)
  __device__ uint32_t byte_offset(int j, int scale_log2) const {
    return __builtin_amdgcn_ubfe(w[j >> 2], 8 * (j & 3), 8) << scale_log2;
  }
};

template <int NBITS, int NKS, int NQB, int NW, int PI, int PR>
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
    const int64_t c0 = sload_i64(P.cand_off, a), c1 = sload_i64(P.cand_off, a + 1);
    p0 = c0 + ((c1 - c0) * chunk) / P.n_chunks;
    p1 = c0 + ((c1 - c0) * (chunk + 1)) / P.n_chunks;
  }
  p0 = uniform64(p0);
  p1 = uniform64(p1);
  if (p0 >= p1) return;  // uniform for the whole workgroup

  // LUT: entry b holds the residual values of the FPB fields of byte b,
  // lowest field first (fields fill a byte from its least significant bit)
  for (int e = threadIdx.x; e < 256 * FPB; e += NW * 64) {
    const int b = e / FPB, f = e % FPB;
    lut[e] = ((const _Float16*)P.weights)[(b >> (f * NBITS)) & ((1 << NBITS) - 1)];
  }

  // query operand (the MFMA's rows): block nb, row r is query token
  // 16 nb + r of query a, zero past its end
  const int64_t qa0 = uniform64(sload_i64(P.q_off, a));
  const int nq = uniform((int)(sload_i64(P.q_off, a + 1) - qa0));
  f16x8 qa[NQB][NKS];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) {
    const int t = 16 * nb + r;
    const bool live = t < nq;
    const _Float16* qrow = (const _Float16*)P.q_tok + (qa0 + (live ? t : 0)) * DIM + g * (DIM / 4);
#pragma unroll
    for (int s = 0; s < NKS; ++s) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (live) v = *(const u32x4*)(qrow + 8 * s);
      qa[nb][s] = __builtin_bit_cast(f16x8, v);
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
  // positions relative to p0 in 32 bits (the host keeps a span below 2^31),
  // so the cursor tests are scalar compares
  const int span = (int)(p1 - p0);
  int cp = wave;
  int64_t ct0 = 0, nx_s = 0, nx_e = 0;
  int cnd = 0, ctile = 0;
  if (cp < span) {
    const int64_t b0 = doc_of(p0 + cp);
    ct0 = sload_i64(P.d_off, b0);
    cnd = (int)(sload_i64(P.d_off, b0 + 1) - ct0);
    if (cp + NW < span) {
      const int64_t b1 = doc_of(p0 + cp + NW);
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
    Tile t{p0 + cp, 0, 1, 0};
    if (cp < span) {
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
        if (cp + NW < span) {
          const int64_t b1 = doc_of(p0 + cp + NW);
          nx_s = sload_i64(P.d_off, b1);
          nx_e = sload_i64(P.d_off, b1 + 1);
        }
      } else {
        ++ctile;
      }
    }
    return t;
  };

  // Every tile issues the same loads (a tile without tokens reads the zero
  // row, and table row 0, instead), so the count of loads in flight is the
  // same on every path and the compiler's waits stay exact across the ring.
  // The document streams are read once: non-temporal loads keep them from
  // displacing the centroid table in the caches. The host keeps n_centroids
  // and the table's row length below 2^24 and the table below 2^32 entries,
  // so table indices are 24 x 24-bit products in 32 bits.
  const uint32_t max_c = (uint32_t)(P.n_centroids - 1);
  const uint32_t ncols = (uint32_t)P.n_cols;
  const uint32_t col0 = (uint32_t)a * (uint32_t)(16 * NQB) + 4 * g;
  const char* zrow = P.zero_row;
  // centroid id of tile row r (clamped to the tile's rows; clamped to the
  // table where it is used, so a bad id cannot read outside it)
  auto load_ids = [&](const Tile& t, uint32_t& id) {
    const int row = r < t.rows ? r : t.rows - 1;
    const int32_t* src = (t.flags & F_TOK) ? P.ids + t.tok0 + row : (const int32_t*)zrow;
    id = (uint32_t)__builtin_nontemporal_load(src);
  };
  // residual codes of row r, and the table entries that seed the
  // accumulator: this row's centroid, query tokens 16 nb + 4g .. + 3
  auto load_rest = [&](const Tile& t, uint32_t id, ResWords<RB>& rw, f32x4 (&pv)[NQB]) {
    const int row = r < t.rows ? r : t.rows - 1;
    rw.load((t.flags & F_TOK) ? P.residuals + (t.tok0 + row) * ROWB + g * RB
                              : (const uint8_t*)zrow);
    const uint32_t idc = id < max_c ? id : max_c;
    const f32x4* src = (const f32x4*)(P.table + (__umul24(idc, ncols) + col0));
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) pv[nb] = src[4 * nb];
  };

  auto store = [&](int64_t pp, float v) {
    if (poison) v = __builtin_bit_cast(float, 0x7fc00000u);
    P.scores[has_cand ? pp : a * P.n_docs + pp] = v;
  };

  // running max per (query block, accumulator row) over this lane's document
  // rows; reduced over the 16 rows of the tile at the document's end
  f32x4 mx[NQB];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) mx[nb] = f32x4{-__builtin_inff(), -__builtin_inff(),
                                                  -__builtin_inff(), -__builtin_inff()};
  const char* lutb = (const char*)lut;

  // max over the 16 lanes of a row group (rotations by 8, 4, 2, 1)
  auto row_max = [](float v) {
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                               0, __builtin_bit_cast(int, v), 0x128, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                               0, __builtin_bit_cast(int, v), 0x124, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                               0, __builtin_bit_cast(int, v), 0x122, 0xF, 0xF, false)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                               0, __builtin_bit_cast(int, v), 0x121, 0xF, 0xF, false)));
    return v;
  };

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
      u32x4 bv;
      if constexpr (NBITS == 1) {
        bv = *(const u32x4*)(lutb + rw.byte_offset(s, EB_LOG2));
      } else if constexpr (NBITS == 2) {
        const uint2 lo = *(const uint2*)(lutb + rw.byte_offset(2 * s, EB_LOG2));
        const uint2 hi = *(const uint2*)(lutb + rw.byte_offset(2 * s + 1, EB_LOG2));
        bv = u32x4{lo.x, lo.y, hi.x, hi.y};
      } else {
        bv = u32x4{*(const uint32_t*)(lutb + rw.byte_offset(4 * s, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 1, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 2, EB_LOG2)),
                   *(const uint32_t*)(lutb + rw.byte_offset(4 * s + 3, EB_LOG2))};
      }
      const f16x8 bh = __builtin_bit_cast(f16x8, bv);
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qa[nb][s], bh, acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) mx[nb][v] = fmaxf(mx[nb][v], acc[nb][v]);
    if (t.flags & F_DLAST) {
      // max over the document's rows (lanes r), then the sum over query
      // tokens: per row position 4g + v over the blocks in order, then over
      // v and g in a fixed tree
      float sv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sv[v] += row_max(mx[nb][v]);
        mx[nb] = f32x4{-__builtin_inff(), -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      }
      const float qsum = sum_rows4((sv[0] + sv[1]) + (sv[2] + sv[3]));
      if (lane == 0) store(t.pp, qsum);
    }
  };

  // Software pipeline over S = PI + PR tile slots: a tile's ids are loaded
  // S tiles before it is consumed, its residual codes and table entries
  // (whose addresses need the ids) PR tiles before. Slot indices are
  // compile-time constants in the unrolled loop, so the ring stays in VGPRs.
  constexpr int S = PI + PR;
  Tile tq[S];
  uint32_t idq[S];
  ResWords<RB> rq[S];
  f32x4 pq[S][NQB];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    tq[k] = next_tile();
    load_ids(tq[k], idq[k]);
  }
#pragma unroll
  for (int k = 0; k < PR; ++k) load_rest(tq[k], idq[k], rq[k], pq[k]);
  // whole rounds of S steps: the tiles after a wave's last one carry no
  // flags, so their steps compute on zero rows and store nothing
  while (tq[0].flags & F_VALID) {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int jr = (j + PR) % S;
      load_rest(tq[jr], idq[jr], rq[jr], pq[jr]);
      consume(tq[j], rq[j], pq[j]);
      tq[j] = next_tile();
      load_ids(tq[j], idq[j]);
    }
  }
}

template <int NKS>
hipError_t launch_table_t(const ResParams& P, hipStream_t s) {
  const int64_t waves = (P.n_centroids + 15) / 16;
  hipLaunchKernelGGL(centroid_table_kernel<NKS>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                     s, P);
  return hipGetLastError();
}

template <int NBITS, int NKS, int NQB, int PI, int PR>
hipError_t launch_score_p(const ResParams& P, hipStream_t s) {
  constexpr int NW = 4;
  hipLaunchKernelGGL((residual_maxsim_kernel<NBITS, NKS, NQB, NW, PI, PR>),
                     dim3((unsigned)(P.n_q * P.n_chunks)), dim3(NW * 64), 0, s, P);
  return hipGetLastError();
}

// pipeline depths (ids lead, table/residual lead) of the selectable variants
template <int NBITS, int NKS, int NQB>
hipError_t launch_score_t(const ResParams& P, hipStream_t s) {
  switch (P.pipe) {
    case 0: return launch_score_p<NBITS, NKS, NQB, 1, 1>(P, s);
    case 1: return launch_score_p<NBITS, NKS, NQB, 1, 2>(P, s);
    case 2: return launch_score_p<NBITS, NKS, NQB, 2, 2>(P, s);
    default: return launch_score_p<NBITS, NKS, NQB, 2, 3>(P, s);
  }
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

// Device address of this file's zero row, per device (the kernels take it as
// an argument).
hipError_t zero_row_address(const char** out) {
  static std::mutex mu;
  static std::map<int, const char*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_zero_row));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, (const char*)p).first;
  }
  *out = it->second;
  return hipSuccess;
}

hipError_t launch_residual(const ResParams& Pin, hipStream_t s) {
  ResParams P = Pin;
  hipError_t e = zero_row_address(&P.zero_row);
  if (e != hipSuccess) return e;
  {
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
