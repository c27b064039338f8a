// fused_impl.h -- fused MaxSim scoring and the unfused (materialised S) comparator.
//
// Fused kernel: Algorithm 3 ("V2-MQ") of the paper with the query block equal
// to the whole query (BQ = Nq), so each document byte crosses HBM once
// (Theorem 1), re-designed for gfx950:
//   * a document tile is 16 rows x one d-chunk (DCH = 128, the paper's
//     dimension tiling; 64 when d is not a multiple of 128; 256 for 1- and
//     2-byte rows of d >= 512, the same k order in longer contiguous reads);
//     lane (r, g) = (lane % 16, lane / 16) consumes row r, bytes
//     [c*64 + g*16, +16) of the chunk for c < NL as its MFMA A operand, either
//     loaded straight into VGPRs or staged through a per-wave LDS ring by
//     non-temporal global_load_lds (STAGE); PF steps per wave are in flight;
//   * rows past a document's end are clamped to its last row: a duplicated
//     token never changes a max (Eq. 1), costs no HBM traffic (the line is
//     already in cache) and needs no -inf masking; the FP32 form, bound by
//     its matrix rate, fills them with the next document's rows instead and
//     splits the row max at the boundary;
//   * Q (B operand) lives in VGPRs when d fits one chunk, else in LDS in the
//     B-operand layout [query block nb][16-byte column group][lane], one copy
//     per wave or per workgroup; S_t^T = D_t Q^T runs on
//     v_mfma_f32_16x16x{32 f16/bf16, 128 f8f6f4, 4 f32}; the d-chunks of a
//     tile accumulate into the same FP32 registers before the max;
//   * FP8: per-token power-of-two scales go into the E8M0 scale operands of
//     v_mfma_scale_f32_16x16x128_f8f6f4 (doc row scale on A, query token
//     scale on B), which is exact for powers of two;
//   * the running max of query token n (= lane % 16 of block nb) is in-lane
//     over the 4 accumulator rows; at a document's end two xor-shuffles finish
//     the max over rows and four more sum a query's tokens; one lane stores
//     the score (no atomics, fixed order: bit-reproducible);
//   * without candidate lists, queries are grouped into units whose blocks
//     share every tile read (one document read for several queries);
//   * persistent grid: the (unit, doc) work list is cut into token-balanced
//     contiguous ranges, one per wave (64-ary wave search over the offsets).
#pragma once
#include "device_common.h"
#include "kernels.h"
#include "select_impl.h"

namespace fused_detail {

using ::DT_F32;
using ::DT_BF16;
using ::DT_F16;
using ::DT_FP8;

constexpr int F_VALID = 1, F_EMPTY = 2, F_TFIRST = 4, F_TLAST = 8, F_DLAST = 16, F_SPLIT = 32;
constexpr int SPLIT_SHIFT = 24;  // rows of the ending document in a split tile

// Work pair (unit, doc) where wave w of W starts: equal shares of the
// document tokens (every unit reads all of them), or of the candidate pairs.
__device__ int64_t wave_range_begin(const FusedParams& P, int64_t w, int64_t W) {
  if (w >= W) return P.n_upairs;
  if (P.cand_off != nullptr || P.tokens_per_query <= 0) {
    return (P.n_upairs / W) * w + ((P.n_upairs % W) * w) / W;
  }
  const int64_t T = P.tokens_per_query;
  const int64_t total = P.n_units * T;
  // tau = floor(w * total / W) without 128-bit arithmetic
  int64_t tau = (total / W) * w + ((total % W) * w) / W;
  int64_t a = tau / T;
  int64_t rem = tau - a * T;
  int64_t b = wave_lower_bound(P.d_off, P.n_docs, rem);
  return a * P.n_docs + b;
}

template <int DT, int NL>
__device__ __forceinline__ f32x4 mma_step(f32x4 acc, const u32x4 (&a)[NL], const u32x4 (&b)[NL],
                                          int sa, int sb) {
  if constexpr (DT == DT_F16) {
#pragma unroll
    for (int c = 0; c < NL; ++c)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a[c]),
                                                   __builtin_bit_cast(f16x8, b[c]), acc, 0, 0, 0);
  } else if constexpr (DT == DT_BF16) {
#pragma unroll
    for (int c = 0; c < NL; ++c)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[c]),
                                                    __builtin_bit_cast(bf16x8, b[c]), acc, 0, 0,
                                                    0);
  } else if constexpr (DT == DT_F32) {
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[c].x), __uint_as_float(b[c].x),
                                                 acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[c].y), __uint_as_float(b[c].y),
                                                 acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[c].z), __uint_as_float(b[c].z),
                                                 acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[c].w), __uint_as_float(b[c].w),
                                                 acc, 0, 0, 0);
    }
  } else {  // FP8: 32 bytes per lane per MFMA; an odd tail is zero-extended
#pragma unroll
    for (int c = 0; c < NL; c += 2) {
      u32x4 a1 = (c + 1 < NL) ? a[c + 1 < NL ? c + 1 : c] : u32x4{0, 0, 0, 0};
      u32x4 b1 = (c + 1 < NL) ? b[c + 1 < NL ? c + 1 : c] : u32x4{0, 0, 0, 0};
      i32x8 A = {(int)a[c].x, (int)a[c].y, (int)a[c].z, (int)a[c].w,
                 (int)a1.x,   (int)a1.y,   (int)a1.z,   (int)a1.w};
      i32x8 B = {(int)b[c].x, (int)b[c].y, (int)b[c].z, (int)b[c].w,
                 (int)b1.x,   (int)b1.y,   (int)b1.z,   (int)b1.w};
      acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(A, B, acc, 0, 0, 0, sa, 0, sb);
    }
  }
  return acc;
}

// The query (0 <= qa < n_q) behind block nb of unit u, or -1, and the row of
// that query the block's lane row r holds.
__device__ __forceinline__ int64_t unit_query(const FusedParams& P, int64_t u, int nb) {
  const int gq = nb / P.bpq;
  const int64_t qa = u * P.group + gq;
  return (gq < P.group && qa < P.n_q) ? qa : -1;
}

// Stage the NQB query blocks of unit u into LDS in the B-operand layout,
// threads t0, t0 + nthreads, ... of the caller's group doing the copy; rows
// past a query's end and columns past d (up to the whole last chunk) are zero.
template <int NQB>
__device__ void stage_unit(const FusedParams& P, int64_t u, u32x4* q_lds, int t0, int nthreads) {
  const int ncg = P.ncg;  // 64-byte column groups of the chunk-padded row
  const int total = NQB * ncg * 64;
  for (int idx = t0; idx < total; idx += nthreads) {
    int ln = idx & 63, rest = idx >> 6;
    int cg = rest % ncg, nb = rest / ncg;
    const int64_t qa = unit_query(P, u, nb);
    u32x4 v = {0, 0, 0, 0};
    if (qa >= 0) {
      const int64_t q0 = P.q_off[qa];
      const int nq = (int)(P.q_off[qa + 1] - q0);
      const int row = (nb % P.bpq) * 16 + (ln & 15);
      const int beta = cg * 4 + (ln >> 4);
      if (row < nq && beta * 16 < P.row_bytes)
        v = *(const u32x4*)(P.q_tok + (q0 + row) * P.row_bytes + beta * 16);
    }
    q_lds[idx] = v;
  }
}

// LDS bytes of the per-wave staging ring of the STAGE variant.
template <int DT, int DCH, int PF, int NW>
constexpr size_t stage_ring_bytes() {
  return (size_t)NW * PF * 16 * DCH * elem_size<DT>::value;
}

// s_waitcnt immediate for "at most n vector memory operations outstanding"
// (vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt left at their maxima).
constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }
// ... and for "no LDS (or scalar memory) operation outstanding", vmcnt and
// expcnt at their maxima
constexpr int lgkmcnt0_imm() { return 0xF | (0x3 << 14) | (0x7 << 4); }

// Fused top-k, after every wave of the workgroup has stored its keys: for
// each query with work pairs in the workgroup's range, the k best ranking keys
// of those pairs (exact radix select over the workgroup's contiguous key
// array, or over the wave key slots and the spill array for waves whose
// ranges did not fit them) go to the query's part slot.
// ranges[w], ranges[NW + w]: first and end work pair of wave w (contiguous).
template <int NW>
__device__ void topk_epilogue(const FusedParams& P, u32x4* lds, const int64_t* ranges) {
  using namespace topk_detail;
  const int k = P.topk_k, cap = P.sel_cap, G = P.group;
  uint64_t* buf = (uint64_t*)lds;
  uint32_t* hist = (uint32_t*)((char*)lds + (size_t)cap * 8);
  const uint32_t* lkeys = (const uint32_t*)((const char*)lds + P.lds_keys_off);
  const int key_slots = P.key_cap / NW;
  const int64_t lo = ranges[0], hi = ranges[2 * NW - 1];
  if (threadIdx.x == 0) P.wg_lo[blockIdx.x] = lo;
  if (lo >= hi) return;
  const bool dense = P.cand_off == nullptr;
  // keys in one contiguous array from the first pair (as the scorer stored them)
  const bool contig = (hi - lo) * G <= P.key_cap;
  int64_t a0, a1;  // units with pairs in [lo, hi)
  if (dense) {
    a0 = lo / P.n_docs;
    a1 = (hi - 1) / P.n_docs;
  } else {
    a0 = wave_owner(P.cand_off, P.n_q, lo);
    a1 = wave_owner(P.cand_off, P.n_q, hi - 1);
  }
  for (int64_t a = a0; a <= a1; ++a) {
    const int64_t s0 = dense ? a * P.n_docs : P.cand_off[a];
    const int64_t s1 = dense ? s0 + P.n_docs : P.cand_off[a + 1];
    const int64_t p0 = lo > s0 ? lo : s0, p1 = hi < s1 ? hi : s1;
    if (p0 >= p1) continue;
    for (int gq = 0; gq < G; ++gq) {
      if (a * G + gq >= P.n_q) break;
      auto get = [&](int64_t i) -> uint64_t {
        const int64_t p = p0 + i;
        const uint32_t id = dense ? (uint32_t)(p - s0) : (uint32_t)P.cand_ids[p];
        if (contig) return rank_key(lkeys[(p - lo) * G + gq], id);
        int w = 0;  // the wave whose range holds p: the last one starting at or before it
#pragma unroll
        for (int v = 1; v < NW; ++v)
          if (ranges[v] <= p) w = v;
        const int64_t wl = ranges[w], wh = ranges[NW + w];
        const uint32_t key = (wh - wl) * G <= key_slots ? lkeys[w * key_slots + (p - wl) * G + gq]
                                                        : P.key_spill[p * G + gq];
        return rank_key(key, id);
      };
      const int64_t slot = ((int64_t)blockIdx.x + a) * G + gq;
      const int cnt = block_topk(p1 - p0, k, get, hist, buf, cap, P.part_keys + slot * k);
      if (threadIdx.x == 0) P.part_cnt[slot] = (uint32_t)cnt;
    }
  }
}

// Where a wave's query operand lives (QM):
//   Q_SHARED  one LDS copy per workgroup (large d); the workgroup's waves
//             stage each query they cross together, with barriers;
//   Q_REGS    VGPRs, loaded by each wave itself (d fits one chunk);
//   Q_WAVE    one LDS copy per wave, staged by that wave alone.
// The per-wave forms need no barrier, so a wave never waits for the others
// when their ranges cross different queries.
constexpr int Q_SHARED = 0, Q_REGS = 1, Q_WAVE = 2;

template <int DT, int NQB, int DCH, int PF, int NW, int QM, bool STAGE, int RT = 16>
__global__ __launch_bounds__(NW * 64) void fused_maxsim_kernel(FusedParams P) {
  extern __shared__ u32x4 q_lds[];
  constexpr bool QREG = QM == Q_REGS;
  constexpr bool PERWAVE = QM != Q_SHARED;
  // RT: document rows per step. 32 (two 16-row MFMA tiles) doubles the bytes
  // each step moves for narrow rows (FP8 at d = 128: 2 KiB -> 4 KiB); staged
  // tiles with the query operand in VGPRs only.
  static_assert(RT == 16 || (RT == 32 && STAGE && QREG), "32-row steps: staged, Q in VGPRs");
  constexpr int SUB = RT / 16;
  constexpr int ESZ = elem_size<DT>::value;
  constexpr int CB = DCH * ESZ;  // bytes of one row within one chunk
  constexpr int NL = CB / 64;    // 16-byte loads per lane per step
  static_assert(NL >= 1, "chunk too narrow");
  // STAGE: each step's tile (16 rows x CB bytes) arrives in a per-wave LDS
  // ring through global_load_lds_dwordx4 (non-temporal): every wave
  // instruction moves 1 KiB of consecutive rows, the fastest way this device
  // streams HBM. Chunk p of tile row rho lands in LDS slot rho*CPR +
  // (p ^ swz(rho)), so the 16 rows an MFMA operand read touches fall in 16
  // different bank groups.
  constexpr int TILE = RT * CB;
  constexpr int CPR = CB / 16;                    // 16-byte chunks per tile row
  constexpr int SW = CPR < 16 ? CPR : 16;         // XOR width
  constexpr int SWD = 16 / SW;                    // rows sharing a bank-group offset
  constexpr int NLS = NL * SUB;                   // LDS-DMA instructions per step
  constexpr int LOADS_PER_FILL = (STAGE ? NLS : NL) + (DT == DT_FP8 ? SUB : 0);

  const int lane = lane_id();
  const int r = lane & 15, g = lane >> 4;
  const int wave = uniform(threadIdx.x >> 6);
  const char* const zrow = zero_row_ptr();
  const int nch = P.nch;
  const int ncg = P.ncg;

  const int64_t W = (int64_t)gridDim.x * NW;
  const int64_t wg0 = (int64_t)blockIdx.x * NW;
  const int64_t my_lo = uniform64(wave_range_begin(P, wg0 + wave, W));
  const int64_t my_hi = uniform64(wave_range_begin(P, wg0 + wave + 1, W));
  // segments: the query-sized pieces of the workgroup's range (shared Q) or
  // of this wave's own range (per-wave Q)
  int64_t pb = PERWAVE ? my_lo : uniform64(wave_range_begin(P, wg0, W));
  const int64_t pe = PERWAVE ? my_hi : uniform64(wave_range_begin(P, wg0 + NW, W));
  // this wave's query operand in LDS (shared: the workgroup's copy)
  u32x4* qw = q_lds + (QM == Q_WAVE ? (size_t)wave * NQB * ncg * 64 : 0);
  // fused top-k: when the workgroup's whole range fits the LDS key slots,
  // one contiguous array indexed from its first pair (the selection then
  // reads keys by position); else this wave's share of the slots when its
  // range fits them, else the spill array
  const int key_slots = P.key_cap / NW;
  const bool keys_in_lds = (my_hi - my_lo) * P.group <= key_slots;
  uint32_t* const wg_keys = (uint32_t*)((char*)q_lds + P.lds_keys_off);
  uint32_t* const wave_keys = wg_keys + wave * key_slots;
  // the wave ranges, published next to the key slots (read by the
  // selection at the end as well)
  int64_t* const ranges = (int64_t*)((char*)q_lds + P.lds_keys_off + (size_t)P.key_cap * 4);
  int64_t wg_lo = 0;
  bool keys_contig = false;
  if (P.topk_k > 0) {
    if (lane == 0) {
      ranges[wave] = my_lo;
      ranges[NW + wave] = my_hi;
    }
    __syncthreads();
    wg_lo = uniform64(ranges[0]);
    keys_contig = (uniform64(ranges[2 * NW - 1]) - wg_lo) * P.group <= P.key_cap;
  }

  while (pb < pe) {
    int64_t a, qend;  // a: the unit (with candidate lists: the query)
    if (P.cand_off == nullptr) {
      a = pb / P.n_docs;
      qend = (a + 1) * P.n_docs;
    } else {
      a = uniform64(wave_owner(P.cand_off, P.n_q, pb));
      qend = P.cand_off[a + 1];
    }
    const int64_t se = qend < pe ? qend : pe;
    if constexpr (QM == Q_SHARED) {
      __syncthreads();
      stage_unit<NQB>(P, a, q_lds, threadIdx.x, NW * 64);
      __syncthreads();
    } else if constexpr (QM == Q_WAVE) {
      // the wave's own LDS ops complete in order; the fence keeps the
      // compiler from moving the operand reads above the staging writes
      __builtin_amdgcn_wave_barrier();
      stage_unit<NQB>(P, a, qw, lane, 64);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // per query gq of the unit, in one word: bit gq = exists, bit 8 + gq =
    // has tokens, bit 16 + gq = exceeds the caller's length bound (then its
    // scores are NaN: never an overrun)
    // (a unit holds at most 8 queries: the host never groups more)
    constexpr int NG = NQB < 8 ? NQB : 8;
    const int bpq = P.bpq;
    uint32_t qmask = 0;
#pragma unroll
    for (int gq = 0; gq < NG; ++gq) {
      const int64_t qa = a * P.group + gq;
      if (gq < P.group && qa < P.n_q) {
        const int n = (int)(P.q_off[qa + 1] - P.q_off[qa]);
        qmask |= 1u << gq;
        if (n > 0) qmask |= 1u << (8 + gq);
        if (n > bpq * 16) qmask |= 1u << (16 + gq);
      }
    }
    qmask = __builtin_amdgcn_readfirstlane(qmask);

    int64_t lo = my_lo > pb ? my_lo : pb;
    const int64_t hi = my_hi < se ? my_hi : se;
    const int64_t pair_base = (P.cand_off == nullptr) ? a * P.n_docs : 0;

    // Query operand registers (one d-chunk, loaded by the wave itself) and
    // FP8 query scales, block nb from query unit_query(a, nb).
    u32x4 qreg[QREG ? NQB : 1][NL];
    int qsc[NQB];
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) {
      const int64_t qa = unit_query(P, a, nb);
      int64_t q0 = 0;
      int nq = 0;
      if (qa >= 0) {
        q0 = P.q_off[qa];
        nq = (int)(P.q_off[qa + 1] - q0);
      }
      const int row = (nb % bpq) * 16 + r;
      if constexpr (QREG) {
        const char* qrow = P.q_tok + (q0 + row) * P.row_bytes + g * 16;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
          u32x4 v = {0u, 0u, 0u, 0u};  // zero past the query's end and past d
          if (row < nq && c * 64 + g * 16 < P.row_bytes) v = *(const u32x4*)(qrow + c * 64);
          qreg[nb][c] = v;
        }
      }
      qsc[nb] = 127;
      if constexpr (DT == DT_FP8) {
        if (row < nq) qsc[nb] = e8m0_of(P.q_scales[q0 + row]);
      }
    }
    // score index of query gq of the unit for work pair pp: pp + sbase +
    // gq * n_docs (with candidate lists the unit is one query, sbase 0)
    const int64_t sbase = (P.cand_off == nullptr) ? a * (P.group - 1) * P.n_docs : 0;
    // Top-k ranking keys are buffered one per lane and written 64 at a time
    // (one LDS store instruction per 64 documents instead of one per
    // document, which measured about 3.5% slower at one wave per SIMD).
    // Entry e = pair * group + query of the unit; lane j holds entry
    // kb_e0 + j. Consecutive entries have consecutive slots in each of the
    // three key homes, so a run of buffered entries is one contiguous write.
    uint32_t kb = 0u;
    int kb_n = 0;
    int64_t kb_e0 = 0;
    auto key_flush = [&]() {
      if (kb_n == 0) return;
      if (lane < kb_n) {
        const int64_t e = kb_e0 + lane;
        if (keys_contig)
          wg_keys[e - wg_lo * P.group] = kb;
        else if (keys_in_lds)
          wave_keys[e - my_lo * P.group] = kb;
        else
          P.key_spill[e] = kb;
      }
      kb_n = 0;
    };
    // Whole wave; the score is lane 0's (after the row sums every lane holds
    // the sum, lane 0 in the order the result is defined by).
    auto store = [&](int64_t pp, int gq, float v) {
      v = __builtin_bit_cast(float,
                             __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
      // (NaN as a bit pattern: this file is compiled assuming no NaN arithmetic)
      if ((qmask >> (16 + gq)) & 1u) v = __builtin_bit_cast(float, 0x7fc00000u);
      if (P.topk_k > 0) {
        const int64_t e = pp * P.group + gq;
        if (kb_n == 64 || (kb_n > 0 && e != kb_e0 + kb_n)) key_flush();
        if (kb_n == 0) kb_e0 = e;
        const uint32_t key = topk_detail::score_key(v);
        kb = lane == kb_n ? key : kb;
        ++kb_n;
      } else if (lane == 0) {
        P.scores[pp + sbase + (int64_t)gq * P.n_docs] = v;
      }
    };

    // ---- prefetch cursor over the (pair, tile, chunk) steps of [lo, hi) ----
    // Document offsets (and candidate ids) are read with scalar loads from
    // the constant address space, one document ahead: they are counted by
    // lgkmcnt, so waiting for them never waits for the tile loads in flight.
    const bool has_cand = P.cand_off != nullptr;
    const int64_t* __restrict__ doff = P.d_off;
    auto doc_of = [&](int64_t p, int nxt_id) -> int64_t {
      return has_cand ? (int64_t)nxt_id : p - pair_base;
    };
    // Packed tiles (FP32, one chunk per tile, no candidate lists): the
    // matrix cores bound the FP32 form, and clamping a document's last,
    // partial tile to its last row spends about 11% of them on duplicate
    // rows. Instead, when the next document (the next one in memory) runs
    // past the tile, the tile takes its first rows, and the consumer splits
    // the row max at the boundary: the ending document's rows go to its
    // score, the rest start the next document's running max (cbase = rows
    // of the document already scored that way). Every row's dot product is
    // the same MFMA output either way, so the scores are the same bits.
    constexpr bool PACK = DT == DT_F32 && QREG && RT == 16;
    const bool pack = PACK && !has_cand;
    int64_t cp = lo;  // cursor pair
    int64_t ct0 = 0;
    int cnd = 0, ctile = 0, cchunk = 0, cbase = 0;
    int64_t nx_s = 0, nx_e = 0;  // offsets of pair cp + 1 (raw)
    int nx2_id = 0;              // candidate id of pair cp + 2
    if (cp < hi) {
      int id0 = has_cand ? sload_i32(P.cand_ids, cp) : 0;
      int64_t b0 = doc_of(cp, id0);
      ct0 = sload_i64(doff, b0);
      cnd = (int)(sload_i64(doff, b0 + 1) - ct0);
      if (cp + 1 < hi) {
        int id1 = has_cand ? sload_i32(P.cand_ids, cp + 1) : 0;
        int64_t b1 = doc_of(cp + 1, id1);
        nx_s = sload_i64(doff, b1);
        nx_e = sload_i64(doff, b1 + 1);
      }
      if (has_cand && cp + 2 < hi) nx2_id = sload_i32(P.cand_ids, cp + 2);
    }

    auto next_pair = [&]() {
      ++cp;
      ctile = 0;
      cchunk = 0;
      cbase = 0;
      ct0 = nx_s;
      cnd = (int)(nx_e - nx_s);
      if (cp + 1 < hi) {
        int64_t b1 = doc_of(cp + 1, nx2_id);
        nx_s = sload_i64(doff, b1);
        nx_e = sload_i64(doff, b1 + 1);
        if (has_cand && cp + 2 < hi) nx2_id = sload_i32(P.cand_ids, cp + 2);
      }
    };

    u32x4 buf[STAGE ? 1 : PF][NL];
    int bsc[PF][SUB];
    int flags[PF];
    int64_t fp[PF];
    constexpr int Q_COPIES = QM == Q_SHARED ? 1 : (QM == Q_WAVE ? NW : 0);
    char* ring =
        (char*)q_lds + (size_t)Q_COPIES * NQB * 16 * ncg * 64 + (size_t)wave * PF * TILE;
    auto swz = [](int row) { return (row / SWD) & (SW - 1); };

    // Every fill issues exactly NL (+1 for FP8) loads, from a harmless address
    // when there is nothing left to load, so the compiler's vmcnt accounting
    // sees a fixed depth of PF steps in flight. Columns of the last chunk past
    // d are read from the row's last 16 bytes instead (inside the row; the
    // query operand is zero there, so they add exact zeros).
    auto fill = [&](const int s) {
      int f = 0;
      const char* base = zrow;
      const bool live = cp < hi && cnd != 0;
      const int rb = (PACK ? cbase : 0) + ctile * RT;  // first document row of this step
      // packed: this document's rows in the tile (1-15), the rest the next one's
      int ra = 0;
      if (PACK && pack && live && rb + RT > cnd && cp + 1 < hi && nx_e - nx_s > RT - (cnd - rb))
        ra = cnd - rb;
      // largest in-row offset from this step's chunk start (idle: none needed)
      const int cmax = live ? P.row_bytes - 16 - cchunk * CB : CB;
      fp[s] = cp;
      if (cp < hi) {
        if (cnd == 0) {
          f = F_VALID | F_EMPTY;
        } else {
          int row = rb + r;
          if (ra == 0) row = row < cnd ? row : cnd - 1;
          base = P.d_tok + (ct0 + row) * P.row_bytes + cchunk * CB;
          f = F_VALID | (cchunk == 0 ? F_TFIRST : 0) | (cchunk << 8);
          if (cchunk == nch - 1) {
            f |= F_TLAST;
            if (rb + RT >= cnd) f |= F_DLAST;
            if (ra != 0) f |= F_SPLIT | (ra << SPLIT_SHIFT);
          }
        }
      }
      if constexpr (STAGE) {
        // uniform tile base + per-lane 32-bit offset; an idle fill reads row
        // 0 of the zero block (offsets stay below CB <= 1 KiB)
        const char* tb = zrow;
        int lim = 0;
        if (live) {
          tb = P.d_tok + (ct0 + rb) * P.row_bytes + cchunk * CB;
          lim = ra != 0 ? RT - 1 : cnd - 1 - rb;
        }
        char* slot = ring + s * TILE;
#pragma unroll
        for (int w = 0; w < NLS; ++w) {
          const int ch = 64 * w + lane;  // LDS slot of this lane's 16 bytes
          const int rho = ch / CPR, p = ch % CPR;
          const int col = (p ^ swz(rho)) * 16;
          const unsigned off =
              (unsigned)((rho < lim ? rho : lim) * P.row_bytes + (col < cmax ? col : cmax));
          __builtin_amdgcn_global_load_lds((const void*)(tb + off),
                                           (__attribute__((address_space(3))) void*)(slot + w * 1024),
                                           16, 0, 2 /* non-temporal */);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NL; ++c) {
          const int col = c * 64 + g * 16;
          buf[s][c] = *(const u32x4*)(base + (col < cmax ? col : cmax));
        }
      }
#pragma unroll
      for (int h = 0; h < SUB; ++h) {
        if constexpr (DT == DT_FP8) {
          const float* sptr = (const float*)zrow;
          if (live) {
            int row = rb + h * 16 + r;
            row = row < cnd ? row : cnd - 1;
            sptr = P.d_scales + ct0 + row;
          }
          bsc[s][h] = e8m0_of(*sptr);
        } else {
          bsc[s][h] = 127;
        }
      }
      flags[s] = f;
      if (cp < hi) {
        if (cnd == 0) {
          next_pair();
        } else if (++cchunk == nch) {
          cchunk = 0;
          ++ctile;
          if (ra != 0) {
            next_pair();
            cbase = RT - ra;
          } else if (rb + RT >= cnd) {
            next_pair();
          }
        }
      }
    };

    f32x4 acc[NQB];
    float mx[NQB];
    float mxn[PACK ? NQB : 1];  // packed: the next document's rows of a split tile
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) {
      acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      mx[nb] = -__builtin_inff();
    }

    // document end: per query, max over the 16 rows (two row swaps per
    // block), sum over its blocks and then its 16 columns (four DPP
    // rotations); register to register, so a wave alone on its SIMD keeps
    // issuing (with LDS shuffles here a launch measured up to 7% slower)
    auto finalize = [&](int64_t pp) {
      float tot = 0.f;
#pragma unroll
      for (int nb = 0; nb < NQB; ++nb) {
        tot += max_rows4(mx[nb]);
        mx[nb] = -__builtin_inff();
        if ((nb + 1) % bpq == 0) {
          const int gq = nb / bpq;
          if ((qmask >> gq) & 1u) store(pp, gq, row_sum16(tot));
          tot = 0.f;
        }
      }
    };

    // A one-chunk tile's MFMA result t for query block nb into the running
    // maxima; in a split tile, rows 4g + i below ra end this document and
    // the rest start the next one.
    auto tile_max = [&](const int nb, const f32x4 t, const int fl) {
      if (PACK && (fl & F_SPLIT)) {
        const int ra = fl >> SPLIT_SHIFT;
        float a = -__builtin_inff(), b = -__builtin_inff();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (4 * g + i < ra)
            a = fmaxf(a, t[i]);
          else
            b = fmaxf(b, t[i]);
        }
        mx[nb] = fmaxf(mx[nb], a);
        mxn[nb] = b;
      } else {
        mx[nb] = fmaxf(mx[nb], fmaxf(fmaxf(t.x, t.y), fmaxf(t.z, t.w)));
      }
    };
    // after a step: a document that ends in it is scored; a split tile's
    // rows of the next document become that document's running maxima
    auto end_step = [&](const int fl, const int64_t pp) {
      if (PACK && (fl & F_SPLIT)) {
        finalize(pp);
#pragma unroll
        for (int nb = 0; nb < NQB; ++nb) mx[nb] = mxn[nb];
      } else if (fl & F_DLAST) {
        finalize(pp);
      }
    };

    auto consume = [&](const int s) {
      const int fl = flags[s], sc = bsc[s][0];
      const int64_t pp = fp[s];
      if (!(fl & F_VALID)) return;
      if (fl & F_EMPTY) {
        for (int gq = 0; gq < NG; ++gq)
          if ((qmask >> gq) & 1u)
            store(pp, gq, ((qmask >> (8 + gq)) & 1u) ? -__builtin_inff() : 0.f);
        return;
      }
      u32x4 bb[NL];
      if constexpr (STAGE) {
        // every later fill issued LOADS_PER_FILL vector memory operations
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((PF - 1) * LOADS_PER_FILL));
      }
      if constexpr (QREG) {
        // one chunk per tile: every step starts and ends its tiles
#pragma unroll
        for (int h = 0; h < SUB; ++h) {
          if constexpr (STAGE) {
            const char* slot = ring + s * TILE;
            const int row = h * 16 + r;
#pragma unroll
            for (int c = 0; c < NL; ++c)
              bb[c] = *(const u32x4*)(slot + (row * CPR + ((c * 4 + g) ^ swz(row))) * 16);
          } else {
#pragma unroll
            for (int c = 0; c < NL; ++c) bb[c] = buf[s][c];
          }
#pragma unroll
          for (int nb = 0; nb < NQB; ++nb)
            tile_max(nb,
                     mma_step<DT, NL>(f32x4{0.f, 0.f, 0.f, 0.f}, bb, qreg[nb], bsc[s][h], qsc[nb]),
                     fl);
        }
      } else {
        if constexpr (STAGE) {
          const char* slot = ring + s * TILE;
#pragma unroll
          for (int c = 0; c < NL; ++c)
            bb[c] = *(const u32x4*)(slot + (r * CPR + ((c * 4 + g) ^ swz(r))) * 16);
        } else {
#pragma unroll
          for (int c = 0; c < NL; ++c) bb[c] = buf[s][c];
        }
        const int chunk = fl >> 8;
        const bool first = (fl & F_TFIRST) != 0;
#pragma unroll
        for (int nb = 0; nb < NQB; ++nb) {
          u32x4 qb[NL];
#pragma unroll
          for (int c = 0; c < NL; ++c) qb[c] = qw[(nb * ncg + chunk * NL + c) * 64 + lane];
          f32x4 base = first ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[nb];
          acc[nb] = mma_step<DT, NL>(base, bb, qb, sc, qsc[nb]);
        }
        if (fl & F_TLAST) {
#pragma unroll
          for (int nb = 0; nb < NQB; ++nb) {
            f32x4 t = acc[nb];
            mx[nb] = fmaxf(mx[nb], fmaxf(fmaxf(t.x, t.y), fmaxf(t.z, t.w)));
          }
        }
      }
      end_step(fl, pp);
    };

    // The arithmetic-heaviest forms (eight query blocks over LDS-staged
    // 2-byte tiles; FP32, whose 16x16x4 MFMAs take the longest per byte)
    // split a step in two: take() copies the slot's flags, pair and tile rows
    // into registers, fill() reuses the slot at once, and compute() runs the
    // MFMAs, maxima and document epilogue while the refill is in flight, so
    // PF steps rather than PF - 1 stay in flight during the arithmetic
    // (measured about 3% faster for eight FP16 blocks, 0.6% for FP32; for
    // fewer blocks, FP8 and register-direct tiles the refill after consume()
    // is as fast or faster).
    constexpr bool EARLY = STAGE && QREG && RT == 16 &&
                           ((NQB == 8 && (DT == DT_F16 || DT == DT_BF16)) || DT == DT_F32);
    auto take = [&](const int s, u32x4 (&bb)[NL], int& fl, int64_t& pp) {
      fl = flags[s];
      pp = fp[s];
      // every later fill issued LOADS_PER_FILL vector memory operations; the
      // wait is on every path, so the compiler's own accounting also sees the
      // segment's query operand loads complete before any MFMA
      __builtin_amdgcn_s_waitcnt(vmcnt_imm((PF - 1) * LOADS_PER_FILL));
      if (!(fl & F_VALID) || (fl & F_EMPTY)) return;
      const char* slot = ring + s * TILE;
#pragma unroll
      for (int c = 0; c < NL; ++c)
        bb[c] = *(const u32x4*)(slot + (r * CPR + ((c * 4 + g) ^ swz(r))) * 16);
      // the slot's LDS reads complete before its refill can land
      __builtin_amdgcn_s_waitcnt(lgkmcnt0_imm());
    };
    auto compute = [&](const u32x4 (&bb)[NL], const int fl, const int64_t pp) {
      if (!(fl & F_VALID)) return;
      if (fl & F_EMPTY) {
        for (int gq = 0; gq < NG; ++gq)
          if ((qmask >> gq) & 1u)
            store(pp, gq, ((qmask >> (8 + gq)) & 1u) ? -__builtin_inff() : 0.f);
        return;
      }
      if constexpr (EARLY) {
#pragma unroll
        for (int nb = 0; nb < NQB; ++nb)
          tile_max(nb, mma_step<DT, NL>(f32x4{0.f, 0.f, 0.f, 0.f}, bb, qreg[nb], 127, 127), fl);
      }
      end_step(fl, pp);
    };

#pragma unroll
    for (int s = 0; s < PF; ++s) fill(s);

    if (flags[0] & F_VALID) {
      while (true) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
          if constexpr (EARLY) {
            u32x4 bb[NL];
            int fl;
            int64_t pp;
            take(s, bb, fl, pp);
            fill(s);
            compute(bb, fl, pp);
          } else {
            consume(s);
            fill(s);
          }
        }
        // slots are filled in order: an invalid refill of slot 0 means the
        // cursor was exhausted before this round's refills, and every valid
        // slot has now been consumed
        if (!(flags[0] & F_VALID)) break;
      }
    }
    // the idle refills still target this wave's ring: let them land before
    // the next segment's fills reuse the slots
    if constexpr (STAGE) __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    key_flush();
    pb = se;
  }

  if (P.topk_k > 0) {
    // once every wave is done the query operand and ring area is free for
    // the selection
    __syncthreads();
    topk_epilogue<NW>(P, q_lds, ranges);
  }
}

// ---------------------------------------------------------------------------
// Unfused comparator, step 1: S[a][t][n] = sum_k d_tk q_an (FP32, to HBM).
// Each wave takes a contiguous run of 16-row tiles of the document tokens,
// streams them through an LDS ring as the fused scorer does, contracts them
// with query a (blockIdx.y, staged in LDS) and writes the tiles' S rows with
// non-temporal stores that cover whole rows.
// ---------------------------------------------------------------------------
// The comparator's query operand: block nb's MFMA column c holds query token
// c * NQB + nb, so a lane's NQB accumulators of one S row are NQB adjacent
// columns and one tile row is written by 16 lanes as one contiguous run.
template <int NQB>
__device__ void stage_query_interleaved(const FusedParams& P, int64_t a, u32x4* q_lds, int t0,
                                        int nthreads) {
  const int ncg = P.ncg;
  const int total = NQB * ncg * 64;
  const int64_t q0 = P.q_off[a];
  const int nq = (int)(P.q_off[a + 1] - q0);
  for (int idx = t0; idx < total; idx += nthreads) {
    const int ln = idx & 63, rest = idx >> 6;
    const int cg = rest % ncg, nb = rest / ncg;
    const int tok = (ln & 15) * NQB + nb;
    const int beta = cg * 4 + (ln >> 4);
    u32x4 v = {0, 0, 0, 0};
    if (tok < nq && beta * 16 < P.row_bytes)
      v = *(const u32x4*)(P.q_tok + (q0 + tok) * P.row_bytes + beta * 16);
    q_lds[idx] = v;
  }
}

template <int N>
struct f32vec;
template <>
struct f32vec<1> {
  typedef float type;
};
template <>
struct f32vec<2> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct f32vec<4> {
  typedef float type __attribute__((ext_vector_type(4)));
};

template <int DT, int NQB, int DCH, int NW, int PF>
__global__ __launch_bounds__(NW * 64) void sim_matrix_kernel(FusedParams P, float* S) {
  extern __shared__ u32x4 q_lds[];
  constexpr int ESZ = elem_size<DT>::value;
  constexpr int CB = DCH * ESZ;  // bytes of one row within one chunk
  constexpr int NL = CB / 64;    // 16-byte operand reads per lane per step
  constexpr int NQP = NQB * 16;
  constexpr int TILE = 16 * CB;
  constexpr int CPR = CB / 16;             // 16-byte pieces per tile row
  constexpr int SW = CPR < 16 ? CPR : 16;  // XOR width
  constexpr int SWD = 16 / SW;             // rows sharing a bank-group offset
  constexpr int NLS = TILE / 1024;         // LDS-DMA instructions per step
  constexpr int LOADS_PER_FILL = NLS + (DT == DT_FP8 ? 1 : 0);
  static_assert(TILE % 1024 == 0, "a step is whole 1 KiB DMA rounds");
  typedef typename f32vec<NQB>::type outv;
  const int lane = lane_id();
  const int r = lane & 15, g = lane >> 4;
  const int wave = uniform(threadIdx.x >> 6);
  const int64_t a = blockIdx.y;
  const int64_t T = P.tokens_per_query;
  const int64_t ntiles = (T + 15) / 16;
  const int ncg = P.ncg;
  const int nch = P.nch;

  stage_query_interleaved<NQB>(P, a, q_lds, threadIdx.x, NW * 64);
  const int nq = uniform((int)(P.q_off[a + 1] - P.q_off[a]));
  __syncthreads();  // the only barrier: every wave passes it before any exits
  int qsc[NQB];
#pragma unroll
  for (int nb = 0; nb < NQB; ++nb) {
    qsc[nb] = 127;
    if constexpr (DT == DT_FP8) {
      const int tok = r * NQB + nb;
      if (tok < nq) qsc[nb] = e8m0_of(P.q_scales[P.q_off[a] + tok]);
    }
  }
  float* Sa = S + a * T * NQP;
  // this wave's contiguous share of the tiles
  const int64_t W = (int64_t)gridDim.x * NW, w = (int64_t)blockIdx.x * NW + wave;
  const int64_t tile_lo = (ntiles / W) * w + ((ntiles % W) * w) / W;
  const int64_t tile_hi = (ntiles / W) * (w + 1) + ((ntiles % W) * (w + 1)) / W;
  if (tile_lo >= tile_hi) return;

  // Each (tile, chunk) step arrives in a per-wave LDS ring by non-temporal
  // global_load_lds (1 KiB of consecutive row bytes per instruction); piece
  // p of tile row rho lands at rho * CPR + (p ^ swz(rho)), so the operand
  // reads (lane (r, g) takes row r) hit 16 different bank groups. Rows past
  // T repeat row T - 1 and columns past d repeat the row's last 16 bytes
  // (the query operand is zero there); rows past T are not stored.
  char* ring = (char*)q_lds + (size_t)NQB * ncg * 1024 + (size_t)wave * PF * TILE;
  auto swz = [](int row) { return (row / SWD) & (SW - 1); };
  int64_t ct = tile_lo;  // fill cursor: tile and chunk
  int cc = 0;
  int64_t ftile[PF];
  int fchunk[PF], fsc[PF];
  bool flive[PF];
  const char* const zrow = zero_row_ptr();
  auto fill = [&](const int sl) {
    const bool live = ct < tile_hi;
    const char* tb = zrow;
    int lim = 0, cmax = CB;
    if (live) {
      tb = P.d_tok + ct * 16 * P.row_bytes + cc * CB;
      const int64_t left = T - 1 - ct * 16;
      lim = left < 15 ? (int)left : 15;
      cmax = P.row_bytes - 16 - cc * CB;
    }
    char* slot = ring + sl * TILE;
#pragma unroll
    for (int i = 0; i < NLS; ++i) {
      const int ch = 64 * i + lane;
      const int rho = ch / CPR, p = ch % CPR;
      const int col = (p ^ swz(rho)) * 16;
      const unsigned off =
          (unsigned)((rho < lim ? rho : lim) * P.row_bytes + (col < cmax ? col : cmax));
      __builtin_amdgcn_global_load_lds((const void*)(tb + off),
                                       (__attribute__((address_space(3))) void*)(slot + i * 1024),
                                       16, 0, 2 /* non-temporal */);
    }
    if constexpr (DT == DT_FP8) {
      const float* sp = (const float*)zrow;
      if (live) sp = P.d_scales + ct * 16 + (r < lim ? r : lim);
      fsc[sl] = e8m0_of(*sp);
    } else {
      fsc[sl] = 127;
    }
    flive[sl] = live;
    ftile[sl] = ct;
    fchunk[sl] = cc;
    if (live && ++cc == nch) {
      cc = 0;
      ++ct;
    }
  };

  f32x4 acc[NQB];
  auto consume = [&](const int sl) {
    // every later fill issued LOADS_PER_FILL vector memory operations
    __builtin_amdgcn_s_waitcnt(vmcnt_imm((PF - 1) * LOADS_PER_FILL));
    if (!flive[sl]) return;
    const char* slot = ring + sl * TILE;
    const int ch = fchunk[sl];
    u32x4 bb[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c)
      bb[c] = *(const u32x4*)(slot + (r * CPR + ((c * 4 + g) ^ swz(r))) * 16);
#pragma unroll
    for (int nb = 0; nb < NQB; ++nb) {
      u32x4 qb[NL];
#pragma unroll
      for (int c = 0; c < NL; ++c) qb[c] = q_lds[(nb * ncg + ch * NL + c) * 64 + lane];
      const f32x4 base = ch == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[nb];
      acc[nb] = mma_step<DT, NL>(base, bb, qb, fsc[sl], qsc[nb]);
    }
    if (ch == nch - 1) {
      // lane (r, g) holds S rows 4g..4g+3, columns r*NQB .. r*NQB + NQB - 1:
      // one non-temporal store per row, the 16 lanes of a row writing its
      // NQP columns contiguously
      const int64_t tile = ftile[sl];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t orow = tile * 16 + 4 * g + i;
        outv v;
        if constexpr (NQB == 1) {
          v = acc[0][i];
        } else {
#pragma unroll
          for (int nb = 0; nb < NQB; ++nb) v[nb] = acc[nb][i];
        }
        if (orow < T) __builtin_nontemporal_store(v, (outv*)(Sa + orow * NQP + r * NQB));
      }
    }
  };

#pragma unroll
  for (int sl = 0; sl < PF; ++sl) fill(sl);
  while (true) {
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      consume(sl);
      fill(sl);
    }
    // slots are filled in order: a dead refill of slot 0 means every live
    // slot has now been consumed
    if (!flive[0]) break;
  }
  // the idle refills target this wave's ring: let them land before exit
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
}

// Unfused comparator, step 2: read S back, max over each document's rows,
// sum over the query tokens. One wave per (query, doc) pair: the document's
// rows of S are one contiguous block, read with 16-byte non-temporal loads
// (lane l: row l / LPR of each group of RPL rows, columns 4 (l % LPR) ..
// + 3), U loads in flight; rows past the document's end repeat its last row.
template <int NQP>
__global__ __launch_bounds__(256) void seg_maxsum_kernel(FusedParams P, const float* S) {
  constexpr int LPR = NQP / 4;   // lanes per S row
  constexpr int RPL = 64 / LPR;  // rows per wave load
  constexpr int U = 4;           // loads in flight per lane
  const int lane = lane_id();
  const int cg = lane % LPR, rsub = lane / LPR;
  const int64_t T = P.tokens_per_query;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < P.n_pairs; p += nw) {
    const int64_t a = p / P.n_docs, b = p - a * P.n_docs;
    const int nq = (int)(P.q_off[a + 1] - P.q_off[a]);
    const int64_t t0 = P.d_off[b], t1 = P.d_off[b + 1];
    const f32x4* Sa = (const f32x4*)(S + a * T * NQP);
    f32x4 m = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    for (int64_t t = t0; t < t1; t += RPL * U) {
      f32x4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int64_t tt = t + u * RPL + rsub;
        tt = tt < t1 ? tt : t1 - 1;
        v[u] = __builtin_nontemporal_load(Sa + tt * LPR + cg);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        m.x = fmaxf(m.x, v[u].x);
        m.y = fmaxf(m.y, v[u].y);
        m.z = fmaxf(m.z, v[u].z);
        m.w = fmaxf(m.w, v[u].w);
      }
    }
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1) {
      m.x = fmaxf(m.x, xor_shfl(m.x, off));
      m.y = fmaxf(m.y, xor_shfl(m.y, off));
      m.z = fmaxf(m.z, xor_shfl(m.z, off));
      m.w = fmaxf(m.w, xor_shfl(m.w, off));
    }
    float v = (m.x + m.y) + (m.z + m.w);
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) v += xor_shfl(v, off);
    if (lane == 0) P.scores[p] = (nq == 0) ? 0.f : (t1 == t0 ? -__builtin_inff() : v);
  }
}

}  // namespace fused_detail

