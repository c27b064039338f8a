// topk.hip -- exact per-segment top-k by (score descending, id ascending).
//
// Every entry maps to a 64-bit key that orders exactly like the required
// ranking: the high 32 bits are the score's bits made order-preserving as an
// unsigned integer (NaN -> 0, below -inf), the low 32 bits are ~id so smaller
// ids rank higher. Five launches:
//   init     zero the per-segment histograms and counters;
//   hist0    4096-bin histogram of the top 12 key bits (LDS, then global);
//   hist1    each block re-derives the bin b0 holding the k-th largest entry
//            from hist0, then histograms the next 12 bits of the entries in
//            b0; this fixes a 24-bit prefix P;
//   compact  entries whose top 24 bits exceed P are certainly selected
//            (fewer than k of them); entries equal to P form the boundary
//            set, copied to a buffer of BOUND_CAP keys;
//   sort     one workgroup per segment sorts the selected and boundary keys
//            with a bitonic network in LDS and writes the first k. If the
//            boundary set overflowed its buffer (massive exact ties), the
//            workgroup instead finishes the selection with 8-bit radix passes
//            over the segment, which is slower but exact.
// Integer keys only: the result is exact and independent of launch shape.
#include "device_common.h"
#include "kernels.h"
#include "select_impl.h"

namespace {

using topk_detail::bitonic_desc;
using topk_detail::key_score;
using topk_detail::score_key;

constexpr int TK_THREADS = 256;
constexpr int TK_SORT_THREADS = 1024;
constexpr int TK_MAXK = 1024;
constexpr int BOUND_CAP = 4096;
constexpr int SORT_CAP = 8192;  // >= TK_MAXK + BOUND_CAP, power of two

struct SegWs {
  uint32_t hist0[4096];
  uint32_t hist1[4096];
  uint32_t n_above;  // entries with a 24-bit prefix above P
  uint32_t n_bound;  // entries with prefix P (may exceed BOUND_CAP)
  uint32_t prefix;   // P
  uint32_t rem;      // how many boundary entries belong to the top k
  uint32_t pad[4];
  // followed by uint64 above[TK_MAXK] and uint64 bound[BOUND_CAP]
};

__host__ __device__ inline size_t seg_ws_bytes() {
  size_t b = sizeof(SegWs) + (size_t)(TK_MAXK + BOUND_CAP) * 8;
  return (b + 255) & ~(size_t)255;
}

__device__ __forceinline__ uint64_t full_key(uint32_t sk, const int32_t* ids, int64_t i,
                                             int64_t start) {
  uint32_t id = ids ? (uint32_t)ids[i] : (uint32_t)(i - start);
  return ((uint64_t)sk << 32) | (uint64_t)(0xFFFFFFFFu - id);
}

__device__ __forceinline__ SegWs* seg_ws(void* ws, int64_t s) {
  return (SegWs*)((char*)ws + (size_t)s * seg_ws_bytes());
}

// Block-wide: the bin holding the rem-th largest entry of a 4096-bin
// histogram, and how many entries lie in higher bins. Every thread returns
// the same values.
__device__ void select_bin(const uint32_t* __restrict__ hist, uint32_t rem, uint32_t* sh,
                           uint32_t& bin, uint32_t& above) {
  // sh: 4096 + 2 words of shared scratch. Suffix sums over bins, high to low.
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = 4096 / nt;  // bins per thread (nt divides 4096)
  // bins of thread t: [4096 - (t+1)*per, 4096 - t*per), visited high to low
  uint32_t local = 0;
  const int hi = 4096 - t * per;
  for (int b = hi - 1; b >= hi - per; --b) local += hist[b];
  sh[t] = local;
  __syncthreads();
  if (t == 0) {  // exclusive prefix over threads (small: nt entries)
    uint32_t run = 0;
    for (int i = 0; i < nt; ++i) {
      uint32_t v = sh[i];
      sh[i] = run;
      run += v;
    }
  }
  __syncthreads();
  uint32_t run = sh[t];
  if (run < rem && run + local >= rem) {
    for (int b = hi - 1; b >= hi - per; --b) {
      uint32_t h = hist[b];
      if (run + h >= rem) {
        sh[4096] = (uint32_t)b;
        sh[4097] = run;
        break;
      }
      run += h;
    }
  }
  __syncthreads();
  bin = sh[4096];
  above = sh[4097];
  __syncthreads();
}

__global__ __launch_bounds__(TK_THREADS) void topk_init_kernel(void* ws) {
  SegWs* w = seg_ws(ws, blockIdx.x);
  for (int i = threadIdx.x; i < 8192; i += TK_THREADS) (&w->hist0[0])[i] = 0u;
  if (threadIdx.x == 0) {
    w->n_above = 0;
    w->n_bound = 0;
    w->prefix = 0;
    w->rem = 0;
  }
}

__global__ __launch_bounds__(TK_THREADS) void topk_hist0_kernel(const float* __restrict__ scores,
                                                                const int64_t* __restrict__ seg_off,
                                                                void* ws, int k) {
  __shared__ uint32_t h[4096];
  const int64_t s = blockIdx.y;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  if (end - start <= k) return;  // everything is selected
  for (int i = threadIdx.x; i < 4096; i += TK_THREADS) h[i] = 0u;
  __syncthreads();
  for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * TK_THREADS)
    atomicAdd(&h[score_key(scores[i]) >> 20], 1u);
  __syncthreads();
  SegWs* w = seg_ws(ws, s);
  for (int i = threadIdx.x; i < 4096; i += TK_THREADS)
    if (h[i]) atomicAdd(&w->hist0[i], h[i]);
}

__global__ __launch_bounds__(TK_THREADS) void topk_hist1_kernel(const float* __restrict__ scores,
                                                                const int64_t* __restrict__ seg_off,
                                                                void* ws, int k) {
  __shared__ uint32_t h[4096 + 2];
  const int64_t s = blockIdx.y;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  if (end - start <= k) return;
  SegWs* w = seg_ws(ws, s);
  uint32_t b0, above0;
  select_bin(w->hist0, (uint32_t)k, h, b0, above0);
  for (int i = threadIdx.x; i < 4096; i += TK_THREADS) h[i] = 0u;
  __syncthreads();
  for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * TK_THREADS) {
    uint32_t key = score_key(scores[i]);
    if ((key >> 20) == b0) atomicAdd(&h[(key >> 8) & 0xFFF], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += TK_THREADS)
    if (h[i]) atomicAdd(&w->hist1[i], h[i]);
}

__global__ __launch_bounds__(TK_THREADS) void topk_compact_kernel(
    const float* __restrict__ scores, const int64_t* __restrict__ seg_off,
    const int32_t* __restrict__ ids, void* ws, int k) {
  __shared__ uint32_t h[4096 + 2];
  const int64_t s = blockIdx.y;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  SegWs* w = seg_ws(ws, s);
  uint64_t* above = (uint64_t*)(w + 1);
  uint64_t* bound = above + TK_MAXK;
  if (end - start <= k) {
    for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
         i += (int64_t)gridDim.x * TK_THREADS)
      above[i - start] = full_key(score_key(scores[i]), ids, i, start);
    return;
  }
  uint32_t b0, above0, b1, above1;
  select_bin(w->hist0, (uint32_t)k, h, b0, above0);
  select_bin(w->hist1, (uint32_t)k - above0, h, b1, above1);
  const uint32_t prefix = (b0 << 12) | b1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    w->prefix = prefix;
    w->rem = (uint32_t)k - above0 - above1;
  }
  for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * TK_THREADS) {
    uint32_t key = score_key(scores[i]);
    uint32_t hi = key >> 8;
    if (hi > prefix) {
      uint32_t slot = atomicAdd(&w->n_above, 1u);
      if (slot < TK_MAXK) above[slot] = full_key(key, ids, i, start);
    } else if (hi == prefix) {
      uint32_t slot = atomicAdd(&w->n_bound, 1u);
      if (slot < BOUND_CAP) bound[slot] = full_key(key, ids, i, start);
    }
  }
}

__global__ __launch_bounds__(TK_SORT_THREADS) void topk_sort_kernel(
    const float* __restrict__ scores, const int64_t* __restrict__ seg_off,
    const int32_t* __restrict__ ids, void* ws, int k, float* __restrict__ out_scores,
    int32_t* __restrict__ out_ids) {
  __shared__ uint64_t keys[SORT_CAP];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_pre;
  __shared__ uint32_t s_cnt[2];
  const int64_t s = blockIdx.x;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  const int64_t n = end - start;
  SegWs* w = seg_ws(ws, s);
  const uint64_t* above = (const uint64_t*)(w + 1);
  const uint64_t* bound = above + TK_MAXK;
  int count;  // keys placed at the front of `keys`, already the top `count`
  if (n <= k) {
    count = (int)n;
    int p2 = 1;
    while (p2 < count) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) keys[i] = i < count ? above[i] : 0ull;
    __syncthreads();
    bitonic_desc(keys, p2);
  } else if (w->n_bound <= BOUND_CAP) {
    const int na = (int)w->n_above, nb = (int)w->n_bound;
    const int tot = na + nb;
    int p2 = 1;
    while (p2 < tot) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += blockDim.x)
      keys[i] = i < na ? above[i] : (i < tot ? bound[i - na] : 0ull);
    __syncthreads();
    bitonic_desc(keys, p2);
    count = k;
  } else {
    // Boundary overflow: the top-k all have key >= (P << 40); finish the
    // radix select on the low 40 bits with 8-bit digits over the segment.
    uint64_t pre = (uint64_t)w->prefix << 40;
    uint32_t rem = w->rem;
    for (int shift = 32; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
      __syncthreads();
      const uint64_t hmask = ~0ull << (shift + 8);
      for (int64_t i = start + threadIdx.x; i < end; i += blockDim.x) {
        uint64_t key = full_key(score_key(scores[i]), ids, i, start);
        if ((key & hmask) == pre) atomicAdd(&hist[(key >> shift) & 255], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t cum = 0;
        int d = 255;
        for (; d > 0; --d) {
          if (cum + hist[d] >= rem) break;
          cum += hist[d];
        }
        s_pre = pre | ((uint64_t)d << shift);
        s_cnt[0] = rem - cum;
      }
      __syncthreads();
      pre = s_pre;
      rem = s_cnt[0];
      __syncthreads();
    }
    // pre is now the exact k-th key; collect every key >= pre (k of them,
    // more only if an (id, score) pair repeats inside the segment)
    if (threadIdx.x == 0) s_cnt[1] = 0;
    __syncthreads();
    for (int64_t i = start + threadIdx.x; i < end; i += blockDim.x) {
      uint64_t key = full_key(score_key(scores[i]), ids, i, start);
      if (key >= pre) {
        uint32_t slot = atomicAdd(&s_cnt[1], 1u);
        if (slot < (uint32_t)SORT_CAP) keys[slot] = key;
      }
    }
    __syncthreads();
    const int got = s_cnt[1] < (uint32_t)SORT_CAP ? (int)s_cnt[1] : SORT_CAP;
    int p2 = 1;
    while (p2 < got || p2 < k) p2 <<= 1;
    for (int i = got + threadIdx.x; i < p2; i += blockDim.x) keys[i] = 0ull;
    __syncthreads();
    bitonic_desc(keys, p2);
    count = k;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    float sc = -__builtin_inff();
    int32_t id = -1;
    if (i < count) {
      uint64_t key = keys[i];
      sc = key_score((uint32_t)(key >> 32));
      id = (int32_t)(0xFFFFFFFFu - (uint32_t)key);
    }
    out_scores[s * k + i] = sc;
    out_ids[s * k + i] = id;
  }
}

}  // namespace

size_t topk_ws_bytes(int64_t n_seg, int k) {
  (void)k;
  return (size_t)n_seg * seg_ws_bytes();
}

hipError_t launch_topk(const float* scores, const int64_t* seg_off, int64_t n_seg, int64_t n_total,
                       const int32_t* ids, int k, float* out_scores, int32_t* out_ids, void* ws,
                       hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  int64_t avg = n_total / n_seg;
  int64_t bps = avg / (TK_THREADS * 16);
  if (bps < 1) bps = 1;
  if (bps > 256) bps = 256;
  const dim3 grid((unsigned)bps, (unsigned)n_seg);
  hipLaunchKernelGGL(topk_init_kernel, dim3((unsigned)n_seg), dim3(TK_THREADS), 0, st, ws);
  hipLaunchKernelGGL(topk_hist0_kernel, grid, dim3(TK_THREADS), 0, st, scores, seg_off, ws, k);
  hipLaunchKernelGGL(topk_hist1_kernel, grid, dim3(TK_THREADS), 0, st, scores, seg_off, ws, k);
  hipLaunchKernelGGL(topk_compact_kernel, grid, dim3(TK_THREADS), 0, st, scores, seg_off, ids, ws,
                     k);
  hipLaunchKernelGGL(topk_sort_kernel, dim3((unsigned)n_seg), dim3(TK_SORT_THREADS), 0, st, scores,
                     seg_off, ids, ws, k, out_scores, out_ids);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Merge of the fused scorer's top-k parts: one workgroup per query. The
// workgroups of the scoring launch whose ranges cover the query's work pairs
// [ps, pe) are b0 .. b1 (wg_lo is non-decreasing); each non-empty one left
// the k best keys of its share in part slot (b + unit) * group + query of the
// unit. Missing part entries read as key 0, below every real key, so the
// query's top-k is the top-k of the concatenated parts; key 0 in the result
// means fewer than k candidates and becomes (-inf, -1).
// ---------------------------------------------------------------------------
namespace {

constexpr int MERGE_THREADS = 1024;
constexpr int MERGE_CAP = 2048;  // sort buffer: >= 2 * max k
static_assert(MERGE_MAX_GRID % MERGE_THREADS == 0, "extras per thread");

__global__ __launch_bounds__(MERGE_THREADS) void topk_merge_kernel(MergeParams M) {
  using namespace topk_detail;
  __shared__ uint64_t buf[MERGE_CAP];
  __shared__ uint32_t hist[SEL_HIST_WORDS];
  __shared__ uint32_t cnts[MERGE_MAX_GRID];
  const int64_t qa = blockIdx.x;
  const int G = M.group, k = M.k;
  const bool dense = M.cand_off == nullptr;
  const int64_t a = dense ? qa / G : qa;
  const int gq = dense ? (int)(qa % G) : 0;
  const int64_t ps = dense ? a * M.n_docs : M.cand_off[qa];
  const int64_t pe = dense ? ps + M.n_docs : M.cand_off[qa + 1];
  float* os = M.out_scores + qa * k;
  int32_t* oi = M.out_ids + qa * k;
  if (ps >= pe) {
    for (int i = threadIdx.x; i < k; i += MERGE_THREADS) {
      os[i] = -__builtin_inff();
      oi[i] = -1;
    }
    return;
  }
  auto R = [&](int64_t b) -> int64_t { return b >= M.grid ? M.n_upairs : M.wg_lo[b]; };
  // One round of loads for every workgroup b of the scoring launch: its
  // first work pair (for b0, the last workgroup with R(b) <= ps, and b1, the
  // last with R(b) <= pe - 1: R is non-decreasing with R(0) = 0, so each is a
  // count minus one) and the size of its part for this query (0 when it
  // scored nothing).
  if (threadIdx.x < 2) hist[threadIdx.x] = 0u;
  __syncthreads();
  uint32_t c0 = 0, c1 = 0;
  for (int b = threadIdx.x; b < M.grid; b += MERGE_THREADS) {
    const int64_t r = R(b), r1 = R(b + 1);
    const uint32_t c = M.part_cnt[(b + a) * G + gq];
    c0 += r <= ps ? 1u : 0u;
    c1 += r <= pe - 1 ? 1u : 0u;
    cnts[b] = r < r1 ? c : 0u;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    c0 += (uint32_t)__shfl_xor((int)c0, o, 64);
    c1 += (uint32_t)__shfl_xor((int)c1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&hist[0], c0);
    atomicAdd(&hist[1], c1);
  }
  __syncthreads();
  const int64_t b0 = (int64_t)hist[0] - 1, b1 = (int64_t)hist[1] - 1;
  __syncthreads();
  const int nb = (int)(b1 - b0 + 1);
  auto part = [&](int bi) -> const uint64_t* {
    return M.part_keys + ((b0 + bi + a) * G + gq) * (int64_t)k;
  };
  auto cnt = [&](int bi) -> uint32_t { return cnts[b0 + bi]; };
  // Fast path: the first m keys of every part (each part is sorted), sorted
  // together; their top k is the answer when no part holds a key left out
  // that could reach it, i.e. when every part with more than m keys has its
  // (m+1)-th key below the k-th of the result. Each part holds about k / nb
  // of the answer on average, so m of twice that plus two rarely misses (and
  // a miss takes the exact path below).
  int m = 2 * ((k + nb - 1) / nb) + 2;
  m = m < k ? m : k;
  m = m < MERGE_CAP / nb ? m : MERGE_CAP / nb;
  bool done = false;
  if (m >= 1 && m < k) {
    int p2 = 64;
    while (p2 < nb * m) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += MERGE_THREADS) {
      const int bi = i / m, j = i - bi * m;
      buf[i] = (i < nb * m && (uint32_t)j < cnt(bi)) ? part(bi)[j] : 0ull;
    }
    // the (m+1)-th key of the parts that have one, loaded in the same round
    // (nb <= MERGE_MAX_GRID = 4 x MERGE_THREADS)
    uint64_t ex[MERGE_MAX_GRID / MERGE_THREADS];
#pragma unroll
    for (int q = 0; q < MERGE_MAX_GRID / MERGE_THREADS; ++q) {
      const int bi = threadIdx.x + q * MERGE_THREADS;
      ex[q] = (bi < nb && cnt(bi) > (uint32_t)m) ? part(bi)[m] : 0ull;
    }
    __syncthreads();
    bitonic_desc(buf, p2);
    const uint64_t kth = buf[k - 1];  // 0: fewer than k keys gathered
    int ok = 1;
#pragma unroll
    for (int q = 0; q < MERGE_MAX_GRID / MERGE_THREADS; ++q) {
      const int bi = threadIdx.x + q * MERGE_THREADS;
      if (bi < nb && cnt(bi) > (uint32_t)m && ex[q] >= kth) ok = 0;
    }
    done = __syncthreads_and(ok) != 0;
  }
  if (!done) {
    auto get = [&](int64_t i) -> uint64_t {
      const int bi = (int)(i / k);
      const int j = (int)(i - (int64_t)bi * k);
      return (uint32_t)j < cnt(bi) ? part(bi)[j] : 0ull;
    };
    block_topk((int64_t)nb * k, k, get, hist, buf, MERGE_CAP, buf);
  }
  for (int i = threadIdx.x; i < k; i += MERGE_THREADS) {
    const uint64_t key = buf[i];
    os[i] = key == 0ull ? -__builtin_inff() : key_score((uint32_t)(key >> 32));
    oi[i] = key == 0ull ? -1 : key_id(key);
  }
}

}  // namespace

size_t fused_topk_scratch_bytes(int sel_cap) {
  return (size_t)sel_cap * 8 + (size_t)topk_detail::SEL_HIST_WORDS * 4;
}

hipError_t launch_topk_merge(const MergeParams& M, hipStream_t st) {
  if (M.n_q <= 0) return hipSuccess;
  hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)M.n_q), dim3(MERGE_THREADS), 0, st, M);
  return hipGetLastError();
}
