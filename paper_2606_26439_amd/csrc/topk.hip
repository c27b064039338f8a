// topk.hip -- exact per-segment top-k by (score descending, id ascending).
//
// Every entry maps to a 64-bit key that orders exactly like the required
// ranking: the high 32 bits are the score's bits made order-preserving as an
// unsigned integer (NaN -> 0, below -inf), the low 32 bits are ~id so smaller
// ids rank higher. The k-th largest key is found by an 8-pass radix select
// (8 bits per pass, 256-bin histograms built in LDS, then merged with global
// atomics); every pass's kernel first re-derives the running prefix from the
// previous pass's histogram, so there is no separate scan launch. A gather
// kernel then copies the (at most k) keys >= the threshold and one workgroup
// per segment sorts them with a bitonic network in LDS. Integer keys only:
// the result is exact and independent of launch shape.
#include "device_common.h"
#include "kernels.h"

namespace {

constexpr int TK_THREADS = 256;
constexpr int TK_MAXK = 1024;

struct SegWs {
  uint32_t hist[8][256];
  uint64_t prefix[9];
  uint32_t remain[9];
  uint32_t n_gt;
  uint32_t n_eq;
  uint32_t pad[5];
  // followed by k uint64 candidate keys
};

__host__ __device__ inline size_t seg_ws_bytes(int k) {
  size_t b = sizeof(SegWs) + (size_t)k * 8;
  return (b + 255) & ~(size_t)255;
}

__device__ __forceinline__ uint32_t score_key(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0u;  // NaN ranks last
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_score(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ uint64_t full_key(const float* scores, const int32_t* ids, int64_t i,
                                             int64_t start) {
  uint32_t id = ids ? (uint32_t)ids[i] : (uint32_t)(i - start);
  return ((uint64_t)score_key(scores[i]) << 32) | (uint64_t)(0xFFFFFFFFu - id);
}

__device__ __forceinline__ SegWs* seg_ws(void* ws, int64_t s, int k) {
  return (SegWs*)((char*)ws + (size_t)s * seg_ws_bytes(k));
}

__global__ __launch_bounds__(TK_THREADS) void topk_init_kernel(void* ws, int k) {
  SegWs* w = seg_ws(ws, blockIdx.x, k);
  for (int i = threadIdx.x; i < 8 * 256; i += TK_THREADS) (&w->hist[0][0])[i] = 0u;
  if (threadIdx.x == 0) {
    w->prefix[0] = 0;
    w->remain[0] = (uint32_t)k;
    w->n_gt = 0;
    w->n_eq = 0;
  }
}

// Given the histogram of pass p (digit bits 56-8p .. 63-8p) and the state
// before it, the state after it: the digit holding the remain-th largest
// element among those that match the prefix.
__device__ void derive_state(const SegWs* w, int p, uint64_t& prefix, uint32_t& remain) {
  uint64_t pre = w->prefix[p];
  uint32_t rem = w->remain[p];
  uint32_t cum = 0;
  int d = 255;
  for (; d > 0; --d) {
    uint32_t h = w->hist[p][d];
    if (cum + h >= rem) break;
    cum += h;
  }
  prefix = pre | ((uint64_t)d << (56 - 8 * p));
  remain = rem - cum;
}

__global__ __launch_bounds__(TK_THREADS) void topk_hist_kernel(const float* __restrict__ scores,
                                                               const int64_t* __restrict__ seg_off,
                                                               const int32_t* __restrict__ ids,
                                                               void* ws, int k, int pass) {
  __shared__ uint32_t h[256];
  __shared__ uint64_t s_prefix;
  const int64_t s = blockIdx.y;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  if (end - start <= k) return;  // everything is selected
  SegWs* w = seg_ws(ws, s, k);
  h[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    uint64_t pre = 0;
    uint32_t rem = (uint32_t)k;
    if (pass > 0) derive_state(w, pass - 1, pre, rem);
    s_prefix = pre;
    if (blockIdx.x == 0 && pass > 0) {
      w->prefix[pass] = pre;
      w->remain[pass] = rem;
    }
  }
  __syncthreads();
  const uint64_t pre = s_prefix;
  const int shift = 56 - 8 * pass;
  const uint64_t hi_mask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
  for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * TK_THREADS) {
    uint64_t key = full_key(scores, ids, i, start);
    if ((key & hi_mask) == pre) atomicAdd(&h[(key >> shift) & 255], 1u);
  }
  __syncthreads();
  uint32_t c = h[threadIdx.x];
  if (c) atomicAdd(&w->hist[pass][threadIdx.x], c);
}

__global__ __launch_bounds__(TK_THREADS) void topk_gather_kernel(const float* __restrict__ scores,
                                                                 const int64_t* __restrict__ seg_off,
                                                                 const int32_t* __restrict__ ids,
                                                                 void* ws, int k) {
  __shared__ uint64_t s_thr;
  __shared__ uint32_t s_rem;
  const int64_t s = blockIdx.y;
  const int64_t start = seg_off[s], end = seg_off[s + 1];
  SegWs* w = seg_ws(ws, s, k);
  uint64_t* cand = (uint64_t*)(w + 1);
  if (end - start <= k) {
    for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
         i += (int64_t)gridDim.x * TK_THREADS)
      cand[i - start] = full_key(scores, ids, i, start);
    return;
  }
  if (threadIdx.x == 0) {
    uint64_t thr;
    uint32_t rem;
    derive_state(w, 7, thr, rem);
    s_thr = thr;
    s_rem = rem;
  }
  __syncthreads();
  const uint64_t thr = s_thr;
  const uint32_t rem = s_rem;
  const uint32_t n_above = (uint32_t)k - rem;
  for (int64_t i = start + (int64_t)blockIdx.x * TK_THREADS + threadIdx.x; i < end;
       i += (int64_t)gridDim.x * TK_THREADS) {
    uint64_t key = full_key(scores, ids, i, start);
    if (key > thr) {
      uint32_t slot = atomicAdd(&w->n_gt, 1u);
      if (slot < n_above) cand[slot] = key;
    } else if (key == thr) {
      uint32_t e = atomicAdd(&w->n_eq, 1u);
      if (e < rem) cand[n_above + e] = key;
    }
  }
}

__global__ __launch_bounds__(TK_MAXK) void topk_sort_kernel(const int64_t* __restrict__ seg_off,
                                                            void* ws, int k, int kpow2,
                                                            float* __restrict__ out_scores,
                                                            int32_t* __restrict__ out_ids) {
  __shared__ uint64_t keys[TK_MAXK];
  const int64_t s = blockIdx.x;
  const int64_t n = seg_off[s + 1] - seg_off[s];
  const int count = n < k ? (int)n : k;
  SegWs* w = seg_ws(ws, s, k);
  const uint64_t* cand = (const uint64_t*)(w + 1);
  for (int i = threadIdx.x; i < kpow2; i += blockDim.x) keys[i] = i < count ? cand[i] : 0ull;
  __syncthreads();
  // bitonic sort, descending
  for (int size = 2; size <= kpow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < kpow2; i += blockDim.x) {
        int j = i ^ stride;
        if (j > i) {
          bool desc = (i & size) == 0;
          uint64_t a = keys[i], b = keys[j];
          if (desc ? (a < b) : (a > b)) {
            keys[i] = b;
            keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
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

size_t topk_ws_bytes(int64_t n_seg, int k) { return (size_t)n_seg * seg_ws_bytes(k); }

hipError_t launch_topk(const float* scores, const int64_t* seg_off, int64_t n_seg, int64_t n_total,
                       const int32_t* ids, int k, float* out_scores, int32_t* out_ids, void* ws,
                       hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  int64_t avg = n_total / n_seg;
  int64_t bps = avg / (TK_THREADS * 16);
  if (bps < 1) bps = 1;
  if (bps > 256) bps = 256;
  hipLaunchKernelGGL(topk_init_kernel, dim3((unsigned)n_seg), dim3(TK_THREADS), 0, st, ws, k);
  for (int p = 0; p < 8; ++p)
    hipLaunchKernelGGL(topk_hist_kernel, dim3((unsigned)bps, (unsigned)n_seg), dim3(TK_THREADS),
                       0, st, scores, seg_off, ids, ws, k, p);
  hipLaunchKernelGGL(topk_gather_kernel, dim3((unsigned)bps, (unsigned)n_seg), dim3(TK_THREADS), 0,
                     st, scores, seg_off, ids, ws, k);
  int kpow2 = 1;
  while (kpow2 < k) kpow2 <<= 1;
  int threads = kpow2 < 64 ? 64 : kpow2;
  hipLaunchKernelGGL(topk_sort_kernel, dim3((unsigned)n_seg), dim3(threads), 0, st, seg_off, ws, k,
                     kpow2, out_scores, out_ids);
  return hipGetLastError();
}
