// select_impl.h -- workgroup-wide exact top-k over 64-bit ranking keys.
//
// A ranking key orders entries exactly as the top-k contract requires
// (score descending, then id ascending): the high 32 bits are the score's
// bits made order-preserving as an unsigned integer (NaN -> 0, below -inf),
// the low 32 bits are ~id. Key 0 never belongs to a real entry (ids are below
// 2^31, so ~id >= 2^31) and serves as padding that ranks below everything.
//
// block_topk() finds the k largest keys of n entries, enumerated by a
// callable get(i), with a radix select: starting from the bits all keys
// share, 12-bit digits fix a key prefix until the entries above the prefix
// plus the entries on it fit the sort buffer; those are collected and sorted
// by a bitonic network. Integer
// keys only, so the result does not depend on the launch shape or on the
// order in which entries are visited.
#pragma once
#include "device_common.h"

namespace topk_detail {

__device__ __forceinline__ uint32_t score_key(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0u;  // NaN ranks last
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_score(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ __forceinline__ uint64_t rank_key(uint32_t sk, uint32_t id) {
  return ((uint64_t)sk << 32) | (uint64_t)(0xFFFFFFFFu - id);
}

__device__ __forceinline__ int32_t key_id(uint64_t key) {
  return (int32_t)(0xFFFFFFFFu - (uint32_t)key);
}

constexpr int SEL_BINS = 4096;
// LDS words of block_topk's histogram area: the bins and a few result words
// (bin, count above it, two collection counters, then 16 wave totals)
constexpr int SEL_HIST_WORDS = SEL_BINS + 24;

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// The bin holding the rem-th largest entry of a SEL_BINS-bin histogram
// (1 <= rem <= total count) and the number of entries in higher bins; every
// thread of the workgroup gets the same answer. hist[SEL_BINS ..] is scratch.
__device__ void select_bin(uint32_t* hist, uint32_t rem, uint32_t& bin, uint32_t& above) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = SEL_BINS / nt;  // nt divides SEL_BINS (256, 512 or 1024)
  const int hi = SEL_BINS - t * per;  // thread t: bins [hi - per, hi), high to low
  uint32_t local = 0;
  for (int b = hi - 1; b >= hi - per; --b) local += hist[b];
  // exclusive prefix over threads in thread order (= bins high to low)
  const uint32_t incl = wave_incl_scan(local);
  const int w = t >> 6;
  uint32_t* wave_tot = hist + SEL_BINS + 8;  // at most 16 waves
  if ((t & 63) == 63) wave_tot[w] = incl;
  __syncthreads();
  uint32_t base = 0;
  for (int i = 0; i < w; ++i) base += wave_tot[i];
  uint32_t run = base + incl - local;
  if (run < rem && run + local >= rem) {
    for (int b = hi - 1; b >= hi - per; --b) {
      const uint32_t h = hist[b];
      if (run + h >= rem) {
        hist[SEL_BINS] = (uint32_t)b;
        hist[SEL_BINS + 1] = run;
        break;
      }
      run += h;
    }
  }
  __syncthreads();
  bin = hist[SEL_BINS];
  above = hist[SEL_BINS + 1];
  __syncthreads();
}

// Sorts n (a power of two) keys descending in LDS, whole workgroup.
__device__ void bitonic_desc(uint64_t* keys, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const uint64_t a = keys[i], b = keys[j];
          if (desc ? (a < b) : (a > b)) {
            keys[i] = b;
            keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// The min(k, n) largest keys of get(0 .. n-1), sorted descending, into
// out[0 ..); returns that count. Whole workgroup; hist has SEL_HIST_WORDS
// words and buf `cap` keys of LDS (cap a power of two, cap >= k, cap >= 64).
template <class Get>
__device__ int block_topk(int64_t n, int k, Get get, uint32_t* hist, uint64_t* buf, int cap,
                          uint64_t* out) {
  const int t = threadIdx.x, nt = blockDim.x;
  int count;
  if (n <= cap) {
    int p2 = 64;
    while (p2 < n) p2 <<= 1;
    for (int i = t; i < p2; i += nt) buf[i] = i < n ? get((int64_t)i) : 0ull;
    __syncthreads();
    bitonic_desc(buf, p2);
    count = n < k ? (int)n : k;
  } else {
    // The score bits every key shares (where the largest and the smallest
    // score key agree) start the prefix, so the first digit already splits
    // the keys: without this, keys of scores in a narrow range all fall into
    // one or two bins of the top digit and their histogram atomics serialise.
    uint32_t hmax = 0u, hmin = ~0u;
    for (int64_t i = t; i < n; i += nt) {
      const uint32_t h = (uint32_t)(get(i) >> 32);
      hmax = h > hmax ? h : hmax;
      hmin = h < hmin ? h : hmin;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      const uint32_t a = (uint32_t)__shfl_xor((int)hmax, m, 64);
      const uint32_t b = (uint32_t)__shfl_xor((int)hmin, m, 64);
      hmax = a > hmax ? a : hmax;
      hmin = b < hmin ? b : hmin;
    }
    // wave partials in the first 32 words of hist, before the bins are used
    const int w = t >> 6, nw = nt >> 6;
    if ((t & 63) == 0) {
      hist[w] = hmax;
      hist[16 + w] = hmin;
    }
    __syncthreads();
    for (int i = 0; i < nw; ++i) {
      hmax = hist[i] > hmax ? hist[i] : hmax;
      hmin = hist[16 + i] < hmin ? hist[16 + i] : hmin;
    }
    __syncthreads();
    int plen = hmax == hmin ? 32 : __builtin_clz(hmax ^ hmin);  // key bits fixed by the prefix
    const uint64_t kmax = (uint64_t)hmax << 32;
    uint64_t prefix = plen == 0 ? 0ull : kmax >> (64 - plen);
    uint32_t rem = (uint32_t)k, n_above = 0;
    while (plen < 64) {
      const int dbits = 64 - plen < 12 ? 64 - plen : 12;
      const int shift = 64 - plen - dbits;
      const uint64_t dmask = (1ull << dbits) - 1ull;
      // keys on the prefix: (key & pmask) == pbits (no shift by 64)
      const uint64_t pmask = plen == 0 ? 0ull : ~0ull << (64 - plen);
      const uint64_t pbits = plen == 0 ? 0ull : prefix << (64 - plen);
      for (int i = t; i < SEL_BINS; i += nt) hist[i] = 0u;
      __syncthreads();
      for (int64_t i = t; i < n; i += nt) {
        const uint64_t key = get(i);
        if ((key & pmask) == pbits) atomicAdd(&hist[(key >> shift) & dmask], 1u);
      }
      __syncthreads();
      uint32_t bin, above;
      select_bin(hist, rem, bin, above);
      const uint32_t on_bin = hist[bin];
      __syncthreads();
      n_above += above;
      rem -= above;
      prefix = (prefix << dbits) | bin;
      plen += dbits;
      if (n_above + on_bin <= (uint32_t)cap) break;
    }
    // entries above the prefix (n_above < k of them) go to the front, the
    // entries on it after them, as many as fit (past the last digit they are
    // equal keys, so which of them are kept does not matter)
    if (t == 0) {
      hist[SEL_BINS + 2] = 0u;
      hist[SEL_BINS + 3] = 0u;
    }
    __syncthreads();
    // the prefix and each key's top plen bits, aligned at the top
    const uint64_t tmask = plen == 64 ? ~0ull : ~(~0ull >> plen);
    const uint64_t pbits = plen == 64 ? prefix : prefix << (64 - plen);
    for (int64_t i = t; i < n; i += nt) {
      const uint64_t key = get(i);
      const uint64_t top = key & tmask;
      if (top > pbits) {
        buf[atomicAdd(&hist[SEL_BINS + 2], 1u)] = key;
      } else if (top == pbits) {
        const uint32_t s = atomicAdd(&hist[SEL_BINS + 3], 1u);
        if (n_above + s < (uint32_t)cap) buf[n_above + s] = key;
      }
    }
    __syncthreads();
    const uint32_t on = hist[SEL_BINS + 3];
    const int got = (int)(n_above + on < (uint32_t)cap ? n_above + on : (uint32_t)cap);
    int p2 = 64;
    while (p2 < got) p2 <<= 1;
    for (int i = got + t; i < p2; i += nt) buf[i] = 0ull;
    __syncthreads();
    bitonic_desc(buf, p2);
    count = k;
  }
  for (int i = t; i < count; i += nt) out[i] = buf[i];
  __syncthreads();
  return count;
}

}  // namespace topk_detail
