// probe.hip -- measured HBM read ceiling: the fastest plain stream read this
// device sustains, so the fused kernels can be reported against it as well
// as against the published peak.
//
// Each wave reads one contiguous share of the buffer with 16-byte loads,
// UNROLL loads in flight per lane, and folds them into an XOR that is stored
// once per wave (so the loads cannot be removed).
//   variant 0: plain loads, lane-contiguous (each wave instruction = 1 KiB)
//   variant 1: the same with the non-temporal hint
//   variant 2: the fused scorer's pattern: 16 rows of 256 B per 4 KiB tile,
//              lane (r, g) reads row r at byte g*16 + c*64 (c < 4)
//   variant 3: variant 2 with the non-temporal hint
//   variant 4: lane-contiguous non-temporal loads straight into LDS
//              (global_load_lds_dwordx4), read back with ds_read_b128
//   variant 5: variant 4 with the 4 KiB tiles dealt round-robin to the waves
//              (all waves sweep the buffer together) instead of one
//              contiguous share per wave
// and the LDS gather ceiling (lds_gather_kernel below).
#include "device_common.h"
#include "kernels.h"

namespace {

template <int VARIANT>
__global__ __launch_bounds__(256) void stream_read_kernel(const u32x4* __restrict__ buf,
                                                          int64_t n16, uint32_t* __restrict__ sink) {
  constexpr int UNROLL = 16;
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  // this wave's [lo, hi) in 16-byte units, whole 4 KiB tiles
  const int64_t tiles = n16 / 256;
  const int64_t t_lo = tiles * w / nw, t_hi = tiles * (w + 1) / nw;
  u32x4 acc = {0, 0, 0, 0};
  for (int64_t t = t_lo; t < t_hi; t += UNROLL / 4) {
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      int64_t tile = t + u / 4;
      if (tile >= t_hi) tile = t_hi - 1;
      int64_t idx;
      if constexpr (VARIANT == 2 || VARIANT == 3) {
        const int r = lane & 15, g = lane >> 4, c = u & 3;
        idx = tile * 256 + r * 16 + c * 4 + g;
      } else {
        idx = tile * 256 + (u & 3) * 64 + lane;
      }
      if constexpr (VARIANT == 1 || VARIANT == 3)
        v[u] = __builtin_nontemporal_load(buf + idx);
      else
        v[u] = buf[idx];
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) acc ^= v[u];
  }
  uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x ^= __shfl_xor(x, m, 64);
  if (lane == 0) sink[w] = x;
}

// Variants 4 and 5: each wave owns a ring of 4 tiles (4 KiB each) in LDS;
// its tile i+3 is requested while tile i is read back. The wave's tiles are
// its i-th local tiles: a contiguous share (variant 4) or every nw-th tile
// starting at its index (variant 5).
template <bool ROUND_ROBIN>
__global__ __launch_bounds__(256) void stream_read_lds_kernel(const u32x4* __restrict__ buf,
                                                              int64_t n16,
                                                              uint32_t* __restrict__ sink) {
  __shared__ u32x4 ring[4][4][256];  // [wave][slot][16-byte chunk]
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t w = (int64_t)blockIdx.x * 4 + wv;
  const int64_t tiles = n16 / 256;
  // local tile indices [t_lo, t_hi) and their buffer tiles
  int64_t t_lo, t_hi;
  if constexpr (ROUND_ROBIN) {
    t_lo = 0;
    t_hi = w < tiles ? (tiles - w + nw - 1) / nw : 0;
  } else {
    t_lo = tiles * w / nw;
    t_hi = tiles * (w + 1) / nw;
  }
  auto tile_of = [&](int64_t t) -> int64_t { return ROUND_ROBIN ? w + t * nw : t; };
  u32x4 acc = {0, 0, 0, 0};
  auto issue = [&](int64_t t, int slot) {
    if (t >= t_hi) t = t_hi - 1;
    const int64_t bt = tile_of(t);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      __builtin_amdgcn_global_load_lds((const void*)(buf + bt * 256 + c * 64 + lane),
                                       (__attribute__((address_space(3))) void*)&ring[wv][slot][c * 64],
                                       16, 0, 2 /* nt */);
  };
  if (t_lo < t_hi) {
    issue(t_lo + 0, 0);
    issue(t_lo + 1, 1);
    issue(t_lo + 2, 2);
    for (int64_t t = t_lo; t < t_hi; t += 4) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        issue(t + s + 3, (s + 3) & 3);
        __builtin_amdgcn_s_waitcnt(0x0F7C);  // vmcnt(12): the oldest tile has landed
#pragma unroll
        for (int c = 0; c < 4; ++c) acc ^= ring[wv][s][c * 64 + lane];
      }
    }
  }
  uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x ^= __shfl_xor(x, m, 64);
  if (lane == 0) sink[w] = x;
}

// LDS gather ceiling: the rate at which the chip serves table lookups from
// LDS, the bound of the PQ scorers (Sec. 4.3 Phase 2 gathers table entries;
// the decode variant gathers codebook rows). Each workgroup (16 waves, one per
// CU) fills a table of `slots` 16-byte entries in LDS, then every wave streams
// its share of a byte buffer from HBM (non-temporal, 16 bytes per lane, four
// steps in flight) and turns each 4-byte word into 8 table indices (its
// rotations by 4-bit steps), each read with one LDS instruction, REPS times
// per word with a different xor mask:
//   variant 0: random 4-byte reads (ds_read_b32), REPS = 4
//   variant 1: random 16-byte reads (ds_read_b128), REPS = 1
//   variant 2: 16-byte reads whose 16 lanes per quarter-wave fall in 16
//              distinct 16-byte bank groups (random row, slot low bits =
//              lane % 16): conflict-free, the LDS read peak, REPS = 1
// Every lane therefore performs 32 * REPS reads per 16 bytes streamed.
template <int VARIANT>
__global__ __launch_bounds__(1024) void lds_gather_kernel(const u32x4* __restrict__ buf, int64_t n16,
                                                          int slots, uint32_t* __restrict__ sink) {
  extern __shared__ u32x4 table[];
  constexpr int REPS = VARIANT == 0 ? 4 : 1;
  for (int i = threadIdx.x; i < slots; i += 1024)
    table[i] = u32x4{(uint32_t)i * 2654435761u, (uint32_t)i ^ 0x9e3779b9u, (uint32_t)i + 7u,
                     ~(uint32_t)i};
  __syncthreads();
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * 16;
  const int64_t w = (int64_t)blockIdx.x * 16 + wv;
  const int64_t units = n16 / 64;  // 1 KiB per wave step
  const int64_t lo = units * w / nw, hi = units * (w + 1) / nw;
  const uint32_t m16 = (uint32_t)slots - 1u, m4 = (uint32_t)slots * 4u - 1u;
  const uint32_t* t4 = (const uint32_t*)table;
  u32x4 acc = {0, 0, 0, 0};
  for (int64_t u = lo; u < hi; u += 4) {
    u32x4 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t uu = u + j < hi ? u + j : hi - 1;
      c[j] = __builtin_nontemporal_load(buf + uu * 64 + lane);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (u + j >= hi) break;  // wave-uniform
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int rep = 0; rep < REPS; ++rep) {
          const uint32_t word = c[j][e] ^ (0x9e3779b9u * (uint32_t)rep);
#pragma unroll
          for (int sft = 0; sft < 8; ++sft) {
            const uint32_t key = __builtin_amdgcn_alignbit(word, word, 4 * sft);
            if constexpr (VARIANT == 0) {
              acc.x ^= t4[key & m4];
            } else if constexpr (VARIANT == 1) {
              acc ^= table[key & m16];
            } else {
              acc ^= table[((key & m16) & ~15u) | (uint32_t)(lane & 15)];
            }
          }
        }
      }
    }
  }
  uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x ^= __shfl_xor(x, m, 64);
  if (lane == 0) sink[w] = x;
}

template <int VARIANT>
hipError_t launch_lds_gather_t(const void* buf, int64_t n16, int slots, uint32_t* sink, int grid,
                               hipStream_t s) {
  auto k = lds_gather_kernel<VARIANT>;
  const size_t lds = (size_t)slots * 16;
  if (lds > 64 * 1024) {
    hipError_t e =
        hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(1024), lds, s, (const u32x4*)buf, n16, slots, sink);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lds_probe(const void* buf, size_t bytes, int variant, int table_bytes,
                            uint32_t* sink, int grid, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const int slots = table_bytes / 16;
  switch (variant) {
    case 0: return launch_lds_gather_t<0>(buf, n16, slots, sink, grid, s);
    case 1: return launch_lds_gather_t<1>(buf, n16, slots, sink, grid, s);
    default: return launch_lds_gather_t<2>(buf, n16, slots, sink, grid, s);
  }
}

hipError_t launch_stream_probe(const void* buf, size_t bytes, int variant, uint32_t* sink,
                               int grid, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  switch (variant) {
    case 1:
      hipLaunchKernelGGL(stream_read_kernel<1>, dim3(grid), dim3(256), 0, s, (const u32x4*)buf,
                         n16, sink);
      break;
    case 2:
      hipLaunchKernelGGL(stream_read_kernel<2>, dim3(grid), dim3(256), 0, s, (const u32x4*)buf,
                         n16, sink);
      break;
    case 3:
      hipLaunchKernelGGL(stream_read_kernel<3>, dim3(grid), dim3(256), 0, s, (const u32x4*)buf,
                         n16, sink);
      break;
    case 4:
      hipLaunchKernelGGL(stream_read_lds_kernel<false>, dim3(grid), dim3(256), 0, s,
                         (const u32x4*)buf, n16, sink);
      break;
    case 5:
      hipLaunchKernelGGL(stream_read_lds_kernel<true>, dim3(grid), dim3(256), 0, s,
                         (const u32x4*)buf, n16, sink);
      break;
    default:
      hipLaunchKernelGGL(stream_read_kernel<0>, dim3(grid), dim3(256), 0, s, (const u32x4*)buf,
                         n16, sink);
      break;
  }
  return hipGetLastError();
}
