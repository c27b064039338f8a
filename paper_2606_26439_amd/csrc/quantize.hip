// quantize.hip -- input conversion for the precision forms.
//
// FP32 -> BF16 / F16: round to nearest even per element (the hardware
// conversions, which round to nearest even in the default mode).
// FP32 -> FP8 E4M3FN: per token, the scale s = 2^k with k the smallest
// integer such that max|x| <= 448 * 2^k (s = 1 for an all-zero token); the
// codes are E4M3FN(x * 2^-k), rounded to nearest even. Multiplying by 2^-k is
// exact, and |x * 2^-k| <= 448 so no code saturates.
#include "device_common.h"
#include "kernels.h"

namespace {

__global__ __launch_bounds__(256) void copy_f32_kernel(const u32x4* __restrict__ src,
                                                       u32x4* __restrict__ dst, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}

// 8 elements per thread: 32 bytes in, 16 bytes out.
template <bool BF>
__global__ __launch_bounds__(256) void to_half_kernel(const float4* __restrict__ src,
                                                      u32x4* __restrict__ dst, int64_t n8) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n8;
       i += (int64_t)gridDim.x * 256) {
    float4 a = src[2 * i], b = src[2 * i + 1];
    float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint16_t lo, hi;
      if constexpr (BF) {
        lo = __builtin_bit_cast(uint16_t, (__bf16)v[2 * j]);
        hi = __builtin_bit_cast(uint16_t, (__bf16)v[2 * j + 1]);
      } else {
        lo = __builtin_bit_cast(uint16_t, (_Float16)v[2 * j]);
        hi = __builtin_bit_cast(uint16_t, (_Float16)v[2 * j + 1]);
      }
      w[j] = (uint32_t)lo | ((uint32_t)hi << 16);
    }
    dst[i] = u32x4{w[0], w[1], w[2], w[3]};
  }
}

// Exponent k of the per-token scale, from the bits of amax (> 0, finite).
__device__ __forceinline__ int fp8_scale_exponent(float amax) {
  int bias = 0;
  if (amax < 1.17549435e-38f) {  // subnormal: renormalise exactly
    amax *= 18446744073709551616.0f;  // 2^64
    bias = 64;
  }
  uint32_t u = __float_as_uint(amax);
  int e = (int)((u >> 23) & 0xFF) - 127;
  uint32_t mant = u & 0x7FFFFF;
  // amax = 1.m * 2^e; 448 * 2^k = 1.75 * 2^(8 + k): k = e - 8 suffices iff 1.m <= 1.75
  return e - 8 + (mant > 0x600000u ? 1 : 0) - bias;
}

// One wavefront per token; dim <= 1024 so each lane holds <= 16 values
// (element j * 64 + lane, for those below dim).
__global__ __launch_bounds__(256) void to_fp8_kernel(const float* __restrict__ src,
                                                     uint8_t* __restrict__ dst,
                                                     float* __restrict__ scales,
                                                     int64_t n_tokens, int dim) {
  const int lane = lane_id();
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < n_tokens;
       t += (int64_t)gridDim.x * 4) {
    const float* x = src + t * dim;
    float v[16];
    float amax = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      v[j] = 0.f;
      if (j * 64 + lane < dim) {
        v[j] = x[j * 64 + lane];
        amax = fmaxf(amax, fabsf(v[j]));
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) amax = fmaxf(amax, __shfl_xor(amax, m, 64));
    int k = amax > 0.f ? fp8_scale_exponent(amax) : 0;
    float inv = __uint_as_float((uint32_t)(127 - k) << 23);  // 2^-k
    if (lane == 0) scales[t] = __uint_as_float((uint32_t)(127 + k) << 23);
    uint8_t* out = dst + t * dim;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j * 64 + lane < dim) {
        unsigned int p = __builtin_amdgcn_cvt_pk_fp8_f32(v[j] * inv, 0.f, 0u, false);
        out[j * 64 + lane] = (uint8_t)(p & 0xFF);
      }
    }
  }
}

int grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_quantize(const float* src, int64_t n_tokens, int dim, int dt, void* dst,
                           float* scales, hipStream_t s) {
  const int64_t n = n_tokens * dim;
  if (n == 0) return hipSuccess;
  switch (dt) {
    case DT_F32:
      hipLaunchKernelGGL(copy_f32_kernel, dim3(grid_for(n / 4, 256)), dim3(256), 0, s,
                         (const u32x4*)src, (u32x4*)dst, n / 4);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(to_half_kernel<true>, dim3(grid_for(n / 8, 256)), dim3(256), 0, s,
                         (const float4*)src, (u32x4*)dst, n / 8);
      break;
    case DT_F16:
      hipLaunchKernelGGL(to_half_kernel<false>, dim3(grid_for(n / 8, 256)), dim3(256), 0, s,
                         (const float4*)src, (u32x4*)dst, n / 8);
      break;
    default:
      hipLaunchKernelGGL(to_fp8_kernel, dim3(grid_for(n_tokens, 4)), dim3(256), 0, s, src,
                         (uint8_t*)dst, scales, n_tokens, dim);
      break;
  }
  return hipGetLastError();
}
