// validate.hip -- device-side checks of the inputs the host cannot see.
//
// The scoring entry points trust what lives in device memory: CSR offsets,
// candidate ids, FP8 scales and PQ codes (reading them on the host would need
// a device-to-host copy per call). These kernels check them on the device and
// OR one bit per violated rule into a caller-owned flag word, so a caller can
// validate a document pool once when it is built, or a batch before scoring.
// Every access stays inside the arrays the descriptors declare, whatever
// their contents.
#include "device_common.h"
#include "kernels.h"

namespace {

__global__ __launch_bounds__(64) void clear_flags_kernel(int32_t* flags) {
  if (threadIdx.x == 0) *flags = 0;
}

// offsets[0] == 0, non-decreasing, offsets[n] == n_tokens; optionally every
// set no longer than max_len.
__global__ __launch_bounds__(256) void check_offsets_kernel(const int64_t* __restrict__ off,
                                                            int64_t n, int64_t n_tokens,
                                                            int32_t max_len, int32_t bit_off,
                                                            int32_t bit_len, int32_t* flags) {
  int32_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * 256) {
    const int64_t v = off[i];
    if (i == 0 && v != 0) bad |= bit_off;
    if (i == n && v != n_tokens) bad |= bit_off;
    if (i < n) {
      const int64_t len = off[i + 1] - v;
      if (len < 0) bad |= bit_off;
      if (max_len >= 0 && len > max_len) bad |= bit_len;
    }
  }
  if (bad) atomicOr(flags, bad);
}

__global__ __launch_bounds__(256) void check_ids_kernel(const int32_t* __restrict__ ids,
                                                        int64_t n, int64_t n_docs, int32_t bit,
                                                        int32_t* flags) {
  int32_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const int32_t v = ids[i];
    if (v < 0 || (int64_t)v >= n_docs) bad = bit;
  }
  if (bad) atomicOr(flags, bad);
}

// FP8 token scales must be normal powers of two (the scale operands of the
// matrix instruction carry only an exponent).
__global__ __launch_bounds__(256) void check_scales_kernel(const float* __restrict__ s, int64_t n,
                                                           int32_t bit, int32_t* flags) {
  int32_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const uint32_t b = __float_as_uint(s[i]);
    const uint32_t e = (b >> 23) & 0xFF;
    if ((b & 0x807FFFFFu) != 0 || e == 0 || e == 0xFF) bad = bit;
  }
  if (bad) atomicOr(flags, bad);
}

__global__ __launch_bounds__(256) void check_codes_kernel(const uint8_t* __restrict__ codes,
                                                          int64_t n, int32_t K, int32_t bit,
                                                          int32_t* flags) {
  int32_t bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    if ((int32_t)codes[i] >= K) bad = bit;
  if (bad) atomicOr(flags, bad);
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_clear_flags(int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, s, flags);
  return hipGetLastError();
}

hipError_t launch_check_offsets(const int64_t* off, int64_t n, int64_t n_tokens, int max_len,
                                int bit_off, int bit_len, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(check_offsets_kernel, dim3(grid_for(n + 1)), dim3(256), 0, s, off, n,
                     n_tokens, max_len, bit_off, bit_len, flags);
  return hipGetLastError();
}

hipError_t launch_check_ids(const int32_t* ids, int64_t n, int64_t n_docs, int bit,
                            int32_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_ids_kernel, dim3(grid_for(n)), dim3(256), 0, s, ids, n, n_docs, bit,
                     flags);
  return hipGetLastError();
}

hipError_t launch_check_scales(const float* sc, int64_t n, int bit, int32_t* flags,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_scales_kernel, dim3(grid_for(n)), dim3(256), 0, s, sc, n, bit, flags);
  return hipGetLastError();
}

hipError_t launch_check_codes(const uint8_t* codes, int64_t n, int K, int bit, int32_t* flags,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_codes_kernel, dim3(grid_for(n)), dim3(256), 0, s, codes, n, K, bit,
                     flags);
  return hipGetLastError();
}
