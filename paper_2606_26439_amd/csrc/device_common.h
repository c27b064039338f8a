// device_common.h -- shared device-side helpers of the gfx950 MaxSim kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Element types, same numbering as maxsim_dtype.
enum : int { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2, DT_FP8 = 3 };

template <int DT>
struct elem_size {
  static constexpr int value = DT == DT_F32 ? 4 : (DT == DT_FP8 ? 1 : 2);
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)v, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float xor_shfl(float v, int m) { return __shfl_xor(v, m, 64); }

// Cross-lane reductions of an MFMA 16x16 result without the LDS pipe (a
// ds_bpermute shuffle is an LDS round trip the wave waits for; register-to-
// register forms keep a wave that is alone on its SIMD issuing).
//
// Max over the four 16-lane rows (lanes i, i ^ 16, i ^ 32, i ^ 48), left in
// every lane: v_permlane16_swap exchanges odd and even rows between two
// copies of v, v_permlane32_swap the two half-waves. Written as assembly so
// the two swapped copies stay distinct values for the compiler. The
// compiler's hazard recognizer does not look inside inline assembly, so the
// block carries its own wait states. The CDNA4 ISA's table of manually
// inserted wait states requires, before a V_PERMLANE16_SWAP or
// V_PERMLANE32_SWAP, 2 wait states after a VALU write of a VGPR it reads and
// 4 after a V_CMPX write of EXEC; "s_nop 3" gives 4, covering both whatever
// the compiler schedules before the block. The "s_nop 1" after it keeps the
// swapped values two states away from their first reader. The whole wave
// executes it. (A CPU test builds kernels using it to gfx950 assembly and
// checks the wait states and that the max after each swap reads both
// registers.)
__device__ __forceinline__ float max_rows4(float v) {
  float a = v, b = v;
  asm volatile("s_nop 3\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
  v = fmaxf(a, b);
  a = v;
  b = v;
  asm volatile("s_nop 3\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
  return fmaxf(a, b);
}

// Sum over the four 16-lane rows by the same two swaps, left in every lane:
// (v_r0 + v_r1) + (v_r2 + v_r3), the pairs and order of an xor butterfly
// over 16 then 32.
__device__ __forceinline__ float sum_rows4(float v) {
  float a = v, b = v;
  asm volatile("s_nop 3\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
  v = a + b;
  a = v;
  b = v;
  asm volatile("s_nop 3\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
  return a + b;
}

// Sum over the 16 lanes of each row, left in every lane of the row: four DPP
// row rotations (by 8, 4, 2, 1) with adds. Lane 0 adds the same pairs in the
// same order as an xor butterfly over 8, 4, 2, 1, so its value does not
// depend on which of the two forms a kernel uses.
__device__ __forceinline__ float row_sum16(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128,
                                                             0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124,
                                                             0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x122,
                                                             0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x121,
                                                             0xF, 0xF, false));
  return v;
}

// First index i in [0, n] with arr[i] >= key, for a non-decreasing arr of
// n + 1 entries with arr[n] >= key. Executed by a whole wavefront: each round
// probes 64 evenly spaced positions and keeps the bracket of the first hit,
// so a 1M-entry array takes 4 dependent loads instead of 20.
__device__ __forceinline__ int64_t wave_lower_bound(const int64_t* __restrict__ arr, int64_t n,
                                                    int64_t key) {
  const int lane = lane_id();
  int64_t lo = 0, hi = n;
  while (hi - lo + 1 > 64) {
    int64_t step = (hi - lo + 64) / 64;  // ceil((hi - lo + 1) / 64)
    int64_t pos = lo + step * lane;
    if (pos > hi) pos = hi;
    bool pred = arr[pos] >= key;
    uint64_t mask = __ballot(pred);
    if (mask & 1ull) return lo;  // arr[lo] >= key
    if (mask == 0) {
      lo = lo + step * 63 + 1;
    } else {
      int f = __ffsll((unsigned long long)mask) - 1;  // f >= 1
      int64_t pf = lo + step * f;
      if (pf > hi) pf = hi;
      lo = lo + step * (f - 1) + 1;
      hi = pf;
    }
  }
  int64_t pos = lo + lane;
  bool pred = pos <= hi && arr[pos < hi ? pos : hi] >= key;
  uint64_t mask = __ballot(pred);
  int f = mask ? __ffsll((unsigned long long)mask) - 1 : (int)(hi - lo);
  return lo + f;
}

// Last index a in [0, n) with arr[a] <= key for arr non-decreasing of n + 1
// entries, arr[0] <= key < arr[n]: the set that owns element `key`.
__device__ __forceinline__ int64_t wave_owner(const int64_t* __restrict__ arr, int64_t n,
                                              int64_t key) {
  // first i with arr[i] >= key + 1, minus one
  return wave_lower_bound(arr, n, key + 1) - 1;
}

// E8M0 exponent byte of a normal power-of-two float (2^k -> k + 127).
__device__ __forceinline__ int e8m0_of(float s) { return (int)((__float_as_uint(s) >> 23) & 0xFF); }

// Scalar (SMEM) loads of wave-uniform indices: reading through the constant
// address space makes the compiler use s_load, whose completion is tracked by
// lgkmcnt and therefore independent of the vector loads in flight.
typedef const __attribute__((address_space(4))) int64_t* const_i64_ptr;
typedef const __attribute__((address_space(4))) int32_t* const_i32_ptr;
__device__ __forceinline__ int64_t sload_i64(const int64_t* p, int64_t i) {
  return ((const_i64_ptr)p)[i];
}
__device__ __forceinline__ int sload_i32(const int32_t* p, int64_t i) {
  return ((const_i32_ptr)p)[i];
}

// 1 KiB of zeros (one wave's worth of 16-byte lanes; at least one chunk row
// of the widest element type): the target of the fixed-count loads a wave
// issues when it has nothing left to load, so those loads never depend on the
// caller's buffers being non-empty.
static __device__ __attribute__((aligned(16))) char g_zero_row[1024];

// The zero row's address, read once into scalar registers. The empty asm
// makes the value opaque, so the compiler keeps it in registers instead of
// re-reading it from the global offset table (a scalar load the wave must
// wait for) at every idle refill of a loop; the pointer stays typed as a
// global one through the asm, so loads from it remain global loads.
typedef const __attribute__((address_space(1))) char global_char;
__device__ __forceinline__ const char* zero_row_ptr() {
  global_char* p = (global_char*)g_zero_row;
  asm volatile("" : "+s"(p));
  return (const char*)p;
}
