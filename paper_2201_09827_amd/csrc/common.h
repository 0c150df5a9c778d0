// Shared device helpers for the gmresir kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gir {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// storage formats of the LU factors (u_f).  Conversions round to nearest
// even; a float64 value is first rounded to odd at fp32 precision so that the
// following rounding to a narrower format is the correctly rounded result
// (24 >= 11 + 2 and 24 >= 8 + 2 bits).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float round_to_odd_f32(double d) {
  float f = (float)d;
  double back = (double)f;
  if (back != d && !__builtin_isinf(f)) {
    uint32_t bits = __float_as_uint(f);
    if ((bits & 1u) == 0u) {
      bits += (back < d) == (f > 0.0f) ? 1u : 0xFFFFFFFFu;
      if (f == 0.0f) bits = (d > 0.0) ? 1u : 0x80000001u;
      f = __uint_as_float(bits);
    }
  }
  return f;
}

struct Fp16 {
  using T = _Float16;
  static __device__ __forceinline__ float to_f(T v) { return (float)v; }
  static __device__ __forceinline__ T from_f(float f) { return (T)f; }
  static __device__ __forceinline__ T from_d(double d) { return (T)round_to_odd_f32(d); }
  static __device__ __forceinline__ bool finite(T v) { return __builtin_isfinite((float)v); }
};

struct Bf16 {
  using T = uint16_t;  // raw bfloat16 bits
  static __device__ __forceinline__ float to_f(T v) {
    return __uint_as_float(((uint32_t)v) << 16);
  }
  static __device__ __forceinline__ T from_f(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u) return (T)(b >> 16);  // inf
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7FFFu + lsb;
    return (T)(b >> 16);
  }
  static __device__ __forceinline__ T from_d(double d) { return from_f(round_to_odd_f32(d)); }
  static __device__ __forceinline__ bool finite(T v) {
    return ((uint32_t)v & 0x7F80u) != 0x7F80u;
  }
};

struct Fp32 {
  using T = float;
  static __device__ __forceinline__ float to_f(T v) { return v; }
  static __device__ __forceinline__ T from_f(float f) { return f; }
  static __device__ __forceinline__ T from_d(double d) { return (float)d; }
  static __device__ __forceinline__ bool finite(T v) { return __builtin_isfinite(v); }
};

// ---------------------------------------------------------------------------
// wave and block reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int64_t b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFF), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((int64_t)(uint32_t)lo) | (((int64_t)hi) << 32));
}

// atomic max of a non-negative double stored as its bit pattern
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// bounded wait on a device-scope flag; returns false on timeout or abort
__device__ __forceinline__ bool wait_geq(const int* flag, int target, int* abort_flag) {
  long long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (((++spins) & 1023) == 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (spins > (1ll << 25)) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  return true;
}

__device__ __forceinline__ bool wait_eq(const int* flag, int target, int* abort_flag) {
  long long spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != target) {
    __builtin_amdgcn_s_sleep(1);
    if (((++spins) & 1023) == 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (spins > (1ll << 25)) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  return true;
}

// Device-side state of one Arnoldi cycle (shared with the host driver).
struct CycleState {
  int done;      // 1 once the residual estimate reached tol or on breakdown
  int jdone;     // completed Arnoldi steps in this cycle
  int abort;     // set when a bounded device wait timed out
  int singular;  // first 1-based zero-pivot column seen by the LU (0: none)
  double tol;    // tau * ||z||_2
  double est;    // Givens residual estimate after the last step
};

// a kernel of Arnoldi step j is skipped when the cycle converged before j
__device__ __forceinline__ bool gated_off(const CycleState* st, int j) {
  return st != nullptr && st->done && st->jdone <= j;
}

}  // namespace gir
