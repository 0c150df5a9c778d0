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

// Wave-wide maximum of a 64-bit unsigned key with DPP row shifts and row
// broadcasts (no LDS round trips); every lane receives the maximum.
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t v, int lo_nb, int hi_nb) {
  return v > (((uint64_t)(uint32_t)hi_nb << 32) | (uint32_t)lo_nb) ? v
         : (((uint64_t)(uint32_t)hi_nb << 32) | (uint32_t)lo_nb);
}

#define GIR_DPP_MAX(v, ctrl, rmask)                                                        \
  do {                                                                                   \
    const int lo_ = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v), ctrl, rmask, 0xf, false); \
    const int hi_ = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((v) >> 32), ctrl, rmask, 0xf, false); \
    v = dpp_max_step(v, lo_, hi_);                                                       \
  } while (0)

// Wave-wide maximum of a 32-bit unsigned value by the same DPP pattern;
// every lane receives the maximum.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#define GIR_DPP_MAX32(ctrl, rmask)                                                          \
  do {                                                                                   \
    const uint32_t o_ = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, rmask, 0xf, false); \
    v = v > o_ ? v : o_;                                                                 \
  } while (0)
  GIR_DPP_MAX32(0x111, 0xf);  // row_shr:1
  GIR_DPP_MAX32(0x112, 0xf);  // row_shr:2
  GIR_DPP_MAX32(0x114, 0xf);  // row_shr:4
  GIR_DPP_MAX32(0x118, 0xf);  // row_shr:8
  GIR_DPP_MAX32(0x142, 0xa);  // row_bcast:15
  GIR_DPP_MAX32(0x143, 0xc);  // row_bcast:31
#undef GIR_DPP_MAX32
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  GIR_DPP_MAX(v, 0x111, 0xf);  // row_shr:1
  GIR_DPP_MAX(v, 0x112, 0xf);  // row_shr:2
  GIR_DPP_MAX(v, 0x114, 0xf);  // row_shr:4
  GIR_DPP_MAX(v, 0x118, 0xf);  // row_shr:8  -> lane 15 of each row holds the row max
  GIR_DPP_MAX(v, 0x142, 0xa);  // row_bcast:15 -> rows 1, 3
  GIR_DPP_MAX(v, 0x143, 0xc);  // row_bcast:31 -> rows 2, 3
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// atomic max of a non-negative double stored as its bit pattern
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// slot of a handle's norms array (as bits) that the residual kernels raise to
// the componentwise backward error max_i |r_i| / (|A| |x| + |b|)_i
constexpr int kNormCw = 4;

// one term of that maximum: 0/0 = 0, r/0 = inf
__device__ __forceinline__ double cw_ratio(double r, double den) {
  if (r == 0.0) return 0.0;
  return den > 0.0 ? r / den : __builtin_inf();
}

// Bounded waits on a device-scope flag.  The flag is polled with relaxed
// loads (an acquire load would invalidate the caches on every poll) and a
// single acquire fence follows the successful poll.  Returns false on
// timeout (which also raises the abort flag) or when another wave aborted.
template <class Pred>
__device__ __forceinline__ bool wait_until(const int* flag, Pred ok, int* abort_flag) {
  long long spins = 0;
  while (!ok(__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
    __builtin_amdgcn_s_sleep(1);
    if (((++spins) & 1023) == 0) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (spins > (1ll << 25)) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__device__ __forceinline__ bool wait_geq(const int* flag, int target, int* abort_flag) {
  return wait_until(flag, [target](int v) { return v >= target; }, abort_flag);
}

__device__ __forceinline__ bool wait_eq(const int* flag, int target, int* abort_flag) {
  return wait_until(flag, [target](int v) { return v == target; }, abort_flag);
}

// Publish the stores of the whole workgroup, then set the flag: the
// workgroup barrier completes every wave's stores, one device-scope release
// fence makes them visible to the other XCDs, then thread 0 stores.
__device__ __forceinline__ void publish_store(int* flag, int value) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ void publish_add(int* flag, int value) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
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

// ---------------------------------------------------------------------------
// factor tiles
// ---------------------------------------------------------------------------
constexpr int kTileCols = 64;

// A tile row of 64 u_f values kept as raw bits (32 registers for 16-bit
// formats) and widened to fp64 when used.
template <class F>
struct RawRow {
  static constexpr int kWords = kTileCols * (int)sizeof(typename F::T) / 4;
  uint32_t w[kWords];

  __device__ __forceinline__ void load(const typename F::T* srow, int cbase, int n, bool valid) {
    if (valid && cbase + kTileCols <= n) {
      const uint4* q = reinterpret_cast<const uint4*>(srow + cbase);
#pragma unroll
      for (int v = 0; v < kWords / 4; ++v) {
        const uint4 x = q[v];
        w[4 * v] = x.x;
        w[4 * v + 1] = x.y;
        w[4 * v + 2] = x.z;
        w[4 * v + 3] = x.w;
      }
    } else {
      using T = typename F::T;
      constexpr int per = 4 / (int)sizeof(T);
#pragma unroll
      for (int i = 0; i < kWords; ++i) {
        uint32_t word = 0;
#pragma unroll
        for (int e = 0; e < per; ++e) {
          const int c = cbase + i * per + e;
          T v{};
          if (valid && c < n) v = srow[c];
          uint32_t bits = 0;
          __builtin_memcpy(&bits, &v, sizeof(T));
          word |= bits << (8 * sizeof(T) * e);
        }
        w[i] = word;
      }
    }
  }

  __device__ __forceinline__ double at(int c) const {
    using T = typename F::T;
    T v;
    if constexpr (sizeof(T) == 2) {
      const uint16_t b = (uint16_t)(w[c >> 1] >> (16 * (c & 1)));
      __builtin_memcpy(&v, &b, 2);
    } else {
      __builtin_memcpy(&v, &w[c], 4);
    }
    return (double)F::to_f(v);
  }
};


}  // namespace gir
