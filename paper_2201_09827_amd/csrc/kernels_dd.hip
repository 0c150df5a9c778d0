// Double-double kernels of RGMRES-IR for the working precision u = fp64,
// where the preconditioned matrix is applied in u^2 (Algorithms 2 and 3 with
// u^2 beyond fp64, Section 3's precision triples) and for a residual
// precision u_r beyond fp64.
//
// A double-double value is an unevaluated sum hi + lo of two fp64 numbers
// with |lo| <= ulp(hi) / 2.  The building blocks are the error-free
// transformations TwoSum (Knuth), FastTwoSum (Dekker) and TwoProduct through
// the fused multiply-add; long sums use the compensated scheme of Ogita, Rump
// and Oishi (Dot2), which keeps a running fp64 sum plus one fp64 correction
// that collects every rounding error exactly produced.  Every operation here
// is written so that no multiply and add are fused by the compiler: the
// transformations are exact only when each operation rounds once, as written.
#include "kernels.h"

#pragma clang fp contract(off)

namespace gir {

namespace {

struct DD {
  double h, l;
};

__device__ __forceinline__ DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ DD two_prod(double a, double b) {
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}

// (a.h + a.l) + (b.h + b.l) with two TwoSums (accurate under cancellation)
__device__ __forceinline__ DD dd_add(DD a, DD b) {
  const DD s = two_sum(a.h, b.h);
  const DD t = two_sum(a.l, b.l);
  DD u = fast_two_sum(s.h, s.l + t.h);
  return fast_two_sum(u.h, u.l + t.l);
}

// x - a y for an fp64 a (a factor entry, exact) and double-double x, y
__device__ __forceinline__ DD dd_sub_mul(DD x, double a, DD y) {
  DD p = two_prod(a, y.h);
  p.l = __builtin_fma(a, y.l, p.l);
  return dd_add(x, DD{-p.h, -p.l});
}

// double-double product a * b (b a double-double reciprocal below)
__device__ __forceinline__ DD dd_mul(DD a, DD b) {
  DD p = two_prod(a.h, b.h);
  p.l = __builtin_fma(a.h, b.l, __builtin_fma(a.l, b.h, p.l));
  return fast_two_sum(p.h, p.l);
}

// compensated accumulator: the sum is s + c, c collects the exact errors
struct Acc {
  double s = 0.0, c = 0.0;

  // += a * (yh + yl), a exact in fp64
  __device__ __forceinline__ void add_prod(double a, double yh, double yl) {
    const DD p = two_prod(a, yh);
    const DD t = two_sum(s, p.h);
    s = t.h;
    c += t.l + __builtin_fma(a, yl, p.l);
  }
  __device__ __forceinline__ void add(const Acc& o) {
    const DD t = two_sum(s, o.s);
    s = t.h;
    c += t.l + o.c;
  }
  __device__ __forceinline__ DD value() const { return fast_two_sum(s, c); }
};

__device__ __forceinline__ Acc wave_sum_acc(Acc a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Acc b;
    b.s = __shfl_xor(a.s, o, kWave);
    b.c = __shfl_xor(a.c, o, kWave);
    a.add(b);
  }
  return a;
}

// ---------------------------------------------------------------------------
// row dot products of an fp64 matrix: one wave per row, 16-byte loads
// ---------------------------------------------------------------------------
// (with kAbs, *abs_sum receives sum |a_c| |v_c| in fp64 on every lane: the
// denominator of the componentwise backward error)
template <bool kAbs = false>
__device__ __forceinline__ Acc row_dot_dd(const double* __restrict__ a,
                                          const double* __restrict__ v, int n, int lane,
                                          double* abs_sum = nullptr) {
  Acc acc0, acc1;
  double s0 = 0.0, s1 = 0.0;
  const int n2 = n & ~1;
  int c = lane * 2;
  for (; c + 128 < n2; c += 256) {
    const double2 a0 = *reinterpret_cast<const double2*>(a + c);
    const double2 a1 = *reinterpret_cast<const double2*>(a + c + 128);
    const double2 x0 = *reinterpret_cast<const double2*>(v + c);
    const double2 x1 = *reinterpret_cast<const double2*>(v + c + 128);
    acc0.add_prod(a0.x, x0.x, 0.0);
    acc1.add_prod(a0.y, x0.y, 0.0);
    acc0.add_prod(a1.x, x1.x, 0.0);
    acc1.add_prod(a1.y, x1.y, 0.0);
    if (kAbs) {
      s0 = fma(fabs(a0.x), fabs(x0.x), s0);
      s1 = fma(fabs(a0.y), fabs(x0.y), s1);
      s0 = fma(fabs(a1.x), fabs(x1.x), s0);
      s1 = fma(fabs(a1.y), fabs(x1.y), s1);
    }
  }
  for (; c < n2; c += 128) {
    const double2 a0 = *reinterpret_cast<const double2*>(a + c);
    const double2 x0 = *reinterpret_cast<const double2*>(v + c);
    acc0.add_prod(a0.x, x0.x, 0.0);
    acc1.add_prod(a0.y, x0.y, 0.0);
    if (kAbs) {
      s0 = fma(fabs(a0.x), fabs(x0.x), s0);
      s1 = fma(fabs(a0.y), fabs(x0.y), s1);
    }
  }
  for (int cc = n2 + lane; cc < n; cc += kWave) {
    acc0.add_prod(a[cc], v[cc], 0.0);
    if (kAbs) s0 = fma(fabs(a[cc]), fabs(v[cc]), s0);
  }
  acc0.add(acc1);
  if (kAbs) *abs_sum = wave_sum(s0 + s1);
  return wave_sum_acc(acc0);
}

__global__ __launch_bounds__(256) void k_gemv_dd(const double* __restrict__ A, int64_t ld,
                                                 const int* __restrict__ permA, int n,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ th,
                                                 double* __restrict__ tl,
                                                 const CycleState* gate, int step) {
  if (gated_off(gate, step)) return;
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= n) return;
  const int prow = permA ? permA[row] : row;
  const DD t = row_dot_dd(A + (int64_t)prow * ld, v, n, lane).value();
  if (lane == 0) {
    th[row] = t.h;
    tl[row] = t.l;
  }
}

// norms[0], norms[1] and norms[kNormCw] cleared
__global__ void k_zero_norms(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
  if (threadIdx.x == 2) p[kNormCw] = 0ull;
}

__global__ __launch_bounds__(256) void k_residual_dd(const double* __restrict__ A, int64_t ld,
                                                     int n, const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     unsigned long long* norms) {
  const int row0 = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const bool rvalid = row0 < n;
  const int row = rvalid ? row0 : n - 1;  // out-of-range waves recompute a valid row
  double axabs;
  const DD ax = row_dot_dd<true>(A + (int64_t)row * ld, x, n, lane, &axabs).value();
  __shared__ double mr[4], mx[4], mc[4];
  const int wave = threadIdx.x / kWave;
  if (lane == 0) {
    // b - (ax.h + ax.l), rounded once to fp64
    const DD t = two_sum(b[row], -ax.h);
    const double ri = t.h + (t.l - ax.l);
    if (rvalid) r[row] = ri;
    mr[wave] = fabs(ri);
    mx[wave] = fabs(x[row]);
    mc[wave] = cw_ratio(fabs(ri), axabs + fabs(b[row]));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0, e = 0.0;
    const int nw = min(4, (n - (int)blockIdx.x * 4));
    for (int w = 0; w < nw; ++w) {
      a = fmax(a, mr[w]);
      c = fmax(c, mx[w]);
      e = fmax(e, mc[w]);
    }
    atomic_max_nonneg(norms + kNormCw, e);
    atomic_max_nonneg(norms + 0, a);
    atomic_max_nonneg(norms + 1, c);
  }
}

// ---------------------------------------------------------------------------
// Blocked triangular solves in double-double, one workgroup (4 waves) per
// 64-row block:
//   lower (unit): y_I = L_II^-1 (t_I - sum_{J < I} L_IJ y_J)
//   upper:        z_I = U_II^-1 (y_I - sum_{J > I} U_IJ z_J)
// The off-diagonal tiles of a block row are spread over the four waves
// (wave w takes every fourth tile), each lane one row, with compensated
// accumulation of the products of the exact u_f entries and the double-double
// solution.  The diagonal block is then solved by substitution in wave 0: lane
// i holds row i of the block and its right-hand side; at step j lane j's value
// is final (after the division by u_jj for the upper solve) and is broadcast to
// the other lanes, which subtract their multiple of it.  A finished block is
// published as four tagged words per row (hi and lo, 32 bits each, tagged with
// the launch's epoch in the upper half), stored with relaxed device-scope
// atomics; readers poll until all four tags of all 64 rows match.
// ---------------------------------------------------------------------------
constexpr int kDB = kTileCols;  // rows per workgroup

__device__ __forceinline__ void put_dd(uint64_t* xw, int row, DD v, uint32_t tag) {
  const uint64_t a = (uint64_t)__double_as_longlong(v.h);
  const uint64_t b = (uint64_t)__double_as_longlong(v.l);
  const uint64_t t = (uint64_t)tag << 32;
  uint64_t* p = xw + (int64_t)kDdWordsPerRow * row;
  __hip_atomic_store(p + 0, t | (a & 0xFFFFFFFFull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, t | (a >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 2, t | (b & 0xFFFFFFFFull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 3, t | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wave-uniform: lane reads row c0 + lane; false on abort (bounded wait)
__device__ __forceinline__ bool get_dd(const uint64_t* xw, int c0, uint32_t tag, DD& v,
                                       int* abortp) {
  const int lane = threadIdx.x % kWave;
  const uint64_t* p = xw + (int64_t)kDdWordsPerRow * (c0 + lane);
  long long spins = 0;
  for (;;) {
    const uint64_t w0 = __hip_atomic_load(p + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w1 = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w2 = __hip_atomic_load(p + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t w3 = __hip_atomic_load(p + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = (uint32_t)(w0 >> 32) == tag && (uint32_t)(w1 >> 32) == tag &&
                    (uint32_t)(w2 >> 32) == tag && (uint32_t)(w3 >> 32) == tag;
    if (__all(ok)) {
      v.h = __longlong_as_double((long long)((w1 << 32) | (w0 & 0xFFFFFFFFull)));
      v.l = __longlong_as_double((long long)((w3 << 32) | (w2 & 0xFFFFFFFFull)));
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    if (((++spins) & 1023) == 0) {
      if (__hip_atomic_load(abortp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (spins > (1ll << 22)) {
        __hip_atomic_store(abortp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
}

template <class F, bool kUpper>
__global__ __launch_bounds__(256) void k_trsv_dd(const typename F::T* __restrict__ S, int64_t ld,
                                                 const int* __restrict__ permS, int n,
                                                 const double* __restrict__ inh,
                                                 const double* __restrict__ inl,
                                                 const int* __restrict__ permIn,
                                                 double* __restrict__ yh, double* __restrict__ yl,
                                                 double scale, double* __restrict__ out64,
                                                 uint64_t* xw, uint32_t epoch,
                                                 const CycleState* gate, int step, int* abortp) {
  if (gated_off(gate, step)) return;
  __shared__ double ysh[4][kDB], ysl[4][kDB];
  __shared__ double ps[4][kDB], pc[4][kDB];
  __shared__ int wok[4];
  const int nt = (n + kDB - 1) / kDB;
  const int blk = kUpper ? nt - 1 - (int)blockIdx.x : (int)blockIdx.x;
  const int r0 = blk * kDB;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int row = r0 + lane;
  const bool valid = row < n;
  const int prow = valid ? (permS ? permS[row] : row) : 0;
  const typename F::T* srow = S + (int64_t)prow * ld;
  // wave 0's inputs of the substitution (the right-hand side and the row of
  // the diagonal block) are loaded before the waits, off the critical path;
  // the loads are unconditional and in bounds, their values used only for
  // valid rows
  DD tin{0.0, 0.0};
  DD rdiag{0.0, 0.0};  // upper: the double-double reciprocal of this row's pivot
  RawRow<F> dv;
  if (wave == 0) {
    dv.load(srow, r0, n, valid);
    const int src = valid ? (permIn ? permIn[row] : row) : 0;
    tin.h = inh[src];
    tin.l = inl ? inl[src] : 0.0;
    if (kUpper) {
      const double d = (double)F::to_f(srow[valid ? row : 0]);
      rdiag.h = 1.0 / d;
      rdiag.l = __builtin_fma(-d, rdiag.h, 1.0) * rdiag.h;
    }
  }
  Acc acc, acc1, acc2, acc3;
  bool ok = true;
  const int t0 = kUpper ? blk + 1 : 0;  // off-diagonal tiles [t0, t1)
  const int t1 = kUpper ? nt : blk;
  // lower: ascending from tile `wave`; upper: descending from the last tile
  for (int i = wave;; i += 4) {
    const int J = kUpper ? t1 - 1 - i : t0 + i;
    if (kUpper ? (J < t0) : (J >= t1)) break;
    RawRow<F> lv;
    lv.load(srow, J * kDB, n, valid);
    DD yv;
    if (!get_dd(xw, J * kDB, epoch, yv, abortp)) {
      ok = false;
      break;
    }
    ysh[wave][lane] = yv.h;
    ysl[wave][lane] = yv.l;
    __builtin_amdgcn_wave_barrier();
    // four interleaved compensated sums: the dependent chain through the
    // running sum is a quarter as long
#pragma unroll
    for (int c = 0; c < kDB; c += 4) {
      acc.add_prod(lv.at(c), ysh[wave][c], ysl[wave][c]);
      acc1.add_prod(lv.at(c + 1), ysh[wave][c + 1], ysl[wave][c + 1]);
      acc2.add_prod(lv.at(c + 2), ysh[wave][c + 2], ysl[wave][c + 2]);
      acc3.add_prod(lv.at(c + 3), ysh[wave][c + 3], ysl[wave][c + 3]);
    }
    __builtin_amdgcn_wave_barrier();
  }
  acc1.add(acc3);
  acc.add(acc2);
  acc.add(acc1);
  ps[wave][lane] = acc.s;
  pc[wave][lane] = acc.c;
  if (lane == 0) wok[wave] = ok ? 1 : 0;
  __syncthreads();
  if (!(wok[0] & wok[1] & wok[2] & wok[3])) return;
  if (wave != 0) return;
  Acc tot;
  tot.s = ps[0][lane];
  tot.c = pc[0][lane];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    Acc o;
    o.s = ps[w][lane];
    o.c = pc[w][lane];
    tot.add(o);
  }
  DD t{0.0, 0.0};
  if (valid) {
    const DD sum = tot.value();
    t = dd_add(tin, DD{-sum.h, -sum.l});
  }
  // substitution with the diagonal block (rows r0 .. r0 + nv - 1)
  const int nv = min(kDB, n - r0);
  if (!kUpper) {
#pragma unroll
    for (int j = 0; j < kDB - 1; ++j) {
      if (j + 1 >= nv) break;
      DD yj;
      yj.h = readlane_d(t.h, j);
      yj.l = readlane_d(t.l, j);
      if (lane > j) t = dd_sub_mul(t, dv.at(j), yj);
    }
  } else {
#pragma unroll
    for (int j = kDB - 1; j >= 0; --j) {
      if (j >= nv) continue;
      if (lane == j) t = dd_mul(t, rdiag);
      if (j == 0) break;
      DD yj;
      yj.h = readlane_d(t.h, j);
      yj.l = readlane_d(t.l, j);
      if (lane < j) t = dd_sub_mul(t, dv.at(j), yj);
    }
  }
  if (valid) {
    if (yh) yh[row] = t.h;
    if (yl) yl[row] = t.l;
    if (out64) out64[row] = (t.h + t.l) * scale;
  }
  put_dd(xw, row, valid ? t : DD{0.0, 0.0}, epoch);
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_gemv_dd(const double* A, int64_t ld, const int* permA, int n, const double* v,
                    double* th, double* tl, const CycleState* gate, int step, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_dd, dim3(nblocks(n, 4)), dim3(256), 0, s, A, ld, permA, n, v, th, tl,
                     gate, step);
}

void launch_residual_dd(const double* A, int64_t ld, int n, const double* b, const double* x,
                        double* r, unsigned long long* norms, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_norms, dim3(1), dim3(64), 0, s, norms);
  hipLaunchKernelGGL(k_residual_dd, dim3(nblocks(n, 4)), dim3(256), 0, s, A, ld, n, b, x, r,
                     norms);
}

void launch_trsv_dd(const void* S, int64_t ld, const int* permS, int store, int n, bool upper,
                    const double* inh, const double* inl, const int* permIn, double* yh,
                    double* yl, double scale, double* out64, uint64_t* xw, int epoch,
                    const CycleState* gate, int step, int* abortp, hipStream_t s) {
  const unsigned grid = nblocks(n, kDB);
#define GIR_TD(F, U)                                                                          \
  hipLaunchKernelGGL((k_trsv_dd<F, U>), dim3(grid), dim3(256), 0, s,                          \
                     reinterpret_cast<const typename F::T*>(S), ld, permS, n, inh, inl, permIn, \
                     yh, yl, scale, out64, xw, (uint32_t)epoch, gate, step, abortp)
  if (store == kStoreF16) {
    if (upper) GIR_TD(Fp16, true); else GIR_TD(Fp16, false);
  } else if (store == kStoreBF16) {
    if (upper) GIR_TD(Bf16, true); else GIR_TD(Bf16, false);
  } else {
    if (upper) GIR_TD(Fp32, true); else GIR_TD(Fp32, false);
  }
#undef GIR_TD
}

}  // namespace gir
