// LU factorisation with partial pivoting in u_f on gfx950 (the factorisation
// step of Algorithms 1-3; GEPP as in Section 1 of the paper).
//
// Blocked right-looking GEPP with "lazy" row interchanges: rows are never
// moved in memory during the factorisation; a permutation vector maps the
// logical (pivoted) row order to physical rows, and every kernel gathers rows
// through it.  The pivot choice is LAPACK's: the first row, in logical order,
// attaining max |a| in the current column.
//
// Rounding points (shared with the CPU reference): a block column of nb
// columns is factored in fp32 (fused multiply-adds, IEEE division) and written
// back in u_f; the block row to its right is solved with the stored u_f unit
// lower triangle in fp32 and written in u_f; the trailing matrix is updated
// with u_f inputs on the matrix cores with fp32 accumulation and rounded to
// u_f once per block column.
//
// Block column = one kernel: every thread keeps one row of the block column
// in registers while the workgroups agree on each pivot through tagged words
// in a small exchange buffer (one record per workgroup and column parity).
#include <type_traits>

#include "kernels.h"

namespace gir {

namespace {

constexpr int kMaxNb = 64;

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// One pass over the caller's A: the fp64 copy (A64, zero padded to ld), the
// fp32 copy A_u (if requested), max |a| and the largest row sum (one atomic
// per block each) and a flag for non-finite entries.  One wave per row.
__global__ __launch_bounds__(256) void k_ingest(const double* __restrict__ A, int64_t n,
                                                int64_t lda, double* __restrict__ A64,
                                                float* __restrict__ Au, int64_t ld,
                                                unsigned long long* norms, int* flag) {
  __shared__ double smax[4], ssum[4];
  __shared__ int sbad[4];
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  double s = 0.0, mx = 0.0;
  int bad = 0;
  if (row < n) {
    const double* a = A + row * lda;
    double* d = A64 + row * ld;
    float* f = Au ? Au + row * ld : nullptr;
    // lane takes columns lane + 64 i in order (the row sum's order); four of
    // them are loaded before any is used, for more loads in flight
    auto put = [&](int64_t c, double v) {
      d[c] = v;
      if (f) f[c] = (float)v;
      if (!__builtin_isfinite(v)) bad = 1;
      const double av = fabs(v);
      s += av;
      mx = fmax(mx, av);
    };
    int64_t c = lane;
    for (; c + 3 * kWave < ld; c += 4 * kWave) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (c + u * kWave < n) ? a[c + u * kWave] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) put(c + u * kWave, v[u]);
    }
    for (; c < ld; c += kWave) put(c, (c < n) ? a[c] : 0.0);
  }
  s = wave_sum(s);
  mx = wave_max_d(mx);
  bad = __any(bad);
  if (lane == 0) {
    smax[wave] = mx;
    ssum[wave] = s;
    sbad[wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0, r = 0.0;
    int b = 0;
    for (int w = 0; w < 4; ++w) {
      m = fmax(m, smax[w]);
      r = fmax(r, ssum[w]);
      b |= sbad[w];
    }
    atomic_max_nonneg(norms + 0, m);
    atomic_max_nonneg(norms + 1, r);
    if (b) atomicOr(flag, 1);
  }
}

// Largest integer e with 2^e * amax * sqrt(n) <= 4094 (exact power-of-two
// scaling of A before rounding to fp16; sqrt(n) is passed in so that host and
// device agree bit for bit).
__device__ __forceinline__ int fp16_scale_exponent_dev(double amax, double sqrtn) {
  if (!(amax > 0.0) || !__builtin_isfinite(amax)) return 0;
  const double t = amax * sqrtn;
  const double limit = 4094.0;
  int e = (int)floor(log2(limit) - log2(t));
  while (ldexp(t, e) > limit) --e;
  while (ldexp(t, e + 1) <= limit) ++e;
  return e;
}

// S = fl_uf(2^e A64) with e from max |a| (norms[0]) when `scaled`, else 0;
// e is also written to e_out; flag[0] = 1 if a u_f value overflowed.
template <class F>
__global__ __launch_bounds__(256) void k_convert_scaled(const double* __restrict__ A64, int64_t n,
                                                        int64_t ld, typename F::T* __restrict__ S,
                                                        const unsigned long long* __restrict__ norms,
                                                        double sqrtn, int scaled, int* e_out,
                                                        int* flag) {
  __shared__ int se;
  if (threadIdx.x == 0) {
    se = scaled ? fp16_scale_exponent_dev(__longlong_as_double((long long)norms[0]), sqrtn) : 0;
    if (blockIdx.x == 0) *e_out = se;
  }
  __syncthreads();
  const int e = se;
  int bad = 0;
  // ld is a multiple of 64: the matrix is a whole number of 2-element pieces
  const int64_t pairs = n * ld / 2;
  const double2* src = reinterpret_cast<const double2*>(A64);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = src[i];
    const typename F::T a = F::from_d(ldexp(v.x, e));
    const typename F::T b = F::from_d(ldexp(v.y, e));
    if (!F::finite(a) || !F::finite(b)) bad = 1;
    S[2 * i] = a;
    S[2 * i + 1] = b;
  }
  if (__any(bad) && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

__global__ void k_iota(int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int)i;
}

__global__ void k_copy_i32(int* __restrict__ dst, const int* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// span blockIdx.y of the list, grid-strided over blockIdx.x
__global__ void k_zero_spans(ZeroSpans z) {
  const int j = blockIdx.y;
  int* p = z.p[j];
  const int64_t n = z.n[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---- block column: one pivot search per column across workgroups -----------
//
// G = ceil(h / 512) workgroups; thread t of workgroup g owns logical row
// q = 512 g + t of the block column and keeps all of its (at most 64) values in
// registers from the gather to the write-back.  Per column c:
//   1. every unpivoted row forms the key (|a_qc| bits, inverted logical index),
//      so that the maximum key is LAPACK's pivot: largest magnitude, first
//      logical row among equals;
//   2. the workgroup maximum is found with DPP reductions and one LDS pass,
//      and the owner of that key copies its row to LDS;
//   3. with G > 1, wave 0 publishes the key and the row as 64-bit words whose
//      upper half carries the column's tag (k0 + c + 1); one poll fetches
//      all G records (keys and rows) and the winner is picked locally.  A
//      word is valid once its tag matches, so no fences or flags are needed;
//      records alternate between two slots by column parity (a workgroup can
//      be at most one column ahead of any other);
//   4. every row eliminates column c with the correctly rounded quotient and
//      one fused multiply-add per remaining column, in the order of the
//      unblocked algorithm.
// Row interchanges stay lazy: lid tracks each row's logical position, and the
// permutation is rewritten once at the end.
constexpr int kRowThreads = 512;
constexpr int kRowWaves = kRowThreads / kWave;
constexpr int kRecWords = 80;  // 64 row words + key word, padded to 640 bytes

__device__ __forceinline__ uint64_t xch_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void xch_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 64 values of a row from a 16-byte aligned address whose 64-element span
// lies inside the padded row (k0 + 64 <= ld); columns >= kb read as zero
template <class F>
__device__ __forceinline__ void load_panel_row(const typename F::T* src, int kb, bool in,
                                               float (&x)[kMaxNb]) {
  using T = typename F::T;
  constexpr int kPer = 16 / sizeof(T);
  if (in) {
#pragma unroll
    for (int v = 0; v < kMaxNb / kPer; ++v) {
      const uint4 w = reinterpret_cast<const uint4*>(src)[v];
      T t[kPer];
      __builtin_memcpy(t, &w, 16);
#pragma unroll
      for (int e = 0; e < kPer; ++e)
        x[v * kPer + e] = (v * kPer + e < kb) ? F::to_f(t[e]) : 0.0f;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kMaxNb; ++c) x[c] = 0.0f;
  }
}

template <class F>
__device__ __forceinline__ void store_panel_row(typename F::T* dst, int kb, float (&x)[kMaxNb]) {
  using T = typename F::T;
  constexpr int kPer = 16 / sizeof(T);
  // fp32 values first, then the rounding to u_f (no fma fused with the
  // narrowing conversion, which would round once instead of twice)
#pragma unroll
  for (int c = 0; c < kMaxNb; ++c) asm volatile("" : "+v"(x[c]));
  if (kb == kMaxNb) {
#pragma unroll
    for (int v = 0; v < kMaxNb / kPer; ++v) {
      T t[kPer];
#pragma unroll
      for (int e = 0; e < kPer; ++e) t[e] = F::from_f(x[v * kPer + e]);
      uint4 w;
      __builtin_memcpy(&w, t, 16);
      reinterpret_cast<uint4*>(dst)[v] = w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kMaxNb; ++c)
      if (c < kb) dst[c] = F::from_f(x[c]);
  }
}

// elimination of column C for one row: x_C <- l, x_j <- fma(-l, u_j, x_j) for
// j > C; returns the row's value in column C + 1 (the next pivot search)
// (u is 16-byte aligned: the aligned part is read four values at a time)
template <int C>
__device__ __forceinline__ float eliminate_col(float (&x)[kMaxNb], float l, const float* u) {
  constexpr int kJ0 = C + 1;
  constexpr int kJA = (kJ0 + 3) & ~3;
  x[C] = l;
#pragma unroll
  for (int j = kJ0; j < kJA && j < kMaxNb; ++j) x[j] = __builtin_fmaf(-l, u[j], x[j]);
#pragma unroll
  for (int j = kJA; j < kMaxNb; j += 4) {
    const float4 w = *reinterpret_cast<const float4*>(u + j);
    x[j] = __builtin_fmaf(-l, w.x, x[j]);
    x[j + 1] = __builtin_fmaf(-l, w.y, x[j + 1]);
    x[j + 2] = __builtin_fmaf(-l, w.z, x[j + 2]);
    x[j + 3] = __builtin_fmaf(-l, w.w, x[j + 3]);
  }
  return x[C + 1 < kMaxNb ? C + 1 : C];
}

constexpr int kMaxPanelWgs = 32;  // h <= 16384

struct PanelSmem {
  uint64_t kw[kRowWaves];
  uint64_t s_win;
  int s_gw;
  int s_abort;
  alignas(16) float rowbuf[kMaxNb];
  alignas(16) float recv[kMaxPanelWgs][kMaxNb];
  alignas(16) float rowsave[kMaxNb][kMaxNb];  // pivot rows owned by this workgroup
};

template <class T>
struct PreSmem;
template <class T>
struct PanelPreSmem;
template <class F, bool kSolve>
__device__ __forceinline__ void block_column_update(PreSmem<typename F::T>& ps,
                                                    const typename F::T* __restrict__ S,
                                                    int64_t ld, int uk0, int phys, bool in,
                                                    const int* __restrict__ perm, int k0,
                                                    float (&x)[kMaxNb]);

// Block column k0 .. k0 + kb - 1 over rows k0 .. k0 + h - 1 (logical), run by
// workgroup g of the G that share it (512 threads each).  With kFold > 0, the
// block column's rows first receive step uk0's trailing update from these
// same workgroups (block_column_update) instead of a launch before; with
// kFold == 2 they also solve step uk0's block row in this block column.
template <class F, int kFold = 0>
__device__ __forceinline__ void panel_rows(PanelSmem& sm, typename F::T* __restrict__ S,
                                           int64_t ld, int* __restrict__ perm, int k0, int kb,
                                           int h, int G, int g, int* __restrict__ ipiv,
                                           int* __restrict__ perm_copy,
                                           uint64_t* __restrict__ xch, CycleState* st,
                                           PreSmem<typename F::T>* ps = nullptr, int uk0 = 0) {
  using T = typename F::T;
  uint64_t* kw = sm.kw;
  float* rowbuf = sm.rowbuf;
  auto& recv = sm.recv;
  auto& rowsave = sm.rowsave;
  uint64_t& s_win = sm.s_win;
  int& s_gw = sm.s_gw;
  int& s_abort = sm.s_abort;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wave = tid / kWave;
  const int q = g * kRowThreads + tid;
  const bool in = q < h;
  int* abortp = &st->abort;

  const int phys = in ? perm[k0 + q] : 0;
  T* row = S + (int64_t)phys * ld + k0;
  float x[kMaxNb];
  if constexpr (kFold > 0)
    block_column_update<F, kFold == 2>(*ps, S, ld, uk0, phys, in, perm, k0, x);  // kb == kMaxNb
  else
    load_panel_row<F>(row, kb, in, x);
  // materialise the fp32 values now (keeps the compiler from carrying the
  // narrow inputs and converting them at every later use)
#pragma unroll
  for (int c = 0; c < kMaxNb; ++c) asm volatile("" : "+v"(x[c]));
  int lid = q;
  bool pv = !in;  // pivoted (or absent) rows take no part in the pivot search
  float xc = x[0];
  if (tid == 0) s_abort = 0;

  for (int c = 0; c < kb; ++c) {
    const uint32_t tag = (uint32_t)(k0 + c + 1);
    const float ac = fabsf(xc);
    const uint32_t ab = (ac == ac) ? __float_as_uint(ac) : 0u;  // NaN ranks as zero
    const uint64_t mykey =
        pv ? 0ull : (((uint64_t)ab << 17) | (uint64_t)(0x1FFFFu - (uint32_t)lid));
    // the wave's largest key by two 32-bit reductions: the largest magnitude
    // (+1, so that an unpivoted zero still outranks the pivoted rows), then,
    // only when several rows attain it, the first of them in logical order
    const uint32_t am = pv ? 0u : ab + 1u;
    const uint32_t mw = wave_max_u32(am);
    const bool cand = mw != 0u && am == mw;
    const uint32_t il = cand ? (0x1FFFFu - (uint32_t)lid) : 0u;
    const unsigned long long bal = __ballot(cand);
    const uint32_t ilw = (__builtin_popcountll(bal) == 1)
                             ? (uint32_t)__builtin_amdgcn_readlane((int)il, __builtin_ctzll(bal))
                             : wave_max_u32(il);
    const uint64_t wmax = mw ? (((uint64_t)(mw - 1u) << 17) | ilw) : 0ull;
    if (lane == 0) kw[wave] = wmax;
    __syncthreads();
    uint64_t K = kw[0];
#pragma unroll
    for (int w = 1; w < kRowWaves; ++w) K = kw[w] > K ? kw[w] : K;
    if (!pv && mykey == K) {
#pragma unroll
      for (int j = 0; j < kMaxNb; j += 4)
        *reinterpret_cast<float4*>(&rowbuf[j]) = make_float4(x[j], x[j + 1], x[j + 2], x[j + 3]);
    }
    __syncthreads();
    uint64_t W = K;
    const float* u = rowbuf;
    if (G > 1) {
      // one round trip: every record's row words are fetched together with
      // the keys, the winner's row is then taken from LDS
      uint64_t* base = xch + (size_t)(c & 1) * G * kRecWords;
      if (wave == 0) {
        uint64_t* mine = base + (size_t)g * kRecWords;
        xch_store(mine + lane, ((uint64_t)tag << 32) | __float_as_uint(rowbuf[lane]));
        if (lane == 0) xch_store(mine + kMaxNb, ((uint64_t)tag << 48) | K);
      }
      bool ok = true;
      uint64_t v[kMaxPanelWgs * kMaxNb / kRowThreads];
      uint64_t kk = 0;  // wave 0, lane < G: the key word of record `lane`
      {
        long long spins = 0;
        for (;;) {
          // every load is issued, unconditionally and in bounds (slots of
          // records >= G lie inside the exchange buffer and are ignored),
          // before any is checked: one memory round trip per poll, where
          // loads under per-record branches were each waited for in turn
#pragma unroll
          for (int i = 0; i < kMaxPanelWgs * kMaxNb / kRowThreads; ++i) {
            const int f = tid + kRowThreads * i;
            v[i] = xch_load(base + (size_t)(f >> 6) * kRecWords + (f & 63));
          }
          if (wave == 0)
            kk = xch_load(base + (size_t)(lane & (kMaxPanelWgs - 1)) * kRecWords + kMaxNb);
          bool got = true;
#pragma unroll
          for (int i = 0; i < kMaxPanelWgs * kMaxNb / kRowThreads; ++i) {
            const int f = tid + kRowThreads * i;
            got = got && ((f >> 6) >= G || (uint32_t)(v[i] >> 32) == tag);
          }
          if (wave == 0) got = got && (lane >= G || (uint32_t)(kk >> 48) == tag);
          if (__all(got)) break;
          __builtin_amdgcn_s_sleep(1);
          if (((++spins) & 1023) == 0) {
            if (__hip_atomic_load(abortp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                spins > (1ll << 22)) {
              __hip_atomic_store(abortp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ok = false;
              break;
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < kMaxPanelWgs * kMaxNb / kRowThreads; ++i) {
        const int f = tid + kRowThreads * i;
        if ((f >> 6) < G) recv[f >> 6][f & 63] = __uint_as_float((uint32_t)v[i]);
      }
      if (wave == 0) {
        const uint64_t kv = (lane < G) ? (kk & 0xFFFFFFFFFFFFull) : 0ull;
        const uint64_t wk = wave_max_u64(kv);
        const unsigned long long bal = __ballot(lane < G && kv == wk);
        if (lane == 0) {
          s_win = wk;
          s_gw = (int)__builtin_ctzll(bal);
        }
      }
      if (!ok) s_abort = 1;
      __syncthreads();
      if (s_abort) return;
      W = s_win;
      u = recv[s_gw];
    }
    // the workgroup that owns the pivot row keeps its values (final once
    // chosen) for the write-back at the end
    if (wave == 0 && (G == 1 || s_gw == g)) rowsave[c][lane] = rowbuf[lane];
    const int wl = (int)(0x1FFFFu - (uint32_t)(W & 0x1FFFFull));
    const float piv = u[c];
    if (g == 0 && tid == 0) {
      ipiv[k0 + c] = k0 + wl;
      if (piv == 0.0f) atomicCAS(&st->singular, 0, k0 + c + 1);
    }
    if (!pv && lid == wl) {
      // the pivot row: its final values are in rowsave[c]; its registers are
      // eliminated with the others below (to zeros) and not stored
      lid = c;
      pv = true;
    } else if (!pv && lid == c) {
      lid = wl;
    }
    if (piv != 0.0f) {
      // fl32(a / piv) from the reciprocal, the product and one fused
      // correction (Markstein); quotients near the subnormal range and an
      // infinite reciprocal fall back to the division
      const float a = xc;
      const float rinv = 1.0f / piv;
      float l;
      if (__builtin_isfinite(rinv)) {
        const float q0 = a * rinv;
        const float e = __builtin_fmaf(-q0, piv, a);
        l = __builtin_fmaf(e, rinv, q0);
        if (__builtin_expect(fabsf(l) < 0x1p-100f, 0) && a != 0.0f) l = a / piv;
      } else {
        l = a / piv;
      }
      switch (c) {
#define GIR_ELIM(C) \
  case C:           \
    xc = eliminate_col<C>(x, l, u); \
    break;
#define GIR_ELIM8(C) \
  GIR_ELIM(C) GIR_ELIM(C + 1) GIR_ELIM(C + 2) GIR_ELIM(C + 3) GIR_ELIM(C + 4) GIR_ELIM(C + 5) \
  GIR_ELIM(C + 6) GIR_ELIM(C + 7)
        GIR_ELIM8(0)
        GIR_ELIM8(8)
        GIR_ELIM8(16)
        GIR_ELIM8(24)
        GIR_ELIM8(32)
        GIR_ELIM8(40)
        GIR_ELIM8(48)
        GIR_ELIM8(56)
#undef GIR_ELIM8
#undef GIR_ELIM
        default:
          break;
      }
    } else {
      // singular column: nothing is eliminated (LAPACK's convention)
      switch (c) {
#define GIR_NEXT(C) \
  case C:           \
    xc = x[C + 1 < kMaxNb ? C + 1 : C]; \
    break;
#define GIR_NEXT8(C) \
  GIR_NEXT(C) GIR_NEXT(C + 1) GIR_NEXT(C + 2) GIR_NEXT(C + 3) GIR_NEXT(C + 4) GIR_NEXT(C + 5) \
  GIR_NEXT(C + 6) GIR_NEXT(C + 7)
        GIR_NEXT8(0)
        GIR_NEXT8(8)
        GIR_NEXT8(16)
        GIR_NEXT8(24)
        GIR_NEXT8(32)
        GIR_NEXT8(40)
        GIR_NEXT8(48)
        GIR_NEXT8(56)
#undef GIR_NEXT8
#undef GIR_NEXT
        default:
          break;
      }
    }
  }
  if constexpr (kFold == 2) {
    // U12 of the block row of step uk0 in this block column: every
    // workgroup has read the unsolved values (its prologue precedes its
    // first pivot record, and all records of the last column are in)
    if (g == 0) {
      constexpr int V = 16 / (int)sizeof(T);
      const auto& pp = *reinterpret_cast<const PanelPreSmem<T>*>(ps);
      const int t = tid / (kMaxNb / V), pc = tid % (kMaxNb / V);
      *reinterpret_cast<uint4*>(S + (int64_t)perm[uk0 + t] * ld + k0 + pc * V) =
          *reinterpret_cast<const uint4*>(&pp.u12[t][pc * V]);
    }
  }
  if (in) {
    if (pv) {
#pragma unroll
      for (int j = 0; j < kMaxNb; ++j) x[j] = rowsave[lid][j];
    }
    store_panel_row<F>(row, kb, x);
    // every workgroup read its permutation entries before publishing its
    // first key, and no workgroup gets here before it has read every
    // workgroup's last key: the in-place rewrite is safe
    perm[k0 + lid] = phys;
    if (perm_copy) perm_copy[k0 + lid] = phys;
  }
}

template <class F>
__global__ __launch_bounds__(kRowThreads) void k_panel(typename F::T* __restrict__ S, int64_t ld,
                                                       int* __restrict__ perm, int k0, int kb,
                                                       int h, int* __restrict__ ipiv,
                                                       int* __restrict__ perm_copy,
                                                       uint64_t* __restrict__ xch,
                                                       CycleState* st) {
  __shared__ PanelSmem sm;
  panel_rows<F>(sm, S, ld, perm, k0, kb, h, (int)gridDim.x, (int)blockIdx.x, ipiv, perm_copy, xch,
                st);
}

// U12 = L11^-1 A12 in fp32 with the stored (u_f) unit lower triangle L11
// (the block column is always 64 wide here: a narrower one is the last and
// has nothing to its right).  Four lanes share a column: lane p of a quad
// keeps rows 4 i + p (i < 16) in registers, and at step t the quad's owner of
// row t hands y_t to the other three by a DPP quad broadcast.  L11 is staged
// in LDS by row class (Lq[t][p][i] = L11[4 i + p][t]) and read as 16-byte
// broadcast vectors.  Step t updates rows r > t with one fused multiply-add
// each, so every entry receives its terms in the order t = 0, 1, ... of
// forward substitution.
constexpr int kTrsmThreads = 64;
constexpr int kTrsmCols = kTrsmThreads / 4;  // columns per workgroup
constexpr int kTrsmLq = 20;                   // padded row class (floats): no bank conflicts

template <int P>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), P * 0x55, 0xf, 0xf, false));
}

// L11 (unit lower, pivot rows prow[0 .. 63] of the block column at k0) by row
// class: Lq[t][r % 4][r / 4] = L(r, t).  Called by threads 0 .. 63 (row = tid).
template <class F>
__device__ __forceinline__ void stage_l11(float (&Lq)[kMaxNb][4][kTrsmLq],
                                          const typename F::T* __restrict__ S, int64_t ld,
                                          int prow_t, int k0, int tid) {
  // entries on and above the diagonal are never read
  float lrow[kMaxNb];
  load_panel_row<F>(S + (int64_t)prow_t * ld + k0, kMaxNb, true, lrow);
#pragma unroll
  for (int t = 0; t < kMaxNb; ++t) Lq[t][tid & 3][tid >> 2] = lrow[t];
}

// Forward substitution with the unit lower L11 for one column of the block
// row, held by a quad of lanes: lane p of the quad keeps rows 4 i + p in
// y[i].  Row r receives -l_rt y_t for t = 0, 1, ..., r - 1 in that order,
// one fused multiply-add each in fp32; y_t reaches the quad from its owner by
// a DPP quad broadcast.
__device__ __forceinline__ void trsm_quad(float (&y)[kMaxNb / 4],
                                          const float (&Lq)[kMaxNb][4][kTrsmLq], int p) {
#define GIR_TRSM_STEP(T)                                                                  \
  {                                                                                       \
    constexpr int ti = (T) >> 2, tp = (T) & 3;                                            \
    const float yt = quad_bcast<tp>(y[ti]);                                               \
    const float* lq = &Lq[T][p][0];                                                       \
    _Pragma("unroll") for (int j = ti & ~3; j < kMaxNb / 4; j += 4) {                     \
      const float4 lv = *reinterpret_cast<const float4*>(lq + j);                         \
      const float l4[4] = {lv.x, lv.y, lv.z, lv.w};                                       \
      _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                     \
        const int i = j + e;                                                              \
        if (i > ti)                                                                       \
          y[i] = __builtin_fmaf(-l4[e], yt, y[i]);                                        \
        else if (i == ti)                                                                 \
          y[i] = (p > tp) ? __builtin_fmaf(-l4[e], yt, y[i]) : y[i];                      \
      }                                                                                   \
    }                                                                                     \
  }
#define GIR_TRSM_STEP4(T) GIR_TRSM_STEP(T) GIR_TRSM_STEP(T + 1) GIR_TRSM_STEP(T + 2) GIR_TRSM_STEP(T + 3)
  GIR_TRSM_STEP4(0) GIR_TRSM_STEP4(4) GIR_TRSM_STEP4(8) GIR_TRSM_STEP4(12)
  GIR_TRSM_STEP4(16) GIR_TRSM_STEP4(20) GIR_TRSM_STEP4(24) GIR_TRSM_STEP4(28)
  GIR_TRSM_STEP4(32) GIR_TRSM_STEP4(36) GIR_TRSM_STEP4(40) GIR_TRSM_STEP4(44)
  GIR_TRSM_STEP4(48) GIR_TRSM_STEP4(52) GIR_TRSM_STEP4(56) GIR_TRSM_STEP(60)
  GIR_TRSM_STEP(61) GIR_TRSM_STEP(62)
#undef GIR_TRSM_STEP4
#undef GIR_TRSM_STEP
  // the fp32 result is rounded to u_f in a separate step by the caller (an
  // fma fused with the narrowing conversion would round only once)
#pragma unroll
  for (int i = 0; i < kMaxNb / 4; ++i) asm volatile("" : "+v"(y[i]));
}

template <class F>
__global__ __launch_bounds__(kTrsmThreads) void k_trsm(typename F::T* __restrict__ S, int64_t ld,
                                                       const int* __restrict__ perm, int k0,
                                                       int c_begin, int c_end) {
  __shared__ __align__(16) float Lq[kMaxNb][4][kTrsmLq];
  __shared__ int prow[kMaxNb];
  const int tid = threadIdx.x;
  const int p = tid & 3;
  const int64_t c = (int64_t)c_begin + (int64_t)blockIdx.x * kTrsmCols + (tid >> 2);
  prow[tid] = perm[k0 + tid];
  __syncthreads();
  // this lane's rows of its column, loaded together with the L11 row below
  // (one memory round trip for both); a lane beyond c_end reads a valid
  // column and discards it
  const int64_t cc = c < c_end ? c : (int64_t)c_begin;
  typename F::T yraw[kMaxNb / 4];
#pragma unroll
  for (int i = 0; i < kMaxNb / 4; ++i) yraw[i] = S[(int64_t)prow[4 * i + p] * ld + cc];
  stage_l11<F>(Lq, S, ld, prow[tid], k0, tid);
  __syncthreads();
  if (c >= c_end) return;  // whole quads: the four lanes of a column leave together
  float y[kMaxNb / 4];
#pragma unroll
  for (int i = 0; i < kMaxNb / 4; ++i) y[i] = F::to_f(yraw[i]);
#pragma unroll
  for (int i = 0; i < kMaxNb / 4; ++i) asm volatile("" : "+v"(y[i]));
  trsm_quad(y, Lq, p);
#pragma unroll
  for (int i = 0; i < kMaxNb / 4; ++i) S[(int64_t)prow[4 * i + p] * ld + c] = F::from_f(y[i]);
}

// ---- trailing update on the matrix cores ----------------------------------

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));
typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;
constexpr int kKP = kMaxNb + 8;  // padded LDS row of -L21 and U12^T (elements, 16-byte multiple)

template <class F>
struct Mfma;

// gfx950's 16-deep fp16 / bf16 products: A rows i = lane % 32 with k =
// 8 (lane / 32) + e, B columns j = lane % 32 with the same k, e = 0 .. 7 (one
// 16-byte LDS read per operand); the 32 x 32 fp32 result as with the 8-deep
// form
template <>
struct Mfma<Fp16> {
  static __device__ __forceinline__ float16_t step(const _Float16* a, const _Float16* b,
                                                   float16_t acc) {
    const half8_t av = *reinterpret_cast<const half8_t*>(a);
    const half8_t bv = *reinterpret_cast<const half8_t*>(b);
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc, 0, 0, 0);
  }
};

template <>
struct Mfma<Bf16> {
  static __device__ __forceinline__ float16_t step(const uint16_t* a, const uint16_t* b,
                                                   float16_t acc) {
    bf16x8_t av, bv;
    __builtin_memcpy(&av, a, 16);
    __builtin_memcpy(&bv, b, 16);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
};

// C tile 128 x 128 of the trailing matrix, rows gathered through `rows`:
// C <- fl_uf(C + sum_k (-L21)(:,k) U12(k,:)).  The product is accumulated on
// the matrix cores from zero and added to C once: in fp32 for fp16 / bf16
// factors (32 x 32 blocks), in fp64 for fp32 factors (16 x 16 x 4 fp64
// blocks: the fp32 products are exact and their sum is rounded to fp32 once,
// as fp32 accumulation of 64 terms would not be for an fp32 result).  Every
// operand moves between HBM and LDS in 16-byte coalesced pieces (the -L21
// block, U12 transposed, and C both ways).
constexpr int kCP = kTile + 8;  // padded LDS row of the C tile (elements)

template <class T>
struct GemmSmem {
  alignas(16) T As[kTile][kKP];
  alignas(16) T Bt[kTile][kKP];
  alignas(16) T Cs[kTile][kCP];
  int rowp[kTile];
  int krow[kMaxNb];
};

// The update tiles of a block column launch that also solve their part of
// the block row (see gemm_tile)
template <class T>
struct GemmTrsmSmem {
  GemmSmem<T> g;
  alignas(16) float Lq[kMaxNb][4][kTrsmLq];
  int arrived;
};

// One 128 x 128 tile (bx, by) of the trailing update for columns
// [c_begin, c_end), rows through `rows`, by a workgroup of 512 threads
// (8 waves: 2 x 4 blocks of 64 x 32).
//
// With kTrsm the tile also solves its 128 columns of the block row (U12 =
// L11^-1 A12, a quad per column as k_trsm solves them) instead of reading
// them solved: every tile of a column strip forms the same U12 from the
// unsolved values, and the last of the strip's tiles to finish (counted in
// strip_cnt[bx], ty tiles per strip) writes U12 back, when every tile of the
// strip has read the unsolved values.
template <class F, bool kTrsm = false>
__device__ __forceinline__ void gemm_tile(GemmSmem<typename F::T>& sm,
                                          typename F::T* __restrict__ S, int64_t ld,
                                          const int* __restrict__ perm,
                                          const int* __restrict__ rows, int k0, int kb, int n,
                                          int c_begin, int c_end, int bx, int by,
                                          int* __restrict__ strip_cnt = nullptr, int ty = 0) {
  using T = typename F::T;
  constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte piece
  constexpr int NT = kRowThreads;
  auto& As = sm.As;
  auto& Bt = sm.Bt;
  auto& Cs = sm.Cs;
  int* rowp = sm.rowp;
  int* krow = sm.krow;
  const int tid = threadIdx.x;
  const int M = n - k0 - kb;  // trailing rows (logical k0 + kb ..), through `rows`
  const int tm = by * kTile;
  const int tn = c_begin + bx * kTile;  // first column of the tile
  if (tid < kTile) rowp[tid] = (tm + tid < M) ? rows[k0 + kb + tm + tid] : -1;
  if (tid < kMaxNb) krow[tid] = (tid < kb) ? perm[k0 + tid] : -1;
  __syncthreads();
  // -L21: 128 rows x 64 (kb == 64 whenever there is a trailing matrix)
  for (int q = tid; q < kTile * (kMaxNb / V); q += NT) {
    const int r = q / (kMaxNb / V), kc = q % (kMaxNb / V);
    T t[V];
    if (rowp[r] >= 0) {
      const uint4 w = *reinterpret_cast<const uint4*>(S + (int64_t)rowp[r] * ld + k0 + kc * V);
      __builtin_memcpy(t, &w, 16);
#pragma unroll
      for (int e = 0; e < V; ++e) t[e] = F::from_f(-F::to_f(t[e]));
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) t[e] = F::from_f(0.0f);
    }
    uint4 w2;
    __builtin_memcpy(&w2, t, 16);
    *reinterpret_cast<uint4*>(&As[r][kc * V]) = w2;
  }
  // U12 rows k, columns tn .. tn + 127, stored transposed
  [[maybe_unused]] T yraw[kMaxNb / 4];
  [[maybe_unused]] auto& gt = reinterpret_cast<GemmTrsmSmem<T>&>(sm);
  if constexpr (!kTrsm) {
    for (int q = tid; q < kMaxNb * (kTile / V); q += NT) {
      const int k = q / (kTile / V), cc = q % (kTile / V);
      const int c = tn + cc * V;
      T t[V];
      if (c < ld) {
        const uint4 w = *reinterpret_cast<const uint4*>(S + (int64_t)krow[k] * ld + c);
        __builtin_memcpy(t, &w, 16);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) Bt[cc * V + e][k] = (c + e < c_end) ? t[e] : F::from_f(0.0f);
    }
  } else {
    // quad tid / 4 takes column tn + tid / 4 of the unsolved block row (a
    // quad past c_end reads column tn and discards it), threads 0 .. 63 L11
    static_assert(kTile * 4 == NT, "a quad per column of the tile");
    const int c = tn + (tid >> 2);
    const int cc = c < c_end ? c : tn;
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i)
      yraw[i] = S[(int64_t)krow[4 * i + (tid & 3)] * ld + cc];
    if (tid < kMaxNb) stage_l11<F>(gt.Lq, S, ld, krow[tid], k0, tid);
  }
  // C tile
  for (int q = tid; q < kTile * (kTile / V); q += NT) {
    const int r = q / (kTile / V), cc = q % (kTile / V);
    const int c = tn + cc * V;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (rowp[r] >= 0 && c < ld) w = *reinterpret_cast<const uint4*>(S + (int64_t)rowp[r] * ld + c);
    *reinterpret_cast<uint4*>(&Cs[r][cc * V]) = w;
  }
  __syncthreads();
  if constexpr (kTrsm) {
    const int cq = tid >> 2, pq = tid & 3;
    float y[kMaxNb / 4];
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) y[i] = F::to_f(yraw[i]);
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) asm volatile("" : "+v"(y[i]));
    trsm_quad(y, gt.Lq, pq);
    const bool live = tn + cq < c_end;
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i)
      Bt[cq][4 * i + pq] = live ? F::from_f(y[i]) : F::from_f(0.0f);
    __syncthreads();
  }
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int wr = (wave / 4) * 64;
  const int wc = (wave % 4) * 32;
  if constexpr (sizeof(T) == 4) {
    // 4 x 2 blocks of 16 x 16 per wave; a 4-deep step takes A(i = lane % 16,
    // k = lane / 16) and B(k = lane / 16, j = lane % 16); lane holds
    // D(4 r + lane / 16, lane % 16) in element r
    const int l16 = lane % 16;
    const int q = lane / 16;
    double4_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;
#pragma unroll 4
    for (int kk = 0; kk < kMaxNb / 4; ++kk) {
      const int k = kk * 4 + q;
      double av[4], bv[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = (double)F::to_f(As[wr + i * 16 + l16][k]);
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = (double)F::to_f(Bt[wc + j * 16 + l16][k]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    // C + product in fp64, rounded to fp32 once
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr + i * 16 + 4 * e + q;
          const int c = wc + j * 16 + l16;
          Cs[r][c] = F::from_d((double)F::to_f(Cs[r][c]) + acc[i][j][e]);
        }
  } else {
    const int l32 = lane % 32;
    const int hi = lane / 32;
    float16_t acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][e] = 0.0f;
#pragma unroll
    for (int kk = 0; kk < kMaxNb / 16; ++kk) {
      const int ko = kk * 16 + 8 * hi;
#pragma unroll
      for (int i = 0; i < 2; ++i)
        acc[i] = Mfma<F>::step(&As[wr + i * 32 + l32][ko], &Bt[wc + l32][ko], acc[i]);
    }
    // C + product in fp32, rounded to u_f once
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr + i * 32 + 8 * g + 4 * hi + e;
          const int c = wc + l32;
          Cs[r][c] = F::from_f(F::to_f(Cs[r][c]) + acc[i][4 * g + e]);
        }
  }
  __syncthreads();
  for (int q = tid; q < kTile * (kTile / V); q += NT) {
    const int r = q / (kTile / V), cc = q % (kTile / V);
    const int c = tn + cc * V;
    if (rowp[r] < 0 || c >= c_end) continue;
    T* dst = S + (int64_t)rowp[r] * ld + c;
    if (c + V <= c_end) {
      *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(&Cs[r][cc * V]);
    } else {
      for (int e = 0; c + e < c_end; ++e) dst[e] = Cs[r][cc * V + e];
    }
  }
  if constexpr (kTrsm) {
    // every thread has consumed its unsolved values (the barrier after the
    // solve): count this tile in, and the strip's last tile writes U12
    if (tid == 0) gt.arrived = atomicAdd(strip_cnt + bx, 1);
    __syncthreads();
    if (gt.arrived == ty - 1) {
      for (int q = tid; q < kMaxNb * (kTile / V); q += NT) {
        const int k = q / (kTile / V), cc = q % (kTile / V);
        const int c = tn + cc * V;
        if (c >= c_end) continue;
        T t[V];
#pragma unroll
        for (int e = 0; e < V; ++e) t[e] = Bt[cc * V + e][k];
        T* dst = S + (int64_t)krow[k] * ld + c;
        if (c + V <= c_end) {
          uint4 w;
          __builtin_memcpy(&w, t, 16);
          *reinterpret_cast<uint4*>(dst) = w;
        } else {
          for (int e = 0; c + e < c_end; ++e) dst[e] = t[e];
        }
      }
    }
  }
}

// The trailing update of step uk0 restricted to block column k0 (the next
// one), formed by the block column's own workgroups before its pivot search:
// the separate launch it replaces sat on the factorisation's critical path
// (≈ 8.5 µs per block column at n = 8192, mostly memory latency).  Every
// product is the one gemm_tile forms for the same entries: the same 32 x 32
// blocks of gfx950's 16-deep fp16 / bf16 products over the same k steps, each
// row and column at the same position in its block, added to C in fp32 and
// rounded to u_f once, so the factors are unchanged.  Each wave forms the
// products of its own 64 rows (2 x 2 blocks) from its own LDS region and
// hands each row's sums to the row's lane through that region, 32 columns at
// a time.  With kSolve, U12 of these 64 columns (the block row's solve with
// L11) is formed here too, by threads 0 .. 255 as k_trsm forms it (a quad per
// column, the same order of fused multiply-adds), and kept in
// PanelPreSmem::u12 for the write-back; without it U12 is read as the launch
// before solved it.  x receives the row's updated values (u_f values in
// fp32).  The
// block column is a full one (a further block column follows it), so no
// column is masked: per-column bounds tests here were kept live by the
// compiler through the whole pivot search, for the write-back's tests, and
// spilled.
template <class T>
struct PreSmem {
  alignas(16) T As[kRowWaves][kWave][kKP];  // per wave: -L21 of its rows, then the sums
  alignas(16) T Bt[kMaxNb][kKP];            // U12 transposed: Bt[j][t] = U12(t, k0 + j)
  alignas(16) float Lq[kMaxNb][4][kTrsmLq];  // L11 of step uk0 by row class
};

// The block column's shared memory with the fold: the pivot search's, then
// U12 of the block column (step uk0's block row), which workgroup 0 writes
// back after the pivot search (PreSmem overlaps both and is dead by then)
template <class T>
struct PanelPreSmem {
  PanelSmem p;
  alignas(16) T u12[kMaxNb][kMaxNb];
};
static_assert(sizeof(PanelPreSmem<_Float16>) <= sizeof(PreSmem<_Float16>) &&
                  sizeof(PanelPreSmem<uint16_t>) <= sizeof(PreSmem<uint16_t>),
              "the block column's fold staging covers the write-back's U12");
constexpr int kPreOutLd = 33;  // padded row of a wave's sums (floats), 32 columns at a time
static_assert(kWave * kPreOutLd * 4 <= kWave * kKP * 2, "a wave's sums fit in its region");

template <class F, bool kSolve>
__device__ __forceinline__ void block_column_update(PreSmem<typename F::T>& ps,
                                                    const typename F::T* __restrict__ S,
                                                    int64_t ld, int uk0, int phys, bool in,
                                                    const int* __restrict__ perm, int k0,
                                                    float (&x)[kMaxNb]) {
  using T = typename F::T;
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int P = kMaxNb / V;  // 16-byte pieces of a 64-element row segment
  static_assert(kMaxNb * P == kRowThreads, "one piece of U12 per thread");
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const T* srow = S + (int64_t)phys * ld;
  uint4 cw[P];
  T yraw[kMaxNb / 4];
  {
    uint4 lw[P];
#pragma unroll
    for (int v = 0; v < P; ++v) {
      lw[v] = in ? *reinterpret_cast<const uint4*>(srow + uk0 + v * V) : make_uint4(0, 0, 0, 0);
      cw[v] = in ? *reinterpret_cast<const uint4*>(srow + k0 + v * V) : make_uint4(0, 0, 0, 0);
    }
    if constexpr (kSolve) {
      // this quad's column of the block row (threads 0 .. 255: column
      // tid / 4, rows 4 i + tid % 4), and L11 (threads 0 .. 63)
      if (tid < 4 * kMaxNb) {
        const int c = tid >> 2, pq = tid & 3;
#pragma unroll
        for (int i = 0; i < kMaxNb / 4; ++i)
          yraw[i] = S[(int64_t)perm[uk0 + 4 * i + pq] * ld + k0 + c];
      }
      if (tid < kMaxNb) stage_l11<F>(ps.Lq, S, ld, perm[uk0 + tid], uk0, tid);
    } else {
      // U12 solved by the launch before: row t (pivot row t of step uk0),
      // piece pc of this block column
      const int t = tid / P, pc = tid % P;
      const uint4 w =
          *reinterpret_cast<const uint4*>(S + (int64_t)perm[uk0 + t] * ld + k0 + pc * V);
      T tv[V];
      __builtin_memcpy(tv, &w, 16);
#pragma unroll
      for (int e = 0; e < V; ++e) ps.Bt[pc * V + e][t] = tv[e];
    }
    // -L21 of this thread's row, as gemm_tile stages it
#pragma unroll
    for (int v = 0; v < P; ++v) {
      T lv[V];
      __builtin_memcpy(lv, &lw[v], 16);
#pragma unroll
      for (int e = 0; e < V; ++e) lv[e] = in ? F::from_f(-F::to_f(lv[e])) : F::from_f(0.0f);
      uint4 w2;
      __builtin_memcpy(&w2, lv, 16);
      *reinterpret_cast<uint4*>(&ps.As[wave][lane][v * V]) = w2;
    }
  }
  __syncthreads();
  [[maybe_unused]] float y[kMaxNb / 4];
  if (kSolve && tid < 4 * kMaxNb) {
    const int c = tid >> 2, pq = tid & 3;
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) y[i] = F::to_f(yraw[i]);
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) asm volatile("" : "+v"(y[i]));
    trsm_quad(y, ps.Lq, pq);
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) ps.Bt[c][4 * i + pq] = F::from_f(y[i]);
  }
  if constexpr (kSolve) __syncthreads();
  const int l32 = lane % 32, hi = lane / 32;
  float16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
#pragma unroll
  for (int kk = 0; kk < kMaxNb / 16; ++kk) {
    const int ko = kk * 16 + 8 * hi;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = Mfma<F>::step(&ps.As[wave][i * 32 + l32][ko], &ps.Bt[j * 32 + l32][ko],
                                  acc[i][j]);
  }
  // the wave's region now takes its sums, 32 columns at a time (the wave's
  // own LDS operations complete in order: no barrier)
  float* out = reinterpret_cast<float*>(&ps.As[wave][0][0]);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int gq = 0; gq < 4; ++gq)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          out[(i * 32 + 8 * gq + 4 * hi + e) * kPreOutLd + l32] = acc[i][j][4 * gq + e];
#pragma unroll
    for (int v = 0; v < 32 / V; ++v) {
      T tv[V];
      __builtin_memcpy(tv, &cw[j * (32 / V) + v], 16);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int c = v * V + e;  // column within this half
        const float v = F::to_f(F::from_f(F::to_f(tv[e]) + out[lane * kPreOutLd + c]));
        x[j * 32 + c] = in ? v : 0.0f;
      }
    }
  }
  __syncthreads();  // the regions are reused by the pivot search
  // U12 kept for the write-back (outside the pivot search's region)
  if (kSolve && tid < 4 * kMaxNb) {
    auto& pp = *reinterpret_cast<PanelPreSmem<T>*>(&ps);
    const int c = tid >> 2, pq = tid & 3;
#pragma unroll
    for (int i = 0; i < kMaxNb / 4; ++i) pp.u12[4 * i + pq][c] = F::from_f(y[i]);
  }
}

template <class F>
__global__ __launch_bounds__(kRowThreads) void k_gemm_update(typename F::T* __restrict__ S,
                                                             int64_t ld,
                                                             const int* __restrict__ perm,
                                                             const int* __restrict__ rows, int k0,
                                                             int kb, int n, int c_begin,
                                                             int c_end) {
  __shared__ GemmSmem<typename F::T> sm;
  gemm_tile<F>(sm, S, ld, perm, rows, k0, kb, n, c_begin, c_end, (int)blockIdx.x,
               (int)blockIdx.y);
}

// Block column k + 1 and the remainder of step k's trailing update in one
// launch: workgroups 0 .. G-1 factor the block column (dispatched first, so
// they are resident together), the others take the update tiles (columns
// right of block column k + 1, disjoint from it; the trailing rows are
// located through the permutation copy of step k, since the block column
// rewrites perm meanwhile).
template <class F, int kFold>
__global__ __launch_bounds__(kRowThreads) void k_panel_update(
    typename F::T* __restrict__ S, int64_t ld, int* __restrict__ perm, int pk0, int pkb, int ph,
    int G, int* __restrict__ ipiv, int* __restrict__ perm_copy, uint64_t* __restrict__ xch,
    CycleState* st, const int* __restrict__ rows, int k0, int kb, int n, int c_begin, int c_end,
    int tiles_x, int* __restrict__ strip_cnt) {
  // the staging of the fold only where it is used (fp32 factors would not fit)
  using T = typename F::T;
  using Pre = std::conditional_t<(kFold > 0), PreSmem<T>, PanelSmem>;
  using Gem = std::conditional_t<kFold == 2, GemmTrsmSmem<T>, GemmSmem<T>>;
  __shared__ union {
    PanelSmem p;
    Gem g;
    Pre pre;
  } sm;
  if ((int)blockIdx.x < G) {
    panel_rows<F, kFold>(sm.p, S, ld, perm, pk0, pkb, ph, G, (int)blockIdx.x, ipiv, perm_copy, xch,
                        st, reinterpret_cast<PreSmem<T>*>(&sm.pre), k0);
  } else {
    const int t = (int)blockIdx.x - G;
    const int ty = (n - k0 - kb + kTile - 1) / kTile;
    gemm_tile<F, kFold == 2>(reinterpret_cast<GemmSmem<T>&>(sm.g), S, ld, perm, rows, k0, kb, n,
                       c_begin, c_end, t % tiles_x, t / tiles_x, strip_cnt, ty);
  }
}

// Non-finite entries of the n x n factor.  Each thread tests one 16-byte
// vector of a row (rows start on 128-byte boundaries: ld is a multiple of 64
// elements); the thread just past the last whole vector tests the row's tail
// element by element.
template <class F>
__global__ void k_check(const typename F::T* __restrict__ S, int64_t n, int64_t ld, int* flag) {
  using T = typename F::T;
  constexpr int kV = 16 / (int)sizeof(T);
  const int64_t nv = n / kV;  // whole vectors per row
  int bad = 0;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y) {
    const T* row = S + r * ld;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= nv;
         v += (int64_t)gridDim.x * blockDim.x) {
      if (v < nv) {
        const uint4 w = *reinterpret_cast<const uint4*>(row + v * kV);
        T e[kV];
        __builtin_memcpy(e, &w, sizeof(w));
#pragma unroll
        for (int i = 0; i < kV; ++i)
          if (!F::finite(e[i])) bad = 1;
      } else {
        for (int64_t c = nv * kV; c < n; ++c)
          if (!F::finite(row[c])) bad = 1;
      }
    }
  }
  if (__any(bad) && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

template <class F>
void panel_step_t(const PanelArgs& a, hipStream_t s) {
  using T = typename F::T;
  const int h = a.n - a.k0;
  const int G = (h + kRowThreads - 1) / kRowThreads;
  hipLaunchKernelGGL(k_panel<F>, dim3(G), dim3(kRowThreads), 0, s, reinterpret_cast<T*>(a.S),
                     a.ld, a.perm, a.k0, a.kb, h, a.ipiv, a.perm_copy, a.xch, a.st);
}

template <class F, int kFold>
void panel_update_t(const PanelArgs& p, const PanelArgs& u, const int* rows, int c_begin,
                    int c_end, int* strip_cnt, hipStream_t s) {
  using T = typename F::T;
  const int h = p.n - p.k0;
  const int G = (h + kRowThreads - 1) / kRowThreads;
  const int M = u.n - u.k0 - u.kb;
  const int tx = (c_end - c_begin + kTile - 1) / kTile;
  const int ty = (M + kTile - 1) / kTile;
  hipLaunchKernelGGL((k_panel_update<F, kFold>), dim3(G + tx * ty), dim3(kRowThreads), 0, s,
                     reinterpret_cast<T*>(p.S), p.ld, p.perm, p.k0, p.kb, h, G, p.ipiv,
                     p.perm_copy, p.xch, p.st, rows, u.k0, u.kb, u.n, c_begin, c_end, tx,
                     strip_cnt);
}

template <class F>
void trsm_t(const PanelArgs& a, int c_begin, int c_end, hipStream_t s) {
  using T = typename F::T;
  if (c_end <= c_begin) return;  // kb == 64 whenever a column lies right of the panel
  hipLaunchKernelGGL(k_trsm<F>, dim3((c_end - c_begin + kTrsmCols - 1) / kTrsmCols),
                     dim3(kTrsmThreads), 0, s, reinterpret_cast<T*>(a.S), a.ld, a.perm, a.k0,
                     c_begin, c_end);
}

template <class F>
void gemm_update_t(const PanelArgs& a, const int* rows, int c_begin, int c_end, hipStream_t s) {
  using T = typename F::T;
  const int M = a.n - a.k0 - a.kb;
  if (M <= 0 || c_end <= c_begin) return;
  const dim3 grid((c_end - c_begin + kTile - 1) / kTile, (M + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gemm_update<F>, grid, dim3(kRowThreads), 0, s, reinterpret_cast<T*>(a.S),
                     a.ld, a.perm, rows, a.k0, a.kb, a.n, c_begin, c_end);
}

}  // namespace

void launch_ingest(const double* A, int64_t n, int64_t lda, double* A64, float* Au, int64_t ld,
                   unsigned long long* norms, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ingest, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, A, n, lda, A64, Au,
                     ld, norms, flag);
}

void launch_convert_scaled(const double* A64, int64_t n, int64_t ld, int store, void* S,
                           const unsigned long long* norms, double sqrtn, int scaled, int* e_out,
                           int* flag, hipStream_t s) {
  const dim3 grid((unsigned)std::min<int64_t>((n * ld / 2 + 255) / 256, 4096));
  if (store == kStoreF16)
    hipLaunchKernelGGL(k_convert_scaled<Fp16>, grid, dim3(256), 0, s, A64, n, ld,
                       reinterpret_cast<_Float16*>(S), norms, sqrtn, scaled, e_out, flag);
  else if (store == kStoreBF16)
    hipLaunchKernelGGL(k_convert_scaled<Bf16>, grid, dim3(256), 0, s, A64, n, ld,
                       reinterpret_cast<uint16_t*>(S), norms, sqrtn, scaled, e_out, flag);
  else
    hipLaunchKernelGGL(k_convert_scaled<Fp32>, grid, dim3(256), 0, s, A64, n, ld,
                       reinterpret_cast<float*>(S), norms, sqrtn, scaled, e_out, flag);
}

void launch_iota(int* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256),
                     0, s, p, n);
}

void launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, s, p, v, n);
}

void launch_zero_spans(const ZeroSpans& z, hipStream_t s) {
  if (z.count <= 0) return;
  int64_t most = 0;
  for (int j = 0; j < z.count; ++j) most = std::max(most, z.n[j]);
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((most + 255) / 256, 1024));
  hipLaunchKernelGGL(k_zero_spans, dim3(gx, (unsigned)z.count), dim3(256), 0, s, z);
}

void launch_panel_step(const PanelArgs& a, int store, hipStream_t s) {
  if (store == kStoreF16)
    panel_step_t<Fp16>(a, s);
  else if (store == kStoreBF16)
    panel_step_t<Bf16>(a, s);
  else
    panel_step_t<Fp32>(a, s);
}

void launch_trsm(const PanelArgs& a, int store, int c_begin, int c_end, hipStream_t s) {
  if (store == kStoreF16)
    trsm_t<Fp16>(a, c_begin, c_end, s);
  else if (store == kStoreBF16)
    trsm_t<Bf16>(a, c_begin, c_end, s);
  else
    trsm_t<Fp32>(a, c_begin, c_end, s);
}

void launch_gemm_update(const PanelArgs& a, int store, const int* rows, int c_begin, int c_end,
                        hipStream_t s) {
  if (store == kStoreF16)
    gemm_update_t<Fp16>(a, rows, c_begin, c_end, s);
  else if (store == kStoreBF16)
    gemm_update_t<Bf16>(a, rows, c_begin, c_end, s);
  else
    gemm_update_t<Fp32>(a, rows, c_begin, c_end, s);
}

void launch_panel_update(const PanelArgs& p, const PanelArgs& u, int store, const int* rows,
                         int c_begin, int c_end, int fold, int* strip_cnt, hipStream_t s) {
  // fp16 / bf16 factors: the block column takes the next block column's part
  // of step u's update (fold >= 1) and the block-row solve (fold == 2)
  // itself; fp32 factors (fp64 matrix-core products) keep the separate
  // launches
  if (store == kStoreF16) {
    if (fold == 2)
      panel_update_t<Fp16, 2>(p, u, rows, c_begin, c_end, strip_cnt, s);
    else if (fold == 1)
      panel_update_t<Fp16, 1>(p, u, rows, c_begin, c_end, strip_cnt, s);
    else
      panel_update_t<Fp16, 0>(p, u, rows, c_begin, c_end, strip_cnt, s);
  } else if (store == kStoreBF16) {
    if (fold == 2)
      panel_update_t<Bf16, 2>(p, u, rows, c_begin, c_end, strip_cnt, s);
    else if (fold == 1)
      panel_update_t<Bf16, 1>(p, u, rows, c_begin, c_end, strip_cnt, s);
    else
      panel_update_t<Bf16, 0>(p, u, rows, c_begin, c_end, strip_cnt, s);
  } else {
    panel_update_t<Fp32, 0>(p, u, rows, c_begin, c_end, strip_cnt, s);
  }
}

bool panel_update_folds(int store) { return store != kStoreF32; }

void launch_copy_i32(int* dst, const int* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, s, dst, src, n);
}

void launch_check_factors(const void* S, int64_t n, int64_t ld, int store, int* flag,
                          hipStream_t s) {
  // one thread per 16-byte vector of a row, plus one for the tail
  const int64_t nvec = n * (store == kStoreF32 ? 4 : 2) / 16 + 1;
  dim3 grid((unsigned)((nvec + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
  if (store == kStoreF16)
    hipLaunchKernelGGL(k_check<Fp16>, grid, dim3(256), 0, s,
                       reinterpret_cast<const _Float16*>(S), n, ld, flag);
  else if (store == kStoreBF16)
    hipLaunchKernelGGL(k_check<Bf16>, grid, dim3(256), 0, s,
                       reinterpret_cast<const uint16_t*>(S), n, ld, flag);
  else
    hipLaunchKernelGGL(k_check<Fp32>, grid, dim3(256), 0, s, reinterpret_cast<const float*>(S),
                       n, ld, flag);
}

}  // namespace gir
