// LU factorisation with partial pivoting in u_f on gfx950 (Algorithm 1-3,
// line 1; GEPP as in Section 1 of the paper).
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
// Block column = one persistent kernel: workgroup 0 (the leader) holds the
// unfactored rows of W columns in registers and performs the pivot searches
// (one workgroup barrier per column); the other workgroups apply the rank-W
// updates to the rest of the block column.  They synchronise through two
// device-scope counters with bounded waits.
#include "kernels.h"

// Phase hooks of the block-column kernel; empty unless a timing harness
// defines them before including this file.
#ifndef GIR_PANEL_MARK
#define GIR_PANEL_MARK(tag)
#define GIR_PANEL_MARK_INIT
#endif

namespace gir {

namespace {

constexpr int kPanelThreads = 512;
constexpr int kMaxNb = 64;

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__global__ void k_scan(const double* __restrict__ A, int64_t n, int64_t lda,
                       unsigned long long* out, int* flag) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= n) return;
  const double* a = A + row * lda;
  double s = 0.0, mx = 0.0;
  int bad = 0;
  for (int64_t c = lane; c < n; c += kWave) {
    double v = a[c];
    if (!__builtin_isfinite(v)) bad = 1;
    v = fabs(v);
    s += v;
    mx = fmax(mx, v);
  }
  s = wave_sum(s);
  mx = wave_max_d(mx);
  bad = __any(bad);
  if (lane == 0) {
    atomic_max_nonneg(out + 0, mx);
    atomic_max_nonneg(out + 1, s);
    if (bad) atomicOr(flag, 1);
  }
}

template <class F>
__global__ void k_convert(const double* __restrict__ A, int64_t n, int64_t lda, int e,
                          typename F::T* __restrict__ S, float* __restrict__ Au, int64_t ld,
                          int* flag) {
  int bad = 0;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ld;
         c += (int64_t)gridDim.x * blockDim.x) {
      const double a = (c < n) ? A[r * lda + c] : 0.0;
      if (S) {
        const typename F::T v = F::from_d(ldexp(a, e));
        if (!F::finite(v)) bad = 1;
        S[r * ld + c] = v;
      }
      if (Au) {
        const float f = (float)a;
        if (!__builtin_isfinite(f)) bad = 1;
        Au[r * ld + c] = f;
      }
    }
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_iota(int* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int)i;
}

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// P[c][q] = S[perm[k0 + q]][k0 + c]  (column-major fp32 panel)
template <class F>
__global__ void k_panel_gather(const typename F::T* __restrict__ S, int64_t ld,
                               const int* __restrict__ perm, int k0, int kb, int h,
                               float* __restrict__ P, int ldp, int* pstep, int* sync) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < 2) sync[threadIdx.x] = 0;
  if (q >= h) return;
  const typename F::T* row = S + (int64_t)perm[k0 + q] * ld + k0;
  for (int c = 0; c < kb; ++c) P[(int64_t)c * ldp + q] = F::to_f(row[c]);
  pstep[q] = -1;
}

struct Cand {
  float val;
  int lidx;
  int prow;
  int pad;
  float row[kMaxNb];
};

template <int R, int W>
__device__ __forceinline__ void panel_leader(float* __restrict__ P, int ldp, int h, int kb, int k0,
                             int* __restrict__ pstep, int* __restrict__ piv_prow,
                             int* __restrict__ lidx_out, int* __restrict__ ipiv, int* sync,
                             CycleState* st, int nhelpers) {
  __shared__ Cand cand[2][kPanelThreads / kWave];
  __shared__ float Lblk[W][W];
  __shared__ int blk_prow[W];
  __shared__ int s_abort;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  int* abortp = &st->abort;

  int lid[R];
  bool pv[R];
  float x[R][W];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int q = tid + kPanelThreads * s;
    lid[s] = q;
    pv[s] = (q >= h);
  }
  if (tid == 0) s_abort = 0;
  __syncthreads();
  GIR_PANEL_MARK_INIT

  const int nblk = (kb + W - 1) / W;
  for (int ib = 0; ib < nblk; ++ib) {
    const int c0 = ib * W;
    const int wcols = min(W, kb - c0);
    GIR_PANEL_MARK(0);
    if (ib > 0) {
      if (lane == 0) {
        if (!wait_geq(&sync[1], ib * nhelpers, abortp)) s_abort = 1;
      }
      __syncthreads();
      if (s_abort) return;
    }
    GIR_PANEL_MARK(1);
    bool pvb[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
      pvb[s] = pv[s];
      const int q = tid + kPanelThreads * s;
#pragma unroll
      for (int c = 0; c < W; ++c)
        x[s][c] = (!pv[s] && c < wcols) ? P[(int64_t)(c0 + c) * ldp + q] : 0.0f;
    }
    GIR_PANEL_MARK(2);

#pragma unroll
    for (int c = 0; c < W; ++c) {
      if (c < wcols) {
        const int cc = c0 + c;
        float bv = -1.0f;
        int bl = 0x7fffffff;
        int bs = -1;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const float a = pv[s] ? -1.0f : fabsf(x[s][c]);
          const bool better = a > bv || (a == bv && lid[s] < bl);
          bv = better ? a : bv;
          bl = better ? lid[s] : bl;
          bs = better ? s : bs;
        }
        if (bv < 0.0f) bs = -1;
        float wv = bv;
        int wl = bl;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const float ov = __shfl_xor(wv, o, kWave);
          const int ol = __shfl_xor(wl, o, kWave);
          if (ov > wv || (ov == wv && ol < wl)) {
            wv = ov;
            wl = ol;
          }
        }
        GIR_PANEL_MARK(10 + c);
        Cand* cb = &cand[c & 1][wave];
        if (bs >= 0 && bl == wl && bv == wv) {
          cb->val = bv;
          cb->lidx = bl;
          cb->prow = tid + kPanelThreads * bs;
#pragma unroll
          for (int s = 0; s < R; ++s) {
            if (s == bs) {
#pragma unroll
              for (int c2 = 0; c2 < W; ++c2) cb->row[c2] = x[s][c2];
            }
          }
        }
        if (wv < 0.0f && lane == 0) {
          cb->val = -1.0f;
          cb->lidx = 0x7fffffff;
          cb->prow = -1;
        }
        __syncthreads();
        GIR_PANEL_MARK(20 + c);
        float gv = -1.0f;
        int gl = 0x7fffffff;
        int gw = 0;
#pragma unroll
        for (int w2 = 0; w2 < kPanelThreads / kWave; ++w2) {
          const float v = cand[c & 1][w2].val;
          const int l = cand[c & 1][w2].lidx;
          if (v > gv || (v == gv && l < gl)) {
            gv = v;
            gl = l;
            gw = w2;
          }
        }
        const Cand* win = &cand[c & 1][gw];
        const int p = win->prow;
        const float* u = win->row;  // pivot row, read from LDS (broadcast)
        const float piv = u[c];
        if (tid == 0) {
          ipiv[k0 + cc] = k0 + gl;
          piv_prow[cc] = p;
          blk_prow[c] = p;
          if (piv == 0.0f) atomicCAS(&st->singular, 0, k0 + cc + 1);
        }
        if (tid < W) Lblk[c][tid] = u[tid];
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int q = tid + kPanelThreads * s;
          lid[s] = (!pv[s] && lid[s] == cc) ? gl : lid[s];
          lid[s] = (q == p) ? cc : lid[s];
          pv[s] = pv[s] || (q == p);
        }
        if (piv != 0.0f) {
          // multipliers fl32(a / piv): reciprocal, product and one fused
          // correction give the correctly rounded quotient (Markstein); a
          // quotient in the subnormal range falls back to the division
          const float rinv = 1.0f / piv;
          const bool rok = __builtin_isfinite(rinv);
          float ucol[W];
#pragma unroll
          for (int c2 = c + 1; c2 < W; ++c2) ucol[c2] = u[c2];
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const float a = x[s][c];
            float l;
            if (rok) {
              const float q0 = a * rinv;
              const float e = __builtin_fmaf(-q0, piv, a);
              l = __builtin_fmaf(e, rinv, q0);
              if (__builtin_expect(fabsf(l) < 0x1p-100f, 0) && a != 0.0f) l = a / piv;
            } else {
              l = a / piv;
            }
            const bool upd = !pv[s];
            x[s][c] = upd ? l : a;
#pragma unroll
            for (int c2 = c + 1; c2 < W; ++c2)
              x[s][c2] = upd ? __builtin_fmaf(-l, ucol[c2], x[s][c2]) : x[s][c2];
          }
        }
      }
    }

    GIR_PANEL_MARK(3);
    // write the block back (rows that were not pivots before this block)
#pragma unroll
    for (int s = 0; s < R; ++s) {
      if (!pvb[s]) {
        const int q = tid + kPanelThreads * s;
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < wcols) P[(int64_t)(c0 + c) * ldp + q] = x[s][c];
        if (pv[s]) pstep[q] = ib;
      }
    }
    __syncthreads();
    GIR_PANEL_MARK(4);
    // U part of the new pivot rows in the remaining columns of the panel
    const int rem0 = c0 + W;
    for (int cr = rem0 + tid; cr < kb; cr += kPanelThreads) {
      float y[W];
#pragma unroll
      for (int t = 0; t < W; ++t) y[t] = P[(int64_t)cr * ldp + blk_prow[t]];
#pragma unroll
      for (int t = 1; t < W; ++t) {
#pragma unroll
        for (int s2 = 0; s2 < t; ++s2) y[t] = __builtin_fmaf(-Lblk[t][s2], y[s2], y[t]);
      }
#pragma unroll
      for (int t = 0; t < W; ++t) P[(int64_t)cr * ldp + blk_prow[t]] = y[t];
    }
    if (ib < nblk - 1) publish_store(&sync[0], ib + 1);
    GIR_PANEL_MARK(5);
  }
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int q = tid + kPanelThreads * s;
    if (q < h) lidx_out[q] = lid[s];
  }
}

template <int W>
__device__ __forceinline__ void panel_helper(float* __restrict__ P, int ldp, int h, int kb,
                             const int* __restrict__ pstep, const int* __restrict__ piv_prow,
                             int* sync, CycleState* st, int nhelpers, int hid) {
  __shared__ float Ush[W][kMaxNb];
  __shared__ int prow_sh[W];
  __shared__ int s_abort;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  int* abortp = &st->abort;
  const int nblk = (kb + W - 1) / W;
  const int slab = (h + nhelpers - 1) / nhelpers;
  const int qb = hid * slab;
  const int qe = min(h, qb + slab);
  const int nrows = max(0, qe - qb);
  if (tid == 0) s_abort = 0;
  __syncthreads();
  for (int ib = 0; ib < nblk - 1; ++ib) {
    const int c0 = ib * W;
    const int rem0 = c0 + W;
    const int nrem = kb - rem0;
    if (lane == 0) {
      if (!wait_geq(&sync[0], ib + 1, abortp)) s_abort = 1;
    }
    __syncthreads();
    if (s_abort) return;
    if (tid < W) prow_sh[tid] = piv_prow[c0 + tid];
    __syncthreads();
    for (int idx = tid; idx < W * nrem; idx += kPanelThreads) {
      const int t = idx / nrem;
      const int cr = idx - t * nrem;
      Ush[t][cr] = P[(int64_t)(rem0 + cr) * ldp + prow_sh[t]];
    }
    __syncthreads();
    // lane -> row, wave -> group of columns; the row's W multipliers are
    // loaded once and applied to every remaining column it owns
    const int rl = tid % kWave;
    const int cg = tid / kWave;
    constexpr int kGroups = kPanelThreads / kWave;
    for (int q = qb + rl; q < qb + nrows; q += kWave) {
      if (pstep[q] >= 0) continue;
      float l[W];
#pragma unroll
      for (int t = 0; t < W; ++t) l[t] = P[(int64_t)(c0 + t) * ldp + q];
      for (int cr = cg; cr < nrem; cr += kGroups) {
        float a = P[(int64_t)(rem0 + cr) * ldp + q];
#pragma unroll
        for (int t = 0; t < W; ++t) a = __builtin_fmaf(-l[t], Ush[t][cr], a);
        P[(int64_t)(rem0 + cr) * ldp + q] = a;
      }
    }
    publish_add(&sync[1], 1);
  }
}

template <int R, int W>
__global__ __launch_bounds__(kPanelThreads) void k_panel(float* P, int ldp, int h, int kb, int k0,
                                                         int* pstep, int* piv_prow, int* lidx,
                                                         int* ipiv, int* sync, CycleState* st,
                                                         int nhelpers) {
  if (blockIdx.x == 0)
    panel_leader<R, W>(P, ldp, h, kb, k0, pstep, piv_prow, lidx, ipiv, sync, st, nhelpers);
  else
    panel_helper<W>(P, ldp, h, kb, pstep, piv_prow, sync, st, nhelpers, blockIdx.x - 1);
}

template <class F>
__global__ void k_panel_scatter(typename F::T* __restrict__ S, int64_t ld,
                                const int* __restrict__ perm, int k0, int kb, int h,
                                const float* __restrict__ P, int ldp,
                                const int* __restrict__ lidx, int* __restrict__ ptmp) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= h) return;
  const int phys = perm[k0 + q];
  typename F::T* row = S + (int64_t)phys * ld + k0;
  for (int c = 0; c < kb; ++c) row[c] = F::from_f(P[(int64_t)c * ldp + q]);
  ptmp[lidx[q]] = phys;
}

__global__ void k_perm_copy(int* perm, const int* ptmp, int k0, int h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < h) perm[k0 + i] = ptmp[i];
}

// U12 = L11^-1 A12 in fp32 with the stored (u_f) unit lower triangle L11.
// A workgroup owns 64 columns staged in LDS; elimination step t updates rows
// r > t with one fused multiply-add each, so every entry receives its terms
// in the order t = 0, 1, ... of forward substitution.
constexpr int kTrsmCols = 64;
template <class F>
__global__ __launch_bounds__(256) void k_trsm(typename F::T* __restrict__ S, int64_t ld,
                                              const int* __restrict__ perm, int k0, int kb,
                                              int n) {
  __shared__ float Lsh[kMaxNb][kMaxNb + 1];
  __shared__ float Y[kMaxNb][kTrsmCols + 1];
  __shared__ int prow[kMaxNb];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)k0 + kb + (int64_t)blockIdx.x * kTrsmCols;
  if (tid < kMaxNb) prow[tid] = (tid < kb) ? perm[k0 + tid] : 0;
  __syncthreads();
  for (int idx = tid; idx < kMaxNb * kMaxNb; idx += blockDim.x) {
    const int t = idx / kMaxNb;
    const int s = idx % kMaxNb;
    Lsh[t][s] = (t < kb && s < t) ? F::to_f(S[(int64_t)prow[t] * ld + k0 + s]) : 0.0f;
  }
  for (int idx = tid; idx < kMaxNb * kTrsmCols; idx += blockDim.x) {
    const int t = idx / kTrsmCols;
    const int c = idx % kTrsmCols;
    Y[t][c] = (t < kb && c0 + c < n) ? F::to_f(S[(int64_t)prow[t] * ld + c0 + c]) : 0.0f;
  }
  __syncthreads();
  const int c = tid % kTrsmCols;
  const int rg = tid / kTrsmCols;  // 4 row groups
  for (int t = 0; t < kb - 1; ++t) {
    const float yt = Y[t][c];
    for (int r = t + 1 + rg; r < kb; r += 4) Y[r][c] = __builtin_fmaf(-Lsh[r][t], yt, Y[r][c]);
    __syncthreads();
  }
  for (int idx = tid; idx < kMaxNb * kTrsmCols; idx += blockDim.x) {
    const int t = idx / kTrsmCols;
    const int cc = idx % kTrsmCols;
    if (t < kb && c0 + cc < n) S[(int64_t)prow[t] * ld + c0 + cc] = F::from_f(Y[t][cc]);
  }
}

// ---- trailing update on the matrix cores ----------------------------------

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;
constexpr int kKP = kMaxNb + 4;  // padded LDS row (elements)

template <class F>
struct Mfma;

template <>
struct Mfma<Fp16> {
  // 8-deep k chunk: A rows i = lane%32, k = 4*(lane/32)+e; B cols j = lane%32
  static __device__ __forceinline__ float16_t step(const _Float16* a, const _Float16* b,
                                                   float16_t acc) {
    const half4_t av = *reinterpret_cast<const half4_t*>(a);
    const half4_t bv = *reinterpret_cast<const half4_t*>(b);
    return __builtin_amdgcn_mfma_f32_32x32x8f16(av, bv, acc, 0, 0, 0);
  }
};

template <>
struct Mfma<Bf16> {
  static __device__ __forceinline__ float16_t step(const uint16_t* a, const uint16_t* b,
                                                   float16_t acc) {
    const short4_t av = *reinterpret_cast<const short4_t*>(a);
    const short4_t bv = *reinterpret_cast<const short4_t*>(b);
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
  }
};

template <>
struct Mfma<Fp32> {
  // the 8-deep chunk as four 2-deep steps; a/b point at k = 4*(lane/32)
  static __device__ __forceinline__ float16_t step(const float* a, const float* b,
                                                   float16_t acc) {
    // lanes 0-31 hold k = 0..3 of their half, lanes 32-63 k = 4..7; the
    // 2-deep instruction takes k = lane/32 -> issue k pairs (0,4),(1,5),...
    // which covers the same 8 products in a different order.
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], acc, 0, 0, 0);
    return acc;
  }
};

template <class F>
__global__ __launch_bounds__(256) void k_gemm_update(typename F::T* __restrict__ S, int64_t ld,
                                                     const int* __restrict__ perm, int k0,
                                                     int kb, int n) {
  using T = typename F::T;
  __shared__ T As[kTile][kKP];
  __shared__ T Bs[kTile][kKP];
  __shared__ int rowp[kTile];
  __shared__ int krow[kMaxNb];
  const int tid = threadIdx.x;
  const int M = n - k0 - kb;
  const int tm = blockIdx.y * kTile;
  const int tn = blockIdx.x * kTile;
  if (tid < kTile) rowp[tid] = (tm + tid < M) ? perm[k0 + kb + tm + tid] : -1;
  if (tid < kMaxNb) krow[tid] = (tid < kb) ? perm[k0 + tid] : -1;
  __syncthreads();
  // A = -L21 (negated so that the product accumulates C - A B)
  for (int idx = tid; idx < kTile * kMaxNb; idx += 256) {
    const int r = idx / kMaxNb;
    const int k = idx % kMaxNb;
    T v = F::from_f(0.0f);
    if (rowp[r] >= 0 && k < kb) v = F::from_f(-F::to_f(S[(int64_t)rowp[r] * ld + k0 + k]));
    As[r][k] = v;
  }
  // B = U12 transposed into LDS
  for (int idx = tid; idx < kTile * kMaxNb; idx += 256) {
    const int k = idx / kTile;
    const int c = idx % kTile;
    T v = F::from_f(0.0f);
    if (k < kb && tn + c < M) v = S[(int64_t)krow[k] * ld + k0 + kb + tn + c];
    Bs[c][k] = v;
  }
  __syncthreads();
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int wr = (wave / 2) * 64;
  const int wc = (wave % 2) * 64;
  const int l32 = lane % 32;
  const int hi = lane / 32;
  float16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr + i * 32 + 8 * g + 4 * hi + e;
          const int c = wc + j * 32 + l32;
          float v = 0.0f;
          if (rowp[r] >= 0 && tn + c < M) v = F::to_f(S[(int64_t)rowp[r] * ld + k0 + kb + tn + c]);
          acc[i][j][4 * g + e] = v;
        }
  const int kchunks = (kb + 7) / 8;
  for (int kk = 0; kk < kchunks; ++kk) {
    const int ko = kk * 8 + 4 * hi;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = Mfma<F>::step(&As[wr + i * 32 + l32][ko], &Bs[wc + j * 32 + l32][ko], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = wr + i * 32 + 8 * g + 4 * hi + e;
          const int c = wc + j * 32 + l32;
          if (rowp[r] >= 0 && tn + c < M)
            S[(int64_t)rowp[r] * ld + k0 + kb + tn + c] = F::from_f(acc[i][j][4 * g + e]);
        }
}

template <class F>
__global__ void k_check(const typename F::T* __restrict__ S, int64_t n, int64_t ld, int* flag) {
  int bad = 0;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x)
      if (!F::finite(S[r * ld + c])) bad = 1;
  if (__any(bad) && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

template <class F>
void panel_step_t(const PanelArgs& a, int nhelpers, hipStream_t s) {
  using T = typename F::T;
  T* S = reinterpret_cast<T*>(a.S);
  const int h = a.n - a.k0;
  const int blk = 256;
  hipLaunchKernelGGL(k_panel_gather<F>, dim3((h + blk - 1) / blk), dim3(blk), 0, s, S, a.ld,
                     a.perm, a.k0, a.kb, h, a.P, a.ldp, a.pstep, a.sync);
  const int nwg = 1 + nhelpers;
#define GIR_PANEL(R, W)                                                                       \
  hipLaunchKernelGGL((k_panel<R, W>), dim3(nwg), dim3(kPanelThreads), 0, s, a.P, a.ldp, h, \
                     a.kb, a.k0, a.pstep, a.piv_prow, a.lidx, a.ipiv, a.sync, a.st, nhelpers)
  // rows per thread x block width chosen so that the leader's register block
  // stays in registers (no scratch) at 512 threads
  if (h <= 512)
    GIR_PANEL(1, 16);
  else if (h <= 1024)
    GIR_PANEL(2, 16);
  else if (h <= 2048)
    GIR_PANEL(4, 8);
  else if (h <= 4096)
    GIR_PANEL(8, 8);
  else if (h <= 8192)
    GIR_PANEL(16, 8);
  else
    GIR_PANEL(32, 2);  // h <= 16384
#undef GIR_PANEL
  hipLaunchKernelGGL(k_panel_scatter<F>, dim3((h + blk - 1) / blk), dim3(blk), 0, s, S, a.ld,
                     a.perm, a.k0, a.kb, h, a.P, a.ldp, a.lidx, a.ptmp);
  hipLaunchKernelGGL(k_perm_copy, dim3((h + blk - 1) / blk), dim3(blk), 0, s, a.perm, a.ptmp,
                     a.k0, h);
}

template <class F>
void trsm_update_t(const PanelArgs& a, hipStream_t s) {
  using T = typename F::T;
  T* S = reinterpret_cast<T*>(a.S);
  const int M = a.n - a.k0 - a.kb;
  if (M <= 0) return;
  hipLaunchKernelGGL(k_trsm<F>, dim3((M + kTrsmCols - 1) / kTrsmCols), dim3(256), 0, s, S, a.ld,
                     a.perm, a.k0, a.kb, a.n);
  const int t = (M + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_gemm_update<F>, dim3(t, t), dim3(256), 0, s, S, a.ld, a.perm, a.k0, a.kb,
                     a.n);
}

}  // namespace

void launch_scan(const double* A, int64_t n, int64_t lda, unsigned long long* out, int* flag,
                 hipStream_t s) {
  const int rows_per_block = 4;
  const int64_t blocks = (n + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL(k_scan, dim3((unsigned)blocks), dim3(rows_per_block * kWave), 0, s, A, n,
                     lda, out, flag);
}

void launch_convert(const double* A, int64_t n, int64_t lda, int e, int store, void* S,
                    float* Au, int64_t ld, int* flag, hipStream_t s) {
  dim3 grid((unsigned)((ld + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
  if (store == kStoreF16)
    hipLaunchKernelGGL(k_convert<Fp16>, grid, dim3(256), 0, s, A, n, lda, e,
                       reinterpret_cast<_Float16*>(S), Au, ld, flag);
  else if (store == kStoreBF16)
    hipLaunchKernelGGL(k_convert<Bf16>, grid, dim3(256), 0, s, A, n, lda, e,
                       reinterpret_cast<uint16_t*>(S), Au, ld, flag);
  else
    hipLaunchKernelGGL(k_convert<Fp32>, grid, dim3(256), 0, s, A, n, lda, e,
                       reinterpret_cast<float*>(S), Au, ld, flag);
}

void launch_iota(int* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256),
                     0, s, p, n);
}

void launch_fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)),
                     dim3(256), 0, s, p, v, n);
}

void launch_panel_step(const PanelArgs& a, int store, int nhelpers, hipStream_t s) {
  if (store == kStoreF16)
    panel_step_t<Fp16>(a, nhelpers, s);
  else if (store == kStoreBF16)
    panel_step_t<Bf16>(a, nhelpers, s);
  else
    panel_step_t<Fp32>(a, nhelpers, s);
}

void launch_trsm_update(const PanelArgs& a, int store, hipStream_t s) {
  if (store == kStoreF16)
    trsm_update_t<Fp16>(a, s);
  else if (store == kStoreBF16)
    trsm_update_t<Bf16>(a, s);
  else
    trsm_update_t<Fp32>(a, s);
}

void launch_check_factors(const void* S, int64_t n, int64_t ld, int store, int* flag,
                          hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)std::min<int64_t>(n, 65535));
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
