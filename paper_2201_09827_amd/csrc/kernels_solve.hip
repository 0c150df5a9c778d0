// Solve-phase kernels of RGMRES-IR (Algorithm 3 and the GCRO-DR algorithm of
// Section 2) on gfx950.
//
//  * preconditioned product A-tilde v = 2^e U^-1 L^-1 P A_u v in u^2 = fp64:
//    a row-gathered GEMV with fp32 A_u and fp64 accumulation, then two
//    blocked triangular solves with the u_f factors (fp64 arithmetic);
//  * residual r = b - A x in fp64 with the infinity norms of r and x;
//  * Arnoldi orthogonalisation against [C_k, V_j] by classical Gram-Schmidt
//    applied twice; inner products in fp64, vectors stored in fp32; the
//    Hessenberg column, its Givens rotation and the residual estimate are
//    updated on the device so that no host round trip sits inside a cycle;
//  * skinny products with the recycle space (combine, gram, updates).
#include <type_traits>

#include "kernels.h"

namespace gir {

namespace {

constexpr int kTB = 64;  // triangular-solve block (rows per workgroup)

// ---------------------------------------------------------------------------
// GEMV: t[i] = sum_c Au[permA[i]][c] v[c], one wave per row, fp64 accumulate
// ---------------------------------------------------------------------------
// one row of the product, summed over the wave (every lane gets the sum);
// with kAhead > 1 the loads of kAhead loop iterations are issued before
// their products are taken, in the same order (the same sums bit for bit),
// for waves that run at low occupancy
template <typename VT, int kAhead = 1>
__device__ __forceinline__ double gemv_au_row(const float* __restrict__ a,
                                              const VT* __restrict__ v, int n, int lane) {
  double acc0 = 0.0, acc1 = 0.0;
  const int n4 = n & ~3;
  int c = lane * 4;
  if (kAhead > 1) {
    for (; c + 512 * (kAhead - 1) + 256 < n4; c += 512 * kAhead) {
      float4 x0[kAhead], x1[kAhead];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        x0[u] = *reinterpret_cast<const float4*>(a + c + 512 * u);
        x1[u] = *reinterpret_cast<const float4*>(a + c + 512 * u + 256);
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const int cu = c + 512 * u;
        acc0 = fma((double)x0[u].x, (double)v[cu + 0], acc0);
        acc1 = fma((double)x0[u].y, (double)v[cu + 1], acc1);
        acc0 = fma((double)x0[u].z, (double)v[cu + 2], acc0);
        acc1 = fma((double)x0[u].w, (double)v[cu + 3], acc1);
        acc0 = fma((double)x1[u].x, (double)v[cu + 256], acc0);
        acc1 = fma((double)x1[u].y, (double)v[cu + 257], acc1);
        acc0 = fma((double)x1[u].z, (double)v[cu + 258], acc0);
        acc1 = fma((double)x1[u].w, (double)v[cu + 259], acc1);
      }
    }
  }
  for (; c + 256 < n4; c += 512) {
    const float4 x0 = *reinterpret_cast<const float4*>(a + c);
    const float4 x1 = *reinterpret_cast<const float4*>(a + c + 256);
    acc0 = fma((double)x0.x, (double)v[c + 0], acc0);
    acc1 = fma((double)x0.y, (double)v[c + 1], acc1);
    acc0 = fma((double)x0.z, (double)v[c + 2], acc0);
    acc1 = fma((double)x0.w, (double)v[c + 3], acc1);
    acc0 = fma((double)x1.x, (double)v[c + 256], acc0);
    acc1 = fma((double)x1.y, (double)v[c + 257], acc1);
    acc0 = fma((double)x1.z, (double)v[c + 258], acc0);
    acc1 = fma((double)x1.w, (double)v[c + 259], acc1);
  }
  for (; c < n4; c += 256) {
    const float4 x0 = *reinterpret_cast<const float4*>(a + c);
    acc0 = fma((double)x0.x, (double)v[c + 0], acc0);
    acc1 = fma((double)x0.y, (double)v[c + 1], acc1);
    acc0 = fma((double)x0.z, (double)v[c + 2], acc0);
    acc1 = fma((double)x0.w, (double)v[c + 3], acc1);
  }
  for (int cc = n4 + lane; cc < n; cc += kWave) acc0 = fma((double)a[cc], (double)v[cc], acc0);
  return wave_sum(acc0 + acc1);
}

template <typename VT>
__global__ __launch_bounds__(256) void k_gemv_au(const float* __restrict__ Au, int64_t ld,
                                                 const int* __restrict__ permA, int n,
                                                 const VT* __restrict__ v, double* __restrict__ t,
                                                 const CycleState* gate, int step) {
  if (gated_off(gate, step)) return;
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= n) return;
  const int prow = permA ? permA[row] : row;
  const double s = gemv_au_row(Au + (int64_t)prow * ld, v, n, lane);
  if (lane == 0) t[row] = s;
}

// T[:, r] = A_u[permA] Y[:, r] for nr <= NR fp64 columns of Y (ld ldy) at
// once (the recycle set-up): one wave takes kMultiRows rows and each lane the
// columns 4 lane + 256 i, summed per row and column in fp64 in that order and
// then over the wave, as k_gemv_au sums one column.  Each chunk of kChunk
// columns of Y is staged once per workgroup in LDS (two buffers, one barrier
// per chunk) instead of being read by every wave from the cache: with eight
// or more columns those reads, four times the bytes of A_u, had set the pace.
// The next chunk's rows of A_u and of Y are loaded before the current chunk's
// multiply-adds; what remains exposed is one memory latency per chunk, so
// wider chunks pay where the registers allow them.
constexpr int kMultiThreads = 512;
template <int NR, int kMultiRows, int kChunk>
__global__ __launch_bounds__(kMultiThreads) void k_gemv_au_multi(
    const float* __restrict__ Au, int64_t ld, const int* __restrict__ permA, int n,
    const double* __restrict__ Y, int64_t ldy, int nr, double* __restrict__ T, int64_t ldt) {
  constexpr int kRowThreads = kChunk / 2;               // threads staging one row of a chunk
  constexpr int kPass = kMultiThreads / kRowThreads;    // chunk rows staged per pass
  static_assert(NR % kPass == 0, "the staging covers whole passes of rows");
  constexpr int kStage = NR / kPass;                    // double2 per thread and chunk
  constexpr int kSub = kChunk / 256;                    // float4 per lane, row and chunk
  __shared__ double ysh[2][NR][kChunk];
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int row0 = (blockIdx.x * (kMultiThreads / kWave) + tid / kWave) * kMultiRows;
  const float* a[kMultiRows];
#pragma unroll
  for (int q = 0; q < kMultiRows; ++q) {
    // rows beyond n repeat the last one (not stored); a wave wholly beyond n
    // still takes part in the staging and the barriers
    const int rw = min(row0 + q, n - 1);
    a[q] = Au + (int64_t)(permA ? permA[rw] : rw) * ld;
  }
  double acc[kMultiRows][NR];
#pragma unroll
  for (int q = 0; q < kMultiRows; ++q)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[q][r] = 0.0;
  const int n4 = n & ~3;
  const int nchunk = (n4 + kChunk - 1) / kChunk;
  // staging: thread t moves the double2 at column 2 (t % kRowThreads) of rows
  // t / kRowThreads + kPass e of the chunk (columns at or past n4 enter as zero)
  double2 st[kStage];
  auto load_stage = [&](int c0) {
#pragma unroll
    for (int e = 0; e < kStage; ++e) {
      const int r = tid / kRowThreads + kPass * e;
      const int c = c0 + 2 * (tid % kRowThreads);
      const double* src = Y + (int64_t)min(r, nr - 1) * ldy + min(c, max(n4 - 2, 0));
      const double2 v = *reinterpret_cast<const double2*>(src);
      st[e] = (c < n4) ? v : make_double2(0.0, 0.0);
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < kStage; ++e)
      *reinterpret_cast<double2*>(
          &ysh[buf][tid / kRowThreads + kPass * e][2 * (tid % kRowThreads)]) = st[e];
  };
  auto load_a = [&](int c0, float4 (&x)[kSub][kMultiRows]) {
#pragma unroll
    for (int u = 0; u < kSub; ++u) {
      const int c = min(c0 + 256 * u + lane * 4, max(n4 - 4, 0));
#pragma unroll
      for (int q = 0; q < kMultiRows; ++q) x[u][q] = *reinterpret_cast<const float4*>(a[q] + c);
    }
  };
  if (nchunk > 0) {
    float4 x[kSub][kMultiRows];
    load_stage(0);
    load_a(0, x);
    store_stage(0);
    __syncthreads();
    for (int i = 0; i < nchunk; ++i) {
      const int c0 = i * kChunk;
      const bool more = i + 1 < nchunk;
      float4 xn[kSub][kMultiRows];
      if (more) {
        load_stage(c0 + kChunk);
        load_a(c0 + kChunk, xn);
      }
      const double(*yb)[kChunk] = ysh[i & 1];
#pragma unroll
      for (int u = 0; u < kSub; ++u) {
        if (c0 + 256 * u + lane * 4 < n4) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double2 y0 = *reinterpret_cast<const double2*>(&yb[r][256 * u + lane * 4]);
            const double2 y1 =
                *reinterpret_cast<const double2*>(&yb[r][256 * u + lane * 4 + 2]);
#pragma unroll
            for (int q = 0; q < kMultiRows; ++q) {
              acc[q][r] = fma((double)x[u][q].x, y0.x, acc[q][r]);
              acc[q][r] = fma((double)x[u][q].y, y0.y, acc[q][r]);
              acc[q][r] = fma((double)x[u][q].z, y1.x, acc[q][r]);
              acc[q][r] = fma((double)x[u][q].w, y1.y, acc[q][r]);
            }
          }
        }
      }
      if (more) {
        store_stage((i + 1) & 1);
#pragma unroll
        for (int u = 0; u < kSub; ++u)
#pragma unroll
          for (int q = 0; q < kMultiRows; ++q) x[u][q] = xn[u][q];
      }
      __syncthreads();
    }
  }
  if (row0 >= n) return;
  for (int cc = n4 + lane; cc < n; cc += kWave) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double yv = Y[(int64_t)min(r, nr - 1) * ldy + cc];
#pragma unroll
      for (int q = 0; q < kMultiRows; ++q) acc[q][r] = fma((double)a[q][cc], yv, acc[q][r]);
    }
  }
#pragma unroll
  for (int q = 0; q < kMultiRows; ++q) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double sres = wave_sum(acc[q][r]);
      if (lane == 0 && r < nr && row0 + q < n) T[(int64_t)r * ldt + row0 + q] = sres;
    }
  }
}

// t[i] = sum_c A[permA[i]][c] v[c] with fp64 A and v (the uniform-precision
// product for u = fp64): one wave per row, double2 loads
__global__ __launch_bounds__(256) void k_gemv_a64(const double* __restrict__ A, int64_t ld,
                                                  const int* __restrict__ permA, int n,
                                                  const double* __restrict__ v,
                                                  double* __restrict__ t, const CycleState* gate,
                                                  int step) {
  if (gated_off(gate, step)) return;
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= n) return;
  const int prow = permA ? permA[row] : row;
  const double* a = A + (int64_t)prow * ld;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  const int n2 = n & ~1;
  int c = lane * 2;
  for (; c + 128 < n2; c += 256) {
    const double2 a0 = *reinterpret_cast<const double2*>(a + c);
    const double2 a1 = *reinterpret_cast<const double2*>(a + c + 128);
    const double2 x0 = *reinterpret_cast<const double2*>(v + c);
    const double2 x1 = *reinterpret_cast<const double2*>(v + c + 128);
    acc0 = fma(a0.x, x0.x, acc0);
    acc1 = fma(a0.y, x0.y, acc1);
    acc2 = fma(a1.x, x1.x, acc2);
    acc3 = fma(a1.y, x1.y, acc3);
  }
  for (; c < n2; c += 128) {
    const double2 a0 = *reinterpret_cast<const double2*>(a + c);
    const double2 x0 = *reinterpret_cast<const double2*>(v + c);
    acc0 = fma(a0.x, x0.x, acc0);
    acc1 = fma(a0.y, x0.y, acc1);
  }
  for (int cc = n2 + lane; cc < n; cc += kWave) acc0 = fma(a[cc], v[cc], acc0);
  const double s = wave_sum((acc0 + acc1) + (acc2 + acc3));
  if (lane == 0) t[row] = s;
}

// ---------------------------------------------------------------------------
// residual r = b - A x (fp64), norms[0] = max |r_i|, norms[1] = max |x_i|
// ---------------------------------------------------------------------------
__global__ void k_zero_u64(unsigned long long* p, int k) {
  if (threadIdx.x < k) p[threadIdx.x] = 0ull;
}

// norms[0], norms[1] and norms[kNormCw] cleared
__global__ void k_zero_resid_norms(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
  if (threadIdx.x == 2) p[kNormCw] = 0ull;
}

// One wave takes R rows: each lane's loads of x serve all of them (one wave
// per row had read x from the cache once per row, as many bytes as A).
// Every row keeps its own four accumulators, summed in the order of the
// one-row form, so r does not depend on R.
constexpr int kResidRows = 4;
template <int R>
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ A, int64_t ld, int n,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ r,
                                                  unsigned long long* norms) {
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int row0 = (blockIdx.x * (blockDim.x / kWave) + wave) * R;
  const double* a[R];
#pragma unroll
  for (int q = 0; q < R; ++q)  // rows beyond n recompute the last row (not stored)
    a[q] = A + (int64_t)min(row0 + q, n - 1) * ld;
  double acc[R][4], ab[R][2];  // ab: sum |a| |x| (componentwise backward error)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.0;
    ab[q][0] = ab[q][1] = 0.0;
  }
  const int n2 = n & ~1;
  int c = lane * 2;
  for (; c + 384 < n2; c += 512) {
    double2 av[R][4];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) av[q][e] = *reinterpret_cast<const double2*>(a[q] + c + 128 * e);
    double2 xv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) xv[e] = *reinterpret_cast<const double2*>(x + c + 128 * e);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      acc[q][0] = fma(av[q][0].x, xv[0].x, acc[q][0]);
      acc[q][1] = fma(av[q][0].y, xv[0].y, acc[q][1]);
      acc[q][2] = fma(av[q][1].x, xv[1].x, acc[q][2]);
      acc[q][3] = fma(av[q][1].y, xv[1].y, acc[q][3]);
      acc[q][0] = fma(av[q][2].x, xv[2].x, acc[q][0]);
      acc[q][1] = fma(av[q][2].y, xv[2].y, acc[q][1]);
      acc[q][2] = fma(av[q][3].x, xv[3].x, acc[q][2]);
      acc[q][3] = fma(av[q][3].y, xv[3].y, acc[q][3]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        ab[q][0] = fma(fabs(av[q][e].x), fabs(xv[e].x), ab[q][0]);
        ab[q][1] = fma(fabs(av[q][e].y), fabs(xv[e].y), ab[q][1]);
      }
    }
  }
  for (; c < n2; c += 128) {
    const double2 x0 = *reinterpret_cast<const double2*>(x + c);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double2 a0 = *reinterpret_cast<const double2*>(a[q] + c);
      acc[q][0] = fma(a0.x, x0.x, acc[q][0]);
      acc[q][1] = fma(a0.y, x0.y, acc[q][1]);
      ab[q][0] = fma(fabs(a0.x), fabs(x0.x), ab[q][0]);
      ab[q][1] = fma(fabs(a0.y), fabs(x0.y), ab[q][1]);
    }
  }
  for (int cc = n2 + lane; cc < n; cc += kWave) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      acc[q][0] = fma(a[q][cc], x[cc], acc[q][0]);
      ab[q][0] = fma(fabs(a[q][cc]), fabs(x[cc]), ab[q][0]);
    }
  }
  // the maxima of |r_i|, |x_i| and the componentwise ratio over the valid rows
  double mrw = 0.0, mxw = 0.0, mcw = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double s = wave_sum((acc[q][0] + acc[q][2]) + (acc[q][1] + acc[q][3]));
    const double sabs = wave_sum(ab[q][0] + ab[q][1]);
    const int row = row0 + q;
    if (lane == 0 && row < n) {
      const double ri = b[row] - s;
      r[row] = ri;
      mrw = fmax(mrw, fabs(ri));
      mxw = fmax(mxw, fabs(x[row]));
      mcw = fmax(mcw, cw_ratio(fabs(ri), sabs + fabs(b[row])));
    }
  }
  __shared__ double mr[4], mx[4], mc[4];
  if (lane == 0) {
    mr[wave] = mrw;
    mx[wave] = mxw;
    mc[wave] = mcw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double am = 0.0, cm = 0.0, em = 0.0;
    for (int w = 0; w < 4; ++w) {
      am = fmax(am, mr[w]);
      cm = fmax(cm, mx[w]);
      em = fmax(em, mc[w]);
    }
    atomic_max_nonneg(norms + kNormCw, em);
    atomic_max_nonneg(norms + 0, am);
    atomic_max_nonneg(norms + 1, cm);
  }
}

// Basis-column products shared by the orthogonalisation passes and the
// first pass fused into the upper triangular solve.
// fp64 sum over the 64 lanes of a wave by DPP row shifts and row broadcasts
// (no LDS); the total lands in lane 63 (other lanes hold partial sums).  The
// tree is fixed, so the result does not depend on timing.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), Ctrl, RowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, RowMask, 0xf, false);
  return v + __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_to63(double v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8: lane 15 of each row holds the row's sum
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// A term of the passes' reductions (a basis entry times w, or w squared),
// rounded on its own: with contraction off here the compiler cannot fuse the
// product into the reduction's first addition, so every pass and every
// variant that forms these sums gets the same bits however its code is
// arranged.
__device__ __forceinline__ double sum_term(double x, double w) {
#pragma clang fp contract(off)
  return x * w;
}

// rows per workgroup of the orthogonalisation passes (their 256-row chunks)
constexpr int kRowsPerBlock = 256;

// vectors in the working precision u: VT = float (u = fp32) or double (fp64)
template <typename VT>
__device__ __forceinline__ double basis_at(const Basis& X, int c, int row) {
  return (c < X.kc) ? X.c64[(int64_t)c * X.ldc + row]
                    : (double)static_cast<const VT*>(X.v)[(int64_t)(c - X.kc) * X.ldv + row];
}

// fl_u(x) held in fp64
template <typename VT>
__device__ __forceinline__ double round_u(double x) {
  return (double)(VT)x;
}

// s <- fma(X[row, c], coef[c], s) for c = 0 .. kc + nv - 1 in order: the C_k
// columns, then the V columns.  The values of eight columns are loaded before
// any of their products is taken, so a row waits for one memory round trip
// per eight columns instead of one per column; the loads are unconditional
// (a column past the end reads the last one, unused), so that no branch
// separates them.
constexpr int kBatchCols = 8;
template <typename VT>
__device__ __forceinline__ double basis_row_fma(const Basis& X, int row,
                                                const double* __restrict__ coef, double s) {
  for (int c = 0; c < X.kc; c += kBatchCols) {
    double v[kBatchCols];
#pragma unroll
    for (int e = 0; e < kBatchCols; ++e) {
      const int cc = (c + e < X.kc) ? c + e : X.kc - 1;
      v[e] = X.c64[(int64_t)cc * X.ldc + row];
    }
#pragma unroll
    for (int e = 0; e < kBatchCols; ++e)
      if (c + e < X.kc) s = fma(v[e], coef[c + e], s);
  }
  const VT* V = static_cast<const VT*>(X.v);
  const double* cv = coef + X.kc;
  for (int c = 0; c < X.nv; c += kBatchCols) {
    double v[kBatchCols];
#pragma unroll
    for (int e = 0; e < kBatchCols; ++e) {
      const int cc = (c + e < X.nv) ? c + e : X.nv - 1;
      v[e] = (double)V[(int64_t)cc * X.ldv + row];
    }
#pragma unroll
    for (int e = 0; e < kBatchCols; ++e)
      if (c + e < X.nv) s = fma(v[e], cv[c + e], s);
  }
  return s;
}

// products X[row, c] * w for the columns c0 .. c0 + G - 1 (zero for
// columns >= ncol or an invalid row), all loads issued before any is used
// (G = kDotGroup, or fewer where registers are short: each column's product
// is the same whatever the group).  The loads are unconditional: an invalid
// row reads row 0 and a column past ncol the last one, neither used; a group
// that lies wholly in C_k or wholly in V loads one kind only.
constexpr int kDotGroup = 16;
template <typename VT, int G>
__device__ __forceinline__ void basis_products(const Basis& X, int c0, int ncol, int row,
                                               bool valid, double w, double (&pr)[G]) {
  const int r = valid ? row : 0;
  const VT* V = static_cast<const VT*>(X.v);
  if (c0 + G <= X.kc) {
#pragma unroll
    for (int e = 0; e < G; ++e) pr[e] = X.c64[(int64_t)(c0 + e) * X.ldc + r];
  } else if (c0 >= X.kc) {
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int cc = (c0 + e < ncol ? c0 + e : ncol - 1) - X.kc;
      pr[e] = (double)V[(int64_t)cc * X.ldv + r];
    }
  } else if (X.nv == 0) {
#pragma unroll
    for (int e = 0; e < G; ++e)
      pr[e] = X.c64[(int64_t)(c0 + e < X.kc ? c0 + e : X.kc - 1) * X.ldc + r];
  } else {
    // the group straddles C_k and V: both loaded for every column, one kept
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int c = c0 + e < ncol ? c0 + e : ncol - 1;
      const double xc = X.c64[(int64_t)(c < X.kc ? c : X.kc - 1) * X.ldc + r];
      const double xv = (double)V[(int64_t)(c >= X.kc ? c - X.kc : 0) * X.ldv + r];
      pr[e] = c < X.kc ? xc : xv;
    }
  }
#pragma unroll
  for (int e = 0; e < G; ++e) pr[e] = (valid && c0 + e < ncol) ? sum_term(pr[e], w) : 0.0;
}

// s = ((0 + p[0]) + p[stride]) + ... over count values in order, the values
// of eight at a time loaded before any is added (one memory round trip per
// eight instead of per value)
__device__ __forceinline__ double ordered_sum(const double* __restrict__ p, int count,
                                              int64_t stride) {
  double s = 0.0;
  for (int b = 0; b < count; b += 8) {
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = p[(int64_t)(b + e < count ? b + e : count - 1) * stride];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (b + e < count) s += v[e];
  }
  return s;
}


// ---------------------------------------------------------------------------
// Triangular solves with the u_f factors in fp64 arithmetic.
//
// One workgroup (8 waves) per block of 128 rows.  The off-diagonal tiles of a
// block row are consumed as soon as the producing block has published its
// part of the solution (tags == epoch), each lane one row of a 64-column
// tile, with the tile loaded before the wait.  The diagonal block is applied
// through its fp64 inverse and the neighbouring block through its product
// with that inverse (both formed once per factorisation), so no dependent
// chain of substitution steps sits on the critical path.
// ---------------------------------------------------------------------------
// Blocked triangular solve, one workgroup per 128-row block (two 64-row
// tiles), fp64 arithmetic with the u_f factor entries taken exactly:
//   lower: y_I = Dinv_I (in_I - sum_{J < I-1} L_IJ y_J) - P_I y_{I-1}
//   upper: z_I = Dinv_I (y_I  - sum_{J > I+1} U_IJ z_J) - P_I z_{I+1}
// Dinv_I is the fp64 inverse of the 128 x 128 diagonal block and P_I its
// product with the neighbouring off-diagonal block.  For the far tiles waves
// 0-3 own the first 64 rows, waves 4-7 the second; wave w takes the 64-column
// tiles J = w mod 4, stepping by 4, and widens each tile row from raw u_f
// bits.
// Finished blocks are published as tagged words: row i's fp64 value is split
// into two 64-bit words (tag << 32 | half) in xw[2i], xw[2i+1], written with
// relaxed device-scope atomic stores; a reader polls until both tags equal
// this launch's epoch, so a block is consumed one memory round trip after it
// is written, with no flags and no fences.
constexpr int kTS = 128;  // rows per workgroup
constexpr int kTSThreads = 512;

__device__ __forceinline__ void put_tagged(uint64_t* xw, int row, double v, uint32_t tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  __hip_atomic_store(xw + 2 * row, ((uint64_t)tag << 32) | (b & 0xFFFFFFFFull),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(xw + 2 * row + 1, ((uint64_t)tag << 32) | (b >> 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// every lane reads the value of row `row` (wave-uniform result: the wave
// waits until all its lanes see this epoch's tags); false on abort
__device__ __forceinline__ bool get_tagged_row(const uint64_t* xw, int row, uint32_t tag,
                                               double& v, int* abortp) {
  const uint64_t* p = xw + 2 * row;
  long long spins = 0;
  for (;;) {
    const uint64_t lo = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t hi = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = (uint32_t)(lo >> 32) == tag && (uint32_t)(hi >> 32) == tag;
    if (__all(ok)) {
      v = __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
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

// wave-uniform: every lane reads row (c0 + lane)'s value; false on abort
__device__ __forceinline__ bool get_tagged64(const uint64_t* xw, int c0, uint32_t tag, double& v,
                                             int* abortp) {
  return get_tagged_row(xw, c0 + (int)(threadIdx.x % kWave), tag, v, abortp);
}

// lane c's fp64 value, read into scalar registers (c a compile-time constant)
__device__ __forceinline__ double lane_value(double v, int c) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), c);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), c);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// v summed over the lanes of each aligned group of four, as
// ((v0 + v1) + (v2 + v3)), through DPP quad permutations (no LDS)
__device__ __forceinline__ double quad_sum(double v) {
  const long long b = __double_as_longlong(v);
  // quad_perm [1,0,3,2]: the partner lane l ^ 1
  const int lo1 = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), 0xB1, 0xf, 0xf, false);
  const int hi1 = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xf, 0xf, false);
  v += __longlong_as_double(((long long)(unsigned)hi1 << 32) | (unsigned)lo1);
  const long long c = __double_as_longlong(v);
  // quad_perm [2,3,0,1]: the partner lane l ^ 2
  const int lo2 = __builtin_amdgcn_update_dpp(0, (int)(c & 0xFFFFFFFFll), 0x4E, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, (int)(c >> 32), 0x4E, 0xf, 0xf, false);
  return v + __longlong_as_double(((long long)(unsigned)hi2 << 32) | (unsigned)lo2);
}

// One wave fetches the 128 published values of rows base .. base + 127
// (lane l: rows base + l and base + 64 + l).  Wave-uniform; false on abort.
__device__ __forceinline__ bool get_tagged_block(const uint64_t* xw, int base, uint32_t tag,
                                                 double& v0, double& v1, int* abortp) {
  const int lane = threadIdx.x % kWave;
  const uint64_t* p0 = xw + 2 * (base + lane);
  const uint64_t* p1 = xw + 2 * (base + kWave + lane);
  long long spins = 0;
  for (;;) {
    const uint64_t a0 = __hip_atomic_load(p0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t a1 = __hip_atomic_load(p0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t a2 = __hip_atomic_load(p1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t a3 = __hip_atomic_load(p1 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = (uint32_t)(a0 >> 32) == tag && (uint32_t)(a1 >> 32) == tag &&
                    (uint32_t)(a2 >> 32) == tag && (uint32_t)(a3 >> 32) == tag;
    if (__all(ok)) {
      v0 = __longlong_as_double((long long)((a1 << 32) | (a0 & 0xFFFFFFFFull)));
      v1 = __longlong_as_double((long long)((a3 << 32) | (a2 & 0xFFFFFFFFull)));
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

// Several right-hand sides are independent solves in one launch: column c
// reads in + c * cs.in and writes y + c * cs.y, out64 + c * cs.out, exchanging
// its values through xw + c * cs.xw.  The grid runs over groups of eight
// block positions: workgroup 8 ncols g + 8 c + e is position 8 g + e of
// column c (workgroups past the last position return at once).  Two
// properties follow.  The chains of all columns advance together when the
// launch holds more workgroups than can be resident (a column-major order
// started the later columns only as the earlier ones drained: 231 us for
// eight columns at n = 8192, against 115 us for one).  And since workgroup w
// runs on XCD w mod 8, every column's block at one position runs on the same
// XCD and reads that block row of the factor through one L2 (ten columns:
// 165 us, against 185 us in plain position-major order).  A block waits only
// for blocks of its own column at earlier positions, which have smaller
// workgroup indices and were dispatched before it.  With one column the
// order is the identity.
struct ColStrides {
  int64_t in, y, out, xw;
  int ncols = 1;
};

// (position in the chain, column) of this workgroup; false past the last
// position
__device__ __forceinline__ bool col_block(const ColStrides& cs, int nb, int& bx, int& col) {
  const int g8 = 8 * cs.ncols;
  const int grp = (int)blockIdx.x / g8, rem = (int)blockIdx.x - grp * g8;
  col = rem >> 3;
  bx = grp * 8 + (rem & 7);
  return bx < nb;
}

inline unsigned col_grid(int n, int ncols) {
  const unsigned nb = (unsigned)((n + kTS - 1) / kTS);
  return ncols == 1 ? nb : ((nb + 7) / 8) * 8 * (unsigned)ncols;
}

// The A-tilde product fused into the lower solve (u = fp32): the launch's
// workgroups beyond the solve's blocks compute t = A_u[permA] v, eight rows
// each (one wave per row, the sums of k_gemv_au), and publish every row as
// two tagged words in xt; a solve block takes its right-hand side from there
// as soon as its rows are published, so the product streams from HBM while
// the chain of blocks is running.
struct FusedGemv {
  const float* Au;
  int64_t ld;
  const int* permA;
  const float* v;
  uint64_t* xt;
};

// vectors read by quarters: quarter q at q * kQS (padded so that the four
// quarters a lane quad reads fall in different LDS banks)
constexpr int kQS = kTS / 4 + 2;

// LDS of one triangular-solve block
struct TrsvShared {
  // this thread's quarter row of the inverse diagonal block, kept in the
  // order it is read (its product is formed two chain steps ahead of need,
  // so it does not have to occupy registers)
  double dsh[kTS / 4][kTSThreads + 2];
  double red[8][kTB];
  double ysh[8][kTB];
  double zsh[4 * kQS];
  double yadj[4 * kQS];
  double yadj2[4 * kQS];
  int wok[8];
};

// One 128-row block of a blocked triangular solve (lower: block blk of L y =
// t; upper: block blk of U z = y), run by a 512-thread workgroup: init()
// stages the block's three fp64 matrices once, solve() runs one solve and
// may be called again (a persistent workgroup keeps its matrices).
template <class F, bool kUpper>
struct TrsvBlock {
  using T = typename F::T;
  int n, nb, nt, blk, r0, tid, wave, lane, wq, di, dq4, adj, adj2;
  bool valid, hasAdj, hasAdj2;
  const T* srow;
  double mq[kTS / 4], qq[kTS / 4];

  __device__ __forceinline__ void init(TrsvShared& sm, const T* S, int64_t ld,
                                       const int* __restrict__ permS, int n_, int blk_,
                                       const double* __restrict__ Dinv) {
    n = n_;
    nb = (n + kTS - 1) / kTS;
    nt = (n + kTB - 1) / kTB;  // 64-column tiles
    blk = blk_;
    r0 = blk * kTS;
    tid = threadIdx.x;
    wave = tid / kWave;
    lane = tid % kWave;
    const int half = wave >> 2;
    wq = wave & 3;
    const int row = r0 + half * kTB + lane;
    valid = row < n;
    const int prow = valid ? (permS ? permS[row] : row) : 0;
    srow = S + (int64_t)prow * ld;
    // the two nearest blocks (the last ones this block waits for) enter
    // through their precomputed products with the inverse diagonal block
    hasAdj = kUpper ? blk < nb - 1 : blk > 0;
    adj = kUpper ? blk + 1 : blk - 1;
    hasAdj2 = kUpper ? blk < nb - 2 : blk > 1;
    adj2 = kUpper ? blk + 2 : blk - 2;
    // the products with the inverse diagonal block and the neighbours'
    // products: wave w takes rows 16 w .. 16 w + 15, lane l the quarter l % 4
    // of row 16 w + l / 4, so a row's four partial sums sit in one lane quad
    di = wave * 16 + lane / 4;
    dq4 = lane % 4;
    // each 128 x 128 block is read whole rows at a time (a wave reads one
    // row per load) into dsh in the per-thread order: thread 64 (r / 16) +
    // 4 (r % 16) + (col / 32) holds row r's columns col / 32 * 32 .. + 31
    const double* dblk = Dinv + (int64_t)blk * kTS * kTS;
    auto stage = [&](const double* M) {
      __syncthreads();
#pragma unroll 4
      for (int k = 0; k < kTS * kTS / 2 / kTSThreads; ++k) {
        const int idx = k * kTSThreads + tid;
        const int r = idx >> 6, col = 2 * (idx & 63);
        const double2 v = *reinterpret_cast<const double2*>(M + (int64_t)r * kTS + col);
        const int t2 = 64 * (r >> 4) + 4 * (r & 15) + (col >> 5);
        sm.dsh[col & 31][t2] = v.x;
        sm.dsh[(col & 31) + 1][t2] = v.y;
      }
      __syncthreads();
    };
    if (hasAdj) {
      stage(dblk + (int64_t)nb * kTS * kTS);
#pragma unroll
      for (int c = 0; c < kTS / 4; ++c) mq[c] = sm.dsh[c][tid];
    } else {
#pragma unroll
      for (int c = 0; c < kTS / 4; ++c) mq[c] = 0.0;
    }
    if (hasAdj2) {
      stage(dblk + 2 * (int64_t)nb * kTS * kTS);
#pragma unroll
      for (int c = 0; c < kTS / 4; ++c) qq[c] = sm.dsh[c][tid];
    } else {
#pragma unroll
      for (int c = 0; c < kTS / 4; ++c) qq[c] = 0.0;
    }
    stage(dblk);
  }

  // One solve: the right-hand side of row r0 + tid (tid < kTS) is in[permIn
  // (row)] (rhs_words null; loaded before the far tiles) or the value
  // published as tagged words in rhs_words (polled after them; rows beyond n
  // read as zero).  The block's results are published in xw with epoch.
  // Returns false on abort; p is the value of row r0 + di (every lane of
  // the row's quad).
  __device__ __forceinline__ bool solve(TrsvShared& sm, uint64_t* xw, uint32_t epoch, int* abortp,
                                        const double* __restrict__ in,
                                        const int* __restrict__ permIn,
                                        const uint64_t* rhs_words, double& p) {
    double rhs = 0.0;
    if (!rhs_words && tid < kTS && r0 + tid < n) {
      const int rr = r0 + tid;
      rhs = in[permIn ? permIn[rr] : rr];
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    bool ok = true;
    // off-diagonal tiles other than the two nearest blocks' four
    const int t0 = kUpper ? 2 * blk + 6 : 0;
    const int t1 = kUpper ? nt : (blk > 2 ? 2 * blk - 4 : 0);
    // lower: ascending from tile wq; upper: descending from the last tile
    for (int i = wq;; i += 4) {
      const int J = kUpper ? t1 - 1 - i : t0 + i;
      if (kUpper ? (J < t0) : (J >= t1)) break;
      RawRow<F> lv;
      lv.load(srow, J * kTB, n, valid);
      double yv;
      if (!get_tagged64(xw, J * kTB, epoch, yv, abortp)) {
        ok = false;
        break;
      }
      sm.ysh[wave][lane] = yv;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int c = 0; c < kTB; c += 4) {
        acc0 = fma(lv.at(c), sm.ysh[wave][c], acc0);
        acc1 = fma(lv.at(c + 1), sm.ysh[wave][c + 1], acc1);
        acc2 = fma(lv.at(c + 2), sm.ysh[wave][c + 2], acc2);
        acc3 = fma(lv.at(c + 3), sm.ysh[wave][c + 3], acc3);
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (rhs_words && ok && tid < kTS) {
      // waves 0 and 1: this block's right-hand side from the published rows
      // (rows beyond n were never published and stay zero)
      double tv = 0.0;
      if (!get_tagged_row(rhs_words, r0 + tid < n ? r0 + tid : r0, epoch, tv, abortp)) ok = false;
      rhs = (r0 + tid < n) ? tv : 0.0;
    }
    sm.red[wave][lane] = (acc0 + acc1) + (acc2 + acc3);
    if (lane == 0) sm.wok[wave] = ok ? 1 : 0;
    __syncthreads();
    int allok = 1;
#pragma unroll
    for (int w = 0; w < 8; ++w) allok &= sm.wok[w];
    if (!allok) return false;
    if (tid < kTS) {
      const int h = tid / kTB, l = tid % kTB;
      const double sum =
          (sm.red[4 * h][l] + sm.red[4 * h + 1][l]) + (sm.red[4 * h + 2][l] + sm.red[4 * h + 3][l]);
      sm.zsh[(tid / (kTS / 4)) * kQS + tid % (kTS / 4)] = (r0 + tid < n) ? rhs - sum : 0.0;
    }
    __syncthreads();
    // Dinv (in - sum over the far blocks) - Q (second neighbour's values) -
    // P (neighbour's values), this thread's quarter of its row, in four
    // interleaved partial sums
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    {
      const double* z = sm.zsh + dq4 * kQS;
#pragma unroll
      for (int c = 0; c < kTS / 4; c += 4) {
        p0 = fma(sm.dsh[c][tid], z[c], p0);
        p1 = fma(sm.dsh[c + 1][tid], z[c + 1], p1);
        p2 = fma(sm.dsh[c + 2][tid], z[c + 2], p2);
        p3 = fma(sm.dsh[c + 3][tid], z[c + 3], p3);
      }
    }
    if (hasAdj2) {
      // the second-nearest block's values, one chain step ahead of need
      if (wave == 0) {
        double ya0 = 0.0, ya1 = 0.0;
        const bool got = get_tagged_block(xw, adj2 * kTS, epoch, ya0, ya1, abortp);
        sm.yadj2[(lane / 32) * kQS + lane % 32] = ya0;
        sm.yadj2[(2 + lane / 32) * kQS + lane % 32] = ya1;
        if (lane == 0) sm.wok[1] = got ? 1 : 0;
      }
      __syncthreads();
      if (!sm.wok[1]) return false;
      const double* ya = sm.yadj2 + dq4 * kQS;
#pragma unroll
      for (int c = 0; c < kTS / 4; c += 4) {
        p0 = fma(-qq[c], ya[c], p0);
        p1 = fma(-qq[c + 1], ya[c + 1], p1);
        p2 = fma(-qq[c + 2], ya[c + 2], p2);
        p3 = fma(-qq[c + 3], ya[c + 3], p3);
      }
    }
    if (hasAdj) {
      // wave 0 fetches the neighbour's 128 values for all
      if (wave == 0) {
        double ya0 = 0.0, ya1 = 0.0;
        const bool got = get_tagged_block(xw, adj * kTS, epoch, ya0, ya1, abortp);
        // rows lane and 64 + lane: quarters lane / 32 and 2 + lane / 32
        sm.yadj[(lane / 32) * kQS + lane % 32] = ya0;
        sm.yadj[(2 + lane / 32) * kQS + lane % 32] = ya1;
        if (lane == 0) sm.wok[0] = got ? 1 : 0;
      }
      __syncthreads();
      if (!sm.wok[0]) return false;
      const double* ya = sm.yadj + dq4 * kQS;
#pragma unroll
      for (int c = 0; c < kTS / 4; c += 4) {
        p0 = fma(-mq[c], ya[c], p0);
        p1 = fma(-mq[c + 1], ya[c + 1], p1);
        p2 = fma(-mq[c + 2], ya[c + 2], p2);
        p3 = fma(-mq[c + 3], ya[c + 3], p3);
      }
    }
    p = quad_sum((p0 + p1) + (p2 + p3));
    return true;
  }
};

template <class F, bool kUpper, bool kFused = false, bool kDots = false>
__global__ __launch_bounds__(kTSThreads) void k_trsv(const typename F::T* __restrict__ S,
                                                     int64_t ld, const int* __restrict__ permS,
                                                     int n, const double* __restrict__ in,
                                                     const int* __restrict__ permIn,
                                                     const double* __restrict__ Dinv, double* y,
                                                     double scale, double* __restrict__ out64,
                                                     float* __restrict__ out32, uint64_t* xw,
                                                     uint32_t epoch, const CycleState* gate,
                                                     int step, int* abortp, ColStrides cs,
                                                     FusedGemv fg = FusedGemv{},
                                                     TrsvDots td = TrsvDots{}) {
  if (gated_off(gate, step)) return;
  if (kFused && (int)blockIdx.x >= (n + kTS - 1) / kTS) {
    // a product workgroup: rows 8 (b - nb) + wave
    const int row = ((int)blockIdx.x - (n + kTS - 1) / kTS) * (kTSThreads / kWave) +
                    (int)(threadIdx.x / kWave);
    if (row >= n) return;
    const int prow = fg.permA ? fg.permA[row] : row;
    const double t = gemv_au_row<float, 8>(fg.Au + (int64_t)prow * fg.ld, fg.v, n,
                                           (int)(threadIdx.x % kWave));
    if ((threadIdx.x % kWave) == 0) put_tagged(fg.xt, row, t, epoch);
    return;
  }
  const int nb = (n + kTS - 1) / kTS;
  int bx, col;
  if (!col_block(cs, nb, bx, col)) return;
  in += (int64_t)col * cs.in;
  if (y) y += (int64_t)col * cs.y;
  if (out64) out64 += (int64_t)col * cs.out;
  xw += (int64_t)col * cs.xw;
  __shared__ TrsvShared sm;
  const int blk = kUpper ? nb - 1 - bx : bx;
  TrsvBlock<F, kUpper> tb;
  tb.init(sm, S, ld, permS, n, blk, Dinv);
  double p = 0.0;
  if (!tb.solve(sm, xw, epoch, abortp, in, permIn, kFused ? fg.xt : nullptr, p)) return;
  const int tid = tb.tid, wave = tb.wave, lane = tb.lane, di = tb.di, dq4 = tb.dq4;
  const int r0 = tb.r0;
  if constexpr (!kDots) {
    if (dq4 != 0) return;
  }
  const int rr = r0 + di;
  const double v = (rr < n) ? p : 0.0;
  if (dq4 == 0) {
    if (rr < n) {
      if (y) y[rr] = v;
      if (out64) out64[rr] = v * scale;
      if (out32) out32[rr] = (float)(v * scale);
    }
    put_tagged(xw, rr, v, epoch);
  }
  if constexpr (kDots) {
    // the first classical Gram-Schmidt pass of the Arnoldi step on this
    // block's rows of w = fl_u(2^e z): lane = row, each basis column summed
    // over a wave's 64 rows by the orthogonalisation's DPP tree, the two
    // waves added as the passes add a chunk's first (or second) pair of
    // waves; the last block adds the pairs of each 256-row chunk and then
    // the chunks in order, so h1 is bit-identical to the separate pass
    __shared__ double wsh[kTS];
    __shared__ double hsum[2][kDotsMaxCols];
    __shared__ unsigned int s_ticket;
    if (dq4 == 0) wsh[di] = (rr < n) ? (double)(float)(v * scale) : 0.0;
    __syncthreads();
    const int ncol = td.X.kc + td.X.nv;
    if (wave < 2) {
      const int lrow = wave * kWave + lane;
      const int grow = r0 + lrow;
      const double wv = wsh[lrow];
      for (int c0 = 0; c0 < ncol; c0 += kDotGroup) {
        double pr[kDotGroup];
        basis_products<float>(td.X, c0, ncol, grow, grow < n, wv, pr);
#pragma unroll
        for (int e = 0; e < kDotGroup; ++e) pr[e] = wave_sum_to63(pr[e]);
        if (lane == kWave - 1) {
#pragma unroll
          for (int e = 0; e < kDotGroup; ++e)
            if (c0 + e < ncol) hsum[wave][c0 + e] = pr[e];
        }
      }
    }
    __syncthreads();
    for (int c = tid; c < ncol; c += kTSThreads)
      td.partial[(int64_t)blk * ncol + c] = hsum[0][c] + hsum[1][c];
    __threadfence();
    __syncthreads();
    if (tid == 0) s_ticket = atomicAdd(td.counter, 1u);
    __syncthreads();
    if (s_ticket != (unsigned)nb - 1) return;
    __threadfence();
    for (int c = tid; c < ncol; c += kTSThreads) {
      double sum = 0.0;
      for (int b = 0; b < nb; b += 16) {
        double v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
          v[e] = (b + e < nb) ? td.partial[(int64_t)(b + e) * ncol + c] : 0.0;
#pragma unroll
        for (int e = 0; e < 16; e += 2)
          if (b + e < nb) sum += v[e] + v[e + 1];
      }
      td.h1[c] = sum;
    }
    if (tid == 0) *td.counter = 0u;
  }
}

// 128 x 128 inverses of the diagonal blocks from the 64 x 64 ones (D64):
//   lower [A 0; B C]^-1 = [A^-1 0; -C^-1 B A^-1  C^-1]
//   upper [A B; 0 C]^-1 = [A^-1  -A^-1 B C^-1; 0 C^-1]
// (fp64, B taken exactly from the u_f factor; a missing second 64-block or
// rows beyond n act as the identity).
template <class F, bool kUpper>
__device__ __forceinline__ void diag_combine(const typename F::T* __restrict__ S, int64_t ld,
                                             const int* __restrict__ permS, int n,
                                             const double* __restrict__ D64,
                                             double* __restrict__ D128, double (&Ai)[kTB][kTB + 1],
                                             double (&Ci)[kTB][kTB + 1],
                                             double (&Bm)[kTB][kTB + 1],
                                             double (&T)[kTB][kTB + 1]) {
  const int blk = blockIdx.x;
  const int tid = threadIdx.x;
  const int nt = (n + kTB - 1) / kTB;
  const int ta = 2 * blk, tc = 2 * blk + 1;
  const bool hasC = tc < nt;
  for (int idx = tid; idx < kTB * kTB; idx += 256) {
    const int r = idx / kTB, c = idx % kTB;
    Ai[r][c] = D64[(int64_t)ta * kTB * kTB + idx];
    Ci[r][c] = hasC ? D64[(int64_t)tc * kTB * kTB + idx] : (r == c ? 1.0 : 0.0);
    // off-diagonal block: lower B = L[rows of C][cols of A]; upper B = U[rows of A][cols of C]
    const int gr = kUpper ? ta * kTB + r : tc * kTB + r;
    const int gc = kUpper ? tc * kTB + c : ta * kTB + c;
    double bv = 0.0;
    if (hasC && gr < n && gc < n) {
      const int pr = permS ? permS[gr] : gr;
      bv = (double)F::to_f(S[(int64_t)pr * ld + gc]);
    }
    Bm[r][c] = bv;
  }
  __syncthreads();
  // lower: T = B A^-1, X = -C^-1 T;  upper: T = B C^-1, X = -A^-1 T
  for (int idx = tid; idx < kTB * kTB; idx += 256) {
    const int r = idx / kTB, c = idx % kTB;
    double sum = 0.0;
    for (int t = 0; t < kTB; ++t) sum = fma(Bm[r][t], kUpper ? Ci[t][c] : Ai[t][c], sum);
    T[r][c] = sum;
  }
  __syncthreads();
  double* out = D128 + (int64_t)blk * kTS * kTS;
  for (int idx = tid; idx < kTS * kTS; idx += 256) {
    const int r = idx / kTS, c = idx % kTS;
    const int rh = r / kTB, ch = c / kTB, rl = r % kTB, cl = c % kTB;
    double v = 0.0;
    if (rh == 0 && ch == 0) {
      v = Ai[rl][cl];
    } else if (rh == 1 && ch == 1) {
      v = Ci[rl][cl];
    } else if (kUpper ? (rh == 0 && ch == 1) : (rh == 1 && ch == 0)) {
      double sum = 0.0;
      for (int t = 0; t < kTB; ++t) sum = fma(kUpper ? Ai[rl][t] : Ci[rl][t], T[t][cl], sum);
      v = -sum;
    }
    out[idx] = v;
  }
}

// both triangles in one launch: blockIdx.y = 0 for L, 1 for U
template <class F>
__global__ __launch_bounds__(256) void k_diag_combine(const typename F::T* __restrict__ S,
                                                      int64_t ld, const int* __restrict__ permS,
                                                      int n, const double* __restrict__ D64L,
                                                      const double* __restrict__ D64U,
                                                      double* __restrict__ Linv,
                                                      double* __restrict__ Uinv) {
  __shared__ double Ai[kTB][kTB + 1];
  __shared__ double Ci[kTB][kTB + 1];
  __shared__ double Bm[kTB][kTB + 1];
  __shared__ double T[kTB][kTB + 1];
  if (blockIdx.y == 0)
    diag_combine<F, false>(S, ld, permS, n, D64L, Linv, Ai, Ci, Bm, T);
  else
    diag_combine<F, true>(S, ld, permS, n, D64U, Uinv, Ai, Ci, Bm, T);
}

// Products of each 128 x 128 inverse diagonal block with the neighbouring
// off-diagonal block of the same triangle, in fp64 with the u_f entries
// taken exactly:
//   lower: P_I = Dinv_I L_{I,I-1}  (I >= 1)
//   upper: P_I = Dinv_I U_{I,I+1}  (I <= nb - 2)
// so that the blocked solve needs one 128 x 128 product once the neighbour's
// values arrive.  Grid (nb - 1, 4, 2): blockIdx.y picks 32 columns of P_I,
// blockIdx.z the triangle (0: L, 1: U).  Rows or columns beyond n enter as
// zeros.
template <class F, bool kUpper>
__device__ __forceinline__ void adjacent_product(const typename F::T* __restrict__ S, int64_t ld,
                                                 const int* __restrict__ permS, int n,
                                                 const double* __restrict__ Dinv,
                                                 double* __restrict__ P, int dist,
                                                 double (&B)[kTS][kTS / 4 + 1]) {
  constexpr int kC = kTS / 4;
  const int blk = kUpper ? (int)blockIdx.x : (int)blockIdx.x + dist;
  const int adj = kUpper ? blk + dist : blk - dist;
  const int c0 = adj * kTS + (int)blockIdx.y * kC;  // first global column
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kTS * kC; idx += 256) {
    const int t = idx / kC, c = idx % kC;
    const int gr = blk * kTS + t, gc = c0 + c;
    double v = 0.0;
    if (gr < n && gc < n) v = (double)F::to_f(S[(int64_t)(permS ? permS[gr] : gr) * ld + gc]);
    B[t][c] = v;
  }
  __syncthreads();
  const int r = tid / 2;
  const int cb = (tid % 2) * (kC / 2);
  const double* drow = Dinv + ((int64_t)blk * kTS + r) * kTS;
  double acc[kC / 2];
#pragma unroll
  for (int j = 0; j < kC / 2; ++j) acc[j] = 0.0;
  for (int t = 0; t < kTS; t += 2) {
    const double2 d = *reinterpret_cast<const double2*>(drow + t);
#pragma unroll
    for (int j = 0; j < kC / 2; ++j) {
      acc[j] = fma(d.x, B[t][cb + j], acc[j]);
      acc[j] = fma(d.y, B[t + 1][cb + j], acc[j]);
    }
  }
  double* out = P + ((int64_t)blk * kTS + r) * kTS + (int)blockIdx.y * kC + cb;
#pragma unroll
  for (int j = 0; j < kC / 2; ++j) out[j] = acc[j];
}

template <class F>
__global__ __launch_bounds__(256) void k_adjacent_product(const typename F::T* __restrict__ S,
                                                          int64_t ld,
                                                          const int* __restrict__ permS, int n,
                                                          const double* __restrict__ Linv,
                                                          double* __restrict__ PL,
                                                          const double* __restrict__ Uinv,
                                                          double* __restrict__ PU, int dist) {
  __shared__ double B[kTS][kTS / 4 + 1];
  if (blockIdx.z == 0)
    adjacent_product<F, false>(S, ld, permS, n, Linv, PL, dist, B);
  else
    adjacent_product<F, true>(S, ld, permS, n, Uinv, PU, dist, B);
}

// The products the transposed solves need, the neighbouring off-diagonal
// block times the inverse diagonal block (fp64, u_f entries exact):
//   U^T solve (block I >= 1):      Q_I = U_{I-1,I} Uinv_I
//   L^T solve (block I <= nb - 2): Q_I = L_{I+1,I} Linv_I
// Q_I^T is the block of the transposed system's product.  Grid (nb - 1, 4):
// blockIdx.y picks 32 columns of Q_I; B and the inverse are staged through
// LDS 32 contraction columns at a time.  Rows or columns beyond n enter as
// zeros.
template <class F, bool kUpperSrc>
__global__ __launch_bounds__(256) void k_adjacent_product_t(const typename F::T* __restrict__ S,
                                                            int64_t ld,
                                                            const int* __restrict__ permS, int n,
                                                            const double* __restrict__ Dinv,
                                                            double* __restrict__ Q) {
  constexpr int kC = kTS / 4;
  __shared__ double B[kTS][kC + 1];
  __shared__ double D[kC][kC + 1];
  const int blk = kUpperSrc ? (int)blockIdx.x + 1 : (int)blockIdx.x;
  const int brow0 = kUpperSrc ? (blk - 1) * kTS : (blk + 1) * kTS;  // rows of B
  const int bcol0 = blk * kTS;                                        // columns of B
  const int c0 = (int)blockIdx.y * kC;
  const int tid = threadIdx.x;
  const int r = tid / 2;
  const int cb = (tid % 2) * (kC / 2);
  const double* Db = Dinv + (int64_t)blk * kTS * kTS;
  double acc[kC / 2];
#pragma unroll
  for (int j = 0; j < kC / 2; ++j) acc[j] = 0.0;
  for (int t0 = 0; t0 < kTS; t0 += kC) {
    __syncthreads();
    for (int idx = tid; idx < kTS * kC; idx += 256) {
      const int rr = idx / kC, t = idx % kC;
      const int gr = brow0 + rr, gc = bcol0 + t0 + t;
      double v = 0.0;
      if (gr < n && gc < n) v = (double)F::to_f(S[(int64_t)(permS ? permS[gr] : gr) * ld + gc]);
      B[rr][t] = v;
    }
    for (int idx = tid; idx < kC * kC; idx += 256) {
      const int t = idx / kC, c = idx % kC;
      D[t][c] = Db[(int64_t)(t0 + t) * kTS + c0 + c];
    }
    __syncthreads();
#pragma unroll 4
    for (int t = 0; t < kC; ++t) {
      const double b = B[r][t];
#pragma unroll
      for (int j = 0; j < kC / 2; ++j) acc[j] = fma(b, D[t][cb + j], acc[j]);
    }
  }
  double* out = Q + ((int64_t)blk * kTS + r) * kTS + c0 + cb;
#pragma unroll
  for (int j = 0; j < kC / 2; ++j) out[j] = acc[j];
}

// Inverse of each 64 x 64 diagonal block of L (unit lower) or U (upper) in
// fp64, row-major per block; rows/columns beyond n get the identity.
template <class F, bool kUpper>
__device__ __forceinline__ void diag_inverse(const typename F::T* __restrict__ S, int64_t ld,
                                             const int* __restrict__ permS, int n,
                                             double* __restrict__ Dinv, double (&B)[kTB][kTB + 1],
                                             double (&X)[kTB][kTB + 1]) {
  const int blk = blockIdx.x;
  const int r0 = blk * kTB;
  const int j = threadIdx.x;  // column of the inverse
  for (int r = 0; r < kTB; ++r) {
    const int row = r0 + r;
    double v = (r == j) ? 1.0 : 0.0;
    if (row < n && r0 + j < n) {
      const int prow = permS ? permS[row] : row;
      v = (double)F::to_f(S[(int64_t)prow * ld + r0 + j]);
      if (!kUpper && r == j) v = 1.0;
    }
    B[r][j] = v;
  }
  __syncthreads();
  if (!kUpper) {
    for (int r = 0; r < kTB; ++r) {
      double v = (r == j) ? 1.0 : 0.0;
      for (int t = 0; t < r; ++t) v = fma(-B[r][t], X[t][j], v);
      X[r][j] = v;
    }
  } else {
    for (int r = kTB - 1; r >= 0; --r) {
      double v = (r == j) ? 1.0 : 0.0;
      for (int t = r + 1; t < kTB; ++t) v = fma(-B[r][t], X[t][j], v);
      X[r][j] = v / B[r][r];
    }
  }
  for (int r = 0; r < kTB; ++r) {
    const bool lowerpart = kUpper ? (j >= r) : (j <= r);
    Dinv[((int64_t)blk * kTB + r) * kTB + j] = lowerpart ? X[r][j] : 0.0;
  }
}

// both triangles in one launch: blockIdx.y = 0 for L, 1 for U
template <class F>
__global__ __launch_bounds__(64) void k_diag_inverse(const typename F::T* __restrict__ S, int64_t ld,
                                                     const int* __restrict__ permS, int n,
                                                     double* __restrict__ DinvL,
                                                     double* __restrict__ DinvU) {
  __shared__ double B[kTB][kTB + 1];
  __shared__ double X[kTB][kTB + 1];
  if (blockIdx.y == 0)
    diag_inverse<F, false>(S, ld, permS, n, DinvL, B, X);
  else
    diag_inverse<F, true>(S, ld, permS, n, DinvU, B, X);
}

// ---------------------------------------------------------------------------
// orthogonalisation passes (CGS2) with last-block reduction
// ---------------------------------------------------------------------------
// lane i's value of a per-index vector held as two registers (indices i and
// 64 + i); i is the same for the whole wave
__device__ __forceinline__ double lane_pick(double lo, double hi, int i) {
  return i < kWave ? readlane_d(lo, i) : readlane_d(hi, i - kWave);
}

// The finish of Arnoldi step j by one whole wave (every lane calls it): the
// Hessenberg column h = h1 + h2 (and the B column of the recycle part) is
// stored, the j earlier Givens rotations are applied to it, the new rotation
// annihilating beta = sqrt(norm2) is formed, and g, the residual estimate and
// the cycle state are updated.  The lanes load the coefficients in parallel;
// the rotations then run as one chain in registers (of the rotated column
// only the running entry matters: the entries above it are not used again).
__device__ __forceinline__ void arnoldi_finish(const OrthoArgs& a, const double* __restrict__ h1,
                                               const double* __restrict__ h2, double norm2) {
  const int lane = threadIdx.x % kWave;
  const int j = a.step;
  const int kc = a.X.kc;
  if (a.B)
    for (int i = lane; i < kc; i += kWave) a.B[(int64_t)j * a.ldb + i] = h1[i] + h2[i];
  double hc0 = 0.0, hc1 = 0.0, cs0 = 0.0, cs1 = 0.0, sn0 = 0.0, sn1 = 0.0;
  if (lane <= j) hc0 = h1[kc + lane] + h2[kc + lane];
  if (kWave + lane <= j) hc1 = h1[kc + kWave + lane] + h2[kc + kWave + lane];
  if (lane < j) {
    cs0 = a.cs[lane];
    sn0 = a.sn[lane];
  }
  if (kWave + lane < j) {
    cs1 = a.cs[kWave + lane];
    sn1 = a.sn[kWave + lane];
  }
  if (a.H && lane <= j) a.H[(int64_t)j * a.ldh + lane] = hc0;
  if (a.H && kWave + lane <= j) a.H[(int64_t)j * a.ldh + kWave + lane] = hc1;
  const double beta = sqrt(norm2);
  double carry = lane_pick(hc0, hc1, 0);
  for (int i = 0; i < j; ++i) {
    const double nxt = lane_pick(hc0, hc1, i + 1);
    carry = -lane_pick(sn0, sn1, i) * carry + lane_pick(cs0, cs1, i) * nxt;
  }
  if (lane != 0) return;
  if (a.H) a.H[(int64_t)j * a.ldh + j + 1] = beta;
  const double aa = carry, bb = beta;
  const double rr = hypot(aa, bb);
  double c = 1.0, s = 0.0;
  if (rr != 0.0) {
    c = aa / rr;
    s = bb / rr;
  }
  a.cs[j] = c;
  a.sn[j] = s;
  const double gj = a.g[j];
  a.g[j + 1] = -s * gj;
  a.g[j] = c * gj;
  const double est = fabs(a.g[j + 1]);
  a.st->est = est;
  a.st->jdone = j + 1;
  if (est <= a.st->tol || beta == 0.0) a.st->done = 1;
  if (a.st_out) {
    // the state after this step (the abort and singular flags were set by
    // earlier kernels, if at all) for the host's poll
    CycleState o;
    o.done = a.st->done;
    o.jdone = j + 1;
    o.abort = a.st->abort;
    o.singular = a.st->singular;
    o.tol = a.st->tol;
    o.est = est;
    *a.st_out = o;
  }
}

// v = fl_u(w / beta) (zero when beta is not positive) over n rows by one
// workgroup: 16-byte pieces, eight of them loaded per thread before any is
// used, then the scalar tail
template <typename VT>
__device__ __forceinline__ void normalize_by_block(const VT* __restrict__ w, VT* __restrict__ v,
                                                   int n, double beta) {
  constexpr int kPer = 16 / (int)sizeof(VT);
  using Vec = typename std::conditional<sizeof(VT) == 4, float4, double2>::type;
  const int nchunk = n / kPer;
  const int nt = (int)blockDim.x;
  const int tid = (int)threadIdx.x;
  for (int c0 = tid; c0 < nchunk; c0 += 8 * nt) {
    Vec x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (c0 + e * nt < nchunk) x[e] = reinterpret_cast<const Vec*>(w)[c0 + e * nt];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (c0 + e * nt >= nchunk) continue;
      VT in[kPer], out[kPer];
      __builtin_memcpy(in, &x[e], 16);
#pragma unroll
      for (int q = 0; q < kPer; ++q) out[q] = (beta > 0.0) ? (VT)((double)in[q] / beta) : (VT)0;
      Vec y;
      __builtin_memcpy(&y, out, 16);
      reinterpret_cast<Vec*>(v)[c0 + e * nt] = y;
    }
  }
  for (int i = nchunk * kPer + tid; i < n; i += nt)
    v[i] = (beta > 0.0) ? (VT)((double)w[i] / beta) : (VT)0;
}

template <typename VT>
__global__ __launch_bounds__(256) void k_ortho(OrthoArgs a, int mode) {
  if (gated_off(a.gate, a.step)) return;
  __shared__ double wsh[kRowsPerBlock];
  __shared__ double red[4][kWave + 1];
  __shared__ double coef_sh[256];
  __shared__ double colsum[4][256];
  __shared__ unsigned int s_ticket;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int ncol = a.X.kc + a.X.nv;
  const int rbase = blockIdx.x * kRowsPerBlock;
  const int row = rbase + tid;
  const bool valid = row < a.n;
  if (mode & kOrthoUpdate) {
    for (int c = tid; c < ncol; c += 256) coef_sh[c] = a.coef[c];
    __syncthreads();
  }
  const VT* w_in = static_cast<const VT*>(a.w_in);
  double wv = valid ? (double)w_in[row] : 0.0;
  if ((mode & kOrthoUpdate) && valid) {
    const double s = basis_row_fma<VT>(a.X, row, coef_sh, 0.0);
    wv = round_u<VT>(wv - s);
    static_cast<VT*>(a.w_out)[row] = (VT)wv;
  }
  wsh[tid] = wv;
  __syncthreads();
  const int nout = ncol + 1;  // dots then the squared norm
  double* part = a.partial + (int64_t)blockIdx.x * nout;
  if (mode & kOrthoDots) {
    // lane = row: each column is read coalesced, multiplied by this row's w
    // and summed over the wave's 64 rows by DPP, four columns at a time; the
    // four waves' sums are added through LDS
    for (int c0 = 0; c0 < ncol; c0 += kDotGroup) {
      double pr[kDotGroup];
      basis_products<VT>(a.X, c0, ncol, row, valid, wv, pr);
#pragma unroll
      for (int e = 0; e < kDotGroup; ++e) pr[e] = wave_sum_to63(pr[e]);
      if (lane == kWave - 1) {
#pragma unroll
        for (int e = 0; e < kDotGroup; ++e)
          if (c0 + e < ncol) colsum[wave][c0 + e] = pr[e];
      }
    }
    __syncthreads();
    for (int c = tid; c < ncol; c += 256)
      part[c] = (colsum[0][c] + colsum[1][c]) + (colsum[2][c] + colsum[3][c]);
  }
  if (mode & kOrthoNorm) {
    double sq = wave_sum(sum_term(wv, wv));
    if (lane == 0) red[wave][0] = sq;
    __syncthreads();
    if (tid == 0) part[ncol] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
  }
  // last block reduces the partial results
  __threadfence();
  __syncthreads();
  if (tid == 0) s_ticket = atomicAdd(a.counter, 1u);
  __syncthreads();
  if (s_ticket != gridDim.x - 1) return;
  __threadfence();
  if (mode & kOrthoDots) {
    for (int c = tid; c < ncol; c += 256) {
      a.dots_out[c] = ordered_sum(a.partial + c, (int)gridDim.x, nout);
    }
  }
  if ((mode & kOrthoNorm) && tid == 0) {
    a.norm_out[0] = ordered_sum(a.partial + ncol, (int)gridDim.x, nout);
  }
  if (tid == 0) *a.counter = 0u;
  if (!(mode & kOrthoFinish)) return;
  __syncthreads();
  if (wave == 0) arnoldi_finish(a, a.h_prev, a.coef, a.norm_out[0]);
  // v_{j+1} = fl_u(w / beta) by this (the last) workgroup: every other one
  // wrote its rows of w before taking its ticket
  if (a.vout)
    normalize_by_block<VT>(static_cast<const VT*>(a.w_out), static_cast<VT*>(a.vout), a.n,
                           sqrt(a.norm_out[0]));
}


// The whole classical Gram-Schmidt step (CGS2: dots, update and dots,
// update and norm), the Arnoldi finish (Hessenberg column, Givens rotation,
// residual estimate) and the normalisation of v_{j+1} in one launch of one
// workgroup, for orders up to kOrthoSmallMax.  Every sum is formed as the
// multi-workgroup passes form it -- per 256-row chunk the DPP sum over each
// wave's 64 rows, the chunk's four waves added pairwise, the chunks then
// added in order -- so the results are bit-identical to k_ortho followed by
// k_normalize; what goes away is three launches and three cross-workgroup
// reductions, which dominate the step at these orders.
constexpr int kOrthoSmallThreads = 1024;
constexpr int kOrthoSmallWaves = kOrthoSmallThreads / kWave;          // 16
constexpr int kOrthoSmallChunks = kOrthoSmallMax / kRowsPerBlock;     // 16 chunks of 256 rows
constexpr int kOrthoSmallIters = kOrthoSmallMax / kOrthoSmallThreads;  // rows per thread
constexpr int kOrthoSmallCols = 192;                                  // kc + nv (k + m <= 189)

template <typename VT>
__device__ __forceinline__ void ortho_small_dots(const Basis& X, int ncol, int n, int nbk,
                                                 const double (&wv)[kOrthoSmallIters],
                                                 double (&colsum)[kOrthoSmallWaves][kOrthoSmallCols],
                                                 double (&part)[kOrthoSmallChunks][kOrthoSmallCols],
                                                 double* __restrict__ out_lds,
                                                 double* __restrict__ out_global) {
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    if (4 * it >= nbk) break;
    const int row = it * kOrthoSmallThreads + tid;
    const bool valid = row < n;
    for (int c0 = 0; c0 < ncol; c0 += kDotGroup) {
      double pr[kDotGroup];
      basis_products<VT>(X, c0, ncol, row, valid, wv[it], pr);
#pragma unroll
      for (int e = 0; e < kDotGroup; ++e) pr[e] = wave_sum_to63(pr[e]);
      if (lane == kWave - 1) {
#pragma unroll
        for (int e = 0; e < kDotGroup; ++e)
          if (c0 + e < ncol) colsum[wave][c0 + e] = pr[e];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < 4 * ncol; idx += kOrthoSmallThreads) {
      const int q = idx / ncol, c = idx % ncol;
      if (4 * it + q < nbk)
        part[4 * it + q][c] =
            (colsum[4 * q][c] + colsum[4 * q + 1][c]) + (colsum[4 * q + 2][c] + colsum[4 * q + 3][c]);
    }
    __syncthreads();
  }
  for (int c = tid; c < ncol; c += kOrthoSmallThreads) {
    double s = 0.0;
    for (int b = 0; b < nbk; ++b) s += part[b][c];
    out_lds[c] = s;
    out_global[c] = s;
  }
  __syncthreads();
}

// a.dots_out: the first pass's coefficients (h1); a.coef: the second's (h2);
// a.norm_out: the squared norm; a.w_out: w after both updates; vout: v_{j+1}
template <typename VT>
__global__ __launch_bounds__(kOrthoSmallThreads) void k_ortho_small(OrthoArgs a, VT* vout) {
  if (gated_off(a.gate, a.step)) return;
  __shared__ double colsum[kOrthoSmallWaves][kOrthoSmallCols];
  __shared__ double part[kOrthoSmallChunks][kOrthoSmallCols];
  __shared__ double c1[kOrthoSmallCols];
  __shared__ double c2[kOrthoSmallCols];
  __shared__ double red[kOrthoSmallWaves];
  __shared__ double npart[kOrthoSmallChunks];
  __shared__ double s_beta;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int n = a.n;
  const int ncol = a.X.kc + a.X.nv;
  const int nbk = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  const VT* w_in = static_cast<const VT*>(a.w_in);
  double wv[kOrthoSmallIters];
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    const int row = it * kOrthoSmallThreads + tid;
    wv[it] = row < n ? (double)w_in[row] : 0.0;
  }
  // pass 1: h1 = X^T w
  ortho_small_dots<VT>(a.X, ncol, n, nbk, wv, colsum, part, c1, a.dots_out);
  // pass 2: w <- fl_u(w - X h1), h2 = X^T w
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    const int row = it * kOrthoSmallThreads + tid;
    if (row < n) wv[it] = round_u<VT>(wv[it] - basis_row_fma<VT>(a.X, row, c1, 0.0));
  }
  double* h2 = const_cast<double*>(a.coef);
  ortho_small_dots<VT>(a.X, ncol, n, nbk, wv, colsum, part, c2, h2);
  // pass 3: w <- fl_u(w - X h2) and its squared norm
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    const int row = it * kOrthoSmallThreads + tid;
    if (row < n) {
      wv[it] = round_u<VT>(wv[it] - basis_row_fma<VT>(a.X, row, c2, 0.0));
      static_cast<VT*>(a.w_out)[row] = (VT)wv[it];
    }
  }
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    if (4 * it >= nbk) break;
    const double sq = wave_sum(sum_term(wv[it], wv[it]));
    if (lane == 0) red[wave] = sq;
    __syncthreads();
    if (tid < 4 && 4 * it + tid < nbk)
      npart[4 * it + tid] = (red[4 * tid] + red[4 * tid + 1]) + (red[4 * tid + 2] + red[4 * tid + 3]);
    __syncthreads();
  }
  if (wave == 0) {
    double s = 0.0;
    for (int b = 0; b < nbk; ++b) s += npart[b];
    if (lane == 0) {
      a.norm_out[0] = s;
      s_beta = sqrt(s);
    }
    arnoldi_finish(a, c1, c2, s);
  }
  __syncthreads();
  // v_{j+1} = fl_u(w / beta)
  const double beta = s_beta;
#pragma unroll
  for (int it = 0; it < kOrthoSmallIters; ++it) {
    const int row = it * kOrthoSmallThreads + tid;
    if (row < n) vout[row] = (beta > 0.0) ? (VT)(wv[it] / beta) : (VT)0;
  }
}

// out[:, o] = sum_c X[:, c] M[c, o]
template <typename VT>
__global__ __launch_bounds__(256) void k_combine(Basis X, int n, const double* __restrict__ M,
                                                 int nout, double* __restrict__ out, int64_t ldo) {
  __shared__ double Msh[4096];
  const int ncol = X.kc + X.nv;
  for (int i = threadIdx.x; i < ncol * nout; i += blockDim.x) Msh[i] = M[i];
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double xv[96];
  const int nc = min(ncol, 96);
  for (int c = 0; c < nc; ++c) xv[c] = basis_at<VT>(X, c, row);
  for (int o = 0; o < nout; ++o) {
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s = fma(xv[c], Msh[(int64_t)o * ncol + c], s);
    out[(int64_t)o * ldo + row] = s;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_cycle_update(Basis Xd, const double* __restrict__ cd,
                                                      VT* __restrict__ d, Basis Xr,
                                                      const double* __restrict__ cr,
                                                      VT* __restrict__ r, int n) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  if (d) d[row] = (VT)((double)d[row] + basis_row_fma<VT>(Xd, row, cd, 0.0));
  if (r) r[row] = (VT)((double)r[row] - basis_row_fma<VT>(Xr, row, cr, 0.0));
}

// G[o * nx + c] = sum_rows X[row, c] Y[row, o]
// G = X^T Y (nx x ny, column o of Y against column c of X at G[o * nx + c])
// in fp64 (nx <= 192, ny <= 96: m <= 95 and k < m).  Each workgroup takes
// 256 rows in chunks of 32, staged in LDS with coalesced loads; thread t
// accumulates outputs t, t + 256, ... over its rows; the last workgroup adds
// the per-workgroup sums in order.
constexpr int kGramRows = 32;
constexpr int kGramQ = 8;
constexpr int kGramMaxX = 192;
constexpr int kGramMaxY = 96;
template <typename VT>
__global__ __launch_bounds__(256) void k_gram(Basis X, const double* __restrict__ Y, int ny,
                                              int64_t ldy, int n, double* __restrict__ G,
                                              double* __restrict__ partial,
                                              unsigned int* counter) {
  __shared__ double xs[kGramRows][kGramMaxX + 1];
  __shared__ double ys[kGramRows][kGramMaxY + 1];
  __shared__ unsigned int s_ticket;
  const int tid = threadIdx.x;
  const int nx = X.kc + X.nv;
  const int rbase = blockIdx.x * kRowsPerBlock;
  const int nout = nx * ny;
  double* part = partial + (int64_t)blockIdx.x * nout;
  // outputs in groups of 256 kGramQ (one group for the usual sizes)
  for (int g0 = 0; g0 < nout; g0 += 256 * kGramQ) {
    double acc[kGramQ];
#pragma unroll
    for (int q = 0; q < kGramQ; ++q) acc[q] = 0.0;
    for (int r0 = rbase; r0 < rbase + kRowsPerBlock; r0 += kGramRows) {
      for (int idx = tid; idx < kGramRows * nx; idx += 256) {
        const int r = idx % kGramRows, c = idx / kGramRows;
        xs[r][c] = (r0 + r < n) ? basis_at<VT>(X, c, r0 + r) : 0.0;
      }
      for (int idx = tid; idx < kGramRows * ny; idx += 256) {
        const int r = idx % kGramRows, o = idx / kGramRows;
        ys[r][o] = (r0 + r < n) ? Y[(int64_t)o * ldy + r0 + r] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kGramQ; ++q) {
        const int idx = g0 + tid + 256 * q;
        if (idx < nout) {
          const int c = idx % nx, o = idx / nx;
          double sacc = acc[q];
#pragma unroll 8
          for (int r = 0; r < kGramRows; ++r) sacc = fma(xs[r][c], ys[r][o], sacc);
          acc[q] = sacc;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kGramQ; ++q) {
      const int idx = g0 + tid + 256 * q;
      if (idx < nout) part[idx] = acc[q];
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) s_ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (s_ticket != gridDim.x - 1) return;
  __threadfence();
  for (int c = tid; c < nout; c += 256) G[c] = ordered_sum(partial + c, (int)gridDim.x, nout);
  if (tid == 0) *counter = 0u;
}

template <typename VT>
__global__ void k_scale_round(const double* __restrict__ r, double s, double* __restrict__ out,
                              int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = round_u<VT>(r[i] / s);
}

template <typename VT>
__global__ void k_x_update(double* __restrict__ x, const VT* __restrict__ d, double s, int n) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double t = s * (double)d[i];
    x[i] = x[i] + t;
  }
}

template <typename VT>
__global__ void k_div_u(const VT* __restrict__ w, double s, VT* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (VT)((double)w[i] / s);
}

__global__ void k_maxabs(const double* __restrict__ v, int n, unsigned long long* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double a = (i < n) ? fabs(v[i]) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, kWave));
  if ((threadIdx.x % kWave) == 0) atomic_max_nonneg(out, a);
}

// word copy for small transfers between device memory and mapped pinned host
// memory (the kernel reads or writes the host side directly)
__global__ void k_copy_words(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// several such copies in one launch (grid row p copies piece p)
__global__ void k_copy_pieces(CopyPieces c) {
  const int p = blockIdx.y;
  if (p >= c.count) return;
  uint32_t* __restrict__ dst = static_cast<uint32_t*>(c.dst[p]);
  const uint32_t* __restrict__ src = static_cast<const uint32_t*>(c.src[p]);
  const int64_t n = c.words[p];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_copy_f32_f64(const float* __restrict__ a, double* __restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------
// Products with the transpose of a row-major matrix (the adjoint system
// A^T lambda = g): t_j = sum_i A[i][j] v_i.  Pass 1: workgroup (bx, by) sums
// rows [by R, (by + 1) R) for 256 consecutive columns (each row segment is
// one coalesced read), fp64 accumulation, partial sums by chunk; pass 2 adds
// the chunks in order (deterministic) and, for the residual, forms b - t and
// the infinity norms.
// ---------------------------------------------------------------------------
constexpr int kColRows = 128;  // rows per chunk

template <typename AT, typename VT>
__global__ __launch_bounds__(256) void k_colsum_partial(const AT* __restrict__ A, int64_t ld,
                                                        int n, const VT* __restrict__ v,
                                                        double* __restrict__ partial,
                                                        const CycleState* gate, int step) {
  if (gated_off(gate, step)) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i0 = blockIdx.y * kColRows;
  const int i1 = min(n, i0 + kColRows);
  if (j >= n) return;
  const AT* a = A + (int64_t)i0 * ld + j;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int i = i0;
  for (; i + 4 <= i1; i += 4, a += 4 * ld) {
    acc0 = fma((double)a[0], (double)v[i], acc0);
    acc1 = fma((double)a[ld], (double)v[i + 1], acc1);
    acc2 = fma((double)a[2 * ld], (double)v[i + 2], acc2);
    acc3 = fma((double)a[3 * ld], (double)v[i + 3], acc3);
  }
  for (; i < i1; ++i, a += ld) acc0 = fma((double)a[0], (double)v[i], acc0);
  partial[(int64_t)blockIdx.y * n + j] = (acc0 + acc1) + (acc2 + acc3);
}

// column sums of |A| (fp64, row-major) by chunks, as k_colsum_partial
__global__ __launch_bounds__(256) void k_colsum_abs_partial(const double* __restrict__ A,
                                                            int64_t ld, int n,
                                                            double* __restrict__ partial) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i0 = blockIdx.y * kColRows;
  const int i1 = min(n, i0 + kColRows);
  if (j >= n) return;
  double acc = 0.0;
  for (int i = i0; i < i1; ++i) acc += fabs(A[(int64_t)i * ld + j]);
  partial[(int64_t)blockIdx.y * n + j] = acc;
}

// t = sum of the chunks; with b: t = b - sum, norms[0] = max|t|, norms[1] =
// max|x| (x: the vector the product was taken with)
__global__ __launch_bounds__(256) void k_colsum_finish(const double* __restrict__ partial,
                                                       int nchunks, int n,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ t,
                                                       unsigned long long* norms,
                                                       const CycleState* gate, int step) {
  if (gated_off(gate, step)) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (j < n)
    for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * n + j];
  double ra = 0.0, xa = 0.0;
  if (j < n) {
    const double v = b ? b[j] - s : s;
    t[j] = v;
    ra = fabs(v);
    xa = x ? fabs(x[j]) : 0.0;
  }
  if (norms) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ra = fmax(ra, __shfl_xor(ra, o, kWave));
      xa = fmax(xa, __shfl_xor(xa, o, kWave));
    }
    if ((threadIdx.x % kWave) == 0) {
      atomic_max_nonneg(norms + 0, ra);
      atomic_max_nonneg(norms + 1, xa);
    }
  }
}

// ---------------------------------------------------------------------------
// Blocked solves with the transposed factors (the adjoint preconditioner
// M^-T = 2^e P^T L^-T U^-T):
//   U^T y = w  (lower triangular): y_I = (U_II^-1)^T (w_I - sum_{J<I} U_JI^T y_J)
//   L^T z = y  (unit upper):       z_I = (L_II^-1)^T (y_I - sum_{J>I} L_JI^T z_J)
// Same scheme as k_trsv (128-row blocks of the transposed system, 8 waves,
// wave-strided 64-column tiles, epoch-tagged partial solutions), but a tile
// row of the transposed factor is a column of the stored one: lane c of a
// wave reads S[row j][c] for the 64 logical rows j of the tile (each read
// coalesced across the wave).  The result of the L^T solve is scattered
// through P^T: out[permOut[i]] = scale * z_i.
// ---------------------------------------------------------------------------
template <class F, bool kUpperT>
__global__ __launch_bounds__(kTSThreads) void k_trsv_t(
    const typename F::T* __restrict__ S, int64_t ld, const int* __restrict__ permS, int n,
    const double* __restrict__ in, const double* __restrict__ Dinv,
    const double* __restrict__ Q, double* __restrict__ y,
    double scale, const int* __restrict__ permOut, double* __restrict__ out64,
    float* __restrict__ out32, uint64_t* xw, uint32_t epoch, const CycleState* gate, int step,
    int* abortp, ColStrides cs) {
  if (gated_off(gate, step)) return;
  int bx, cidx;  // the launch order of k_trsv
  if (!col_block(cs, (n + kTS - 1) / kTS, bx, cidx)) return;
  in += (int64_t)cidx * cs.in;
  if (y) y += (int64_t)cidx * cs.y;
  if (out64) out64 += (int64_t)cidx * cs.out;
  xw += (int64_t)cidx * cs.xw;
  __shared__ double red[8][kTB];
  __shared__ double ysh[8][kTB];
  __shared__ double zsh[kTS];
  __shared__ double part[4][kTS];
  __shared__ int wok[8];
  using T = typename F::T;
  const int nb = (n + kTS - 1) / kTS;
  const int nt = (n + kTB - 1) / kTB;
  const int blk = kUpperT ? nb - 1 - bx : bx;
  const int r0 = blk * kTS;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int half = wave >> 2;
  const int wq = wave & 3;
  const int col = r0 + half * kTB + lane;  // this thread's row of the transposed system
  // the neighbouring block (the last one waited for) enters through Q^T
  const bool hasAdj = kUpperT ? blk < nb - 1 : blk > 0;
  const int adj = kUpperT ? blk + 1 : blk - 1;
  // this thread's quarter of its row of (D^-1)^T and of Q^T, i.e. of column
  // di of D^-1 and of Q
  const int di = tid % kTS;
  const int dq4 = tid / kTS;
  double dq[kTS / 4], mq[kTS / 4];
  {
    const int64_t off = (int64_t)blk * kTS * kTS + (int64_t)(dq4 * (kTS / 4)) * kTS + di;
#pragma unroll
    for (int c = 0; c < kTS / 4; ++c) dq[c] = Dinv[off + (int64_t)c * kTS];
#pragma unroll
    for (int c = 0; c < kTS / 4; ++c) mq[c] = hasAdj ? Q[off + (int64_t)c * kTS] : 0.0;
  }
  double rhs = 0.0;
  if (tid < kTS && r0 + tid < n) rhs = in[r0 + tid];
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  bool ok = true;
  // off-diagonal tiles other than the neighbouring block's two
  const int t0 = kUpperT ? 2 * blk + 4 : 0;
  const int t1 = kUpperT ? nt : (blk > 0 ? 2 * blk - 2 : 0);
  for (int i = wq;; i += 4) {
    const int J = kUpperT ? t1 - 1 - i : t0 + i;
    if (kUpperT ? (J < t0) : (J >= t1)) break;
    // the 64 physical rows of tile J, then one column read per row: all
    // loads are issued unconditionally (a column beyond the padded row reads
    // the last one; its results are discarded) and converted only after the
    // wait for the published values, so they overlap one another and the wait
    const int jr = J * kTB + lane;
    const int pr = (jr < n) ? (permS ? permS[jr] : jr) : 0;
    const T* scol = S + min(col, (int)ld - 1);
    T tv[kTB];
#pragma unroll
    for (int jj = 0; jj < kTB; ++jj)
      tv[jj] = scol[(int64_t)__builtin_amdgcn_readlane(pr, jj) * ld];
    double yv;
    if (!get_tagged64(xw, J * kTB, epoch, yv, abortp)) {
      ok = false;
      break;
    }
    ysh[wave][lane] = yv;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < kTB; c += 4) {
      acc0 = fma((double)F::to_f(tv[c]), ysh[wave][c], acc0);
      acc1 = fma((double)F::to_f(tv[c + 1]), ysh[wave][c + 1], acc1);
      acc2 = fma((double)F::to_f(tv[c + 2]), ysh[wave][c + 2], acc2);
      acc3 = fma((double)F::to_f(tv[c + 3]), ysh[wave][c + 3], acc3);
    }
    __builtin_amdgcn_wave_barrier();
  }
  red[wave][lane] = (acc0 + acc1) + (acc2 + acc3);
  if (lane == 0) wok[wave] = ok ? 1 : 0;
  __syncthreads();
  int allok = 1;
#pragma unroll
  for (int w = 0; w < 8; ++w) allok &= wok[w];
  if (!allok) return;
  if (tid < kTS) {
    const int h = tid / kTB, l = tid % kTB;
    const double sum = (red[4 * h][l] + red[4 * h + 1][l]) + (red[4 * h + 2][l] + red[4 * h + 3][l]);
    zsh[tid] = (r0 + tid < n) ? rhs - sum : 0.0;
  }
  __syncthreads();
  double p = 0.0;
#pragma unroll
  for (int c = 0; c < kTS / 4; ++c) p = fma(dq[c], zsh[dq4 * (kTS / 4) + c], p);
  if (hasAdj) {
    // lanes c and c + 32 both read row dq4 * 32 + c of the neighbour
    double ya;
    const bool got = get_tagged_row(xw, adj * kTS + dq4 * (kTS / 4) + (lane & 31), epoch, ya,
                                    abortp);
    if (got) {
#pragma unroll
      for (int c = 0; c < kTS / 4; ++c) p = fma(-mq[c], lane_value(ya, c), p);
    }
    if (lane == 0) wok[wave] = got ? 1 : 0;
  }
  part[dq4][di] = p;
  __syncthreads();
  if (hasAdj) {
#pragma unroll
    for (int w = 0; w < 8; ++w) allok &= wok[w];
    if (!allok) return;
  }
  if (tid >= kTS) return;
  const int rr = r0 + tid;
  const double v = (rr < n) ? (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]) : 0.0;
  if (rr < n) {
    if (y) y[rr] = v;
    const int o = permOut ? permOut[rr] : rr;
    if (out64) out64[o] = v * scale;
    if (out32) out32[o] = (float)(v * scale);
  }
  put_tagged(xw, rr, v, epoch);
}

// out = alpha x y^T (n x n, row-major, leading dimension ld)
__global__ __launch_bounds__(256) void k_rank1(double alpha, const double* __restrict__ x,
                                               const double* __restrict__ yv, int n, int64_t ld,
                                               double* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (j < n) out[(int64_t)i * ld + j] = alpha * x[i] * yv[j];
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


// ---------------------------------------------------------------------------
// One GMRES cycle of a small system in one persistent launch
// ---------------------------------------------------------------------------
// 3 nb workgroups (nb = ceil(n / 128) <= 16) stay resident for the whole
// cycle, in three roles of nb each:
//   upper solve: workgroup u takes block nb - 1 - u (the chain's order);
//   lower solve: workgroup nb + l takes block l;
//   rows: workgroup 2 nb + b takes the 128 rows of block b for the
//         Gram-Schmidt passes and a share of the product's rows.
// The solve blocks stage their fp64 matrices once and keep them (in LDS and
// registers) for the cycle; a rows workgroup keeps its rows of the basis
// [C_k V] in LDS.  Per Arnoldi step j, with the tag epoch0 + j on every word
// the step publishes:
//   1. the rows workgroups take v_j (step 0: from V; later: from the words
//      they published) and form the rows of A_u[permA] v_j in row order,
//      published as tagged words;
//   2. the lower chain runs on those rows, the upper chain on the lower
//      chain's published values;
//   3. rows workgroup b takes its block's values of z, forms w = fl32(2^e z)
//      and runs the three classical Gram-Schmidt passes on its rows,
//      publishing its per-block sums and reading every block's, added in
//      the order of the multi-workgroup passes;
//   4. every rows workgroup runs the finish on its own copy of the rotations
//      (the same arithmetic, so the same values; workgroup 2 nb also writes H
//      and B and publishes the step's verdict, which the solve blocks wait
//      for), normalises its rows of v_{j+1} and publishes them.
// Every sum is formed as in the separate launches of a step, so the results
// are bit-identical to them.  Every wait is bounded and watches the abort
// flag; a workgroup that gives up leaves the flag set and the others follow.
constexpr int kCycleBlocks = kCycleMaxN / kTS;
// the exchanges' reduction: blocks polled per thread
constexpr int kCycleReduceBlocks = 8;
constexpr int kCycleRowPieces = 16;  // 16-byte pieces a lane of the product loads per round

// LDS of a rows workgroup: its block's rows of the basis, column after
// column (kc fp64 columns of C_k, then the fp32 columns of V; at most
// kCycleMaxM columns of 128 doubles in all, since kc + steps + 1 <= m + 1
// and an fp32 column takes half the room), v_j, w, the passes' sums, the
// rotations and the cycle state
struct CycleRowsShared {
  double basis[kCycleMaxM * kTS];
  float vsh[kCycleMaxN];
  double wsh[kTS];
  double hsum[2][kCycleMaxM];
  double c1[kCycleMaxM];
  double c2[kCycleMaxM];
  double scr[kCycleMaxM * (kCycleBlocks / 2)];  // the exchanges' chunk sums
  double nrm[2];
  double cs[kCycleMaxM], sn[kCycleMaxM], g[kCycleMaxM + 1];
  CycleState st;
};
union CycleShared {
  TrsvShared t;
  CycleRowsShared r;
};

// one lane's value of entry idx of a tagged double array (two words per
// entry); per lane, no wave vote; false on abort
__device__ __forceinline__ bool get_tagged_lane(const uint64_t* xw, int idx, uint32_t tag,
                                                double& v, int* abortp) {
  const uint64_t* p = xw + 2 * idx;
  long long spins = 0;
  for (;;) {
    const uint64_t lo = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t hi = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(lo >> 32) == tag && (uint32_t)(hi >> 32) == tag) {
      v = __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
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

// v_j in LDS from the fp32 words the previous step published (one word per
// row: tag << 32 | bits); false (for the whole workgroup) on abort
__device__ __forceinline__ bool cycle_fetch_v(const uint64_t* vw, int n, uint32_t tag, float* vsh,
                                              int* abortp) {
  constexpr int kPer = kCycleMaxN / kTSThreads;  // words per thread in flight
  bool ok = true;
  for (int i0 = 0; i0 < n && ok; i0 += kPer * kTSThreads) {
    // every word of the round in flight, then poll until all carry the tag
    uint64_t x[kPer];
    long long spins = 0;
    for (;;) {
      bool all = true;
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = i0 + e * kTSThreads + (int)threadIdx.x;
        x[e] = __hip_atomic_load(vw + (i < n ? i : 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = i0 + e * kTSThreads + (int)threadIdx.x;
        all = all && (i >= n || (uint32_t)(x[e] >> 32) == tag);
      }
      if (all) break;
      __builtin_amdgcn_s_sleep(1);
      if (((++spins) & 1023) == 0) {
        if (__hip_atomic_load(abortp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = false;
          break;
        }
        if (spins > (1ll << 22)) {
          __hip_atomic_store(abortp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
          break;
        }
      }
    }
    if (ok) {
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = i0 + e * kTSThreads + (int)threadIdx.x;
        if (i < n) vsh[i] = __uint_as_float((uint32_t)x[e]);
      }
    }
  }
  return !__syncthreads_or(!ok);
}

// The product's rows, formed by the rows workgroups in row order, so that
// the lower chain's blocks find their rows ahead of need.  A row's 256-column
// pieces number P = ceil(n4 / 256) <= 32 (n4 = n rounded down to a multiple
// of 4); a wave takes R = kCycleRowPieces / P rows at a time (one row, in
// batches of kCycleRowPieces pieces, when P is larger) and issues every load
// of a batch before any product, and its rows' indices in A_u sit in one
// register (lane e: the e-th row it takes), so no permutation load waits in
// the step.  Rows workgroup u's wave w takes, in its k-th round, rows
// ((k nb + u) 8 + w) R .. + R - 1.
__device__ __forceinline__ int cycle_product_pieces(int n) {
  const int p = ((n & ~3) + 255) / 256;
  return p < 1 ? 1 : p;
}

__device__ __forceinline__ int cycle_product_rows_per_wave(int n) {
  const int p = cycle_product_pieces(n);
  return p < kCycleRowPieces ? kCycleRowPieces / p : 1;
}

// lane e of the result: the row of A_u for the e-th row this wave takes
// (-1 past n; at most 64 rows, since k R < 16 for every round k that starts
// below n)
__device__ __forceinline__ int cycle_product_rowlist(const CycleArgs& a, int nb, int u) {
  const int R = cycle_product_rows_per_wave(a.n);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int k = lane / R, r = lane % R;
  const int row = ((k * nb + u) * 8 + wave) * R + r;
  if (row >= a.n) return -1;
  return a.permA ? a.permA[row] : row;
}

// one step's rows of A_u[permA] v (v in LDS), each row's sum formed as
// gemv_au_row forms it: the pieces in increasing order, their elements
// alternately into two accumulators, the tail element into the first, then
// the wave sum of the two
template <int P>
__device__ __forceinline__ void cycle_product_rows(const CycleArgs& a, const float* v, int rowlist,
                                                   int nb, int u, uint32_t tag) {
  constexpr int R = kCycleRowPieces / P;
  const int n = a.n, n4 = n & ~3;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int cc = n4 + lane;  // this lane's tail column (n - n4 < 4)
  for (int k = 0;; ++k) {
    const int base = ((k * nb + u) * 8 + wave) * R;
    if (base >= n) break;
    // every load is issued unconditionally (an index outside the row reads
    // its first piece, a row past n reads row 0 of A_u; neither is used), so
    // that no branch splits the loads and they all wait together
    const float* rp[R];
    bool ok[R];
    float4 x[R][P];
    float tl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pr = __builtin_amdgcn_readlane(rowlist, k * R + r);
      ok[r] = pr >= 0;
      rp[r] = a.Au + (int64_t)(pr >= 0 ? pr : 0) * a.lda;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int c = lane * 4 + 256 * i;
        x[r][i] = *reinterpret_cast<const float4*>(rp[r] + (c < n4 ? c : 0));
      }
      tl[r] = rp[r][cc < n ? cc : 0];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!ok[r]) continue;
      double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int c = lane * 4 + 256 * i;
        if (c < n4) {
          acc0 = fma((double)x[r][i].x, (double)v[c + 0], acc0);
          acc1 = fma((double)x[r][i].y, (double)v[c + 1], acc1);
          acc0 = fma((double)x[r][i].z, (double)v[c + 2], acc0);
          acc1 = fma((double)x[r][i].w, (double)v[c + 3], acc1);
        }
      }
      if (cc < n) acc0 = fma((double)tl[r], (double)v[cc], acc0);
      const double t = wave_sum(acc0 + acc1);
      if (lane == 0) put_tagged(a.xt, base + r, t, tag);
    }
  }
}

// rows of more than kCycleRowPieces pieces: one row per wave at a time, its
// pieces in batches of kCycleRowPieces (the same order of sums)
__device__ __forceinline__ void cycle_product_long_rows(const CycleArgs& a, const float* v,
                                                        int rowlist, int nb, int u, uint32_t tag) {
  constexpr int B = kCycleRowPieces;
  const int n = a.n, n4 = n & ~3, P = cycle_product_pieces(n);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int cc = n4 + lane;
  for (int k = 0;; ++k) {
    const int row = (k * nb + u) * 8 + wave;
    if (row >= n) break;
    const int pr = __builtin_amdgcn_readlane(rowlist, k);
    const float* rp = a.Au + (int64_t)(pr >= 0 ? pr : 0) * a.lda;
    double acc0 = 0.0, acc1 = 0.0;
    for (int i0 = 0; i0 < P; i0 += B) {
      float4 x[B];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const int c = lane * 4 + 256 * (i0 + i);
        x[i] = *reinterpret_cast<const float4*>(rp + (c < n4 ? c : 0));
      }
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const int c = lane * 4 + 256 * (i0 + i);
        if (c < n4) {
          acc0 = fma((double)x[i].x, (double)v[c + 0], acc0);
          acc1 = fma((double)x[i].y, (double)v[c + 1], acc1);
          acc0 = fma((double)x[i].z, (double)v[c + 2], acc0);
          acc1 = fma((double)x[i].w, (double)v[c + 3], acc1);
        }
      }
    }
    if (cc < n) acc0 = fma((double)rp[cc], (double)v[cc], acc0);
    const double t = wave_sum(acc0 + acc1);
    if (lane == 0) put_tagged(a.xt, row, t, tag);
  }
}

__device__ __forceinline__ void cycle_product(const CycleArgs& a, const float* v, int rowlist,
                                              int nb, int u, uint32_t tag) {
  if (cycle_product_pieces(a.n) > 8) {
    cycle_product_long_rows(a, v, rowlist, nb, u, tag);
    return;
  }
  switch (cycle_product_pieces(a.n)) {
    case 1: cycle_product_rows<1>(a, v, rowlist, nb, u, tag); break;
    case 2: cycle_product_rows<2>(a, v, rowlist, nb, u, tag); break;
    case 3: cycle_product_rows<3>(a, v, rowlist, nb, u, tag); break;
    case 4: cycle_product_rows<4>(a, v, rowlist, nb, u, tag); break;
    case 5: cycle_product_rows<5>(a, v, rowlist, nb, u, tag); break;
    case 6: cycle_product_rows<6>(a, v, rowlist, nb, u, tag); break;
    case 7: cycle_product_rows<7>(a, v, rowlist, nb, u, tag); break;
    default: cycle_product_rows<8>(a, v, rowlist, nb, u, tag); break;
  }
}

// The per-block sums of one exchange (cnt values per block; block b's pair
// sum of column c at entry b cnt + c of x): per 256-row chunk the two
// blocks' sums added, then the chunks in order from zero, into out[c].
// ceil(nb / kCycleReduceBlocks) threads per column (in rounds of the
// workgroup's threads), each polling its kCycleReduceBlocks blocks' words
// at once (every load unconditional: a block past nb reads block 0's,
// unused) and leaving its chunk sums in scr; then one thread per column adds
// the chunks in order.  False (for the whole workgroup) on abort.
__device__ __forceinline__ bool cycle_reduce(const uint64_t* x, int nb, int cnt, uint32_t tag,
                                             double* out, double* scr, int* abortp) {
  constexpr int B = kCycleReduceBlocks, Q = B / 2;
  const int T = (nb + B - 1) / B;
  bool ok = true;
  for (int p0 = 0; p0 < cnt * T; p0 += kTSThreads) {
    const int pidx = p0 + (int)threadIdx.x;
    if (pidx < cnt * T && ok) {
      const int c = pidx / T, g = pidx % T, b0 = B * g;
      double v[B];
      long long spins = 0;
      for (;;) {
        bool all = true;
        uint64_t lo[B], hi[B];
#pragma unroll
        for (int e = 0; e < B; ++e) {
          const uint64_t* p = x + 2 * ((b0 + e < nb ? b0 + e : 0) * cnt + c);
          lo[e] = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          hi[e] = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int e = 0; e < B; ++e) {
          const bool in = b0 + e < nb;
          all = all &&
                (!in || ((uint32_t)(lo[e] >> 32) == tag && (uint32_t)(hi[e] >> 32) == tag));
          v[e] = in ? __longlong_as_double((long long)((hi[e] << 32) | (lo[e] & 0xFFFFFFFFull)))
                    : 0.0;
        }
        if (all) break;
        __builtin_amdgcn_s_sleep(1);
        if (((++spins) & 1023) == 0) {
          if (__hip_atomic_load(abortp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = false;
            break;
          }
          if (spins > (1ll << 22)) {
            __hip_atomic_store(abortp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) scr[c * (kCycleBlocks / 2) + g * Q + q] = v[2 * q] + v[2 * q + 1];
    }
  }
  if (__syncthreads_or(!ok)) return false;
  if ((int)threadIdx.x < cnt) {
    const int c = threadIdx.x;
    double sum = 0.0;
    for (int k = 0; 2 * k < nb; ++k) sum += scr[c * (kCycleBlocks / 2) + k];
    out[c] = sum;
  }
  __syncthreads();
  return true;
}

// the solve blocks: after each solve, the step's verdict (0: go on; 1: the
// cycle ended); false when the cycle ended or on abort
__device__ __forceinline__ bool cycle_verdict(const CycleArgs& a, uint32_t tag) {
  bool ok = true;
  double verdict = 0.0;
  if (threadIdx.x == 0) ok = get_tagged_lane(a.ctrl, 0, tag, verdict, a.abortp);
  return !__syncthreads_or(!ok || verdict != 0.0);
}

template <class F, bool kUpper>
__device__ __forceinline__ void cycle_solve(const CycleArgs& a, TrsvShared& sm, int blk) {
  const int n = a.n;
  TrsvBlock<F, kUpper> tb;
  tb.init(sm, static_cast<const typename F::T*>(a.S), a.ld, a.permS, n, blk,
          kUpper ? a.Uinv : a.Linv);
  uint64_t* xw = kUpper ? a.xwU : a.xwL;
  // right-hand sides: the product's rows (lower), the lower chain's values
  // (upper), both published as tagged words
  const uint64_t* rhs = kUpper ? a.xwL : a.xt;
  for (int j = 0; j < a.nsteps; ++j) {
    const uint32_t tag = a.epoch0 + (uint32_t)j;
    double p = 0.0;
    if (!tb.solve(sm, xw, tag, a.abortp, nullptr, nullptr, rhs, p)) return;
    const int rr = tb.r0 + tb.di;
    if (tb.dq4 == 0) put_tagged(xw, rr, rr < n ? p : 0.0, tag);
    if (!cycle_verdict(a, tag)) return;
  }
}

// the block's rows of the basis in LDS: column c < kc is C_k's (fp64), the
// others V's (fp32); the products and sums are those of basis_products and
// basis_row_fma (the same values, the same order)
struct CycleBasis {
  const double* c;
  const float* v;
  int kc;
  __device__ __forceinline__ double at(int col, int lr) const {
    return col < kc ? c[col * kTS + lr] : (double)v[(col - kc) * kTS + lr];
  }
};

__device__ __forceinline__ double cycle_row_fma(const CycleBasis& X, int nv, int lr,
                                                const double* __restrict__ coef) {
  double s = 0.0;
  for (int c = 0; c < X.kc; ++c) s = fma(X.c[c * kTS + lr], coef[c], s);
  for (int c = 0; c < nv; ++c) s = fma((double)X.v[c * kTS + lr], coef[X.kc + c], s);
  return s;
}

__device__ __forceinline__ void cycle_rows(const CycleArgs& a, CycleRowsShared& sm, int nb) {
  const int n = a.n;
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int u = (int)blockIdx.x - 2 * nb;  // this workgroup's block of rows
  const bool lead = u == 0;
  const int kc = a.kc;
  const int r0 = u * kTS;
  // the block's rows of C_k and of v_1, the rotations, the cycle state
  for (int i = tid; i < kc * kTS; i += kTSThreads) {
    const int c = i / kTS, lr = i % kTS;
    sm.basis[i] = (r0 + lr < n) ? a.C[(int64_t)c * a.ldc + r0 + lr] : 0.0;
  }
  float* vb = reinterpret_cast<float*>(sm.basis + (int64_t)kc * kTS);
  for (int lr = tid; lr < kTS; lr += kTSThreads) vb[lr] = (r0 + lr < n) ? a.V[r0 + lr] : 0.0f;
  for (int i = tid; i <= a.m; i += kTSThreads) {
    if (i < a.m) {
      sm.cs[i] = a.cs[i];
      sm.sn[i] = a.sn[i];
    }
    sm.g[i] = a.g[i];
  }
  if (tid == 0) sm.st = *a.st;
  const CycleBasis X{sm.basis, vb, kc};
  const int rowlist = cycle_product_rowlist(a, nb, u);
  const int lrow = wave * kWave + lane;  // waves 0 and 1: lane = row
  const int grow = r0 + lrow;
  const bool vrow = wave < 2 && grow < n;
  // the dot products: wave w takes the rows of half w % 2 and the columns
  // c = 4 i + w / 2 (the sums of every column are the same whoever forms them)
  const int dh = wave & 1, dq = wave >> 1;
  const int dlr = dh * kWave + lane;
  const bool dvalid = r0 + dlr < n;
  __syncthreads();
  for (int j = 0; j < a.nsteps; ++j) {
    const uint32_t tag = a.epoch0 + (uint32_t)j;
    // 1. v_j, then this workgroup's rows of the product
    if (j == 0) {
      for (int i = tid; i < n; i += kTSThreads) sm.vsh[i] = a.V[i];
      __syncthreads();
    } else if (!cycle_fetch_v(a.vw, n, tag, sm.vsh, a.abortp)) {
      return;
    }
    cycle_product(a, sm.vsh, rowlist, nb, u, tag);
    // 2. this block's z from the upper chain; w = fl32(2^e z)
    double wv = 0.0;
    {
      bool ok = true;
      if (wave < 2) {
        double z = 0.0;
        ok = get_tagged_row(a.xwU, grow, tag, z, a.abortp);
        wv = (grow < n) ? (double)(float)(z * a.scale) : 0.0;
        sm.wsh[lrow] = wv;
      }
      if (__syncthreads_or(!ok)) return;
    }
    // 3. the passes: dots; update and dots; update and norm
    const int ncol = kc + j + 1;
    for (int pass = 0; pass < 3; ++pass) {
      uint64_t* px = a.px + (int64_t)pass * kCycleBlocks * kCycleMaxM * 2;
      if (pass > 0 && vrow) wv = round_u<float>(wv - cycle_row_fma(X, j + 1, lrow, pass == 1 ? sm.c1 : sm.c2));
      if (pass < 2) {
        if (pass > 0) {
          if (wave < 2) sm.wsh[lrow] = wv;
          __syncthreads();
        }
        const double wd = sm.wsh[dlr];
        for (int c = dq; c < ncol; c += 4) {
          const double pr = wave_sum_to63(dvalid ? sum_term(X.at(c, dlr), wd) : 0.0);
          if (lane == kWave - 1) sm.hsum[dh][c] = pr;
        }
        __syncthreads();
        for (int c = tid; c < ncol; c += kTSThreads)
          put_tagged(px, u * ncol + c, sm.hsum[0][c] + sm.hsum[1][c], tag);
        if (!cycle_reduce(px, nb, ncol, tag, pass == 0 ? sm.c1 : sm.c2, sm.scr, a.abortp)) return;
      } else {
        const double sq = wave_sum(sum_term(wv, wv));
        if (wave < 2 && lane == 0) sm.nrm[wave] = sq;
        __syncthreads();
        if (tid == 0) put_tagged(px, u, sm.nrm[0] + sm.nrm[1], tag);
        if (!cycle_reduce(px, nb, 1, tag, sm.nrm, sm.scr, a.abortp)) return;
      }
    }
    // 4. the finish on this workgroup's copy (the lead also writes H and B)
    const double norm2 = sm.nrm[0];
    if (wave == 0) {
      OrthoArgs fa{};
      fa.X.kc = kc;
      fa.step = j;
      fa.H = lead ? a.H : nullptr;
      fa.B = lead ? a.B : nullptr;
      fa.ldh = a.ldh;
      fa.ldb = a.ldb;
      fa.cs = sm.cs;
      fa.sn = sm.sn;
      fa.g = sm.g;
      fa.st = &sm.st;
      arnoldi_finish(fa, sm.c1, sm.c2, norm2);
    }
    __syncthreads();
    // v_{j+1} = fl32(w / beta) on this block's rows (LDS, V and the words
    // of the next step); then the verdict
    const double beta = sqrt(norm2);
    const int done = sm.st.done;
    if (wave < 2) {
      const float vv = (vrow && beta > 0.0) ? (float)(wv / beta) : 0.0f;
      vb[(j + 1) * kTS + lrow] = vv;
      if (vrow) {
        a.V[(int64_t)(j + 1) * a.ldv + grow] = vv;
        if (!done && j + 1 < a.nsteps)
          __hip_atomic_store(a.vw + grow, ((uint64_t)(tag + 1) << 32) | __float_as_uint(vv),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (lead && tid == 0) put_tagged(a.ctrl, 0, done ? 1.0 : 0.0, tag);
    if (done) break;
  }
  // the cycle's state for the host (the lead's copy; every copy is the same)
  if (lead) {
    __syncthreads();
    for (int i = tid; i <= a.m; i += kTSThreads) {
      if (i < a.m) {
        a.cs[i] = sm.cs[i];
        a.sn[i] = sm.sn[i];
      }
      a.g[i] = sm.g[i];
    }
    if (tid == 0) {
      a.st->done = sm.st.done;
      a.st->jdone = sm.st.jdone;
      a.st->est = sm.st.est;
    }
  }
}

// The launch goes on only if all its total workgroups are resident at once
// (they wait for one another at every step).  state[0] counts arrivals (one
// fetch-and-add per workgroup); state[1] holds the decision, taken once by
// compare-and-swap from zero: kCycleGo by the arrival that completes the
// count, kCycleGaveUp by a workgroup that has waited bound_us without seeing
// a decision (a bound of zero gives up at once).  Every workgroup then reads
// the decision, so all take the same one.  Returns it (workgroup-uniform).
__device__ __forceinline__ bool cycle_arrive(unsigned* state, unsigned total, int bound_us,
                                             int& verdict) {
  if (threadIdx.x == 0) {
    unsigned* count = state;
    unsigned* decision = state + 1;
    unsigned expect = 0;
    if (bound_us <= 0) {
      __hip_atomic_compare_exchange_strong(decision, &expect, kCycleGaveUp, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned before =
          __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (before + 1 == total)
        __hip_atomic_compare_exchange_strong(decision, &expect, kCycleGo, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();  // 100 MHz
    unsigned d;
    for (;;) {
      d = __hip_atomic_load(decision, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (d != 0) break;
      if (__builtin_amdgcn_s_memrealtime() - t0 > (uint64_t)bound_us * 100) {
        expect = 0;
        __hip_atomic_compare_exchange_strong(decision, &expect, kCycleGaveUp, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        continue;  // read the decision taken
      }
      __builtin_amdgcn_s_sleep(2);
    }
    verdict = (d == kCycleGo) ? 1 : 0;
  }
  __syncthreads();
  return verdict != 0;
}

template <class F>
__global__ __launch_bounds__(kTSThreads) void k_cycle(CycleArgs a) {
  __shared__ CycleShared sm;
  __shared__ int s_verdict;
  const int nb = (a.n + kTS - 1) / kTS;
  if (!cycle_arrive(a.arrive, 3u * (unsigned)nb, a.arrive_us, s_verdict)) return;
  const int role = (int)blockIdx.x / nb, i = (int)blockIdx.x % nb;
  if (role == 0)
    cycle_solve<F, true>(a, sm.t, nb - 1 - i);
  else if (role == 1)
    cycle_solve<F, false>(a, sm.t, i);
  else
    cycle_rows(a, sm.r, nb);
}

}  // namespace

void launch_copy_words(void* dst, const void* src, int64_t words, hipStream_t s) {
  if (words <= 0) return;
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 64)),
                     dim3(256), 0, s, reinterpret_cast<uint32_t*>(dst),
                     reinterpret_cast<const uint32_t*>(src), words);
}

void launch_copy_pieces(const CopyPieces& c, hipStream_t s) {
  if (c.count <= 0) return;
  int64_t most = 0;
  for (int p = 0; p < c.count; ++p) most = std::max(most, c.words[p]);
  if (most <= 0) return;
  hipLaunchKernelGGL(k_copy_pieces,
                     dim3((unsigned)std::min<int64_t>((most + 255) / 256, 64), (unsigned)c.count),
                     dim3(256), 0, s, c);
}

void launch_gemv_au(const float* Au, int64_t ld, const int* permA, int n, const float* v32,
                    const double* v64, double* t, const CycleState* gate, int step,
                    hipStream_t s) {
  const unsigned grid = nblocks(n, 4);
  if (v32)
    hipLaunchKernelGGL(k_gemv_au<float>, dim3(grid), dim3(256), 0, s, Au, ld, permA, n, v32, t,
                       gate, step);
  else
    hipLaunchKernelGGL(k_gemv_au<double>, dim3(grid), dim3(256), 0, s, Au, ld, permA, n, v64, t,
                       gate, step);
}

void launch_gemv_au_multi(const float* Au, int64_t ld, const int* permA, int n, const double* Y,
                          int64_t ldy, int nr, double* T, int64_t ldt, hipStream_t s) {
  // four rows per wave (each staged entry of Y serves four rows: the LDS
  // reads keep pace with the fp64 multiply-adds); 512-column chunks where
  // the registers allow (up to eight columns).  Measured at n = 8192: eight
  // columns 72 us (87 with 256-column chunks), ten columns in the twelve-
  // column form 101 us (150 with two rows per wave and sixteen columns)
  constexpr int kWaves = kMultiThreads / kWave;
  const dim3 grid(nblocks(n, kWaves * 4)), block(kMultiThreads);
  if (nr <= 4)
    hipLaunchKernelGGL((k_gemv_au_multi<4, 4, 256>), grid, block, 0, s, Au, ld, permA, n, Y, ldy,
                       nr, T, ldt);
  else if (nr <= 8)
    hipLaunchKernelGGL((k_gemv_au_multi<8, 4, 512>), grid, block, 0, s, Au, ld, permA, n, Y, ldy,
                       nr, T, ldt);
  else if (nr <= 12)
    hipLaunchKernelGGL((k_gemv_au_multi<12, 4, 256>), grid, block, 0, s, Au, ld, permA, n, Y,
                       ldy, nr, T, ldt);
  else
    hipLaunchKernelGGL((k_gemv_au_multi<16, 4, 256>), grid, block, 0, s, Au, ld, permA, n, Y,
                       ldy, nr, T, ldt);
}

void launch_gemv_a64(const double* A, int64_t ld, const int* permA, int n, const double* v,
                     double* t, const CycleState* gate, int step, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_a64, dim3(nblocks(n, 4)), dim3(256), 0, s, A, ld, permA, n, v, t,
                     gate, step);
}

void launch_residual(const double* A, int64_t ld, int n, const double* b, const double* x,
                     double* r, unsigned long long* norms, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_resid_norms, dim3(1), dim3(64), 0, s, norms);
  hipLaunchKernelGGL(k_residual<kResidRows>, dim3(nblocks(n, 4 * kResidRows)), dim3(256), 0, s, A,
                     ld, n, b, x, r, norms);
}

template <class F>
void trsv_pair(const void* S, int64_t ld, const int* permS, int n, bool upper, const double* in,
               const int* permIn, const double* Dinv, double* y, double scale, double* out64,
               float* out32, uint64_t* xw, int epoch, const CycleState* gate, int step,
               int* abortp, hipStream_t s, int ncols = 1, ColStrides cs = ColStrides{0, 0, 0, 0}) {
  using T = typename F::T;
  const dim3 grid(col_grid(n, ncols));
  cs.ncols = ncols;
  const T* Sp = reinterpret_cast<const T*>(S);
  if (upper)
    hipLaunchKernelGGL((k_trsv<F, true>), grid, dim3(kTSThreads), 0, s, Sp, ld, permS, n, in,
                       permIn, Dinv, y, scale, out64, out32, xw, (uint32_t)epoch, gate, step,
                       abortp, cs);
  else
    hipLaunchKernelGGL((k_trsv<F, false>), grid, dim3(kTSThreads), 0, s, Sp, ld, permS, n, in,
                       permIn, Dinv, y, 1.0, nullptr, nullptr, xw, (uint32_t)epoch, gate, step,
                       abortp, cs);
}

template <class F>
void atilde_lower_t(const void* S, int64_t ld, const int* permS, int n, const float* Au,
                    int64_t lda, const int* permA, const float* v, const double* Linv, double* y,
                    uint64_t* xw, uint64_t* xt, int epoch, const CycleState* gate, int step,
                    int* abortp, hipStream_t s) {
  using T = typename F::T;
  const unsigned nb = nblocks(n, kTS);
  const unsigned ng = nblocks(n, kTSThreads / kWave);
  const T* Sp = reinterpret_cast<const T*>(S);
  hipLaunchKernelGGL((k_trsv<F, false, true>), dim3(nb + ng), dim3(kTSThreads), 0, s, Sp, ld,
                     permS, n, nullptr, nullptr, Linv, y, 1.0, nullptr, nullptr, xw,
                     (uint32_t)epoch, gate, step, abortp, ColStrides{0, 0, 0, 0},
                     FusedGemv{Au, lda, permA, v, xt});
}

void launch_atilde_lower(const void* S, int64_t ld, const int* permS, int store, int n,
                         const float* Au, int64_t lda, const int* permA, const float* v,
                         const double* Linv, double* y, uint64_t* xw, uint64_t* xt, int epoch,
                         const CycleState* gate, int step, int* abort, hipStream_t s) {
  if (store == kStoreF16)
    atilde_lower_t<Fp16>(S, ld, permS, n, Au, lda, permA, v, Linv, y, xw, xt, epoch, gate, step,
                         abort, s);
  else if (store == kStoreBF16)
    atilde_lower_t<Bf16>(S, ld, permS, n, Au, lda, permA, v, Linv, y, xw, xt, epoch, gate, step,
                         abort, s);
  else
    atilde_lower_t<Fp32>(S, ld, permS, n, Au, lda, permA, v, Linv, y, xw, xt, epoch, gate, step,
                         abort, s);
}

template <class F>
void trsv_cols_t(const void* S, int64_t ld, const int* permS, int n, bool upper,
                 const double* in, int64_t ldi, int nr, const double* Dinv, double* out,
                 int64_t ldo, double scale, uint64_t* xw, int64_t xstride, int epoch,
                 int* abortp, hipStream_t s) {
  if (upper)
    trsv_pair<F>(S, ld, permS, n, true, in, nullptr, Dinv, nullptr, scale, out, nullptr, xw,
                 epoch, nullptr, 0, abortp, s, nr, ColStrides{ldi, 0, ldo, xstride});
  else  // the lower solve writes its (unscaled) result through y
    trsv_pair<F>(S, ld, permS, n, false, in, nullptr, Dinv, out, 1.0, nullptr, nullptr, xw,
                 epoch, nullptr, 0, abortp, s, nr, ColStrides{ldi, ldo, 0, xstride});
}

void launch_trsv_cols(const void* S, int64_t ld, const int* permS, int store, int n, bool upper,
                      const double* in, int64_t ldi, int nr, const double* Dinv, double* out,
                      int64_t ldo, double scale, uint64_t* xw, int64_t xstride, int epoch,
                      int* abortp, hipStream_t s) {
  if (nr <= 0) return;
  if (store == kStoreF16)
    trsv_cols_t<Fp16>(S, ld, permS, n, upper, in, ldi, nr, Dinv, out, ldo, scale, xw, xstride,
                      epoch, abortp, s);
  else if (store == kStoreBF16)
    trsv_cols_t<Bf16>(S, ld, permS, n, upper, in, ldi, nr, Dinv, out, ldo, scale, xw, xstride,
                      epoch, abortp, s);
  else
    trsv_cols_t<Fp32>(S, ld, permS, n, upper, in, ldi, nr, Dinv, out, ldo, scale, xw, xstride,
                      epoch, abortp, s);
}

void launch_trsv_lower(const void* S, int64_t ld, const int* permS, int store, int n,
                       const double* in, const int* permIn, const double* Linv, double* y,
                       uint64_t* xw, int epoch, const CycleState* gate, int step, int* abortp,
                       hipStream_t s) {
  if (store == kStoreF16)
    trsv_pair<Fp16>(S, ld, permS, n, false, in, permIn, Linv, y, 1.0, nullptr, nullptr, xw,
                    epoch, gate, step, abortp, s);
  else if (store == kStoreBF16)
    trsv_pair<Bf16>(S, ld, permS, n, false, in, permIn, Linv, y, 1.0, nullptr, nullptr, xw,
                    epoch, gate, step, abortp, s);
  else
    trsv_pair<Fp32>(S, ld, permS, n, false, in, permIn, Linv, y, 1.0, nullptr, nullptr, xw,
                    epoch, gate, step, abortp, s);
}

template <class F>
using T_of = typename F::T;

template <class F>
void trsv_upper_dots_t(const void* S, int64_t ld, const int* permS, int n, const double* yin,
                       const double* Uinv, double* z, double scale, double* out64, float* out32,
                       uint64_t* xw, int epoch, const CycleState* gate, int step, int* abortp,
                       const TrsvDots& td, hipStream_t s) {
  const T_of<F>* Sp = reinterpret_cast<const T_of<F>*>(S);
  hipLaunchKernelGGL((k_trsv<F, true, false, true>), dim3(nblocks(n, kTS)), dim3(kTSThreads), 0,
                     s, Sp, ld, permS, n, yin, nullptr, Uinv, z, scale, out64, out32, xw,
                     (uint32_t)epoch, gate, step, abortp, ColStrides{0, 0, 0, 0}, FusedGemv{},
                     td);
}

void launch_trsv_upper(const void* S, int64_t ld, const int* permS, int store, int n,
                       const double* yin, const double* Uinv, double* z, double scale,
                       double* out64, float* out32, uint64_t* xw, int epoch,
                       const CycleState* gate, int step, int* abortp, hipStream_t s,
                       const TrsvDots* dots) {
  if (dots) {
    if (store == kStoreF16)
      trsv_upper_dots_t<Fp16>(S, ld, permS, n, yin, Uinv, z, scale, out64, out32, xw, epoch,
                              gate, step, abortp, *dots, s);
    else if (store == kStoreBF16)
      trsv_upper_dots_t<Bf16>(S, ld, permS, n, yin, Uinv, z, scale, out64, out32, xw, epoch,
                              gate, step, abortp, *dots, s);
    else
      trsv_upper_dots_t<Fp32>(S, ld, permS, n, yin, Uinv, z, scale, out64, out32, xw, epoch,
                              gate, step, abortp, *dots, s);
    return;
  }
  if (store == kStoreF16)
    trsv_pair<Fp16>(S, ld, permS, n, true, yin, nullptr, Uinv, z, scale, out64, out32, xw,
                    epoch, gate, step, abortp, s);
  else if (store == kStoreBF16)
    trsv_pair<Bf16>(S, ld, permS, n, true, yin, nullptr, Uinv, z, scale, out64, out32, xw,
                    epoch, gate, step, abortp, s);
  else
    trsv_pair<Fp32>(S, ld, permS, n, true, yin, nullptr, Uinv, z, scale, out64, out32, xw,
                    epoch, gate, step, abortp, s);
}

void launch_diag_inverses(const void* S, int64_t ld, const int* permS, int store, int n,
                          double* Linv, double* Uinv, double* tmp, hipStream_t s) {
  const unsigned g64 = nblocks(n, kTB);
  const unsigned g128 = nblocks(n, kTS);
#define GIR_DINV(F)                                                                          \
  do {                                                                                       \
    const typename F::T* Sp = reinterpret_cast<const typename F::T*>(S);                     \
    double* tmpU = tmp + (int64_t)g64 * kTB * kTB;                                           \
    hipLaunchKernelGGL((k_diag_inverse<F>), dim3(g64, 2), dim3(kTB), 0, s, Sp, ld, permS, n,  \
                       tmp, tmpU);                                                           \
    hipLaunchKernelGGL((k_diag_combine<F>), dim3(g128, 2), dim3(256), 0, s, Sp, ld, permS, n, \
                       tmp, tmpU, Linv, Uinv);                                               \
    for (int d = 1; d <= 2 && (unsigned)d < g128; ++d)                                      \
      hipLaunchKernelGGL((k_adjacent_product<F>), dim3(g128 - d, 4, 2), dim3(256), 0, s, Sp,  \
                         ld, permS, n, Linv, Linv + (int64_t)d * g128 * kTS * kTS, Uinv,      \
                         Uinv + (int64_t)d * g128 * kTS * kTS, d);                            \
  } while (0)
  if (store == kStoreF16) {
    GIR_DINV(Fp16);
  } else if (store == kStoreBF16) {
    GIR_DINV(Bf16);
  } else {
    GIR_DINV(Fp32);
  }
#undef GIR_DINV
}

void launch_adjacent_products_t(const void* S, int64_t ld, const int* permS, int store, int n,
                                const double* Linv, const double* Uinv, double* Lq, double* Uq,
                                hipStream_t s) {
  const unsigned g128 = nblocks(n, kTS);
  if (g128 < 2) return;
#define GIR_QT(F)                                                                              \
  do {                                                                                         \
    const typename F::T* Sp = reinterpret_cast<const typename F::T*>(S);                       \
    hipLaunchKernelGGL((k_adjacent_product_t<F, true>), dim3(g128 - 1, 4), dim3(256), 0, s, Sp, \
                       ld, permS, n, Uinv, Uq);                                                \
    hipLaunchKernelGGL((k_adjacent_product_t<F, false>), dim3(g128 - 1, 4), dim3(256), 0, s,    \
                       Sp, ld, permS, n, Linv, Lq);                                            \
  } while (0)
  if (store == kStoreF16) {
    GIR_QT(Fp16);
  } else if (store == kStoreBF16) {
    GIR_QT(Bf16);
  } else {
    GIR_QT(Fp32);
  }
#undef GIR_QT
}

void launch_ortho(const OrthoArgs& a, int mode, hipStream_t s) {
  if (a.X.v64)
    hipLaunchKernelGGL(k_ortho<double>, dim3(nblocks(a.n, kRowsPerBlock)), dim3(256), 0, s, a,
                       mode);
  else
    hipLaunchKernelGGL(k_ortho<float>, dim3(nblocks(a.n, kRowsPerBlock)), dim3(256), 0, s, a,
                       mode);
}

void launch_ortho_small(const OrthoArgs& a, void* vout, hipStream_t s) {
  if (a.X.v64)
    hipLaunchKernelGGL(k_ortho_small<double>, dim3(1), dim3(kOrthoSmallThreads), 0, s, a,
                       static_cast<double*>(vout));
  else
    hipLaunchKernelGGL(k_ortho_small<float>, dim3(1), dim3(kOrthoSmallThreads), 0, s, a,
                       static_cast<float*>(vout));
}

void launch_cycle(const CycleArgs& a, int store, hipStream_t s) {
  const int nb = (a.n + kTS - 1) / kTS;
  const dim3 grid(3 * nb), block(kTSThreads);
  if (store == kStoreF16)
    hipLaunchKernelGGL(k_cycle<Fp16>, grid, block, 0, s, a);
  else if (store == kStoreBF16)
    hipLaunchKernelGGL(k_cycle<Bf16>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_cycle<Fp32>, grid, block, 0, s, a);
}

void launch_combine(const Basis& X, int n, const double* M, int nout, double* out, int64_t ldo,
                    hipStream_t s) {
  if (X.v64)
    hipLaunchKernelGGL(k_combine<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, X, n, M, nout,
                       out, ldo);
  else
    hipLaunchKernelGGL(k_combine<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, X, n, M, nout,
                       out, ldo);
}

void launch_cycle_update(const Basis& Xd, const double* cd, void* d, const Basis& Xr,
                         const double* cr, void* r, int n, int v64, hipStream_t s) {
  if (v64)
    hipLaunchKernelGGL(k_cycle_update<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, Xd, cd,
                       static_cast<double*>(d), Xr, cr, static_cast<double*>(r), n);
  else
    hipLaunchKernelGGL(k_cycle_update<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, Xd, cd,
                       static_cast<float*>(d), Xr, cr, static_cast<float*>(r), n);
}

void launch_gram(const Basis& X, const double* Y, int ny, int64_t ldy, int n, double* G,
                 double* partial, unsigned int* counter, hipStream_t s) {
  if (X.v64)
    hipLaunchKernelGGL(k_gram<double>, dim3(nblocks(n, kRowsPerBlock)), dim3(256), 0, s, X, Y,
                       ny, ldy, n, G, partial, counter);
  else
    hipLaunchKernelGGL(k_gram<float>, dim3(nblocks(n, kRowsPerBlock)), dim3(256), 0, s, X, Y, ny,
                       ldy, n, G, partial, counter);
}

void launch_scale_round(const double* r, double sc, double* out, int n, int v64, hipStream_t s) {
  if (v64)
    hipLaunchKernelGGL(k_scale_round<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, r, sc, out,
                       n);
  else
    hipLaunchKernelGGL(k_scale_round<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, r, sc, out,
                       n);
}

void launch_x_update(double* x, const void* d, int v64, double sc, int n, hipStream_t s) {
  if (v64)
    hipLaunchKernelGGL(k_x_update<double>, dim3(nblocks(n, 256)), dim3(256), 0, s, x,
                       static_cast<const double*>(d), sc, n);
  else
    hipLaunchKernelGGL(k_x_update<float>, dim3(nblocks(n, 256)), dim3(256), 0, s, x,
                       static_cast<const float*>(d), sc, n);
}

void launch_div_u(const void* w, double sc, void* out, int v64, int n, hipStream_t s) {
  if (v64)
    hipLaunchKernelGGL(k_div_u<double>, dim3(nblocks(n, 256)), dim3(256), 0, s,
                       static_cast<const double*>(w), sc, static_cast<double*>(out), n);
  else
    hipLaunchKernelGGL(k_div_u<float>, dim3(nblocks(n, 256)), dim3(256), 0, s,
                       static_cast<const float*>(w), sc, static_cast<float*>(out), n);
}

// out[0] = max |x - x_true|, out[1] = max |x_true| (bits; zeroed here)
__global__ void k_ferr(const double* __restrict__ x, const double* __restrict__ xt, int n,
                       unsigned long long* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0, t = 0.0;
  if (i < n) {
    d = fabs(x[i] - xt[i]);
    t = fabs(xt[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d = fmax(d, __shfl_xor(d, o, kWave));
    t = fmax(t, __shfl_xor(t, o, kWave));
  }
  if ((threadIdx.x % kWave) == 0) {
    atomic_max_nonneg(out, d);
    atomic_max_nonneg(out + 1, t);
  }
}

// one wave per row, lanes strided over the columns as in k_ingest, then the
// same wave reduction: the same sums bit for bit
__global__ __launch_bounds__(256) void k_rowsum_max(const double* __restrict__ A, int64_t n,
                                                    int64_t lda, unsigned long long* out) {
  __shared__ double ssum[4];
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  double s = 0.0;
  if (row < n) {
    const double* a = A + row * lda;
    for (int64_t c = lane; c < n; c += kWave) s += fabs(a[c]);
  }
  s = wave_sum(s);
  if (lane == 0) ssum[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < 4; ++w) r = fmax(r, ssum[w]);
    atomic_max_nonneg(out, r);
  }
}

void launch_rowsum_max(const double* A, int64_t n, int64_t lda, unsigned long long* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out, 1);
  hipLaunchKernelGGL(k_rowsum_max, dim3(nblocks(n, 4)), dim3(256), 0, s, A, n, lda, out);
}

// out[0..2] from the reduction words of an error report (layout of
// launch_errors_finish); one thread
__global__ void k_errors_finish(const unsigned long long* __restrict__ w, int has_xt,
                                double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double rmax = __longlong_as_double((long long)w[0]);
  const double xmax = __longlong_as_double((long long)w[1]);
  const double bmax = __longlong_as_double((long long)w[2]);
  const double na = __longlong_as_double((long long)w[3]);
  const double den = na * xmax + bmax;
  out[0] = (rmax == 0.0) ? 0.0 : (den > 0.0 ? rmax / den : __builtin_inf());
  out[1] = __longlong_as_double((long long)w[kNormCw]);
  out[2] = __builtin_nan("");
  if (has_xt) {
    const double dmax = __longlong_as_double((long long)w[5]);
    const double tmax = __longlong_as_double((long long)w[6]);
    out[2] = (dmax == 0.0) ? 0.0 : (tmax > 0.0 ? dmax / tmax : __builtin_inf());
  }
}

void launch_errors_finish(const unsigned long long* w, int has_xt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_errors_finish, dim3(1), dim3(64), 0, s, w, has_xt, out);
}

void launch_ferr(const double* x, const double* xt, int n, unsigned long long* out,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out, 2);
  hipLaunchKernelGGL(k_ferr, dim3(nblocks(n, 256)), dim3(256), 0, s, x, xt, n, out);
}

void launch_maxabs(const double* v, int n, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out, 1);
  hipLaunchKernelGGL(k_maxabs, dim3(nblocks(n, 256)), dim3(256), 0, s, v, n, out);
}

void launch_copy_f32_to_f64(const float* a, double* b, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32_f64, dim3(nblocks(n, 256)), dim3(256), 0, s, a, b, n);
}

void launch_colsum(const void* A, int a64, int64_t ld, int n, const void* v, int v64,
                   double* partial, const double* b, const double* x, double* t,
                   unsigned long long* norms, const CycleState* gate, int step, hipStream_t s) {
  const int nchunks = (n + kColRows - 1) / kColRows;
  const dim3 g1(nblocks(n, 256), (unsigned)nchunks);
#define GIR_CS(AT, VT)                                                                       \
  hipLaunchKernelGGL((k_colsum_partial<AT, VT>), g1, dim3(256), 0, s,                         \
                     static_cast<const AT*>(A), ld, n, static_cast<const VT*>(v), partial, gate, \
                     step)
  if (a64) {
    if (v64) GIR_CS(double, double); else GIR_CS(double, float);
  } else {
    if (v64) GIR_CS(float, double); else GIR_CS(float, float);
  }
#undef GIR_CS
  if (norms) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, norms, 2);
  hipLaunchKernelGGL(k_colsum_finish, dim3(nblocks(n, 256)), dim3(256), 0, s, partial, nchunks, n,
                     b, x, t, norms, gate, step);
}

void launch_colsum_abs(const double* A, int64_t ld, int n, double* partial, double* t,
                       unsigned long long* out, hipStream_t s) {
  const int nchunks = (n + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(k_colsum_abs_partial, dim3(nblocks(n, 256), (unsigned)nchunks), dim3(256), 0,
                     s, A, ld, n, partial);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out, 2);
  hipLaunchKernelGGL(k_colsum_finish, dim3(nblocks(n, 256)), dim3(256), 0, s, partial, nchunks, n,
                     nullptr, nullptr, t, out, nullptr, 0);
}

void launch_trsv_t_cols(const void* S, int64_t ld, const int* permS, int store, int n,
                        bool upperT, const double* in, int64_t ldi, int nr, const double* Dinv,
                        const double* Q, double* y, int64_t ldy, double scale,
                        const int* permOut, double* out64, int64_t ldo, uint64_t* xw,
                        int64_t xstride, int epoch, int* abortp, hipStream_t s) {
  if (nr <= 0) return;
  const dim3 grid(col_grid(n, nr));
  const ColStrides cs{ldi, ldy, ldo, xstride, nr};
#define GIR_TT(F, U)                                                                          \
  hipLaunchKernelGGL((k_trsv_t<F, U>), grid, dim3(kTSThreads), 0, s,                          \
                     reinterpret_cast<const typename F::T*>(S), ld, permS, n, in, Dinv, Q, y,  \
                     scale, permOut, out64, nullptr, xw, (uint32_t)epoch, nullptr, 0, abortp, cs)
  if (store == kStoreF16) {
    if (upperT) GIR_TT(Fp16, true); else GIR_TT(Fp16, false);
  } else if (store == kStoreBF16) {
    if (upperT) GIR_TT(Bf16, true); else GIR_TT(Bf16, false);
  } else {
    if (upperT) GIR_TT(Fp32, true); else GIR_TT(Fp32, false);
  }
#undef GIR_TT
}

void launch_trsv_t(const void* S, int64_t ld, const int* permS, int store, int n, bool upperT,
                   const double* in, const double* Dinv, const double* Q, double* y, double scale,
                   const int* permOut, double* out64, float* out32, uint64_t* xw, int epoch,
                   const CycleState* gate, int step, int* abortp, hipStream_t s) {
  const unsigned grid = nblocks(n, kTS);
  const ColStrides cs{0, 0, 0, 0};
#define GIR_TT(F, U)                                                                        \
  hipLaunchKernelGGL((k_trsv_t<F, U>), dim3(grid), dim3(kTSThreads), 0, s,                  \
                     reinterpret_cast<const typename F::T*>(S), ld, permS, n, in, Dinv, Q,   \
                     y, scale, permOut, out64, out32, xw, (uint32_t)epoch, gate, step, abortp, \
                     cs)
  if (store == kStoreF16) {
    if (upperT) GIR_TT(Fp16, true); else GIR_TT(Fp16, false);
  } else if (store == kStoreBF16) {
    if (upperT) GIR_TT(Bf16, true); else GIR_TT(Bf16, false);
  } else {
    if (upperT) GIR_TT(Fp32, true); else GIR_TT(Fp32, false);
  }
#undef GIR_TT
}

void launch_rank1(double alpha, const double* x, const double* y, int n, int64_t ld, double* out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_rank1, dim3(nblocks(n, 256), (unsigned)n), dim3(256), 0, s, alpha, x, y,
                     n, ld, out);
}

}  // namespace gir
