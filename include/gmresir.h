/*
 * gmresir.h -- C ABI of the MI355X mixed-precision GMRES-IR solver with
 * Krylov subspace recycling (RGMRES-IR).
 *
 * Method: Oktay & Carson, "Mixed Precision GMRES-based Iterative Refinement
 * with Recycling".  gmresir_factor is the factorisation step of Algorithm 3
 * (LU factorisation in precision u_f); gmresir_solve is the rest of
 * Algorithm 3 (the initial solve and the refinement loop, whose correction
 * equation U^-1 L^-1 A d = U^-1 L^-1 r is solved by the
 * GCRO-DR algorithm of Section 2, with the preconditioned product computed in
 * precision u^2).  With k = 0 the correction solver is restarted GMRES(m),
 * i.e. Algorithm 2 (GMRES-IR).
 *
 * Conventions shared by every entry point
 *   - Matrices are dense, row-major (C order), float64, leading dimension
 *     lda >= n (elements).  Vectors are float64 and contiguous (stride 1).
 *   - "device pointer": memory allocated on the HIP device that is current
 *     when the call is made (hipMalloc, or a torch CUDA tensor on ROCm).
 *     "host pointer": ordinary CPU memory.
 *   - stream: a hipStream_t passed as void*; NULL means the null stream.
 *     Every call is blocking: it synchronises the stream before returning,
 *     so inputs may be reused and outputs read as soon as it returns.
 *   - Return value: 0 on success.  Negative values are caller or runtime
 *     errors, positive values are numerical outcomes (see gmresir_status).
 *     No C++ exception crosses this interface.
 *   - A handle is not re-entrant: calls on one handle must not overlap.
 *     Distinct handles are independent.
 */
#ifndef GMRESIR_H
#define GMRESIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMRESIR_ABI_VERSION 3

typedef enum {
  GMRESIR_OK = 0,
  GMRESIR_EINVAL = -1,      /* invalid argument (null pointer, n <= 0, lda < n,
                               m <= k, k < 0, tau <= 0, unsupported or
                               mis-ordered precisions, struct_size mismatch) */
  GMRESIR_ENOMEM = -2,      /* device or host allocation failed             */
  GMRESIR_EHIP = -3,        /* HIP runtime error (text: gmresir_last_error) */
  GMRESIR_EINTERNAL = -4,   /* a device-side wait exceeded its bound        */
  GMRESIR_ESINGULAR = 1,    /* exact zero pivot in u_f (column in info)     */
  GMRESIR_ERANGE = 2,       /* non-finite input, or overflow to u_f         */
  GMRESIR_ENOCONV = 3       /* i_max refinement steps without reaching the
                               backward-error target; x holds the last
                               iterate                                       */
} gmresir_status;

/* Precisions of Algorithm 3 (Section 3): u_f factorisation, u working
 * precision of GCRO-DR, u_r residual.  u^2 (the precision of the
 * preconditioned product) is fp64 for u = fp32 and double-double for
 * u = fp64.  Supported triples: u_f in {FP16, BF16, FP32}, u in {FP32, FP64},
 * u_r in {FP64, DD}, with unit roundoff u_f >= u >= u_r. */
typedef enum {
  GMRESIR_BF16 = 1,
  GMRESIR_FP16 = 2,
  GMRESIR_FP32 = 3,
  GMRESIR_FP64 = 4,
  GMRESIR_DD = 5
} gmresir_prec;

typedef struct {
  uint32_t struct_size;   /* must equal sizeof(gmresir_opts)                 */
  int32_t uf, u, ur;      /* gmresir_prec values                             */
  int32_t m;              /* restart length (maximum subspace size), m >= 1  */
  int32_t k;              /* recycled dimension, 0 <= k < m (0: GMRES(m))    */
  double tau;             /* GMRES tolerance on the relative preconditioned
                             residual (Section 4), tau > 0                    */
  int32_t imax;           /* maximum refinement steps (Algorithm 3 i_max)     */
  int32_t maxit;          /* Arnoldi steps per correction solve; 0 -> 10 m    */
  double berr_target;     /* stop when ||r||_inf / (||A||_inf ||x||_inf +
                             ||b||_inf) <= berr_target                        */
  int32_t scale_pow2;     /* -1 auto (on for FP16), 0 off, 1 on: multiply A by
                             2^e before rounding to u_f (exact; undone in the
                             preconditioner)                                  */
  int32_t keep_recycle;   /* 1: the recycled pair survives between
                             gmresir_solve calls on the same handle          */
  int32_t timing;         /* bit c (classes 0-7) or bit c + 8 (classes 8-15)
                             set: bracket every launch of kernel class c (the
                             order listed at gmresir_kernel_stats) with HIP
                             events on the stream it runs on; bits 8-15 =
                             s > 1: only every s-th launch of each timed
                             class (fewer events in the stream); 0: off     */
  int32_t matvec_u;       /* 1: the correction solve applies M^-1 and A-tilde in
                             u instead of u^2 (SGMRES-IR / RSGMRES-IR, Section 3;
                             u = FP64 only); x0 keeps u^2.  Default 0.          */
  int32_t reuse_recycle;  /* 1: keep C_k and U_k of the previous correction solve
                             (same A: A-tilde U_k = C_k still holds) instead of
                             recomputing QR(A-tilde U_k).  Default 0.           */
  int32_t ortho;          /* orthogonalisation of each Arnoldi vector against
                             [C_k V_j]: 0 classical Gram-Schmidt applied
                             twice (CGS2, default), 1 modified Gram-Schmidt
                             (one column at a time; slower, two launches per
                             basis column)                                   */
  /* Optional device allocator (both or neither): when alloc is not NULL,
   * every device buffer of a handle is carved from memory obtained with
   * alloc(bytes, alloc_user) -- which must return device memory on the
   * current device, 256-byte aligned, or NULL (then the call fails with
   * ENOMEM) -- and handed back with free_(ptr, alloc_user) by gmresir_free.
   * This routes the library's memory through a caller's pool (for example
   * torch's caching allocator).  With gmresir_solve_batched the callbacks
   * are called from the worker threads and must be thread-safe.  NULL: the
   * library's own allocation and its process-wide cache.                    */
  void* (*alloc)(size_t bytes, void* alloc_user);
  void (*free_)(void* ptr, void* alloc_user);
  void* alloc_user;
} gmresir_opts;

/* Per-solve record, filled by gmresir_solve (host struct). */
#define GMRESIR_MAX_STEPS 64
typedef struct {
  int32_t status;                      /* gmresir_status of the solve       */
  int32_t steps;                       /* corrections applied               */
  int32_t total_its;                   /* sum of its[]                      */
  int32_t its[GMRESIR_MAX_STEPS];      /* Arnoldi steps per correction, the
                                          paper's "total (i1, i2, ...)"     */
  double berr[GMRESIR_MAX_STEPS + 1];  /* normwise backward error before
                                          each correction and at the end:
                                          ||r||_inf / (||A||_inf ||x||_inf +
                                          ||b||_inf), r from the u_r residual */
  int32_t singular_col;                /* 1-based column of the zero pivot  */
  int32_t recycle_dim;                 /* dimension of U_k at the end       */
  double t_factor_s;                   /* wall time of gmresir_factor       */
  double t_solve_s;                    /* wall time of this gmresir_solve   */
  double berr_cw[GMRESIR_MAX_STEPS + 1];  /* componentwise backward error at
                                          the same points, max_i |r_i| /
                                          (|A| |x| + |b|)_i with 0/0 = 0 (the
                                          error measures of Table 2); NaN for
                                          gmresir_solve_transposed            */
  /* Stream time of the solve's phases (seconds; HIP events at the phase
   * boundaries, so host decisions between launches count in the phase they
   * interrupt).  They add up to the solve's device span.                   */
  double t_x0_s;                       /* x0 = M^-1 b                        */
  double t_residual_s;                 /* residuals, backward errors, test  */
  double t_precond_s;                  /* r-hat and z = M^-1 r-hat           */
  double t_recycle_s;                  /* QR(A-tilde U_k), projection of z,
                                          deferred recycle refreshes         */
  double t_arnoldi_s;                  /* Arnoldi cycles, least squares,
                                          cycle updates and refreshes, x
                                          update                             */
  int32_t cycles_persistent;           /* GMRES cycles whose Arnoldi steps ran
                                          in one persistent launch (u = FP32,
                                          CGS2, n <= 8192 and 3 ceil(n/128)
                                          compute units on the device)       */
  int32_t cycles_fallback;             /* persistent launches that gave up
                                          (not all their workgroups resident
                                          together: the device was shared)
                                          and ran as separate launches       */
} gmresir_info;

typedef struct gmresir_ctx gmresir_ctx;

/* Fill *opts with defaults: (FP16, FP32, FP64), m = 30, k = 10, tau = 1e-4,
 * imax = 10, maxit = 0, berr_target = 1e-14, scale_pow2 = -1,
 * keep_recycle = 0, timing = 0, ortho = 0 (CGS2). */
void gmresir_default_opts(gmresir_opts* opts);

/*
 * gmresir_factor -- Algorithm 3, factorisation step: LU with partial
 * pivoting of A in precision u_f (Section 1, GEPP), plus the copies of A
 * the solve needs (A in fp64 for the residual, A_u = fl_u(A) for the
 * preconditioned product) and ||A||_inf.
 *
 *   A      device pointer, n x n float64, row-major, leading dimension lda.
 *          Read only; the library copies what it needs.
 *   n      order of A, 1 <= n <= 16384 (EINVAL beyond: the pivot search
 *          of a block column runs in at most 32 workgroups of 512 rows);
 *          lda >= n.
 *   opts   host pointer to options (copied).
 *   stream hipStream_t or NULL.
 *   out    host pointer receiving a new handle (set to NULL on failure).
 *
 * Returns 0, GMRESIR_ESINGULAR (a handle is still returned so the caller can
 * inspect or free it; gmresir_solve on it returns ESINGULAR),
 * GMRESIR_ERANGE (non-finite entry or overflow in u_f; handle returned
 * likewise), EINVAL, ENOMEM, EHIP or EINTERNAL (no handle).
 * The handle owns all device memory it uses; release it with gmresir_free.
 */
int gmresir_factor(const double* A, int64_t n, int64_t lda,
                   const gmresir_opts* opts, void* stream, gmresir_ctx** out);

/*
 * gmresir_solve -- Algorithm 3 after the factorisation: x0 = M^-1 b, then refinement
 * steps r = b - A x (in u_r), r-hat = r / ||r||_inf, GCRO-DR(m, k) on
 * U^-1 L^-1 P A d = U^-1 L^-1 P r-hat with the product in u^2, and
 * x = x + ||r||_inf d, until the backward error reaches opts.berr_target.
 *
 *   h      handle from gmresir_factor or gmresir_import_factors.
 *   b      device pointer, nrhs right-hand sides of length n, column j at
 *          b + j * ldb (ldb >= n).  Read only.
 *   x      device pointer, same layout as b; receives the solutions.
 *   nrhs   >= 1; the columns are solved one after another, and the recycled
 *          space carries over between them when opts.keep_recycle = 1.
 *   stream hipStream_t or NULL (overrides the factor stream for this call).
 *   info   host pointer or NULL; describes the LAST right-hand side.
 *
 * Returns the status of the last column (0, ENOCONV, ESINGULAR, ERANGE for a
 * non-finite b) or a negative error.  On ENOCONV x holds the last iterate.
 */
int gmresir_solve(gmresir_ctx* h, const double* b, double* x, int64_t nrhs,
                  int64_t ldb, void* stream, gmresir_info* info);

/*
 * gmresir_solve_transposed -- the adjoint system A^T lambda = g by the same
 * refinement with the transposed factors (A^T = 2^-e U^T L^T P):
 * lambda0 = M^-T g with M^-T = 2^e P^T L^-T U^-T, residual g - A^T lambda in
 * fp64, GCRO-DR(m, k) on M^-T A_u^T with the product in u^2 = fp64, and a
 * recycle space of its own, separate from gmresir_solve's (kept across calls
 * when opts.keep_recycle = 1).  The backward error uses ||A^T||_inf = ||A||_1
 * (computed on the first call).  Used for the gradient of a loss through
 * x = A^-1 b: with g = dL/dx, dL/db = lambda and dL/dA = -lambda x^T.
 *
 * Arguments, layout, ownership and return values as for gmresir_solve (g in
 * place of b, lambda in place of x).  Supported for u = FP32, ur = FP64; EINVAL
 * for other precision triples.
 */
int gmresir_solve_transposed(gmresir_ctx* h, const double* g, double* lambda,
                             int64_t nrhs, int64_t ldb, void* stream,
                             gmresir_info* info);

/*
 * gmresir_rank1 -- out = alpha x y^T: x, y device pointers of n float64
 * values, out a device pointer to n x n float64, row-major, leading dimension
 * ldo >= n (overwritten).  Forms the matrix gradient -lambda x^T of the
 * adjoint.  Blocks on stream; EINVAL on null pointers or ldo < n.
 */
int gmresir_rank1(double alpha, const double* x, const double* y, int64_t n,
                  double* out, int64_t ldo, void* stream);

/*
 * gmresir_choose_k -- automatic recycle dimension, "finding the knee"
 * (Section 3, the discussion of the total iterations against k): solves
 * A x = b once for every k = 0 .. kmax, without carrying a recycle space
 * between the solves, and sets *k_best to the smallest k with the fewest
 * total Arnoldi steps among the solves that reach the backward-error target.
 * k is limited to (Arnoldi steps of the first refinement step at k = 0) - 1,
 * as the first step runs without recycling and k harmonic Ritz vectors need
 * at least k + 1 Arnoldi steps.
 *
 *   h      handle; kmax <= the k it was created with (its buffers).
 *   b      device pointer, n float64.
 *   k_best host pointer, receives the chosen k.
 *   its    host pointer to kmax + 1 int32 or NULL: total Arnoldi steps per k,
 *          -1 where the solve did not converge or k was beyond the limit.
 *   stream hipStream_t or NULL.
 *
 * Returns 0, ENOCONV (no k converged; *k_best = 0), ESINGULAR / ERANGE as
 * gmresir_solve, or a negative error.  The handle's k is left as it was; a
 * recycle space kept from earlier solves (opts.keep_recycle = 1) is dropped,
 * because the trial solves reuse its buffers, so the next gmresir_solve starts
 * without one (as on a new handle).
 */
int gmresir_choose_k(gmresir_ctx* h, const double* b, int32_t kmax,
                     int32_t* k_best, int32_t* its, void* stream);

/* Release every resource of the handle.  NULL is accepted.  The handle must
 * not be used afterwards.  Its device memory goes to a process-wide cache
 * (at most 16 GiB in all, beyond that it is freed) from which later handles
 * of the same sizes take their buffers, so repeated factorisations do not
 * call hipMalloc / hipFree; cached memory is returned when the process
 * ends. */
void gmresir_free(gmresir_ctx* h);

/* Static description of a status code. */
const char* gmresir_strerror(int status);

/* Text of the last HIP or validation error seen in this thread. */
const char* gmresir_last_error(void);

/*
 * gmresir_import_factors -- build a handle from LU factors computed
 * elsewhere (same meaning as after gmresir_factor): P 2^e A = L U with L unit
 * lower and U upper packed row-major in lu (device pointer, n x n, leading
 * dimension ldlu, element type u_f: 2-byte IEEE half or bfloat16 bits, or
 * float32), ipiv host pointer of n LAPACK-style 0-based interchanges (row i
 * was swapped with row ipiv[i] at step i), e the power-of-two scale.
 * A (device, float64) is the unscaled matrix.  Used to run the solve phase on
 * given factors.  Same return values as gmresir_factor except ESINGULAR.
 */
int gmresir_import_factors(const double* A, int64_t n, int64_t lda,
                           const void* lu, int64_t ldlu, const int32_t* ipiv,
                           int32_t e, const gmresir_opts* opts, void* stream,
                           gmresir_ctx** out);

/*
 * gmresir_export_factors -- copy the factors of a handle: lu (host pointer,
 * n x n row-major, element type u_f as in gmresir_import_factors, leading
 * dimension n), ipiv (host, n int32, LAPACK style, 0-based) and *e.  Any
 * output pointer may be NULL.
 */
int gmresir_export_factors(gmresir_ctx* h, void* lu, int32_t* ipiv, int32_t* e);

/*
 * gmresir_apply -- one preconditioned product of the solve phase, for
 * inspection: op = 0: y = M^-1 v = 2^e U^-1 L^-1 P v; op = 1:
 * y = A-tilde v = M^-1 A_u v; op = 2: y = M^-T v = 2^e P^T L^-T U^-T v;
 * op = 3: y = M^-T A_u^T v (the adjoint's operator; ops 2 and 3 for u = FP32,
 * ur = FP64 only).  All are computed in u^2 and returned rounded to fp64
 * (float64).  v and y are device pointers of n float64 values (v must hold u
 * values for ops 1 and 3).
 */
int gmresir_apply(gmresir_ctx* h, int32_t op, const double* v, double* y,
                  void* stream);

/*
 * gmresir_errors -- the error measures of a computed solution (Table 2's
 * columns), from a residual r = b - A x formed in double-double and rounded
 * to fp64 (independent of the handle's u_r):
 *   out[0]  normwise backward error ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf)
 *   out[1]  componentwise backward error max_i |r_i| / (|A| |x| + |b|)_i
 *           (0/0 = 0)
 *   out[2]  forward error ||x - x_true||_inf / ||x_true||_inf, or NaN when
 *           x_true is NULL
 * b, x, x_true: device pointers of n float64 values (read only); out: host
 * pointer to 3 doubles.  Uses the handle's fp64 copy of A and its scratch
 * vectors (not re-entrant with a solve on the same handle).  Returns 0,
 * EINVAL (null handle, b, x or out), ERANGE (handle from a non-finite A),
 * or EHIP.
 */
int gmresir_errors(gmresir_ctx* h, const double* b, const double* x,
                   const double* x_true, double* out, void* stream);

/*
 * gmresir_errors_noalloc -- gmresir_errors for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): the same three measures, computed by the same
 * kernels, without a handle and without allocating anything.  Its scratch
 * vectors and reduction words live in one static device array per GPU
 * (about 384 KiB, held until the process ends; its device address is taken
 * once per device on the first call).  Results go to device memory in stream
 * order: the call enqueues its kernels and returns without synchronising.
 *
 *   A       device pointer, n x n float64 row-major, leading dimension lda;
 *           16-byte aligned with lda even (its rows are read as 16-byte
 *           pairs).  ||A||_inf is computed here, summed in the same order as
 *           gmresir_factor sums it.
 *   n       1 <= n <= 16384 (EINVAL beyond: the static scratch limit).
 *   b, x    device pointers of n float64 values; x_true as well, or NULL.
 *   out     DEVICE pointer to 3 doubles: normwise backward error,
 *           componentwise backward error, forward error (NaN without
 *           x_true), as gmresir_errors defines them.
 *   stream  hipStream_t or NULL.
 *
 * Every call on one GPU uses that GPU's one scratch array: calls that
 * overlap on the same device (other streams or threads) race and must be
 * serialised by the caller.  Returns 0, EINVAL (null pointer, n out of range,
 * lda < n, misaligned A or odd lda) or EHIP.
 */
int gmresir_errors_noalloc(const double* A, int64_t n, int64_t lda,
                           const double* b, const double* x,
                           const double* x_true, double* out, void* stream);

/*
 * Per-kernel-class launch timing (handles created with opts.timing != 0).
 * One record per timed class that ran since the handle was created: the
 * number of
 * launches, the sum of their durations measured with HIP events recorded on
 * the stream the kernels were launched on (launches an Arnoldi step skipped
 * on the device after convergence are not counted), and the algorithmic work
 * of those launches: bytes that must cross HBM (bound = 0) or floating-point
 * operations (bound = 1).  Classes, in order: "lu_panel" (a block column's
 * GEPP fused with the previous step's trailing update), "lu_trsm", "lu_gemm"
 * (factorisation; flops), "trsv_lower", "trsv_upper", "gemv_au", "residual",
 * "ortho" (solve-phase launches; bytes), "arnoldi_step" (class 8, timing
 * bit 16: one whole Arnoldi step, A-tilde v_j through the normalisation,
 * with n^2 (s_A + s_f) plus one read of the basis as its bytes) and
 * "arnoldi_cycle" (class 9, timing bit 17: a cycle's steps in one persistent
 * launch, used for u = FP32 with classical Gram-Schmidt when n <= 8192; its
 * work is that of the steps it took; GMRESIR_PERSISTENT=0 in the
 * environment at handle creation keeps the separate launches).  Each event
 * pair costs a few microseconds of stream time, so time only the classes of
 * interest, or a sample of their launches (opts.timing bits 8-15).
 *
 *   out    host array of cap records; count receives the number written.
 * Waits for the recorded events.  Returns EINVAL when timing is off.
 */
typedef struct {
  char name[24];
  int32_t launches;
  int32_t bound;      /* 0: HBM bytes, 1: matrix-core flops */
  double total_ms;
  double work;
} gmresir_kernel_stat;

int gmresir_kernel_stats(gmresir_ctx* h, gmresir_kernel_stat* out, int32_t cap,
                         int32_t* count);

/* One system of a batch (host struct; A, b, x are device pointers).
 *   A     n x n row-major fp64, leading dimension lda >= n.
 *   b, x  nrhs right-hand sides and solutions, column j at b + j * ldb and
 *         x + j * ldb (ldb >= n); x is written.
 *   info  host array of nrhs records, one per right-hand side (as
 *         gmresir_solve fills them), or NULL.
 *   status  out: the system's outcome -- the first nonzero gmresir_status
 *         of its factorisation and its right-hand sides in order (a negative
 *         one stops the system), else 0. */
typedef struct {
  const double* A;
  int64_t n;
  int64_t lda;
  const double* b;
  double* x;
  int64_t nrhs;
  int64_t ldb;
  gmresir_info* info;
  int32_t status;
  int32_t reserved;
} gmresir_batch_item;

/* Batched solves (the batching extension of the method: many independent
 * systems of uneven n, each with its own right-hand sides).  Every system is
 * factored and solved exactly as by gmresir_factor + gmresir_solve with
 * `opts` (Algorithm 3; Algorithm 2 for k = 0), so its result does not depend
 * on the batch.  `workers` host threads (<= 0: 8; at most 64), each with a
 * HIP stream of its own, take the systems largest first and keep several in
 * flight on the current device.
 *   stream  hipStream_t or NULL: work queued on it (producing A and b) is
 *           finished before any system is read.
 * Blocks until every system is done and its device memory released.
 * Returns 0 when no system reports a negative status; otherwise the first
 * negative status in item order (EINVAL also for invalid items: null
 * pointers, n <= 0, lda < n, nrhs <= 0, ldb < n -- then nothing runs). */
int gmresir_solve_batched(gmresir_batch_item* items, int64_t count,
                          const gmresir_opts* opts, int32_t workers, void* stream);

/* Size n and ABI version of a handle (either pointer may be NULL). */
int gmresir_query(gmresir_ctx* h, int64_t* n, int32_t* abi_version);

#ifdef __cplusplus
}
#endif

#endif /* GMRESIR_H */
