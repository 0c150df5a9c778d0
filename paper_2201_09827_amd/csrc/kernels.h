// Host-side launchers of the gmresir HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace gir {

enum StoreType { kStoreF16 = 0, kStoreBF16 = 1, kStoreF32 = 2 };

// ---- factorisation ---------------------------------------------------------

// one pass over the caller's A (lda): A64 and Au (if not null) copies with
// zero padding to ld, norms[0] = max |a| bits, norms[1] = max row-sum bits,
// flag[0] = 1 on a non-finite entry (norms/flag zeroed beforehand)
void launch_ingest(const double* A, int64_t n, int64_t lda, double* A64, float* Au, int64_t ld,
                   unsigned long long* norms, int* flag, hipStream_t s);
// S = fl_uf(2^e A64), e = the fp16 scale exponent from norms[0] and sqrtn
// (sqrt(n) as computed on the host) when scaled != 0, else 0; *e_out = e
void launch_convert_scaled(const double* A64, int64_t n, int64_t ld, int store, void* S,
                           const unsigned long long* norms, double sqrtn, int scaled, int* e_out,
                           int* flag, hipStream_t s);
void launch_iota(int* p, int64_t n, hipStream_t s);

struct PanelArgs {
  void* S;          // u_f storage, physical row order
  int64_t ld;
  int n;
  int k0;           // first column of the panel
  int kb;           // panel width (<= nb)
  int* perm;        // logical -> physical rows, rewritten for rows k0.. by the panel
  int* ipiv;        // [n] LAPACK-style (0-based)
  int* perm_copy;   // null, or receives the same rewrite of rows k0.. as perm
  uint64_t* xch;    // [kPanelXchWords] pivot exchange, zeroed before the first panel
  CycleState* st;   // abort + singular reporting
};
// words of the exchange buffer: 2 column parities x 32 workgroups x 80 words
constexpr int64_t kPanelXchWords = 2 * 32 * 80;
// one block column of the blocked right-looking GEPP (lazy row interchanges)
void launch_panel_step(const PanelArgs& a, int store, hipStream_t s);
// the block row to the right of the panel (U12 = L11^-1 A12), columns
// [c_begin, c_end)
void launch_trsm(const PanelArgs& a, int store, int c_begin, int c_end, hipStream_t s);
// the trailing update A22 -= L21 U12 on the matrix cores for columns
// [c_begin, c_end); trailing rows located through rows[k0 + kb ..] (perm or
// a copy of it)
void launch_gemm_update(const PanelArgs& a, int store, const int* rows, int c_begin, int c_end,
                        hipStream_t s);
// block column p and, in the same launch, the trailing update of step u for
// columns [c_begin, c_end) (disjoint from block column p), rows through `rows`.
// Where panel_update_folds(store): block column p's own part of step u's
// update is formed by its workgroups (no launch_gemm_update for it), and with
// fold == 2 the launch also solves step u's block row (no launch_trsm;
// strip_cnt then holds ceil((c_end - c_begin) / 128) zeroed counters for this
// launch alone); with fold == 1 launch_trsm(u, c1, n) runs before; fold == 0
// (or fp32 factors): both run as their own launches before
void launch_panel_update(const PanelArgs& p, const PanelArgs& u, int store, const int* rows,
                         int c_begin, int c_end, int fold, int* strip_cnt, hipStream_t s);
bool panel_update_folds(int store);
void launch_copy_i32(int* dst, const int* src, int64_t n, hipStream_t s);
// copy of `words` 4-byte words; either side may be mapped pinned host memory
void launch_copy_words(void* dst, const void* src, int64_t words, hipStream_t s);
// up to kCopyPieces such copies in one launch
constexpr int kCopyPieces = 8;
struct CopyPieces {
  void* dst[kCopyPieces];
  const void* src[kCopyPieces];
  int64_t words[kCopyPieces];
  int count;
};
void launch_copy_pieces(const CopyPieces& c, hipStream_t s);
// after the last panel: non-finite check of the factors (S 16-byte aligned,
// ld a multiple of 8 elements: rows are read as 16-byte vectors)
void launch_check_factors(const void* S, int64_t n, int64_t ld, int store, int* flag,
                          hipStream_t s);

// ---- solve phase -----------------------------------------------------------

// t[i] = sum_c Au[permA[i]][c] v[c] in fp64 (v float or double)
void launch_gemv_au(const float* Au, int64_t ld, const int* permA, int n, const float* v32,
                    const double* v64, double* t, const CycleState* gate, int step,
                    hipStream_t s);
// T[:, r] = A_u[permA rows] Y[:, r], r < nr <= 16 (fp64 Y and T, leading
// dimensions ldy, ldt; Y's columns 16-byte aligned), fp64 accumulation
void launch_gemv_au_multi(const float* Au, int64_t ld, const int* permA, int n, const double* Y,
                          int64_t ldy, int nr, double* T, int64_t ldt, hipStream_t s);
// t[i] = sum_c A[permA[i]][c] v[c] with fp64 A and v, fp64 accumulation
void launch_gemv_a64(const double* A, int64_t ld, const int* permA, int n, const double* v,
                     double* t, const CycleState* gate, int step, hipStream_t s);
// r = b - A x (fp64); norms[0] = max|r| bits, norms[1] = max|x| bits,
// norms[kNormCw] = componentwise backward error bits (all three zeroed here)
void launch_residual(const double* A, int64_t ld, int n, const double* b, const double* x,
                     double* r, unsigned long long* norms, hipStream_t s);
// y = L^-1 (in gathered by permIn), fp64; L unit lower in S rows permS;
// Linv as written by launch_diag_inverses
// xw: [2 * ceil(n/128) * 128] tagged words, zeroed once; epoch: a new
// nonzero value per launch
void launch_trsv_lower(const void* S, int64_t ld, const int* permS, int store, int n,
                       const double* in, const int* permIn, const double* Linv, double* y,
                       uint64_t* xw, int epoch, const CycleState* gate, int step, int* abort,
                       hipStream_t s);
// y = L^-1 (A_u[permA] v) in fp64 in one launch: the lower solve's blocks
// plus workgroups that form the product (eight rows each, fp64 sums as
// launch_gemv_au) and publish its rows as tagged words in xt (2 words per
// row, sized as xw, zeroed once); epoch tags both xw and xt
void launch_atilde_lower(const void* S, int64_t ld, const int* permS, int store, int n,
                         const float* Au, int64_t lda, const int* permA, const float* v,
                         const double* Linv, double* y, uint64_t* xw, uint64_t* xt, int epoch,
                         const CycleState* gate, int step, int* abort, hipStream_t s);

// a basis [C_k, V]: kc fp64 columns, then nv columns in u
struct Basis {
  const double* c64;  // kc columns, column-major, ld ldc
  int kc;
  int64_t ldc;
  const void* v;      // nv columns in u (fp32, or fp64 when v64), column-major, ld ldv
  int nv;
  int64_t ldv;
  int v64;
};

// The first classical Gram-Schmidt pass of an Arnoldi step fused into its
// upper solve: h1 = X^T w, w = fl32(2^e z), over the basis X = [C_k, V_j]
// (fp32 V, kc + nv <= kDotsMaxCols); partial holds ceil(n/128) x (kc + nv)
// per-block sums; counter is zero on entry and reset by the last block.
// The sums are those of launch_ortho's kOrthoDots pass, bit for bit.
constexpr int kDotsMaxCols = 192;
struct TrsvDots {
  Basis X;
  double* partial;
  unsigned int* counter;
  double* h1;
};
// z = U^-1 y; out64 = 2^e z, out32 = fl32(2^e z) (either may be null); with
// dots (out32 required), also the first Gram-Schmidt pass on out32
void launch_trsv_upper(const void* S, int64_t ld, const int* permS, int store, int n,
                       const double* y, const double* Uinv, double* z, double scale,
                       double* out64, float* out32, uint64_t* xw, int epoch,
                       const CycleState* gate, int step, int* abort, hipStream_t s,
                       const TrsvDots* dots = nullptr);
// the lower (upper = false) or upper solve for nr <= 16 right-hand sides as
// nr independent solves in one launch (block-major grid): in / out
// column-major (ldi / ldo); the upper solve writes scale * solution, the
// lower solve its unscaled solution (scale is ignored);
// xw holds nr slots of xstride >= 2 * ceil(n/128) * 128 tagged words
constexpr int kTrsvMaxRhs = 16;
void launch_trsv_cols(const void* S, int64_t ld, const int* permS, int store, int n, bool upper,
                      const double* in, int64_t ldi, int nr, const double* Dinv, double* out,
                      int64_t ldo, double scale, uint64_t* xw, int64_t xstride, int epoch,
                      int* abortp, hipStream_t s);
// Linv / Uinv: 3 * ceil(n/128) blocks of 128 x 128 fp64, row-major: the
// inverses of the diagonal blocks of L and U, then the products of each
// inverse with the nearest and with the second-nearest off-diagonal block
// the solves read (lower: Linv_I L_{I,I-1}, then Linv_I L_{I,I-2}; upper:
// Uinv_I U_{I,I+1}, then Uinv_I U_{I,I+2});
// tmp: 2 * ceil(n/64) * 64 * 64 doubles (the 64 x 64 inverses of L, then of U)
constexpr int kTrsvBlock = 128;
void launch_diag_inverses(const void* S, int64_t ld, const int* permS, int store, int n,
                          double* Linv, double* Uinv, double* tmp, hipStream_t s);


enum OrthoMode { kOrthoDots = 1, kOrthoUpdate = 2, kOrthoNorm = 4, kOrthoFinish = 8 };
struct OrthoArgs {
  Basis X;
  int n;
  const void* w_in;       // vectors in u: fp32, or fp64 when X.v64
  void* w_out;            // may equal w_in
  const double* coef;     // update coefficients (kc + nv) when kOrthoUpdate
  double* dots_out;       // kc + nv inner products (kOrthoDots)
  double* norm_out;       // squared 2-norm of the (updated) vector (kOrthoNorm)
  double* partial;        // grid * (kc + nv + 1)
  unsigned int* counter;  // zeroed, reset by the last block
  // finish (Arnoldi step j): H (m+1) x m col-major, B k x m col-major
  const double* h_prev;   // first-pass coefficients (h = h_prev + coef)
  double* H;
  double* B;
  int ldh, ldb;
  int step;
  double* cs;
  double* sn;
  double* g;
  CycleState* st;
  const CycleState* gate;
  // when set (kOrthoFinish), the finish also writes the step's whole cycle
  // state there (host-mapped pinned memory the host polls); null: not written
  CycleState* st_out;
  // when set (kOrthoFinish), the finishing workgroup also writes
  // v_{j+1} = fl_u(w_out / beta) there (16-byte aligned; zero when beta is not positive)
  void* vout;
};
void launch_ortho(const OrthoArgs& a, int mode, hipStream_t s);
// the CGS2 step, the finish and the normalisation in one single-workgroup
// launch (n <= kOrthoSmallMax, kc + nv <= 192): a.dots_out = h1, a.coef =
// h2 (written), a.norm_out, a.w_out; vout = v_{j+1}.  Bit-identical to the
// three k_ortho passes and k_normalize.
constexpr int kOrthoSmallMax = 4096;
void launch_ortho_small(const OrthoArgs& a, void* vout, hipStream_t s);

// A whole GMRES cycle of Arnoldi steps (u = fp32, classical Gram-Schmidt
// twice, the forward operator) in one persistent launch of 3 ceil(n/128)
// workgroups that stay resident for the cycle (the upper and the lower
// solve's blocks, and one per 128 rows for the product, the three passes,
// the finish and v_{j+1}), every cross-workgroup hand-over through tagged
// words (the step's tag is epoch0 + j).  Bit-identical to the step's
// separate launches.  Needs n <= kCycleMaxN, m <= kCycleMaxM and all its
// workgroups resident at once (one per compute unit: at most 192 of them;
// the caller checks the device has that many):
// each first arrives on the
// zeroed words arrive[0] (the arrival count) and arrive[1] (the decision);
// when not all have arrived within arrive_us, the launch gives up before
// touching any result (arrive[1] = kCycleGaveUp; kCycleGo when it ran) and
// the caller runs the steps as separate launches instead.
constexpr int kCycleMaxN = 8192;
constexpr unsigned kCycleGo = 1;
constexpr unsigned kCycleGaveUp = 2;
constexpr int kCycleArriveUs = 500;
constexpr int kCycleMaxM = 96;
struct CycleArgs {
  // the u_f factors (rows permS), the fp64 diagonal-block inverses and
  // products (three sets each, as the triangular solves take them)
  const void* S;
  int64_t ld;
  const int* permS;
  const double* Linv;
  const double* Uinv;
  double scale;  // 2^e of the preconditioner
  // A_u (rows permA), ld lda
  const float* Au;
  int64_t lda;
  const int* permA;
  int n, kc, m, nsteps;
  // the basis: C_k (fp64, ld ldc) and V (fp32, ld ldv; column 0 = v_1 on
  // entry, columns 1 .. J written)
  const double* C;
  int64_t ldc;
  float* V;
  int64_t ldv;
  // the Hessenberg and B columns of the steps, the rotations, the Givens
  // right-hand side and the cycle state (as the finish writes them)
  double* H;
  double* B;
  int ldh, ldb;
  double* cs;
  double* sn;
  double* g;
  CycleState* st;
  // tagged exchange words, zeroed once: xt, xwL, xwU 2 ceil(n/128) 128 each
  // (the product, the lower and the upper solve), vw ceil(n/128) 128 (v_{j+1}
  // in fp32), px kCycleExchange (the passes' per-block sums), ctrl 4 (the
// verdict, then the arrival word)
  uint64_t* xt;
  uint64_t* xwL;
  uint64_t* xwU;
  uint64_t* vw;
  uint64_t* px;
  uint64_t* ctrl;
  unsigned* arrive;  // two zeroed words: the arrival count, the decision
  int arrive_us;  // the arrival wait's bound (kCycleArriveUs unless a test sets it)
  uint32_t epoch0;
  int* abortp;
};
constexpr int kCycleExchange = 3 * (kCycleMaxN / kTrsvBlock) * kCycleMaxM * 2;
void launch_cycle(const CycleArgs& a, int store, hipStream_t s);

// out (n x nout, col-major fp64, ld ldo) = X M, M (ncol x nout col-major) on device
void launch_combine(const Basis& X, int n, const double* M, int nout, double* out, int64_t ldo,
                    hipStream_t s);
// d = fl_u(d + Xd cd), r = fl_u(r - Xr cr) (u = fp32, or fp64 when v64); either
// part skipped when its vector is null
void launch_cycle_update(const Basis& Xd, const double* cd, void* d, const Basis& Xr,
                         const double* cr, void* r, int n, int v64, hipStream_t s);
// G (nx x ny, col-major) = X^T Y for fp64 Y (n x ny, ld ldy); nx <= 192,
// ny <= 96 (m <= 95, k < m)
void launch_gram(const Basis& X, const double* Y, int ny, int64_t ldy, int n, double* G,
                 double* partial, unsigned int* counter, hipStream_t s);
// out = fl_u(r / s), held in fp64 (u = fp32, or fp64 when v64)
void launch_scale_round(const double* r, double s, double* out, int n, int v64, hipStream_t st);
// x = x + s d (two roundings, no fused multiply-add); d in u
void launch_x_update(double* x, const void* d, int v64, double s, int n, hipStream_t st);
// out = fl_u(w / s)
void launch_div_u(const void* w, double s, void* out, int v64, int n, hipStream_t st);
// out[0] = max |v_i| (as bits)
void launch_maxabs(const double* v, int n, unsigned long long* out, hipStream_t st);
// out[0] = max_i sum_j |A[i][j]| (bits; zeroed here), the rows summed in the
// order of launch_ingest's row sums (bit-identical ||A||_inf)
void launch_rowsum_max(const double* A, int64_t n, int64_t lda, unsigned long long* out,
                       hipStream_t s);
// out[0..2] (device) = normwise backward error, componentwise backward error
// and forward error (NaN without has_xt) from the reduction words w:
// w[0] max |r|, w[1] max |x|, w[2] max |b|, w[3] ||A||_inf, w[kNormCw] the
// componentwise error, w[5] max |x - x_true|, w[6] max |x_true| (as bits)
void launch_errors_finish(const unsigned long long* w, int has_xt, double* out, hipStream_t s);
// sets the text gmresir_last_error returns (defined with the C ABI)
void set_last_error(const char* s);
// out[0] = max |x - x_true|, out[1] = max |x_true| (as bits)
void launch_ferr(const double* x, const double* xt, int n, unsigned long long* out,
                 hipStream_t s);
void launch_copy_f32_to_f64(const float* a, double* b, int n, hipStream_t s);
void launch_fill_i32(int* p, int v, int64_t n, hipStream_t s);
// zeroes count (<= kMaxZeroSpans) spans of 4-byte words, p[j][0 .. n[j]), in
// one launch; the spans must not overlap
constexpr int kMaxZeroSpans = 16;
struct ZeroSpans {
  int* p[kMaxZeroSpans];
  int64_t n[kMaxZeroSpans];
  int count;
};
void launch_zero_spans(const ZeroSpans& z, hipStream_t s);

// ---- double-double (u = fp64, u^2 = double-double; u_r = double-double) -----

// th + tl = A[permA[i]] . v for each row i, in double-double (A fp64)
void launch_gemv_dd(const double* A, int64_t ld, const int* permA, int n, const double* v,
                    double* th, double* tl, const CycleState* gate, int step, hipStream_t s);
// r = fl64(b - A x) with A x in double-double; norms as launch_residual
void launch_residual_dd(const double* A, int64_t ld, int n, const double* b, const double* x,
                        double* r, unsigned long long* norms, hipStream_t s);
// Blocked triangular solve with the u_f factor (rows permS of S) in
// double-double arithmetic, 64 rows per workgroup.  Right-hand side
// (inh + inl)[permIn[i]] (inl may be null: zero low parts).  The solution goes
// to yh / yl (either may be null) and, rounded to fp64 and times scale, to
// out64 (may be null).  xw: kDdWordsPerRow * ceil(n/64) * 64 tagged words,
// zeroed once; epoch: a new nonzero value per launch.
constexpr int kDdWordsPerRow = 4;
void launch_trsv_dd(const void* S, int64_t ld, const int* permS, int store, int n, bool upper,
                    const double* inh, const double* inl, const int* permIn, double* yh,
                    double* yl, double scale, double* out64, uint64_t* xw, int epoch,
                    const CycleState* gate, int step, int* abortp, hipStream_t s);

// ---- transposed system (adjoint) --------------------------------------------

// t_j = sum_i A[i][j] v_i (A row-major, fp64 when a64 else fp32; v fp64 when
// v64 else fp32), fp64 accumulation in row chunks of 128 (partial: ceil(n/128)
// x n doubles); with b: t = b - A^T x (x = v) and norms[0] = max|t|,
// norms[1] = max|x| (norms zeroed here)
void launch_colsum(const void* A, int a64, int64_t ld, int n, const void* v, int v64,
                   double* partial, const double* b, const double* x, double* t,
                   unsigned long long* norms, const CycleState* gate, int step, hipStream_t s);
// out[0] = max_j sum_i |A[i][j]| (= ||A||_1, as bits; out[1] cleared); t
// receives the column sums
void launch_colsum_abs(const double* A, int64_t ld, int n, double* partial, double* t,
                       unsigned long long* out, hipStream_t s);
// the products the transposed solves read, one 128 x 128 fp64 block per
// block row (ceil(n/128) blocks each, row-major): Uq_I = U_{I-1,I} Uinv_I,
// Lq_I = L_{I+1,I} Linv_I (Linv / Uinv as written by launch_diag_inverses)
void launch_adjacent_products_t(const void* S, int64_t ld, const int* permS, int store, int n,
                                const double* Linv, const double* Uinv, double* Lq, double* Uq,
                                hipStream_t s);
// U^T y = in (upperT = false) or L^T z = in (upperT = true) with the stored
// factor (rows permS of S), the fp64 inverses of its 128 x 128 diagonal
// blocks (transposed on use) and the products Q (Uq, Lq) above; y (may be
// null) receives the solution, out64 / out32 (either may be null) scale *
// solution scattered through permOut (null: identity); xw / epoch as for
// launch_trsv_lower
void launch_trsv_t(const void* S, int64_t ld, const int* permS, int store, int n, bool upperT,
                   const double* in, const double* Dinv, const double* Q, double* y, double scale,
                   const int* permOut, double* out64, float* out32, uint64_t* xw, int epoch,
                   const CycleState* gate, int step, int* abortp, hipStream_t s);
// the same for nr <= 8 right-hand sides as independent solves in one launch
// (one grid row each): column c reads in + c * ldi, writes y + c * ldy (y may
// be null) and out64 + c * ldo (scattered through permOut), and exchanges
// through xw + c * xstride
void launch_trsv_t_cols(const void* S, int64_t ld, const int* permS, int store, int n,
                        bool upperT, const double* in, int64_t ldi, int nr, const double* Dinv,
                        const double* Q, double* y, int64_t ldy, double scale,
                        const int* permOut, double* out64, int64_t ldo, uint64_t* xw,
                        int64_t xstride, int epoch, int* abortp, hipStream_t s);
// out = alpha x y^T (n x n row-major, leading dimension ld)
void launch_rank1(double alpha, const double* x, const double* y, int n, int64_t ld, double* out,
                  hipStream_t s);

}  // namespace gir
