// Host driver of RGMRES-IR on one MI355X: Algorithm 3 of Oktay & Carson
// (refinement loop) with the GCRO-DR correction solver of Section 2, and the
// extern "C" boundary declared in include/gmresir.h.
//
// Control lives on the host; every vector operation runs in the HIP kernels
// of kernels_lu.hip / kernels_solve.hip.  Inside an Arnoldi cycle the host
// only enqueues work: convergence of the Givens estimate is detected on the
// device, later steps of the cycle turn into no-ops, and the host polls the
// device state one step behind the work it has queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/gmresir.h"
#include "host_la.h"
#include "kernels.h"

namespace {

thread_local std::string g_last_error;

void set_error(const std::string& s) { g_last_error = s; }

}  // namespace

namespace gir {
// the text gmresir_last_error returns, for the entry points of other files
void set_last_error(const char* s) { set_error(s); }
}  // namespace gir

namespace {

#define GIR_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_) + " (" __FILE__ ":" + \
                std::to_string(__LINE__) + ")");                                      \
      return GMRESIR_EHIP;                                                            \
    }                                                                                 \
  } while (0)

#define GIR_TRY(expr)          \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != 0) return rc_;  \
  } while (0)

constexpr int kEventRing = 4;   // events of the Arnoldi loop (> kLaunchAhead + 1)
constexpr int kNb = 64;           // LU block size (sets the u_f rounding points)
constexpr int kMaxM = 95;         // limit from the skinny-product kernels
constexpr int kLaunchAhead = 1;   // Arnoldi steps queued before polling

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int store_of(int uf) {
  switch (uf) {
    case GMRESIR_FP16: return gir::kStoreF16;
    case GMRESIR_BF16: return gir::kStoreBF16;
    default: return gir::kStoreF32;
  }
}

size_t store_bytes(int store) { return store == gir::kStoreF32 ? 4 : 2; }

int prec_rank(int p) {
  switch (p) {
    case GMRESIR_BF16:
    case GMRESIR_FP16: return 0;
    case GMRESIR_FP32: return 1;
    case GMRESIR_FP64: return 2;
    case GMRESIR_DD: return 3;
    default: return -1;
  }
}

// Largest integer e with 2^e * amax * sqrt(n) <= 2^-4 * 65504 (fp16 range
// headroom for the element growth of partial pivoting).
int scale_exponent(double amax, int64_t n) {
  if (!(amax > 0.0) || !std::isfinite(amax)) return 0;
  const double t = amax * std::sqrt((double)std::max<int64_t>(n, 1));
  const double limit = 4094.0;
  int e = (int)std::floor(std::log2(limit) - std::log2(t));
  while (std::ldexp(t, e) > limit) --e;
  while (std::ldexp(t, e + 1) <= limit) ++e;
  return e;
}

// Device memory released by handles is kept by the process (up to
// kCacheBytes in all) and handed out again for requests of the same size on
// the same device, so repeated factorisations of systems of one order call
// neither hipMalloc nor hipFree (which waits for the whole device) after the
// first.  Every entry point is blocking, so a released chunk has no work
// pending on it.  The cache is never torn down: its memory returns to the
// system when the process ends.
constexpr size_t kCacheBytes = size_t(16) << 30;

struct ChunkCache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void*> free_chunks;  // (device, bytes) -> chunk
  size_t cached = 0;
};

ChunkCache& chunk_cache() {
  static ChunkCache* c = new ChunkCache();  // never destroyed (see above)
  return *c;
}

hipError_t chunk_alloc(void** p, size_t bytes, int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  *dev_out = dev;
  {
    ChunkCache& c = chunk_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.free_chunks.find({dev, bytes});
    if (it != c.free_chunks.end()) {
      *p = it->second;
      c.free_chunks.erase(it);
      c.cached -= bytes;
      return hipSuccess;
    }
  }
  return hipMalloc(p, bytes);
}

// the pinned host staging of a handle, kept the same way (a handful of
// small blocks; hipHostMalloc and hipHostFree cost hundreds of microseconds)
struct PinnedCache {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;
};

PinnedCache& pinned_cache() {
  static PinnedCache* c = new PinnedCache();  // never destroyed
  return *c;
}

hipError_t pinned_alloc(void** p, size_t bytes) {
  {
    PinnedCache& c = pinned_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.free_blocks.find(bytes);
    if (it != c.free_blocks.end()) {
      *p = it->second;
      c.free_blocks.erase(it);
      return hipSuccess;
    }
  }
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void pinned_release(void* p, size_t bytes) {
  constexpr size_t kMaxPinnedBlocks = 64;
  PinnedCache& c = pinned_cache();
  {
    std::lock_guard<std::mutex> lock(c.mu);
    if (c.free_blocks.size() < kMaxPinnedBlocks) {
      c.free_blocks.emplace(bytes, p);
      return;
    }
  }
  (void)hipHostFree(p);
}

void chunk_release(void* p, size_t bytes, int dev) {
  ChunkCache& c = chunk_cache();
  {
    std::lock_guard<std::mutex> lock(c.mu);
    if (c.cached + bytes <= kCacheBytes) {
      c.free_chunks.emplace(std::make_pair(dev, bytes), p);
      c.cached += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

// Device memory of a handle: buffers above 4 MiB get their own allocation,
// smaller ones are carved from 32 MiB chunks (256-byte aligned), so that a
// handle costs a handful of chunk allocations.
// With a caller's allocator (opts.alloc / opts.free_) the chunks come from it
// instead and go back to it when the handle is freed.
struct Arena {
  struct Chunk {
    void* p;
    size_t bytes;
    int dev;
    bool user;
  };
  std::vector<Chunk> chunks;
  char* cur = nullptr;
  size_t left = 0;
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_)(void*, void*) = nullptr;
  void* user = nullptr;
  ~Arena() {
    for (const Chunk& c : chunks) {
      if (c.user)
        free_(c.p, user);
      else
        chunk_release(c.p, c.bytes, c.dev);
    }
  }
};

constexpr size_t kOwnAllocation = size_t(4) << 20;
constexpr size_t kChunk = size_t(32) << 20;

template <class T>
int dalloc(Arena& a, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = (sizeof(T) * count + 255) & ~size_t(255);
  if (bytes > kOwnAllocation || bytes > a.left) {
    void* q = nullptr;
    const size_t want = bytes > kOwnAllocation ? bytes : kChunk;
    int dev = 0;
    if (a.alloc) {
      q = a.alloc(want, a.user);
      if (!q) {
        set_error("the caller's allocator returned NULL");
        return GMRESIR_ENOMEM;
      }
      if ((reinterpret_cast<uintptr_t>(q) & 255) != 0) {
        a.free_(q, a.user);
        set_error("the caller's allocator returned memory not 256-byte aligned");
        return GMRESIR_ENOMEM;
      }
      a.chunks.push_back({q, want, 0, true});
    } else {
      hipError_t e = chunk_alloc(&q, want, &dev);
      if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return GMRESIR_ENOMEM;
      }
      a.chunks.push_back({q, want, dev, false});
    }
    if (bytes > kOwnAllocation) {
      *p = reinterpret_cast<T*>(q);
      return 0;
    }
    a.cur = reinterpret_cast<char*>(q);
    a.left = kChunk;
  }
  *p = reinterpret_cast<T*>(a.cur);
  a.cur += bytes;
  a.left -= bytes;
  return 0;
}

// kernel classes of gmresir_kernel_stats
enum KClass { kKcPanel, kKcTrsm, kKcGemm, kKcTrsvL, kKcTrsvU, kKcGemv, kKcResid, kKcOrtho,
              kKcStep, kKcCycle, kKcCount };
const char* const kKcName[kKcCount] = {"lu_panel", "lu_trsm",  "lu_gemm",  "trsv_lower",
                                       "trsv_upper", "gemv_au", "residual", "ortho",
                                       "arnoldi_step", "arnoldi_cycle"};
// the factorisation's classes count matrix-core flops, the others HBM bytes
constexpr bool kKcFlops[kKcCount] = {true,  true,  true,  false, false,
                                     false, false, false, false, false};
// bit of opts.timing that selects class c: bits 0-7 for classes 0-7, bits
// 16-23 for classes 8-15 (bits 8-15 hold the sampling stride)
constexpr int timing_bit(int c) { return c < 8 ? c : c + 8; }
struct TimedRec {
  int cls;
  double work;
  bool gated;  // launched for an Arnoldi step the device may skip
  int step;
  hipEvent_t a, b;
};
struct KStat {
  int64_t launches = 0;
  double ms = 0.0, work = 0.0;
};

}  // namespace

// The host part of a recycle-space refresh at the end of a GCRO-DR cycle (the
// harmonic Ritz problem G^T G z = theta G^T M z, the QR of G P_k) and the
// data it needs; after the last cycle of a correction solve it is deferred
// until the space is next needed, so that it overlaps the device work in
// between (x update, residual, preconditioned right-hand side).
struct Refresh {
  bool active = false;
  int kc = 0, J = 0, rows = 0, cols = 0;
  std::vector<double> Gm, Mm, dk;  // rows x cols each (column-major); D of U
};

struct gmresir_ctx {
  Arena arena;  // declared first: destroyed last
  int64_t n = 0, ld = 0;
  gmresir_opts o{};
  int store = 0;
  hipStream_t stream = nullptr;
  int status = 0;
  int singular_col = 0;
  int e = 0;
  double scale = 1.0;
  double norm_a = 0.0;   // ||A||_inf
  double norm_a1 = -1.0;  // ||A||_1 = ||A^T||_inf (computed on first use)
  int trans = 0;          // the current solve is the adjoint one (A^T lambda = g)
  double t_factor = 0.0;
  int m = 0, k = 0;
  int u64 = 0;    // working precision fp64: vectors in fp64, A-tilde in double-double
  int uni = 0;    // u = fp64 with the correction solve's products in u (uniform)
  int rdd = 0;    // residual in double-double
  size_t ue = 4;  // bytes per element of a vector in u

  // matrices
  double* A64 = nullptr;
  float* Au = nullptr;  // fl32(A) (u = fp32; for u = fp64, A_u is A64)
  void* S = nullptr;
  int* perm = nullptr;    // logical -> physical row of S
  int* permP = nullptr;   // logical -> row of A (P)
  int* permS = nullptr;   // equals perm after gmresir_factor, null after import
  int* ipiv = nullptr;
  // diagonal-block inverses, then the products with the nearest and the
  // second-nearest off-diagonal blocks (three nb x 128 x 128 sets)
  double *Linv = nullptr, *Uinv = nullptr;
  double *Lq = nullptr, *Uq = nullptr;      // the transposed solves' block products
  double* dtmp = nullptr;                    // 64 x 64 inverses of L and U (factor time)
  // LU scratch
  uint64_t* xch = nullptr;  // pivot exchange of the block-column kernel (LU only)
  int* perm_rest = nullptr;  // permutation copy read by the lookahead remainder (LU only)
  // solve buffers (length ld, zero padded)
  double *x = nullptr, *b = nullptr, *r64 = nullptr, *t64 = nullptr, *y64 = nullptr,
         *z64 = nullptr;
  // vectors in u (fp32, or fp64 when u64)
  void *zu = nullptr, *wu = nullptr, *du = nullptr, *ru = nullptr;
  void* V = nullptr;
  double *tl = nullptr, *yl = nullptr;  // low parts of the double-double products (u64)
  double *C = nullptr, *U = nullptr, *Cn = nullptr, *Un = nullptr;
  int kc_keep = 0;  // columns of U carried to the next correction solve
  // recycle set-up by Householder QR only (environment variable
  // GMRESIR_RECYCLE_QR=householder at handle creation; a test hook for the
  // branch that CholeskyQR2 breakdowns take)
  bool force_hqr = false;
  // Arnoldi steps (u = fp32) run the A_u product inside the lower solve's
  // launch; GMRESIR_FUSED_ATILDE=0 at handle creation selects the separate
  // launches (the same arithmetic)
  bool fuse_atilde = true;
  // the Arnoldi step's Gram-Schmidt passes, finish and normalisation in one
  // single-workgroup launch (1) or as three multi-workgroup passes and a
  // normalisation (0): bit-identical, chosen by timing both on this device
  // for the handle's shape (GMRESIR_ORTHO_SMALL=0/1 at handle creation
  // forces one; -1 until decided)
  int ortho_small = -1;
  // the first Gram-Schmidt pass inside the upper solve (GMRESIR_FUSED_DOTS=0
  // at handle creation: the separate pass; the same sums either way)
  bool fuse_dots = true;
  // a cycle's Arnoldi steps in one persistent launch where the shape allows
  // it (the same sums as the separate launches); GMRESIR_PERSISTENT=0 at
  // handle creation keeps the separate launches
  bool persistent = true;
  // the LU's block-row solve and the next block column's part of each
  // step's update inside the block column's launch (fp16 / bf16 factors;
  // the same factors bit for bit); GMRESIR_LU_FOLD=0 at handle creation
  // keeps their separate launches
  bool lu_fold = true;
  uint64_t *cvw = nullptr, *cpx = nullptr, *cctrl = nullptr;  // its exchange words
  int64_t cycles_run = 0;        // cycles run as one persistent launch
  int64_t cycle_fallbacks = 0;  // persistent launches that gave up (device shared)
  // after a launch gave up, the next cycles run as separate launches
  // without trying (cycle_wait of them), the wait doubling with every
  // further give-up and reset by a launch that runs
  int cycle_backoff = 0, cycle_wait = 0;
  // the persistent launch's arrival bound (GMRESIR_CYCLE_ARRIVE_US at handle
  // creation: a test hook; 0 makes every launch give up and fall back)
  int cycle_arrive_us = gir::kCycleArriveUs;
  Refresh pend;     // deferred refresh of the last cycle (V, C, U untouched meanwhile)
  // the adjoint solve's own recycle space (swapped with C, U, kc_keep while
  // it runs) and the partial sums of the products with A^T
  double *Ct = nullptr, *Ut = nullptr;
  int kc_keep_t = 0;
  double* colpart = nullptr;
  double *Hd = nullptr, *Bd = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  double *h1 = nullptr, *h2 = nullptr, *nrm = nullptr, *coefA = nullptr, *coefB = nullptr,
         *Mdev = nullptr, *Gdev = nullptr, *partial = nullptr;
  unsigned int* counter = nullptr;
  unsigned long long* norms = nullptr;
  gir::CycleState* st = nullptr;
  uint64_t *xwL = nullptr, *xwU = nullptr;  // tagged partial solutions of the two solves
  uint64_t* xt = nullptr;  // tagged rows of A_u v for the fused lower solve (u = fp32)
  uint64_t *xwLm = nullptr, *xwUm = nullptr;  // the same for the multi-vector solves
  double *Tb = nullptr, *Yb = nullptr;        // ld x 8 blocks for the multi-vector product
  int epoch = 0;
  // pinned host staging
  gir::CycleState* st_host = nullptr;  // one slot per queued step
  size_t pinned_bytes = 0;             // the pinned block st_host starts
  double* hbuf = nullptr;              // general small transfers
  size_t hbuf_len = 0;
  char *up_stage = nullptr, *dl_stage = nullptr;  // pinned staging of small transfers
  size_t up_off = 0;
  std::vector<hipEvent_t> ev;
  // launch timing (opts.timing): pooled events and pending records
  std::vector<hipEvent_t> tpool;
  size_t tnext = 0;
  std::vector<TimedRec> trec;
  KStat kstat[kKcCount];
  int64_t tcount[kKcCount] = {};  // launches per class (the timing stride)
  // phase clock of a solve: an event on the stream at each phase boundary,
  // tagged with the phase that ends there
  std::vector<hipEvent_t> pev;
  std::vector<int> pphase;
  size_t pnext = 0;

  ~gmresir_ctx() {
    // device buffers belong to `arena` (freed by its destructor)
    if (st_host) pinned_release(st_host, pinned_bytes);
    for (auto& e2 : ev) (void)hipEventDestroy(e2);
    for (auto& e2 : tpool) (void)hipEventDestroy(e2);
    for (auto& e2 : pev) (void)hipEventDestroy(e2);
  }};

namespace {

// ---------------------------------------------------------------------------
// launch timing
// ---------------------------------------------------------------------------

// bytes per element of the matrix the preconditioned product reads (A_u)
double a_bytes(const gmresir_ctx* h) { return h->u64 ? 8.0 : 4.0; }

// flops of GEPP on an h x kb block column (division and rank-1 update of the
// rows below each pivot)
double panel_flops(double hr, int kb) {
  double f = 0.0;
  for (int c = 0; c < kb; ++c) f += (hr - c - 1.0) * (1.0 + 2.0 * (kb - c - 1.0));
  return f;
}

int pool_event(gmresir_ctx* h, hipEvent_t* e) {
  if (h->tnext == h->tpool.size()) {
    hipEvent_t ne = nullptr;
    GIR_HIP(hipEventCreate(&ne));
    h->tpool.push_back(ne);
  }
  *e = h->tpool[h->tnext++];
  return 0;
}

// launch() may return nothing or a status (nonzero is passed on)
template <class Fn>
int run_launch(Fn&& launch) {
  if constexpr (std::is_same_v<decltype(launch()), int>) {
    return launch();
  } else {
    launch();
    return 0;
  }
}

// Runs launch() bracketed by two events on s when timing is on.
template <class Fn>
int timed(gmresir_ctx* h, int cls, double work, hipStream_t s, const void* gate, int step,
          Fn&& launch) {
  if (!((h->o.timing >> timing_bit(cls)) & 1)) return run_launch(launch);
  // bits 8-15: bracket only every s-th launch of the class
  const int stride = (h->o.timing >> 8) & 0xFF;
  if (stride > 1 && (h->tcount[cls]++ % stride) != 0) return run_launch(launch);
  TimedRec r{cls, work, gate != nullptr, step, nullptr, nullptr};
  GIR_TRY(pool_event(h, &r.a));
  GIR_TRY(pool_event(h, &r.b));
  GIR_HIP(hipEventRecord(r.a, s));
  GIR_TRY(run_launch(launch));
  GIR_HIP(hipEventRecord(r.b, s));
  h->trec.push_back(r);
  return 0;
}

// drop the records of gated launches from step `done` on (skipped on device)
void drop_skipped(gmresir_ctx* h, size_t from, int done) {
  size_t w = from;
  for (size_t i = from; i < h->trec.size(); ++i)
    if (!(h->trec[i].gated && h->trec[i].step >= done)) h->trec[w++] = h->trec[i];
  h->trec.resize(w);
}

int flush_timing(gmresir_ctx* h) {
  for (const TimedRec& r : h->trec) {
    GIR_HIP(hipEventSynchronize(r.b));
    float ms = 0.0f;
    GIR_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    KStat& k = h->kstat[r.cls];
    k.launches += 1;
    k.ms += ms;
    k.work += r.work;
  }
  h->trec.clear();
  h->tnext = 0;
  return 0;
}

// phases of a solve (gmresir_info's timers)
enum { kPhStart = 0, kPhX0, kPhResidual, kPhPrecond, kPhRecycle, kPhArnoldi, kPhCount };

// records the end of phase ph on the handle's stream
int phase_mark(gmresir_ctx* h, int ph) {
  if (h->pnext == h->pev.size()) {
    hipEvent_t e = nullptr;
    GIR_HIP(hipEventCreate(&e));
    h->pev.push_back(e);
    h->pphase.push_back(0);
  }
  h->pphase[h->pnext] = ph;
  GIR_HIP(hipEventRecord(h->pev[h->pnext], h->stream));
  ++h->pnext;
  return 0;
}

// stream time between consecutive marks, summed per phase (seconds); the
// stream must have passed the last mark
int phase_times(gmresir_ctx* h, double* t) {
  for (int p = 0; p < kPhCount; ++p) t[p] = 0.0;
  for (size_t i = 1; i < h->pnext; ++i) {
    float ms = 0.0f;
    GIR_HIP(hipEventElapsedTime(&ms, h->pev[i - 1], h->pev[i]));
    t[h->pphase[i]] += 1e-3 * (double)ms;
  }
  h->pnext = 0;
  return 0;
}

int validate_opts(const gmresir_opts* o) {
  if (!o) {
    set_error("opts is NULL");
    return GMRESIR_EINVAL;
  }
  if (o->struct_size != sizeof(gmresir_opts)) {
    set_error("opts.struct_size mismatch");
    return GMRESIR_EINVAL;
  }
  const int rf = prec_rank(o->uf), ru = prec_rank(o->u), rr = prec_rank(o->ur);
  if (rf != 0 && o->uf != GMRESIR_FP32) {
    set_error("uf must be FP16, BF16 or FP32");
    return GMRESIR_EINVAL;
  }
  if (o->u != GMRESIR_FP32 && o->u != GMRESIR_FP64) {
    set_error("u must be FP32 (u^2 = fp64) or FP64 (u^2 = double-double)");
    return GMRESIR_EINVAL;
  }
  if (o->ur != GMRESIR_FP64 && o->ur != GMRESIR_DD) {
    set_error("ur must be FP64 or DD");
    return GMRESIR_EINVAL;
  }
  if (!(rf <= ru && ru <= rr)) {
    set_error("precisions must satisfy uf >= u >= ur");
    return GMRESIR_EINVAL;
  }
  if (o->m < 1 || o->m > kMaxM || o->k < 0 || o->k >= o->m ||
      (o->m + 1) * std::max(o->k, 1) > 4096) {
    set_error("need 0 <= k < m <= 95 and (m + 1) k <= 4096");
    return GMRESIR_EINVAL;
  }
  if (!(o->tau > 0.0) || o->imax < 0 || o->imax > GMRESIR_MAX_STEPS || o->maxit < 0) {
    set_error("invalid tau, imax or maxit");
    return GMRESIR_EINVAL;
  }
  if (o->timing < 0 || o->timing >= (1 << timing_bit(kKcCount))) {
    set_error("timing must be a bit mask of the kernel classes (bits 0-7 and 16-23) and a "
              "stride (bits 8-15)");
    return GMRESIR_EINVAL;
  }
  if ((o->alloc == nullptr) != (o->free_ == nullptr)) {
    set_error("alloc and free_ must be given together");
    return GMRESIR_EINVAL;
  }
  if (o->ortho != 0 && o->ortho != 1) {
    set_error("ortho must be 0 (CGS2) or 1 (MGS)");
    return GMRESIR_EINVAL;
  }
  if ((o->matvec_u != 0 && o->matvec_u != 1) || (o->reuse_recycle != 0 && o->reuse_recycle != 1)) {
    set_error("matvec_u and reuse_recycle must be 0 or 1");
    return GMRESIR_EINVAL;
  }
  if (o->matvec_u && o->u != GMRESIR_FP64) {
    set_error("uniform-precision products (matvec_u) are supported for u = FP64");
    return GMRESIR_EINVAL;
  }
  return 0;
}

// Small host <-> device transfers go through pinned staging memory.  An
// upload copies into the next free piece of the staging arena and queues the
// copy without waiting; the arena is recycled after the next synchronisation
// (every download synchronises the stream, so all queued uploads are done).
constexpr size_t kStageBytes = 64 * 1024;

// one pinned block: per-step cycle states (m + 2), a general buffer of 8192
// doubles and the two staging areas
int pinned_init(gmresir_ctx* h) {
  if (h->st_host) return 0;
  const size_t st_bytes = (sizeof(gir::CycleState) * (size_t)(h->m + 2) + 255) & ~size_t(255);
  h->hbuf_len = 8192;
  const size_t total = st_bytes + sizeof(double) * h->hbuf_len + 2 * kStageBytes;
  char* p = nullptr;
  GIR_HIP(pinned_alloc(reinterpret_cast<void**>(&p), total));
  h->pinned_bytes = total;
  h->st_host = reinterpret_cast<gir::CycleState*>(p);
  h->hbuf = reinterpret_cast<double*>(p + st_bytes);
  h->up_stage = p + st_bytes + sizeof(double) * h->hbuf_len;
  h->dl_stage = h->up_stage + kStageBytes;
  return 0;
}

int stage_init(gmresir_ctx* h) { return pinned_init(h); }

// Buffers zeroed at set-up, collected and cleared by one kernel per 16 spans
// (a memset call, or a launch per buffer, costs microseconds of latency each).
struct ZeroList {
  std::vector<std::pair<void*, size_t>> spans;  // (pointer, bytes: a multiple of 4)
  void add(void* p, size_t bytes) { spans.emplace_back(p, bytes); }
  void launch(hipStream_t s) {
    for (size_t i = 0; i < spans.size(); i += gir::kMaxZeroSpans) {
      gir::ZeroSpans z{};
      z.count = (int)std::min<size_t>(gir::kMaxZeroSpans, spans.size() - i);
      for (int j = 0; j < z.count; ++j) {
        z.p[j] = static_cast<int*>(spans[i + (size_t)j].first);
        z.n[j] = (int64_t)(spans[i + (size_t)j].second / 4);
      }
      gir::launch_zero_spans(z, s);
    }
    spans.clear();
  }
};

int tune_ortho(gmresir_ctx* h);

int alloc_solve(gmresir_ctx* h) {
  const size_t ld = (size_t)h->ld;
  const int m = h->m, k = std::max(h->k, 1);
  GIR_TRY(dalloc(h->arena, &h->x, ld));
  GIR_TRY(dalloc(h->arena, &h->b, ld));
  GIR_TRY(dalloc(h->arena, &h->r64, ld));
  GIR_TRY(dalloc(h->arena, &h->t64, ld));
  GIR_TRY(dalloc(h->arena, &h->y64, ld));
  GIR_TRY(dalloc(h->arena, &h->z64, ld));
  void** uv[] = {&h->zu, &h->wu, &h->du, &h->ru};
  for (void** p : uv) GIR_TRY(dalloc(h->arena, reinterpret_cast<char**>(p), ld * h->ue));
  GIR_TRY(dalloc(h->arena, reinterpret_cast<char**>(&h->V), ld * (m + 1) * h->ue));
  GIR_TRY(dalloc(h->arena, &h->C, ld * k));
  GIR_TRY(dalloc(h->arena, &h->U, ld * k));
  GIR_TRY(dalloc(h->arena, &h->Cn, ld * k));
  GIR_TRY(dalloc(h->arena, &h->Un, ld * k));
  GIR_TRY(dalloc(h->arena, &h->Hd, (size_t)(m + 1) * m));
  GIR_TRY(dalloc(h->arena, &h->Bd, (size_t)k * m));
  GIR_TRY(dalloc(h->arena, &h->cs, m + 1));
  GIR_TRY(dalloc(h->arena, &h->sn, m + 1));
  GIR_TRY(dalloc(h->arena, &h->g, m + 2));
  GIR_TRY(dalloc(h->arena, &h->h1, 256));
  GIR_TRY(dalloc(h->arena, &h->h2, 256));
  GIR_TRY(dalloc(h->arena, &h->nrm, 4));
  GIR_TRY(dalloc(h->arena, &h->coefA, 256));
  GIR_TRY(dalloc(h->arena, &h->coefB, 256));
  // the small products of the recycle space: [C_k V] (k + m + 1 columns)
  // against at most k + 1 columns
  const size_t small = std::max<size_t>(4096, (size_t)(h->m + h->k + 2) * (size_t)(h->k + 2));
  GIR_TRY(dalloc(h->arena, &h->Mdev, small));
  GIR_TRY(dalloc(h->arena, &h->Gdev, small));
  const size_t grid = (ld + 255) / 256;
  GIR_TRY(dalloc(h->arena, &h->partial, grid * small));
  // tagged words of the two solves: 2 per row in 128-row blocks (fp64), 4 per
  // row in 64-row blocks (double-double)
  const int64_t nxw =
      h->u64 ? gir::kDdWordsPerRow * ((h->n + 63) / 64) * 64
             : 2 * ((h->n + gir::kTrsvBlock - 1) / gir::kTrsvBlock) * gir::kTrsvBlock;
  GIR_TRY(dalloc(h->arena, &h->xwL, (size_t)nxw));
  GIR_TRY(dalloc(h->arena, &h->xwU, (size_t)nxw));
  ZeroList zl;
  zl.add(h->xwL, sizeof(uint64_t) * (size_t)nxw);
  zl.add(h->xwU, sizeof(uint64_t) * (size_t)nxw);
  if (h->u64) {
    GIR_TRY(dalloc(h->arena, &h->tl, ld));
    GIR_TRY(dalloc(h->arena, &h->yl, ld));
  } else {
    // the A_u product's rows, published to the fused lower solve
    GIR_TRY(dalloc(h->arena, &h->xt, (size_t)nxw));
    zl.add(h->xt, sizeof(uint64_t) * (size_t)nxw);
    // the persistent cycle's 3 ceil(n/128) workgroups must all be resident
    // at once, one per compute unit
    int dev = 0, cus = 0;
    GIR_HIP(hipGetDevice(&dev));
    GIR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t cycle_wgs = 3 * ((h->n + gir::kTrsvBlock - 1) / gir::kTrsvBlock);
    if (h->n <= gir::kCycleMaxN && h->m <= gir::kCycleMaxM && cycle_wgs <= cus) {
      // the persistent cycle's own words: v_{j+1}, the passes' sums, the verdict
      GIR_TRY(dalloc(h->arena, &h->cvw, (size_t)nxw / 2));
      GIR_TRY(dalloc(h->arena, &h->cpx, (size_t)gir::kCycleExchange));
      GIR_TRY(dalloc(h->arena, &h->cctrl, 4));
      zl.add(h->cvw, sizeof(uint64_t) * (size_t)nxw / 2);
      zl.add(h->cpx, sizeof(uint64_t) * (size_t)gir::kCycleExchange);
      zl.add(h->cctrl, sizeof(uint64_t) * 4);
    }
  }
  if (!h->u64 && h->k > 0) {
    const int64_t nm = nxw * gir::kTrsvMaxRhs;
    GIR_TRY(dalloc(h->arena, &h->xwLm, (size_t)nm));
    GIR_TRY(dalloc(h->arena, &h->xwUm, (size_t)nm));
    zl.add(h->xwLm, sizeof(uint64_t) * (size_t)nm);
    zl.add(h->xwUm, sizeof(uint64_t) * (size_t)nm);
    GIR_TRY(dalloc(h->arena, &h->Tb, (size_t)h->ld * gir::kTrsvMaxRhs));
    GIR_TRY(dalloc(h->arena, &h->Yb, (size_t)h->ld * gir::kTrsvMaxRhs));
  }
  // zero padding of every vector
  double* dv[] = {h->x, h->b, h->r64, h->t64, h->y64, h->z64};
  for (double* p : dv) zl.add(p, sizeof(double) * ld);
  void* fv[] = {h->zu, h->wu, h->du, h->ru};
  for (void* p : fv) zl.add(p, h->ue * ld);
  zl.add(h->V, h->ue * ld * (m + 1));
  if (h->u64) {
    zl.add(h->tl, sizeof(double) * ld);
    zl.add(h->yl, sizeof(double) * ld);
  }
  zl.launch(h->stream);
  GIR_TRY(pinned_init(h));
  h->ev.resize(kEventRing);
  for (auto& e2 : h->ev) GIR_HIP(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
  return tune_ortho(h);
}

int alloc_common(gmresir_ctx* h) {
  const size_t ld = (size_t)h->ld, n = (size_t)h->n;
  GIR_TRY(dalloc(h->arena, &h->A64, n * ld));
  if (!h->u64) GIR_TRY(dalloc(h->arena, &h->Au, n * ld));
  GIR_TRY(dalloc(h->arena, reinterpret_cast<char**>(&h->S), n * ld * store_bytes(h->store)));
  GIR_TRY(dalloc(h->arena, &h->perm, n));
  GIR_TRY(dalloc(h->arena, &h->ipiv, n));
  if (!h->u64 || h->uni) {
    // fp64 inverses of the diagonal blocks (the double-double solves
    // substitute within the block instead)
    const size_t nb2 = (n + gir::kTrsvBlock - 1) / gir::kTrsvBlock;
    GIR_TRY(dalloc(h->arena, &h->Linv, 3 * nb2 * gir::kTrsvBlock * gir::kTrsvBlock));
    GIR_TRY(dalloc(h->arena, &h->Uinv, 3 * nb2 * gir::kTrsvBlock * gir::kTrsvBlock));
    GIR_TRY(dalloc(h->arena, &h->dtmp, 2 * ((n + 63) / 64) * 64 * 64));
  }
  GIR_TRY(dalloc(h->arena, &h->st, 1));
  GIR_TRY(dalloc(h->arena, &h->counter, 8));
  GIR_TRY(dalloc(h->arena, &h->norms, 8));
  ZeroList zl;
  zl.add(h->st, sizeof(gir::CycleState));
  zl.add(h->counter, sizeof(unsigned) * 8);
  zl.launch(h->stream);
  return 0;
}

// Small transfers (whole 4-byte words) are done by a copy kernel that reads or
// writes the mapped pinned staging memory directly, which keeps them off the
// copy engines (tens of microseconds of latency each).
struct Piece {
  void* dst;
  const void* src;
  size_t bytes;
};
int upload(gmresir_ctx* h, void* dst, const void* src, size_t bytes) {
  GIR_TRY(stage_init(h));
  if (bytes > kStageBytes || bytes % 4 != 0) {
    GIR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
    GIR_HIP(hipStreamSynchronize(h->stream));
    h->up_off = 0;
    return 0;
  }
  if (h->up_off + bytes > kStageBytes) {
    GIR_HIP(hipStreamSynchronize(h->stream));
    h->up_off = 0;
  }
  char* p = h->up_stage + h->up_off;
  std::memcpy(p, src, bytes);
  gir::launch_copy_words(dst, p, (int64_t)(bytes / 4), h->stream);
  GIR_HIP(hipGetLastError());
  h->up_off += (bytes + 255) & ~size_t(255);
  return 0;
}

int download(gmresir_ctx* h, void* dst, const void* src, size_t bytes) {
  GIR_TRY(stage_init(h));
  if (bytes > kStageBytes || bytes % 4 != 0) {
    GIR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
    GIR_HIP(hipStreamSynchronize(h->stream));
  } else {
    gir::launch_copy_words(h->dl_stage, src, (int64_t)(bytes / 4), h->stream);
    GIR_HIP(hipGetLastError());
    GIR_HIP(hipStreamSynchronize(h->stream));
    std::memcpy(dst, h->dl_stage, bytes);
  }
  h->up_off = 0;
  return 0;
}

// Several host-to-device copies in stream order: staged pieces go in one copy
// launch (up to eight per launch); a piece that does not fit is copied as
// upload copies it, after the staged ones before it have been launched.
int upload_many(gmresir_ctx* h, std::initializer_list<Piece> pieces) {
  GIR_TRY(stage_init(h));
  gir::CopyPieces cp{};
  auto flush = [&] {
    gir::launch_copy_pieces(cp, h->stream);
    cp.count = 0;
  };
  for (const Piece& p : pieces) {
    if (p.bytes == 0) continue;
    if (p.bytes > kStageBytes || p.bytes % 4 != 0) {
      flush();
      GIR_TRY(upload(h, p.dst, p.src, p.bytes));
      continue;
    }
    if (h->up_off + p.bytes > kStageBytes) {
      flush();
      GIR_HIP(hipStreamSynchronize(h->stream));
      h->up_off = 0;
    }
    if (cp.count == gir::kCopyPieces) flush();
    char* st = h->up_stage + h->up_off;
    std::memcpy(st, p.src, p.bytes);
    cp.dst[cp.count] = p.dst;
    cp.src[cp.count] = st;
    cp.words[cp.count] = (int64_t)(p.bytes / 4);
    ++cp.count;
    h->up_off += (p.bytes + 255) & ~size_t(255);
  }
  flush();
  GIR_HIP(hipGetLastError());
  return 0;
}

// Several device-to-host copies with one synchronisation: the pieces go
// through the pinned download staging in one copy launch (up to eight per
// launch; hipMemcpyAsync for a piece that does not fit), then the stream is
// synchronised once.
int download_many(gmresir_ctx* h, std::initializer_list<Piece> pieces) {
  GIR_TRY(stage_init(h));
  size_t off = 0;
  std::vector<std::pair<const Piece*, size_t>> staged;
  gir::CopyPieces cp{};
  for (const Piece& p : pieces) {
    if (p.bytes == 0) continue;
    if (p.bytes % 4 == 0 && off + p.bytes <= kStageBytes) {
      if (cp.count == gir::kCopyPieces) {
        gir::launch_copy_pieces(cp, h->stream);
        cp.count = 0;
      }
      cp.dst[cp.count] = h->dl_stage + off;
      cp.src[cp.count] = p.src;
      cp.words[cp.count] = (int64_t)(p.bytes / 4);
      ++cp.count;
      staged.push_back({&p, off});
      off += (p.bytes + 255) & ~size_t(255);
    } else {
      GIR_HIP(hipMemcpyAsync(p.dst, p.src, p.bytes, hipMemcpyDeviceToHost, h->stream));
    }
  }
  gir::launch_copy_pieces(cp, h->stream);
  GIR_HIP(hipGetLastError());
  GIR_HIP(hipStreamSynchronize(h->stream));
  for (const auto& st : staged) std::memcpy(st.first->dst, h->dl_stage + st.second, st.first->bytes);
  h->up_off = 0;
  return 0;
}

// Copies of A (fp64 and fp32, zero padded), ||A||_inf, max |a|, the
// non-finite check and, with make_lu_copy, A_f = fl_uf(2^e A) with the scale
// exponent chosen on the device: no host round trip.  ingest_finish reads the
// results back after the next synchronisation.
int ingest(gmresir_ctx* h, const double* A, int64_t lda, bool make_lu_copy) {
  const int64_t n = h->n, ld = h->ld;
  unsigned long long* norms = h->norms;  // [0] max|a|, [1] max row sum
  int* iflag = reinterpret_cast<int*>(h->counter + 4);
  int* e_dev = reinterpret_cast<int*>(h->counter + 5);
  gir::launch_fill_i32(reinterpret_cast<int*>(norms), 0, 4, h->stream);
  gir::launch_fill_i32(iflag, 0, 2, h->stream);
  gir::launch_ingest(A, n, lda, h->A64, h->Au, ld, norms, iflag, h->stream);
  if (make_lu_copy) {
    const bool scaled =
        (h->o.scale_pow2 < 0) ? (h->o.uf == GMRESIR_FP16) : (h->o.scale_pow2 != 0);
    gir::launch_convert_scaled(h->A64, n, ld, h->store, h->S, norms,
                               std::sqrt((double)std::max<int64_t>(n, 1)), scaled ? 1 : 0, e_dev,
                               iflag, h->stream);
  }
  GIR_HIP(hipGetLastError());
  return 0;
}

// the scalars the ingest leaves on the device: ||A||_inf (bits), the
// non-finite flag and the scale exponent
struct IngestScalars {
  unsigned long long hv[2];
  int hi[2];
};

Piece ingest_piece_norms(gmresir_ctx* h, IngestScalars& r) {
  return Piece{r.hv, h->norms, sizeof(r.hv)};
}
Piece ingest_piece_flags(gmresir_ctx* h, IngestScalars& r) {
  return Piece{r.hi, h->counter + 4, sizeof(r.hi)};
}

void ingest_apply(gmresir_ctx* h, const IngestScalars& r, bool has_e) {
  double rowsum;
  std::memcpy(&rowsum, &r.hv[1], 8);
  h->norm_a = rowsum;
  if (has_e) {
    h->e = r.hi[1];
    h->scale = std::ldexp(1.0, h->e);
  }
  if (r.hi[0]) h->status = GMRESIR_ERANGE;
}

int ingest_finish(gmresir_ctx* h, bool has_e) {
  IngestScalars r{};
  GIR_TRY(download_many(h, {ingest_piece_norms(h, r), ingest_piece_flags(h, r)}));
  ingest_apply(h, r, has_e);
  return 0;
}

int run_lu(gmresir_ctx* h) {
  const int n = (int)h->n;
  gir::launch_iota(h->perm, n, h->stream);
  uint64_t* xch = nullptr;
  GIR_TRY(dalloc(h->arena, &xch, (size_t)gir::kPanelXchWords));
  h->xch = xch;
  gir::launch_fill_i32(reinterpret_cast<int*>(xch), 0, 2 * gir::kPanelXchWords, h->stream);
  gir::PanelArgs a{};
  a.S = h->S;
  a.ld = h->ld;
  a.n = n;
  a.perm = h->perm;
  a.ipiv = h->ipiv;
  a.xch = xch;
  a.st = h->st;
  // Lookahead on one stream.  Step k: the block row right of block column k
  // is solved (TRSM, all columns), the next block column k + 1 is updated
  // (trailing GEMM on its 64 columns), then one launch factors block column
  // k + 1 while its other workgroups apply step k's update to the columns
  // beyond it.  That remainder locates the trailing rows through the copy of
  // the permutation written by block column k (two copies, alternating),
  // because block column k + 1 rewrites perm at the same time.
  hipStream_t s0 = h->stream;
  int* prow = nullptr;
  GIR_TRY(dalloc(h->arena, &prow, 2 * (size_t)n));
  h->perm_rest = prow;
  int dev = 0, cus = 0;
  GIR_HIP(hipGetDevice(&dev));
  GIR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // arrival counters of the update tiles that also solve the block row: one
  // row per step, one counter per 128-column strip, zeroed once
  const int64_t strip_stride = (n + 127) / 128 + 1;
  const int64_t nstrip = ((int64_t)n / kNb + 2) * strip_stride;
  int* strip_cnt = nullptr;
  GIR_TRY(dalloc(h->arena, &strip_cnt, (size_t)nstrip));
  gir::launch_fill_i32(strip_cnt, 0, nstrip, s0);
  // work of each launch for the timing records: flops (panel GEPP, the
  // block-row solve, the rank-kb trailing products)
  int step = 0;
  for (int k0 = 0; k0 < n; k0 += kNb, ++step) {
    a.k0 = k0;
    a.kb = std::min(kNb, n - k0);
    const double hr = (double)(n - k0), kb = (double)a.kb, M = hr - kb;
    int* pcopy = prow + (size_t)(step & 1) * n;  // written by block column `step`
    if (k0 == 0) {
      a.perm_copy = pcopy;
      GIR_TRY(timed(h, kKcPanel, panel_flops(hr, a.kb), s0, nullptr, 0,
                    [&] { gir::launch_panel_step(a, h->store, s0); }));
    }
    if (M <= 0) break;
    const int c1 = k0 + a.kb;                // next block column
    const int c2 = std::min(n, c1 + kNb);    // ... and the columns beyond it
    // the block row's solve and the next block column's part of this step's
    // update: their own launches, or (fp16 / bf16 factors, a further block
    // column beyond the next) formed inside the block column's launch.  The
    // solve moves in only while the update is small: each update tile then
    // solves its own columns again, and beyond about 5.5 rounds of tiles
    // over the compute units that work made the update, not the pivot
    // search, the launch's critical path (measured at n = 8192: from 1 300
    // tiles on, the separate solve launch is cheaper)
    const bool fold = h->lu_fold && c2 < n && gir::panel_update_folds(h->store);
    const int64_t tiles = ((int64_t)(n - c2) + 127) / 128 * (((int64_t)M + 127) / 128);
    const bool fold_solve = fold && tiles * 2 <= 11 * (int64_t)cus;
    if (!fold_solve)
      GIR_TRY(timed(h, kKcTrsm, kb * (kb - 1.0) * (n - c1), s0, nullptr, 0,
                    [&] { gir::launch_trsm(a, h->store, c1, n, s0); }));
    if (!fold)
      GIR_TRY(timed(h, kKcGemm, 2.0 * M * (c2 - c1) * kb, s0, nullptr,
                    0, [&] { gir::launch_gemm_update(a, h->store, h->perm, c1, c2, s0); }));
    gir::PanelArgs an = a;
    an.k0 = c1;
    an.kb = std::min(kNb, n - c1);
    an.perm_copy = prow + (size_t)((step + 1) & 1) * n;
    const double hn = (double)(n - c1);
    const double pflops = panel_flops(hn, an.kb) + (fold ? 2.0 * M * (c2 - c1) * kb : 0.0) +
                          (fold_solve ? kb * (kb - 1.0) * (n - c1) : 0.0);
    if (c2 < n) {
      const double gflops = 2.0 * M * (n - c2) * kb;
      GIR_TRY(timed(h, kKcPanel, pflops + gflops, s0, nullptr, 0, [&] {
        gir::launch_panel_update(an, a, h->store, pcopy, c2, n, fold_solve ? 2 : fold ? 1 : 0,
                                 strip_cnt + (size_t)step * strip_stride, s0);
      }));
    } else {
      GIR_TRY(timed(h, kKcPanel, pflops, s0, nullptr, 0,
                    [&] { gir::launch_panel_step(an, h->store, s0); }));
    }
  }
  GIR_HIP(hipGetLastError());
  int* flag = reinterpret_cast<int*>(h->counter + 2);
  gir::launch_fill_i32(flag, 0, 1, h->stream);
  gir::launch_check_factors(h->S, n, h->ld, h->store, flag, h->stream);
  if (!h->u64 || h->uni)
    gir::launch_diag_inverses(h->S, h->ld, h->perm, h->store, n, h->Linv, h->Uinv, h->dtmp,
                              h->stream);
  // the factorisation's state and the ingest's scalars in one round trip
  gir::CycleState hs{};
  int hflag = 0;
  IngestScalars ir{};
  GIR_TRY(download_many(h, {{&hs, h->st, sizeof(hs)},
                            {&hflag, flag, sizeof(int)},
                            ingest_piece_norms(h, ir),
                            ingest_piece_flags(h, ir)}));
  ingest_apply(h, ir, true);
  if (hs.abort) {
    set_error("LU: a device-side wait exceeded its bound");
    return GMRESIR_EINTERNAL;
  }
  if (h->status == GMRESIR_ERANGE) {
    // non-finite A: the factors are meaningless; nothing more to report
  } else if (hs.singular) {
    h->status = GMRESIR_ESINGULAR;
    h->singular_col = hs.singular;
  } else if (hflag) {
    h->status = GMRESIR_ERANGE;
  }

  return 0;
}

int make_ctx(const double* A, int64_t n, int64_t lda, const gmresir_opts* opts, void* stream,
             gmresir_ctx** out, gmresir_ctx** hp) {
  if (!out) {
    set_error("out is NULL");
    return GMRESIR_EINVAL;
  }
  *out = nullptr;
  GIR_TRY(validate_opts(opts));
  if (!A || n <= 0 || lda < n || n > 16384) {
    set_error("invalid A, n (1..16384) or lda");
    return GMRESIR_EINVAL;
  }
  gmresir_ctx* h = new (std::nothrow) gmresir_ctx();
  if (!h) return GMRESIR_ENOMEM;
  h->n = n;
  h->ld = (n + 63) / 64 * 64;
  {
    const char* q = std::getenv("GMRESIR_RECYCLE_QR");
    h->force_hqr = q && std::strcmp(q, "householder") == 0;
    const char* f = std::getenv("GMRESIR_FUSED_ATILDE");
    h->fuse_atilde = !(f && std::strcmp(f, "0") == 0);
    const char* fd = std::getenv("GMRESIR_FUSED_DOTS");
    h->fuse_dots = !(fd && std::strcmp(fd, "0") == 0);
    const char* pe = std::getenv("GMRESIR_PERSISTENT");
    h->persistent = !(pe && std::strcmp(pe, "0") == 0);
    const char* lf = std::getenv("GMRESIR_LU_FOLD");
    h->lu_fold = !(lf && std::strcmp(lf, "0") == 0);
    const char* au = std::getenv("GMRESIR_CYCLE_ARRIVE_US");
    if (au && *au) h->cycle_arrive_us = std::max(0, std::min(1000000, std::atoi(au)));
    const char* os = std::getenv("GMRESIR_ORTHO_SMALL");
    if (os && (std::strcmp(os, "0") == 0 || std::strcmp(os, "1") == 0))
      h->ortho_small = os[0] - '0';
  }
  h->o = *opts;
  h->arena.alloc = opts->alloc;
  h->arena.free_ = opts->free_;
  h->arena.user = opts->alloc_user;
  h->m = opts->m;
  h->k = opts->k;
  h->store = store_of(opts->uf);
  h->u64 = opts->u == GMRESIR_FP64 ? 1 : 0;
  h->uni = (h->u64 && opts->matvec_u) ? 1 : 0;
  h->rdd = opts->ur == GMRESIR_DD ? 1 : 0;
  h->ue = h->u64 ? 8 : 4;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  *hp = h;
  return 0;
}

// ---------------------------------------------------------------------------
// solve phase
// ---------------------------------------------------------------------------

int next_epoch(gmresir_ctx* h) {
  if (++h->epoch >= 0x3fffffff) h->epoch = 1;
  return h->epoch;
}

// count consecutive epochs; the first is returned
int reserve_epochs(gmresir_ctx* h, int count) {
  if (h->epoch + count + 1 >= 0x3fffffff) h->epoch = 0;
  const int e0 = h->epoch + 1;
  h->epoch += count;
  return e0;
}

// M^-1 in = 2^e U^-1 L^-1 P in (P applied by gather through permIn) in u^2:
// fp64 for u = fp32, double-double for u = fp64 (inl: low parts of in, or
// null).  The result goes to out64 (fp64) or outu (rounded to u), either may
// be null.
// M^-T in = 2^e P^T L^-T U^-T in in fp64 (the adjoint system; u = fp32):
// the solve with U^T, then with L^T, scattered through P^T
int precond_t(gmresir_ctx* h, const double* in, double* out64, void* outu,
              const gir::CycleState* gate, int step) {
  const int n = (int)h->n;
  const double bytes = 0.5 * (double)n * (double)(n + 1) * (double)store_bytes(h->store) +
                       24.0 * (double)n;
  const int eL = next_epoch(h);
  GIR_TRY(timed(h, kKcTrsvL, bytes, h->stream, gate, step, [&] {
    gir::launch_trsv_t(h->S, h->ld, h->permS, h->store, n, false, in, h->Uinv, h->Uq, h->y64, 1.0,
                       nullptr, nullptr, nullptr, h->xwL, eL, gate, step, &h->st->abort,
                       h->stream);
  }));
  const int eU = next_epoch(h);
  GIR_TRY(timed(h, kKcTrsvU, bytes, h->stream, gate, step, [&] {
    gir::launch_trsv_t(h->S, h->ld, h->permS, h->store, n, true, h->y64, h->Linv, h->Lq, nullptr,
                       h->scale, h->permP, out64, static_cast<float*>(outu), h->xwU, eU, gate,
                       step, &h->st->abort, h->stream);
  }));
  return 0;
}

int precond(gmresir_ctx* h, const double* in, const double* inl, const int* permIn, double* out64,
            void* outu, const gir::CycleState* gate, int step, bool correction = false,
            const gir::TrsvDots* dots = nullptr) {
  const int n = (int)h->n;
  if (h->trans) return precond_t(h, in, out64, outu, gate, step);
  if (h->uni && correction) {
    // uniform precision: the fp64 solves (u = fp64)
    const double bytes = 0.5 * (double)n * (double)(n + 1) * (double)store_bytes(h->store) +
                         24.0 * (double)n;
    double* out = out64 ? out64 : static_cast<double*>(outu);
    const int eL = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvL, bytes, h->stream, gate, step, [&] {
      gir::launch_trsv_lower(h->S, h->ld, h->permS, h->store, n, in, permIn, h->Linv, h->y64,
                             h->xwL, eL, gate, step, &h->st->abort, h->stream);
    }));
    const int eU = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvU, bytes, h->stream, gate, step, [&] {
      gir::launch_trsv_upper(h->S, h->ld, h->permS, h->store, n, h->y64, h->Uinv, h->z64,
                             h->scale, out, nullptr, h->xwU, eU, gate, step, &h->st->abort,
                             h->stream);
    }));
    return 0;
  }
  // the stored triangle and the vectors read and written
  const double tri = 0.5 * (double)n * (double)(n + 1) * (double)store_bytes(h->store);
  if (h->u64) {
    double* out = out64 ? out64 : static_cast<double*>(outu);
    const int eL = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvL, tri + 32.0 * n, h->stream, gate, step, [&] {
      gir::launch_trsv_dd(h->S, h->ld, h->permS, h->store, n, false, in, inl, permIn, h->y64,
                          h->yl, 1.0, nullptr, h->xwL, eL, gate, step, &h->st->abort, h->stream);
    }));
    const int eU = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvU, tri + 24.0 * n, h->stream, gate, step, [&] {
      gir::launch_trsv_dd(h->S, h->ld, h->permS, h->store, n, true, h->y64, h->yl, nullptr,
                          nullptr, nullptr, h->scale, out, h->xwU, eU, gate, step,
                          &h->st->abort, h->stream);
    }));
    return 0;
  }
  const double bytes = tri + 24.0 * (double)n;
  float* out32 = static_cast<float*>(outu);
  const int eL = next_epoch(h);
  GIR_TRY(timed(h, kKcTrsvL, bytes, h->stream, gate, step, [&] {
    gir::launch_trsv_lower(h->S, h->ld, h->permS, h->store, n, in, permIn, h->Linv, h->y64,
                           h->xwL, eL, gate, step, &h->st->abort, h->stream);
  }));
  const int eU = next_epoch(h);
  GIR_TRY(timed(h, kKcTrsvU, bytes, h->stream, gate, step, [&] {
    gir::launch_trsv_upper(h->S, h->ld, h->permS, h->store, n, h->y64, h->Uinv, h->z64,
                           h->scale, out64, out32, h->xwU, eU, gate, step, &h->st->abort,
                           h->stream, dots);
  }));
  return 0;
}

// A-tilde v for v in u (vu) or in fp64 (v64): the product with A_u in u^2
// (fp64, or double-double from A itself for u = fp64), then M^-1
// the Arnoldi step's first Gram-Schmidt pass runs inside the upper solve
// (fp32 basis, classical Gram-Schmidt in its multi-workgroup form, the
// forward operator; GMRESIR_FUSED_DOTS=0 at handle creation keeps the
// separate pass)
bool fuse_first_dots(const gmresir_ctx* h) {
  return h->fuse_dots && !h->trans && !h->u64 && !h->uni && h->o.ortho == 0 &&
         h->ortho_small == 0;
}

// dots (u = fp32 only): the Arnoldi step's first Gram-Schmidt pass on the
// result, fused into the upper solve
int atilde(gmresir_ctx* h, const void* vu, const double* v64, double* out64, void* outu,
           const gir::CycleState* gate, int step, const gir::TrsvDots* dots = nullptr) {
  const double nn = (double)h->n;
  if (h->trans) {
    // A_u^T v (column sums in fp64), then M^-T
    GIR_TRY(timed(h, kKcGemv, 4.0 * nn * nn + 12.0 * nn, h->stream, gate, step, [&] {
      gir::launch_colsum(h->Au, 0, h->ld, (int)h->n, vu ? vu : static_cast<const void*>(v64),
                         vu ? 0 : 1, h->colpart, nullptr, nullptr, h->t64, nullptr, gate, step,
                         h->stream);
    }));
    return precond_t(h, h->t64, out64, outu, gate, step);
  }
  if (h->uni) {
    const double* v = vu ? static_cast<const double*>(vu) : v64;
    GIR_TRY(timed(h, kKcGemv, 8.0 * nn * nn + 24.0 * nn, h->stream, gate, step, [&] {
      gir::launch_gemv_a64(h->A64, h->ld, h->permP, (int)h->n, v, h->t64, gate, step,
                           h->stream);
    }));
    return precond(h, h->t64, nullptr, nullptr, out64, outu, gate, step, true);
  }
  if (h->u64) {
    const double* v = vu ? static_cast<const double*>(vu) : v64;
    GIR_TRY(timed(h, kKcGemv, 8.0 * nn * nn + 24.0 * nn, h->stream, gate, step, [&] {
      gir::launch_gemv_dd(h->A64, h->ld, h->permP, (int)h->n, v, h->t64, h->tl, gate, step,
                          h->stream);
    }));
    return precond(h, h->t64, h->tl, nullptr, out64, outu, gate, step);
  }
  const float* v32 = static_cast<const float*>(vu);
  if (v32 && h->fuse_atilde) {
    // the product and the lower solve in one launch, then the upper solve
    const double tri = 0.5 * nn * (nn + 1.0) * (double)store_bytes(h->store);
    const int eL = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvL, 4.0 * nn * nn + 4.0 * nn + tri + 16.0 * nn, h->stream, gate, step,
                  [&] {
                    gir::launch_atilde_lower(h->S, h->ld, h->permS, h->store, (int)h->n, h->Au,
                                             h->ld, h->permP, v32, h->Linv, h->y64, h->xwL, h->xt,
                                             eL, gate, step, &h->st->abort, h->stream);
                  }));
    const int eU = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvU, tri + 24.0 * nn, h->stream, gate, step, [&] {
      gir::launch_trsv_upper(h->S, h->ld, h->permS, h->store, (int)h->n, h->y64, h->Uinv, h->z64,
                             h->scale, out64, static_cast<float*>(outu), h->xwU, eU, gate, step,
                             &h->st->abort, h->stream, dots);
    }));
    return 0;
  }
  GIR_TRY(timed(h, kKcGemv, 4.0 * nn * nn + (v32 ? 4.0 : 8.0) * nn + 8.0 * nn, h->stream, gate,
                step, [&] {
                  gir::launch_gemv_au(h->Au, h->ld, h->permP, (int)h->n, v32, v64, h->t64, gate,
                                      step, h->stream);
                }));
  return precond(h, h->t64, nullptr, nullptr, out64, outu, gate, step, false, dots);
}

// C(:, 0:kk) = A-tilde Y(:, 0:kk) for fp64 columns (ld apart): the products
// with A_u (or A_u^T) for up to sixteen columns, then the two triangular solves
// for those columns in one launch each (double-double: one column at a time)
int atilde_block(gmresir_ctx* h, const double* Y, int kk, double* C) {
  const int n = (int)h->n;
  const int64_t ld = h->ld;
  const int64_t xstride = 2 * ((h->n + gir::kTrsvBlock - 1) / gir::kTrsvBlock) * gir::kTrsvBlock;
  const double nn = (double)n;
  const double tbytes = 0.5 * nn * (nn + 1.0) * (double)store_bytes(h->store);
  if (h->trans && !h->u64) {
    // A_u^T one column at a time, then M^-T for up to sixteen columns at once
    for (int c0 = 0; c0 < kk; c0 += gir::kTrsvMaxRhs) {
      const int nr = std::min(gir::kTrsvMaxRhs, kk - c0);
      for (int c = 0; c < nr; ++c)
        GIR_TRY(timed(h, kKcGemv, 4.0 * nn * nn + 12.0 * nn, h->stream, nullptr, 0, [&] {
          gir::launch_colsum(h->Au, 0, ld, n, Y + (size_t)(c0 + c) * ld, 1, h->colpart, nullptr,
                             nullptr, h->Tb + (size_t)c * ld, nullptr, nullptr, 0, h->stream);
        }));
      const int eL = next_epoch(h);
      GIR_TRY(timed(h, kKcTrsvL, tbytes + 16.0 * nr * nn, h->stream, nullptr, 0, [&] {
        gir::launch_trsv_t_cols(h->S, ld, h->permS, h->store, n, false, h->Tb, ld, nr, h->Uinv,
                                h->Uq, h->Yb, ld, 1.0, nullptr, nullptr, 0, h->xwLm, xstride, eL,
                                &h->st->abort, h->stream);
      }));
      const int eU = next_epoch(h);
      GIR_TRY(timed(h, kKcTrsvU, tbytes + 16.0 * nr * nn, h->stream, nullptr, 0, [&] {
        gir::launch_trsv_t_cols(h->S, ld, h->permS, h->store, n, true, h->Yb, ld, nr, h->Linv,
                                h->Lq, nullptr, 0, h->scale, h->permP, C + (size_t)c0 * ld, ld,
                                h->xwUm, xstride, eU, &h->st->abort, h->stream);
      }));
    }
    return 0;
  }
  if (h->u64) {
    for (int c = 0; c < kk; ++c)
      GIR_TRY(atilde(h, nullptr, Y + (size_t)c * ld, C + (size_t)c * ld, nullptr, nullptr, 0));
    return 0;
  }
  for (int c0 = 0; c0 < kk; c0 += gir::kTrsvMaxRhs) {
    const int nr = std::min(gir::kTrsvMaxRhs, kk - c0);
    // A_u read once for the chunk's columns
    GIR_TRY(timed(h, kKcGemv, 4.0 * nn * nn + 16.0 * nn * nr, h->stream, nullptr, 0, [&] {
      gir::launch_gemv_au_multi(h->Au, ld, h->permP, n, Y + (size_t)c0 * ld, ld, nr, h->Tb, ld,
                                h->stream);
    }));
    const int eL = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvL, tbytes + 16.0 * nr * nn, h->stream, nullptr, 0, [&] {
      gir::launch_trsv_cols(h->S, ld, h->permS, h->store, n, false, h->Tb, ld, nr, h->Linv,
                            h->Yb, ld, 1.0, h->xwLm, xstride, eL, &h->st->abort, h->stream);
    }));
    const int eU = next_epoch(h);
    GIR_TRY(timed(h, kKcTrsvU, tbytes + 16.0 * nr * nn, h->stream, nullptr, 0, [&] {
      gir::launch_trsv_cols(h->S, ld, h->permS, h->store, n, true, h->Yb, ld, nr, h->Uinv,
                            C + (size_t)c0 * ld, ld, h->scale, h->xwUm, xstride, eU,
                            &h->st->abort, h->stream);
    }));
  }
  return 0;
}

// fp64 columns c (kc of them) followed by nv columns v in u
gir::Basis basis(const gmresir_ctx* h, const double* c, int kc, int64_t ldc, const void* v,
                 int nv, int64_t ldv) {
  gir::Basis X;
  X.c64 = c;
  X.kc = kc;
  X.ldc = ldc;
  X.v = v;
  X.nv = nv;
  X.ldv = ldv;
  X.v64 = h->u64;
  return X;
}

// column j of V
void* vcol(gmresir_ctx* h, int j) { return static_cast<char*>(h->V) + (size_t)j * h->ld * h->ue; }

// ---------------------------------------------------------------------------
// Autotuning by measurement.  Where two kernel variants give bit-identical
// results, the faster one on this device for a shape is found by timing both
// once, on the handle's own (scratch) buffers, and the choice is kept for the
// process, per device and shape; results never depend on it.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::array<int, 6>, int> g_tune;

// milliseconds for `reps` runs of `run` on stream s (after one untimed run)
template <class Fn>
int time_runs(hipStream_t s, int reps, Fn&& run, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GIR_HIP(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error(hipGetErrorString(e));
    return GMRESIR_EHIP;
  }
  run();
  e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) run();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    set_error(hipGetErrorString(e));
    return GMRESIR_EHIP;
  }
  return 0;
}

// The Arnoldi step's orthogonalisation: the single-workgroup launch against
// the three multi-workgroup passes (the last one normalising; the first is
// timed as its own launch although a solve runs it inside the upper
// triangular solve), timed at step 0
// with half a cycle's basis ([C_k V_{m/2+1}]) and a scratch cycle state (in
// Mdev), so that nothing the solve keeps is touched.
int tune_ortho(gmresir_ctx* h) {
  if (h->ortho_small >= 0) return 0;
  if (h->o.ortho == 1 || h->n > gir::kOrthoSmallMax || h->k + h->m + 1 > 192) {
    h->ortho_small = 0;
    return 0;
  }
  int dev = 0;
  GIR_HIP(hipGetDevice(&dev));
  const std::array<int, 6> key{dev, 0, h->u64 ? 1 : 0, (int)((h->n + 255) / 256), h->k, h->m};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      h->ortho_small = it->second;
      return 0;
    }
  }
  hipStream_t s = h->stream;
  const int m = h->m, k = h->k, n = (int)h->n;
  const int64_t ld = h->ld;
  double* sc = h->Mdev;  // >= 4096 doubles of scratch
  gir::CycleState* st = reinterpret_cast<gir::CycleState*>(sc);
  gir::OrthoArgs a{};
  a.X = basis(h, h->C, k, ld, h->V, m / 2 + 1, ld);
  a.n = n;
  a.w_in = h->wu;
  a.w_out = h->wu;
  a.partial = h->partial;
  a.counter = h->counter;
  a.gate = st;
  a.step = 0;
  a.h_prev = h->h1;
  a.norm_out = h->nrm;
  a.H = sc + 32;
  a.B = sc + 64;
  a.ldh = m + 1;
  a.ldb = std::max(k, 1);
  a.cs = sc + 160;
  a.sn = sc + 170;
  a.g = sc + 200;
  a.st = st;
  void* vout = vcol(h, m);
  auto multi = [&] {
    gir::OrthoArgs b = a;
    b.dots_out = h->h1;
    gir::launch_ortho(b, gir::kOrthoDots, s);
    b.coef = h->h1;
    b.dots_out = h->h2;
    gir::launch_ortho(b, gir::kOrthoUpdate | gir::kOrthoDots, s);
    b.coef = h->h2;
    b.vout = vout;
    gir::launch_ortho(b, gir::kOrthoUpdate | gir::kOrthoNorm | gir::kOrthoFinish, s);
  };
  auto single = [&] {
    gir::OrthoArgs b = a;
    b.dots_out = h->h1;
    b.coef = h->h2;
    gir::launch_ortho_small(b, vout, s);
  };
  // a zero state: done stays 0 or, with jdone = 1 > step 0, gates nothing
  gir::launch_fill_i32(reinterpret_cast<int*>(sc), 0, 2 * 256, s);
  constexpr int kReps = 10;
  float t_multi = 0.0f, t_single = 0.0f, t_multi2 = 0.0f;
  GIR_TRY(time_runs(s, kReps, multi, &t_multi));
  GIR_TRY(time_runs(s, kReps, single, &t_single));
  GIR_TRY(time_runs(s, kReps, multi, &t_multi2));
  const int choice = t_single < std::min(t_multi, t_multi2) ? 1 : 0;
  h->ortho_small = choice;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = choice;
  return 0;
}

// dots (X^T w) and/or squared norm of a vector in u, synchronous result
// extra: one more device-to-host piece fetched in the same synchronisation
// (null: none)
int dots_norm(gmresir_ctx* h, const gir::Basis& X, const void* w, double* dots, double* nrm2,
              const struct Piece* extra = nullptr) {
  gir::OrthoArgs a{};
  a.X = X;
  a.n = (int)h->n;
  a.w_in = w;
  a.w_out = nullptr;
  a.dots_out = h->h1;
  a.norm_out = h->nrm;
  a.partial = h->partial;
  a.counter = h->counter;
  int mode = gir::kOrthoNorm;
  if (X.kc + X.nv > 0 && dots) mode |= gir::kOrthoDots;
  gir::launch_ortho(a, mode, h->stream);
  GIR_HIP(hipGetLastError());
  const int nc = X.kc + X.nv;
  const size_t db = (nc > 0 && dots) ? sizeof(double) * nc : 0;
  GIR_TRY(download_many(h, {{dots, h->h1, db},
                            {nrm2, h->nrm, sizeof(double)},
                            extra ? *extra : Piece{nullptr, nullptr, 0}}));
  return 0;
}

int gram(gmresir_ctx* h, const gir::Basis& X, const double* Y, int ny, std::vector<double>& G) {
  const int nx = X.kc + X.nv;
  G.assign((size_t)nx * ny, 0.0);
  if (nx == 0 || ny == 0) return 0;
  gir::launch_gram(X, Y, ny, h->ld, (int)h->n, h->Gdev, h->partial, h->counter, h->stream);
  GIR_HIP(hipGetLastError());
  GIR_TRY(download(h, G.data(), h->Gdev, sizeof(double) * nx * ny));
  return 0;
}

int combine(gmresir_ctx* h, const gir::Basis& X, const std::vector<double>& M, int nout,
            double* out) {
  const int nc = X.kc + X.nv;
  if (nout == 0) return 0;
  GIR_TRY(upload(h, h->Mdev, M.data(), sizeof(double) * (size_t)nc * nout));
  gir::launch_combine(X, (int)h->n, h->Mdev, nout, out, h->ld, h->stream);
  GIR_HIP(hipGetLastError());
  return 0;
}

// Harmonic Ritz vectors P_k of the refresh problem, QR of G P_k = Q R, then
// C <- [C V_{J+1}] Q and U <- [U D, V_J] P_k R^-1 on the device; *kc_new is
// the new dimension (unchanged when no vector was found)
int apply_refresh(gmresir_ctx* h, Refresh& rf, int* kc_new) {
  rf.active = false;
  const int64_t ld = h->ld;
  const int rows = rf.rows, cols = rf.cols, kc = rf.kc, J = rf.J, k = h->k;
  *kc_new = kc;
  std::vector<double> Pk((size_t)cols * k);
  const int kn = gir::la::harmonic_ritz(rf.Gm.data(), rf.Mm.data(), rows, cols, k, Pk.data());
  if (kn <= 0) return 0;
  std::vector<double> GP((size_t)rows * kn, 0.0), Q((size_t)rows * kn), R((size_t)kn * kn),
      Ri((size_t)kn * kn), PR((size_t)cols * kn, 0.0);
  for (int o = 0; o < kn; ++o)
    for (int i = 0; i < rows; ++i) {
      double sum = 0.0;
      for (int c = 0; c < cols; ++c) sum += rf.Gm[(size_t)c * rows + i] * Pk[(size_t)o * cols + c];
      GP[(size_t)o * rows + i] = sum;
    }
  if (!gir::la::qr_thin(GP.data(), rows, rows, kn, Q.data(), R.data())) return 0;
  gir::la::inv_upper(R.data(), kn, Ri.data());
  for (int o = 0; o < kn; ++o)
    for (int c = 0; c < cols; ++c) {
      double sum = 0.0;
      for (int t = 0; t < kn; ++t) sum += Pk[(size_t)t * cols + c] * Ri[(size_t)o * kn + t];
      // U-tilde = U D: fold D into the coefficients of the U columns
      PR[(size_t)o * cols + c] = (c < kc) ? sum * rf.dk[c] : sum;
    }
  GIR_TRY(combine(h, basis(h, h->C, kc, ld, h->V, J + 1, ld), Q, kn, h->Cn));
  GIR_TRY(combine(h, basis(h, h->U, kc, ld, h->V, J, ld), PR, kn, h->Un));
  std::swap(h->C, h->Cn);
  std::swap(h->U, h->Un);
  *kc_new = kn;
  return 0;
}

// after a cycle: the refresh now, or, when the cycle is likely the last of
// the correction solve, deferred (*kc stays until it is applied)
int schedule_refresh(gmresir_ctx* h, Refresh& rf, bool likely_last, int* kc) {
  if (likely_last) {
    h->pend = std::move(rf);
    h->pend.active = true;
    return 0;
  }
  return apply_refresh(h, rf, kc);
}

// the deferred refresh (if any) of the previous correction solve
int resolve_pending(gmresir_ctx* h, bool keep) {
  if (!h->pend.active) return 0;
  if (!keep) {
    h->pend.active = false;
    h->kc_keep = 0;
    return 0;
  }
  int kcn = 0;
  GIR_TRY(apply_refresh(h, h->pend, &kcn));
  h->kc_keep = h->k > 0 ? kcn : 0;
  return 0;
}

// C = QR(A-tilde U) by CholeskyQR2 in fp64, U <- U R^-1 (the recycled space
// at the start of a correction solve); *ok = false when a Cholesky factor
// breaks down (the space is then dropped)
// C R = Z (Z = A-tilde U in h->C, n x kk) by Householder QR on the host,
// then U = U R^-1 on the device
int householder_recycle(gmresir_ctx* h, int kk, bool* ok) {
  const int64_t ld = h->ld;
  const int n = (int)h->n;
  std::vector<double> Z((size_t)ld * kk), Q((size_t)n * kk), R((size_t)kk * kk),
      Ri((size_t)kk * kk);
  GIR_TRY(download(h, Z.data(), h->C, sizeof(double) * (size_t)ld * kk));
  *ok = gir::la::qr_thin(Z.data(), (int)ld, n, kk, Q.data(), R.data());
  if (!*ok) return 0;
  std::fill(Z.begin(), Z.end(), 0.0);  // Q in the padded column layout
  for (int j = 0; j < kk; ++j)
    std::copy(Q.begin() + (size_t)j * n, Q.begin() + (size_t)(j + 1) * n,
              Z.begin() + (size_t)j * ld);
  GIR_TRY(upload(h, h->C, Z.data(), sizeof(double) * (size_t)ld * kk));
  gir::la::inv_upper(R.data(), kk, Ri.data());
  GIR_TRY(combine(h, basis(h, h->U, kk, ld, nullptr, 0, ld), Ri, kk, h->Un));
  std::swap(h->U, h->Un);
  return 0;
}

int recompute_recycle(gmresir_ctx* h, int kk, bool* ok) {
  const int64_t ld = h->ld;
  GIR_TRY(atilde_block(h, h->U, kk, h->C));
  GIR_HIP(hipGetLastError());
  if (h->force_hqr) return householder_recycle(h, kk, ok);
  std::vector<double> G1, G2, R1(kk * kk), R2(kk * kk), Ri(kk * kk), Rt(kk * kk);
  GIR_TRY(gram(h, basis(h, h->C, kk, ld, nullptr, 0, ld), h->C, kk, G1));
  *ok = gir::la::cholesky_upper(G1.data(), kk, R1.data());
  if (*ok) {
    gir::la::inv_upper(R1.data(), kk, Ri.data());
    GIR_TRY(combine(h, basis(h, h->C, kk, ld, nullptr, 0, ld), Ri, kk, h->Cn));
    GIR_TRY(gram(h, basis(h, h->Cn, kk, ld, nullptr, 0, ld), h->Cn, kk, G2));
    *ok = gir::la::cholesky_upper(G2.data(), kk, R2.data());
  }
  if (*ok) {
    gir::la::inv_upper(R2.data(), kk, Ri.data());
    GIR_TRY(combine(h, basis(h, h->Cn, kk, ld, nullptr, 0, ld), Ri, kk, h->C));
    // R = R2 R1, U = Y R^-1
    for (int j = 0; j < kk; ++j)
      for (int i = 0; i < kk; ++i) {
        double sum = 0.0;
        for (int t = 0; t < kk; ++t) sum += R2[(size_t)t * kk + i] * R1[(size_t)j * kk + t];
        Rt[(size_t)j * kk + i] = sum;
      }
    gir::la::inv_upper(Rt.data(), kk, Ri.data());
    GIR_TRY(combine(h, basis(h, h->U, kk, ld, nullptr, 0, ld), Ri, kk, h->Un));
    std::swap(h->U, h->Un);
  }
  if (!*ok) {
    // CholeskyQR2 broke down (the Gram matrix of Z = A-tilde U is not
    // numerically positive definite): Householder QR of Z on the host, the
    // factorisation the method states.  h->C still holds Z.  Only an exactly
    // rank-deficient Z (no R^-1) drops the space.
    GIR_TRY(householder_recycle(h, kk, ok));
  }
  return 0;
}

struct SolveStats {
  int its = 0;
};

// a cycle's Arnoldi steps in one persistent launch: u = fp32, classical
// Gram-Schmidt twice, the forward operator, n and m within the kernel's
// limits and 3 ceil(n/128) compute units on the device (its exchange words
// allocated)
bool cycle_eligible(const gmresir_ctx* h) {
  return h->persistent && h->cvw && !h->trans && !h->u64 && !h->uni && h->o.ortho == 0 &&
         h->fuse_atilde;
}

// up to nsteps Arnoldi steps of the cycle with kc recycled columns, one
// launch; the results (V, H, B, the rotations and the cycle state) are where
// the separate launches leave them, unless the launch gave up (its
// workgroups were not all resident together: the decision word after the
// arrival count at cctrl + 2 is then kCycleGaveUp, not kCycleGo), in which
// case it wrote nothing.
int run_cycle(gmresir_ctx* h, int kc, int nsteps) {
  gir::CycleArgs a{};
  a.S = h->S;
  a.ld = h->ld;
  a.permS = h->permS;
  a.Linv = h->Linv;
  a.Uinv = h->Uinv;
  a.scale = h->scale;
  a.Au = h->Au;
  a.lda = h->ld;
  a.permA = h->permP;
  a.n = (int)h->n;
  a.kc = kc;
  a.m = h->m;
  a.nsteps = nsteps;
  a.C = h->C;
  a.ldc = h->ld;
  a.V = static_cast<float*>(h->V);
  a.ldv = h->ld;
  a.H = h->Hd;
  a.B = h->Bd;
  a.ldh = h->m + 1;
  a.ldb = std::max(h->k, 1);
  a.cs = h->cs;
  a.sn = h->sn;
  a.g = h->g;
  a.st = h->st;
  a.xt = h->xt;
  a.xwL = h->xwL;
  a.xwU = h->xwU;
  a.vw = h->cvw;
  a.px = h->cpx;
  a.ctrl = h->cctrl;
  a.arrive = reinterpret_cast<unsigned*>(h->cctrl + 2);
  a.arrive_us = h->cycle_arrive_us;
  a.epoch0 = (uint32_t)reserve_epochs(h, nsteps);
  a.abortp = &h->st->abort;
  gir::launch_fill_i32(reinterpret_cast<int*>(a.arrive), 0, 2, h->stream);
  // the work is set once the number of steps taken is known
  return timed(h, kKcCycle, 0.0, h->stream, nullptr, 0,
               [&] { gir::launch_cycle(a, h->store, h->stream); });
}

// GCRO-DR(m, k) for A-tilde d = z (z in h->zu); result in h->du.
int gcrodr(gmresir_ctx* h, SolveStats& stats) {
  const int n = (int)h->n;
  const int64_t ld = h->ld;
  const int m = h->m, k = h->k;
  const int cap = h->o.maxit > 0 ? h->o.maxit : 10 * m;
  hipStream_t s = h->stream;
  // the previous solve's last refresh runs on the host while the device
  // finishes the preconditioned right-hand side
  GIR_TRY(resolve_pending(h, true));
  double beta0 = 0.0;
  {
    double n2 = 0.0;
    GIR_TRY(dots_norm(h, basis(h, nullptr, 0, ld, nullptr, 0, ld), h->zu, nullptr, &n2));
    beta0 = std::sqrt(n2);
  }
  // small device copies and fills run as kernels (no copy-engine latency)
  const int64_t uw = (int64_t)n * (int64_t)(h->ue / 4);  // 4-byte words of a vector in u
  gir::launch_copy_i32(static_cast<int*>(h->ru), static_cast<const int*>(h->zu), uw, s);
  gir::launch_fill_i32(static_cast<int*>(h->du), 0, uw, s);
  stats.its = 0;
  if (beta0 == 0.0) return 0;
  const double tol = h->o.tau * beta0;
  int kc = 0;

  // recycled space from the previous system: C = QR(A-tilde Y), U = Y R^-1
  if (k > 0 && h->kc_keep > 0) {
    const int kk = h->kc_keep;
    bool ok = true;
    if (h->o.reuse_recycle) {
      // the matrix is unchanged: C and U of the previous solve still satisfy
      // A-tilde U = C with C orthonormal (the reuse variant)
      kc = kk;
    } else {
      GIR_TRY(recompute_recycle(h, kk, &ok));
      if (ok) kc = kk;
    }
    if (ok) {
      // d = U (C^T r), r = r - C (C^T r)
      std::vector<double> ctr(kc);
      double n2;
      GIR_TRY(dots_norm(h, basis(h, h->C, kc, ld, nullptr, 0, ld), h->ru, ctr.data(), &n2));
      GIR_TRY(upload(h, h->coefA, ctr.data(), sizeof(double) * kc));
      gir::launch_cycle_update(basis(h, h->U, kc, ld, nullptr, 0, ld), h->coefA, h->du,
                               basis(h, h->C, kc, ld, nullptr, 0, ld), h->coefA, h->ru, n, h->u64, s);
      GIR_HIP(hipGetLastError());
    }
  }
  GIR_TRY(phase_mark(h, kPhRecycle));

  std::vector<double> Hh((size_t)(m + 1) * m), Bh((size_t)std::max(k, 1) * m), y((size_t)m + 1);
  while (true) {
    std::vector<double> ctr(std::max(kc, 1));
    double n2 = 0.0;
    // C^T r and ||r||, and with them U^T U (its diagonal scales the recycled
    // columns after the cycle; U does not change before then), all in one
    // synchronisation
    std::vector<double> UU((size_t)std::max(kc, 1) * std::max(kc, 1));
    auto start_cycle = [&]() -> int {
      Piece uu{UU.data(), h->Gdev, 0};
      if (kc > 0) {
        gir::launch_gram(basis(h, h->U, kc, ld, nullptr, 0, ld), h->U, kc, ld, n, h->Gdev,
                         h->partial, h->counter, s);
        GIR_HIP(hipGetLastError());
        uu.bytes = sizeof(double) * (size_t)kc * kc;
      }
      return dots_norm(h, basis(h, h->C, kc, ld, nullptr, 0, ld), h->ru,
                       kc ? ctr.data() : nullptr, &n2, &uu);
    };
    GIR_TRY(start_cycle());
    double rn = std::sqrt(n2);
    if (rn <= tol) break;
    if (stats.its >= cap) break;
    if (h->pend.active) {
      // the estimate said converged but the residual did not: refresh now
      GIR_TRY(apply_refresh(h, h->pend, &kc));
      ctr.assign(std::max(kc, 1), 0.0);
      UU.assign((size_t)std::max(kc, 1) * std::max(kc, 1), 0.0);
      GIR_TRY(start_cycle());
      rn = std::sqrt(n2);
    }
    const int nsteps = std::min(m - kc, cap - stats.its);
    // v1 = r / ||r||; device cycle state and Givens right-hand side
    gir::launch_div_u(h->ru, rn, h->V, h->u64, n, s);
    gir::CycleState st0{};
    st0.tol = tol;
    st0.est = rn;
    double* hb = h->hbuf;
    std::fill(hb, hb + m + 2, 0.0);
    hb[0] = rn;
    // the orthogonalisation's reduction ticket starts at zero (a launch
    // that gave up on a bounded wait may have left it counted)
    gir::launch_fill_i32(reinterpret_cast<int*>(h->counter), 0, 1, s);
    // g, and the state but its abort and singular fields
    GIR_TRY(upload_many(h, {{h->g, hb, sizeof(double) * (m + 2)},
                            {h->st, &st0, offsetof(gir::CycleState, abort)},
                            {&h->st->tol, &st0.tol, 2 * sizeof(double)}}));
    int queued = 0;
    const size_t trec0 = h->trec.size();
    // modified Gram-Schmidt's finish pass applies zero coefficients
    if (h->o.ortho == 1)
      gir::launch_fill_i32(reinterpret_cast<int*>(h->h2), 0, 2 * 256, s);
    // one Arnoldi step's work: A_u v_j and the factors once each (the HBM
    // model of the step) plus one read of the basis [C_k V_j]
    auto step_work = [&](int j) {
      return (double)n * (double)n * (double)(a_bytes(h) + store_bytes(h->store)) +
             (8.0 * kc + (double)h->ue * (j + 1)) * n + 4.0 * h->ue * n;
    };
    // the cycle's steps as separate launches, the host polling each step's
    // state (it stops the loop once the cycle has converged)
    auto run_steps = [&]() -> int {
      for (int j = 0; j < nsteps; ++j) {
        // one Arnoldi step, timed as a whole under its own class
        const double step_bytes = step_work(j);
        GIR_TRY(timed(h, kKcStep, step_bytes, s, h->st, j, [&]() -> int {
        const gir::Basis Xj = basis(h, h->C, kc, ld, h->V, j + 1, ld);
        // classical Gram-Schmidt in its multi-workgroup form: the first pass
        // (h1 = X^T w) runs inside the upper solve that produces w
        const bool dots1 = fuse_first_dots(h) && kc + j + 1 <= gir::kDotsMaxCols;
        const gir::TrsvDots td{Xj, h->partial, h->counter, h->h1};
        GIR_TRY(atilde(h, vcol(h, j), nullptr, nullptr, h->wu, h->st, j, dots1 ? &td : nullptr));
        gir::OrthoArgs a{};
        a.X = Xj;
        a.n = n;
        a.w_in = h->wu;
        a.w_out = h->wu;
        a.partial = h->partial;
        a.counter = h->counter;
        a.gate = h->st;
        a.step = j;
        a.dots_out = h->h1;
        // basis read once per pass; the update pass also reads and writes w
        const double xb = (8.0 * kc + (double)h->ue * (j + 1)) * n;
        if (h->o.ortho != 1 && h->ortho_small == 1) {
          // the three passes, the finish and the normalisation in one launch
          // of one workgroup (the same sums; the basis read four times)
          a.coef = h->h2;
          a.norm_out = h->nrm;
          a.H = h->Hd;
          a.B = h->Bd;
          a.ldh = m + 1;
          a.ldb = std::max(k, 1);
          a.cs = h->cs;
          a.sn = h->sn;
          a.g = h->g;
          a.st = h->st;
          a.st_out = &h->st_host[j];
          GIR_TRY(timed(h, kKcOrtho, 4.0 * xb + 4.0 * h->ue * n, s, h->st, j,
                        [&] { gir::launch_ortho_small(a, vcol(h, j + 1), s); }));
          return 0;
        }
        if (h->o.ortho == 1) {
          // modified Gram-Schmidt: one basis column at a time ([C_k V_j] in
          // order), its inner product with the current w, then its update;
          // the coefficients gather in h1 and the finish pass below applies
          // none (h2 is zero) but forms the norm and the Givens update
          for (int i = 0; i < kc + j + 1; ++i) {
            gir::OrthoArgs ai = a;
            ai.X = i < kc ? basis(h, h->C + (size_t)i * ld, 1, ld, nullptr, 0, ld)
                          : basis(h, nullptr, 0, ld, vcol(h, i - kc), 1, ld);
            ai.dots_out = h->h1 + i;
            ai.coef = h->h1 + i;
            const double cb = (double)(i < kc ? 8 : h->ue) * n;
            GIR_TRY(timed(h, kKcOrtho, cb + (double)h->ue * n, s, h->st, j,
                          [&] { gir::launch_ortho(ai, gir::kOrthoDots, s); }));
            GIR_TRY(timed(h, kKcOrtho, cb + 2.0 * h->ue * n, s, h->st, j,
                          [&] { gir::launch_ortho(ai, gir::kOrthoUpdate, s); }));
          }
        } else {
          if (!dots1)
            GIR_TRY(timed(h, kKcOrtho, xb + (double)h->ue * n, s, h->st, j,
                          [&] { gir::launch_ortho(a, gir::kOrthoDots, s); }));
          a.coef = h->h1;
          a.dots_out = h->h2;
          GIR_TRY(timed(h, kKcOrtho, 2.0 * xb + 2.0 * h->ue * n, s, h->st, j,
                        [&] { gir::launch_ortho(a, gir::kOrthoUpdate | gir::kOrthoDots, s); }));
        }
        a.coef = h->h2;
        a.h_prev = h->h1;
        a.norm_out = h->nrm;
        a.H = h->Hd;
        a.B = h->Bd;
        a.ldh = m + 1;
        a.ldb = std::max(k, 1);
        a.cs = h->cs;
        a.sn = h->sn;
        a.g = h->g;
        a.st = h->st;
        a.st_out = &h->st_host[j];
        a.vout = vcol(h, j + 1);  // the normalisation in the finishing workgroup
        GIR_TRY(timed(h, kKcOrtho, xb + 4.0 * h->ue * n, s, h->st, j, [&] {
          gir::launch_ortho(a, gir::kOrthoUpdate | gir::kOrthoNorm | gir::kOrthoFinish, s);
        }));
        return 0;
        }));
        // the step's finish wrote its cycle state to st_host[j]; a step skipped
        // on the device (converged earlier) writes nothing, and its slot is
        // never read: the loop stops at the converged step's own slot
        GIR_HIP(hipEventRecord(h->ev[j % kEventRing], s));
        queued = j + 1;
        if (j >= kLaunchAhead) {
          GIR_HIP(hipEventSynchronize(h->ev[(j - kLaunchAhead) % kEventRing]));
          const gir::CycleState& sj = h->st_host[j - kLaunchAhead];
          if (sj.done || sj.abort) break;
        }
      }
      return 0;
    };
    // one persistent launch for the steps where it applies; its residency
    // word comes back with the cycle's state, and a launch that gave up (not
    // all its workgroups resident together: the device is shared) wrote
    // nothing, so the steps then run as separate launches
    bool one_launch = cycle_eligible(h);
    if (one_launch && h->cycle_wait > 0) {
      --h->cycle_wait;
      one_launch = false;
    }
    if (one_launch)
      GIR_TRY(run_cycle(h, kc, nsteps));
    else
      GIR_TRY(run_steps());
    (void)queued;
    gir::CycleState fin{};
    unsigned gate = 0;
    // W = [C V_{nsteps+1}]^T U for the recycle refresh, formed over every
    // column the cycle may have written (rows past kc + J + 1 are not used)
    // and fetched with the cycle's state
    const int wrows = kc + nsteps + 1;
    std::vector<double> Wall((size_t)wrows * std::max(kc, 1));
    auto fetch_state = [&]() -> int {
      if (kc > 0) {
        gir::launch_gram(basis(h, h->C, kc, ld, h->V, nsteps + 1, ld), h->U, kc, ld, n, h->Gdev,
                         h->partial, h->counter, s);
        GIR_HIP(hipGetLastError());
      }
      return download_many(
          h, {{&fin, h->st, sizeof(fin)},
              {Hh.data(), h->Hd, sizeof(double) * (size_t)(m + 1) * m},
              {Bh.data(), h->Bd, kc > 0 ? sizeof(double) * (size_t)std::max(k, 1) * m : 0},
              {&gate, reinterpret_cast<unsigned*>(h->cctrl + 2) + 1, one_launch ? sizeof(gate) : 0},
              {Wall.data(), h->Gdev, kc > 0 ? sizeof(double) * (size_t)wrows * kc : 0}});
    };
    GIR_TRY(fetch_state());
    if (one_launch && gate != gir::kCycleGo) {
      h->trec.resize(trec0);
      ++h->cycle_fallbacks;
      h->cycle_backoff = std::min(64, std::max(1, 2 * h->cycle_backoff));
      h->cycle_wait = h->cycle_backoff;
      one_launch = false;
      GIR_TRY(run_steps());
      GIR_TRY(fetch_state());
    } else if (one_launch) {
      ++h->cycles_run;
      h->cycle_backoff = 0;
    }
    if (fin.abort) {
      set_error("triangular solve: a device-side wait exceeded its bound");
      return GMRESIR_EINTERNAL;
    }
    const int J = fin.jdone;
    drop_skipped(h, trec0, J);
    if (one_launch && h->trec.size() > trec0 && h->trec.back().cls == kKcCycle) {
      double w = 0.0;
      for (int j = 0; j < J; ++j) w += step_work(j);
      h->trec.back().work = w;
    }
    const int ldh = m + 1, ldb = std::max(k, 1);
    std::fill(y.begin(), y.end(), 0.0);
    gir::la::givens_lsq(Hh.data(), ldh, J, rn, y.data());
    // Hbar y (J+1)
    std::vector<double> hy(J + 1, 0.0);
    for (int c = 0; c < J; ++c)
      for (int i = 0; i <= c + 1 && i <= J; ++i) hy[i] += Hh[(size_t)c * ldh + i] * y[c];
    stats.its += J;
    if (kc == 0) {
      std::vector<double> cdv(y.begin(), y.begin() + J);
      GIR_TRY(upload_many(h, {{h->coefA, cdv.data(), sizeof(double) * std::max(J, 1)},
                              {h->coefB, hy.data(), sizeof(double) * (J + 1)}}));
      gir::launch_cycle_update(basis(h, nullptr, 0, ld, h->V, J, ld), h->coefA, h->du,
                               basis(h, nullptr, 0, ld, h->V, J + 1, ld), h->coefB, h->ru, n, h->u64, s);
      GIR_HIP(hipGetLastError());
      if (k > 0 && J > 0) {
        // first-cycle harmonic Ritz: Hbar^T Hbar z = theta H^T z
        Refresh rf;
        rf.kc = 0;
        rf.J = J;
        rf.rows = J + 1;
        rf.cols = J;
        rf.Gm.assign((size_t)(J + 1) * J, 0.0);
        rf.Mm.assign((size_t)(J + 1) * J, 0.0);
        for (int c = 0; c < J; ++c) {
          for (int i = 0; i <= J; ++i)
            rf.Gm[(size_t)c * (J + 1) + i] = (i <= c + 1) ? Hh[(size_t)c * ldh + i] : 0.0;
          rf.Mm[(size_t)c * (J + 1) + c] = 1.0;
        }
        GIR_TRY(schedule_refresh(h, rf, fin.done || stats.its >= cap, &kc));
      }
    } else {
      // D = diag(1 / ||U e_i||), U^T U fetched at the cycle's start
      std::vector<double> dk(kc);
      for (int i = 0; i < kc; ++i) dk[i] = 1.0 / std::sqrt(UU[(size_t)i * kc + i]);
      std::vector<double> y1(kc), by2(kc, 0.0);
      for (int i = 0; i < kc; ++i) {
        for (int c = 0; c < J; ++c) by2[i] += Bh[(size_t)c * ldb + i] * y[c];
        y1[i] = (ctr[i] - by2[i]) / dk[i];
      }
      std::vector<double> cdv(kc + J), crv(kc + J + 1);
      for (int i = 0; i < kc; ++i) {
        cdv[i] = dk[i] * y1[i];
        crv[i] = dk[i] * y1[i] + by2[i];
      }
      for (int c = 0; c < J; ++c) cdv[kc + c] = y[c];
      for (int i = 0; i <= J; ++i) crv[kc + i] = hy[i];
      GIR_TRY(upload_many(h, {{h->coefA, cdv.data(), sizeof(double) * cdv.size()},
                              {h->coefB, crv.data(), sizeof(double) * crv.size()}}));
      gir::launch_cycle_update(basis(h, h->U, kc, ld, h->V, J, ld), h->coefA, h->du,
                               basis(h, h->C, kc, ld, h->V, J + 1, ld), h->coefB, h->ru, n, h->u64, s);
      GIR_HIP(hipGetLastError());
      if (J > 0) {
        const int rows = kc + J + 1, cols = kc + J;
        std::vector<double> W((size_t)rows * kc);  // [C V_{J+1}]^T U  (rows x kc)
        for (int c = 0; c < kc; ++c)
          std::copy(Wall.begin() + (size_t)c * wrows, Wall.begin() + (size_t)c * wrows + rows,
                    W.begin() + (size_t)c * rows);
        std::vector<double> Gm((size_t)rows * cols, 0.0), Mm((size_t)rows * cols, 0.0);
        for (int i = 0; i < kc; ++i) Gm[(size_t)i * rows + i] = dk[i];
        for (int c = 0; c < J; ++c) {
          for (int i = 0; i < kc; ++i) Gm[(size_t)(kc + c) * rows + i] = Bh[(size_t)c * ldb + i];
          for (int i = 0; i <= J; ++i)
            Gm[(size_t)(kc + c) * rows + kc + i] = (i <= c + 1) ? Hh[(size_t)c * ldh + i] : 0.0;
          Mm[(size_t)(kc + c) * rows + kc + c] = 1.0;
        }
        for (int c = 0; c < kc; ++c)
          for (int i = 0; i < rows; ++i) Mm[(size_t)c * rows + i] = W[(size_t)c * rows + i] * dk[c];
        Refresh rf;
        rf.kc = kc;
        rf.J = J;
        rf.rows = rows;
        rf.cols = cols;
        rf.Gm = std::move(Gm);
        rf.Mm = std::move(Mm);
        rf.dk = dk;
        GIR_TRY(schedule_refresh(h, rf, fin.done || stats.its >= cap, &kc));
      }
    }
  }
  // with a deferred refresh the dimension is set when it is applied
  if (!h->pend.active) h->kc_keep = (k > 0) ? kc : 0;
  return 0;
}

int solve_one(gmresir_ctx* h, const double* bcol, double* xcol, gmresir_info* info) {
  const int n = (int)h->n;
  hipStream_t s = h->stream;
  const double t0 = now_s();
  gmresir_info inf{};
  inf.singular_col = h->singular_col;
  const int64_t cyc0 = h->cycles_run, fb0 = h->cycle_fallbacks;
  if (h->status == GMRESIR_ESINGULAR || h->status == GMRESIR_ERANGE) {
    inf.status = h->status;
    if (info) *info = inf;
    return h->status;
  }
  if (!h->o.keep_recycle) {
    h->kc_keep = 0;
    h->pend.active = false;
  }
  h->pnext = 0;
  GIR_TRY(phase_mark(h, kPhStart));
  gir::launch_copy_i32(reinterpret_cast<int*>(h->b), reinterpret_cast<const int*>(bcol), 2 * n, s);
  gir::launch_maxabs(h->b, n, h->norms + 2, s);
  unsigned long long bbits = 0;
  GIR_TRY(download(h, &bbits, h->norms + 2, 8));
  double bmax;
  std::memcpy(&bmax, &bbits, 8);
  if (!std::isfinite(bmax)) {
    inf.status = GMRESIR_ERANGE;
    if (info) *info = inf;
    return GMRESIR_ERANGE;
  }
  // x0 = M^-1 b in u^2, kept in fp64
  GIR_TRY(precond(h, h->b, nullptr, h->permP, h->x, nullptr, nullptr, 0));
  GIR_TRY(phase_mark(h, kPhX0));
  int status = GMRESIR_ENOCONV;
  const int imax = h->o.imax;
  int i = 0;
  for (;; ++i) {
    GIR_TRY(timed(h, kKcResid, 8.0 * (double)n * (double)n + 24.0 * (double)n, s, nullptr, 0,
                  [&] {
                    if (h->trans)
                      gir::launch_colsum(h->A64, 1, h->ld, n, h->x, 1, h->colpart, h->b, h->x,
                                         h->r64, h->norms, nullptr, 0, s);
                    else if (h->rdd)
                      gir::launch_residual_dd(h->A64, h->ld, n, h->b, h->x, h->r64, h->norms, s);
                    else
                      gir::launch_residual(h->A64, h->ld, n, h->b, h->x, h->r64, h->norms, s);
                  }));
    GIR_HIP(hipGetLastError());
    unsigned long long nb[gir::kNormCw + 1];
    GIR_TRY(download(h, nb, h->norms, sizeof(nb)));
    GIR_TRY(phase_mark(h, kPhResidual));
    double rmax, xmax, etac;
    std::memcpy(&rmax, &nb[0], 8);
    std::memcpy(&xmax, &nb[1], 8);
    std::memcpy(&etac, &nb[gir::kNormCw], 8);
    const double den = (h->trans ? h->norm_a1 : h->norm_a) * xmax + bmax;
    const double eta = (rmax == 0.0) ? 0.0 : (den > 0.0 ? rmax / den : INFINITY);
    if (i <= GMRESIR_MAX_STEPS) {
      inf.berr[i] = eta;
      // the products with A^T do not form |A^T| |lambda|
      inf.berr_cw[i] = h->trans ? NAN : etac;
    }
    if (!std::isfinite(eta)) {
      status = GMRESIR_ERANGE;
      break;
    }
    if (eta <= h->o.berr_target) {
      status = GMRESIR_OK;
      break;
    }
    if (i >= imax) break;
    gir::launch_scale_round(h->r64, rmax, h->t64, n, h->u64, s);  // r-hat = fl_u(r / s)
    GIR_TRY(precond(h, h->t64, nullptr, h->permP, nullptr, h->zu, nullptr, 0, true));
    GIR_TRY(phase_mark(h, kPhPrecond));
    SolveStats ss;
    GIR_TRY(gcrodr(h, ss));
    inf.its[i] = ss.its;
    inf.total_its += ss.its;
    gir::launch_x_update(h->x, h->du, h->u64, rmax, n, s);
    GIR_HIP(hipGetLastError());
    GIR_TRY(phase_mark(h, kPhArnoldi));
  }
  // the last refresh is needed only when the space is kept for the next call
  GIR_TRY(resolve_pending(h, h->o.keep_recycle != 0));
  GIR_TRY(phase_mark(h, kPhRecycle));
  inf.steps = i;
  inf.status = status;
  inf.recycle_dim = h->kc_keep;
  gir::launch_copy_i32(reinterpret_cast<int*>(xcol), reinterpret_cast<const int*>(h->x), 2 * n, s);
  GIR_HIP(hipStreamSynchronize(s));
  inf.t_factor_s = h->t_factor;
  inf.t_solve_s = now_s() - t0;
  inf.cycles_persistent = (int32_t)(h->cycles_run - cyc0);
  inf.cycles_fallback = (int32_t)(h->cycle_fallbacks - fb0);
  {
    double tp[kPhCount];
    GIR_TRY(phase_times(h, tp));
    inf.t_x0_s = tp[kPhX0];
    inf.t_residual_s = tp[kPhResidual];
    inf.t_precond_s = tp[kPhPrecond];
    inf.t_recycle_s = tp[kPhRecycle];
    inf.t_arnoldi_s = tp[kPhArnoldi];
  }
  if (info) *info = inf;
  return status;
}

// The adjoint system A^T lambda = g: buffers on first use (partial sums of
// the products with A^T, the adjoint recycle space), ||A||_1 from the column
// sums of |A| (one product with A^T on a vector of ones would not do: the
// entries' signs matter).
int adjoint_setup(gmresir_ctx* h) {
  const size_t ld = (size_t)h->ld;
  const int n = (int)h->n;
  if (!h->colpart) {
    const size_t nchunks = ((size_t)n + 127) / 128;
    GIR_TRY(dalloc(h->arena, &h->colpart, nchunks * (size_t)n));
  }
  if (h->k > 0 && !h->Ut) {
    GIR_TRY(dalloc(h->arena, &h->Ut, ld * h->k));
    GIR_TRY(dalloc(h->arena, &h->Ct, ld * h->k));
  }
  if (!h->Lq) {
    const size_t nb2 = ((size_t)n + gir::kTrsvBlock - 1) / gir::kTrsvBlock;
    GIR_TRY(dalloc(h->arena, &h->Lq, nb2 * gir::kTrsvBlock * gir::kTrsvBlock));
    GIR_TRY(dalloc(h->arena, &h->Uq, nb2 * gir::kTrsvBlock * gir::kTrsvBlock));
    gir::launch_adjacent_products_t(h->S, h->ld, h->permS, h->store, n, h->Linv, h->Uinv, h->Lq,
                                    h->Uq, h->stream);
    GIR_HIP(hipGetLastError());
  }
  if (h->norm_a1 < 0.0) {
    gir::launch_colsum_abs(h->A64, h->ld, n, h->colpart, h->t64, h->norms + 2, h->stream);
    GIR_HIP(hipGetLastError());
    unsigned long long bits = 0;
    GIR_TRY(download(h, &bits, h->norms + 2, 8));
    std::memcpy(&h->norm_a1, &bits, 8);
  }
  return 0;
}

// swaps the forward and the adjoint recycle spaces
void swap_recycle(gmresir_ctx* h) {
  std::swap(h->C, h->Ct);
  std::swap(h->U, h->Ut);
  std::swap(h->kc_keep, h->kc_keep_t);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void gmresir_default_opts(gmresir_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(gmresir_opts);
  o->uf = GMRESIR_FP16;
  o->u = GMRESIR_FP32;
  o->ur = GMRESIR_FP64;
  o->m = 30;
  o->k = 10;
  o->tau = 1e-4;
  o->imax = 10;
  o->maxit = 0;
  o->berr_target = 1e-14;
  o->scale_pow2 = -1;
  o->keep_recycle = 0;
}

int gmresir_factor(const double* A, int64_t n, int64_t lda, const gmresir_opts* opts,
                   void* stream, gmresir_ctx** out) {
  gmresir_ctx* h = nullptr;
  const double t0 = now_s();
  GIR_TRY(make_ctx(A, n, lda, opts, stream, out, &h));
  int rc = alloc_common(h);
  // the solve's buffers first: their zeroing is then complete by the time
  // the factorisation's results are read back, and the final
  // synchronisation finds an idle stream
  if (rc == 0) rc = alloc_solve(h);
  if (rc == 0) rc = ingest(h, A, lda, true);
  if (rc == 0) {
    h->permP = h->perm;
    h->permS = h->perm;
    rc = run_lu(h);
  }
  if (rc == 0) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
      rc = GMRESIR_EHIP;
    }
  }
  if (rc != 0) {
    delete h;
    return rc;
  }
  h->t_factor = now_s() - t0;
  *out = h;
  return h->status;
}

int gmresir_import_factors(const double* A, int64_t n, int64_t lda, const void* lu, int64_t ldlu,
                           const int32_t* ipiv, int32_t e, const gmresir_opts* opts, void* stream,
                           gmresir_ctx** out) {
  gmresir_ctx* h = nullptr;
  GIR_TRY(make_ctx(A, n, lda, opts, stream, out, &h));
  if (!lu || !ipiv || ldlu < n) {
    delete h;
    set_error("invalid lu, ipiv or ldlu");
    return GMRESIR_EINVAL;
  }
  int rc = alloc_common(h);
  if (rc == 0) rc = ingest(h, A, lda, false);
  if (rc == 0) rc = ingest_finish(h, false);
  if (rc == 0) {
    // factors in logical row order: S is read without a row gather
    const size_t eb = store_bytes(h->store);
    hipError_t err = hipMemcpy2DAsync(h->S, h->ld * eb, lu, ldlu * eb, n * eb, n,
                                      hipMemcpyDeviceToDevice, h->stream);
    if (err != hipSuccess) {
      set_error(std::string("hipMemcpy2DAsync: ") + hipGetErrorString(err));
      rc = GMRESIR_EHIP;
    }
  }
  if (rc == 0 && hipStreamSynchronize(h->stream) != hipSuccess) rc = GMRESIR_EHIP;
  if (rc == 0) {
    h->e = e;
    h->scale = std::ldexp(1.0, e);
    std::vector<int> perm(n), ip(ipiv, ipiv + n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
    for (int64_t i = 0; i < n; ++i) {
      if (ip[i] < 0 || ip[i] >= n) {
        set_error("ipiv out of range");
        rc = GMRESIR_EINVAL;
        break;
      }
      std::swap(perm[i], perm[ip[i]]);
    }
    if (rc == 0) rc = upload(h, h->perm, perm.data(), sizeof(int) * n);
    if (rc == 0) rc = upload(h, h->ipiv, ipiv, sizeof(int) * n);
    h->permP = h->perm;
    h->permS = nullptr;
    if (rc == 0 && (!h->u64 || h->uni)) {
      gir::launch_diag_inverses(h->S, h->ld, nullptr, h->store, (int)n, h->Linv, h->Uinv,
                                h->dtmp, h->stream);
      if (hipGetLastError() != hipSuccess) rc = GMRESIR_EHIP;
    }
  }
  if (rc == 0) rc = alloc_solve(h);
  if (rc == 0 && hipStreamSynchronize(h->stream) != hipSuccess) rc = GMRESIR_EHIP;
  if (rc != 0) {
    delete h;
    return rc;
  }
  *out = h;
  return h->status == GMRESIR_ESINGULAR ? 0 : h->status;
}

int gmresir_solve(gmresir_ctx* h, const double* b, double* x, int64_t nrhs, int64_t ldb,
                  void* stream, gmresir_info* info) {
  if (!h || !b || !x || nrhs < 1 || ldb < h->n) {
    set_error("invalid solve arguments");
    return GMRESIR_EINVAL;
  }
  if (stream) h->stream = reinterpret_cast<hipStream_t>(stream);
  int rc = 0;
  for (int64_t j = 0; j < nrhs; ++j) {
    rc = solve_one(h, b + j * ldb, x + j * ldb, info);
    if (rc < 0) return rc;
  }
  return rc;
}

int gmresir_solve_transposed(gmresir_ctx* h, const double* g, double* lambda, int64_t nrhs,
                             int64_t ldb, void* stream, gmresir_info* info) {
  if (!h || !g || !lambda || nrhs < 1 || ldb < h->n) {
    set_error("invalid solve arguments");
    return GMRESIR_EINVAL;
  }
  if (h->u64 || h->rdd) {
    set_error("the adjoint solve supports u = FP32, ur = FP64");
    return GMRESIR_EINVAL;
  }
  if (stream) h->stream = reinterpret_cast<hipStream_t>(stream);
  if (h->status == GMRESIR_ESINGULAR || h->status == GMRESIR_ERANGE) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = h->status;
      info->singular_col = h->singular_col;
    }
    return h->status;
  }
  GIR_TRY(adjoint_setup(h));
  swap_recycle(h);
  h->trans = 1;
  int rc = 0;
  for (int64_t j = 0; j < nrhs; ++j) {
    rc = solve_one(h, g + j * ldb, lambda + j * ldb, info);
    if (rc < 0) break;
  }
  h->trans = 0;
  swap_recycle(h);
  return rc;
}

int gmresir_choose_k(gmresir_ctx* h, const double* b, int32_t kmax, int32_t* k_best,
                     int32_t* its, void* stream) {
  if (!h || !b || !k_best || kmax < 0 || kmax > h->k) {
    set_error("invalid arguments (need 0 <= kmax <= the handle's k)");
    return GMRESIR_EINVAL;
  }
  if (stream) h->stream = reinterpret_cast<hipStream_t>(stream);
  const int k_saved = h->k, keep_saved = h->o.keep_recycle;
  h->o.keep_recycle = 0;
  int best = 0, best_its = -1, limit = kmax, rc = 0, first_status = 0;
  for (int k = 0; k <= kmax && k <= limit; ++k) {
    h->k = k;
    h->kc_keep = 0;
    gmresir_info inf{};
    rc = solve_one(h, b, h->z64, &inf);
    if (rc < 0) break;
    const int total = inf.status == GMRESIR_OK ? inf.total_its : -1;
    if (its) its[k] = total;
    if (k == 0) {
      first_status = rc;
      // k recycled vectors need at least k + 1 Arnoldi steps in the first
      // refinement step, which runs without recycling
      limit = inf.steps > 0 ? std::max(0, inf.its[0] - 1) : 0;
    }
    if (total >= 0 && (best_its < 0 || total < best_its)) {
      best_its = total;
      best = k;
    }
  }
  if (its)
    for (int k = limit + 1; k <= kmax; ++k) its[k] = -1;
  h->k = k_saved;
  h->o.keep_recycle = keep_saved;
  // the trial solves overwrote (and may have swapped) the buffers of the
  // kept pair, so a space kept from an earlier solve no longer satisfies
  // A-tilde U_k = C_k: it is dropped, and the next solve starts without one
  h->kc_keep = 0;
  h->pend.active = false;
  if (rc < 0) return rc;
  *k_best = best;
  return best_its < 0 ? (first_status ? first_status : GMRESIR_ENOCONV) : GMRESIR_OK;
}

int gmresir_rank1(double alpha, const double* x, const double* y, int64_t n, double* out,
                  int64_t ldo, void* stream) {
  if (!x || !y || !out || n <= 0 || ldo < n || n > (1 << 30)) {
    set_error("invalid rank-1 arguments");
    return GMRESIR_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  gir::launch_rank1(alpha, x, y, (int)n, ldo, out, s);
  GIR_HIP(hipGetLastError());
  GIR_HIP(hipStreamSynchronize(s));
  return 0;
}

void gmresir_free(gmresir_ctx* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

const char* gmresir_strerror(int status) {
  switch (status) {
    case GMRESIR_OK: return "success";
    case GMRESIR_EINVAL: return "invalid argument";
    case GMRESIR_ENOMEM: return "out of memory";
    case GMRESIR_EHIP: return "HIP runtime error";
    case GMRESIR_EINTERNAL: return "device-side wait exceeded its bound";
    case GMRESIR_ESINGULAR: return "exact zero pivot in the factorization precision";
    case GMRESIR_ERANGE: return "non-finite value or overflow in the factorization precision";
    case GMRESIR_ENOCONV: return "backward-error target not reached within imax steps";
    default: return "unknown status";
  }
}

const char* gmresir_last_error(void) { return g_last_error.c_str(); }

int gmresir_export_factors(gmresir_ctx* h, void* lu, int32_t* ipiv, int32_t* e) {
  if (!h) {
    set_error("handle is NULL");
    return GMRESIR_EINVAL;
  }
  const int64_t n = h->n;
  if (e) *e = h->e;
  if (ipiv) GIR_TRY(download(h, ipiv, h->ipiv, sizeof(int) * n));
  if (lu) {
    const size_t eb = store_bytes(h->store);
    std::vector<int> perm(n);
    if (h->permS) {
      GIR_TRY(download(h, perm.data(), h->permS, sizeof(int) * n));
    } else {
      for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
    }
    std::vector<char> row((size_t)h->ld * eb);
    char* dst = reinterpret_cast<char*>(lu);
    for (int64_t i = 0; i < n; ++i) {
      const char* src = reinterpret_cast<const char*>(h->S) + (size_t)perm[i] * h->ld * eb;
      GIR_HIP(hipMemcpyAsync(dst + (size_t)i * n * eb, src, n * eb, hipMemcpyDeviceToHost,
                             h->stream));
    }
    GIR_HIP(hipStreamSynchronize(h->stream));
  }
  return 0;
}

int gmresir_apply(gmresir_ctx* h, int32_t op, const double* v, double* y, void* stream) {
  if (!h || !v || !y || op < 0 || op > 3) {
    set_error("invalid apply arguments");
    return GMRESIR_EINVAL;
  }
  if (op >= 2 && (h->u64 || h->rdd)) {
    set_error("the adjoint products support u = FP32, ur = FP64");
    return GMRESIR_EINVAL;
  }
  if (h->status == GMRESIR_ERANGE) return GMRESIR_ERANGE;
  if (stream) h->stream = reinterpret_cast<hipStream_t>(stream);
  const int n = (int)h->n;
  GIR_HIP(hipMemcpyAsync(h->r64, v, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
  if (op >= 2) GIR_TRY(adjoint_setup(h));
  h->trans = op >= 2 ? 1 : 0;
  int rc = 0;
  if (op == 0 || op == 2)
    rc = precond(h, h->r64, nullptr, h->permP, h->x, nullptr, nullptr, 0);
  else
    rc = atilde(h, nullptr, h->r64, h->x, nullptr, nullptr, 0);
  h->trans = 0;
  GIR_TRY(rc);
  GIR_HIP(hipGetLastError());
  GIR_HIP(hipMemcpyAsync(y, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
  GIR_HIP(hipStreamSynchronize(h->stream));
  gir::CycleState hs{};
  GIR_TRY(download(h, &hs, h->st, sizeof(hs)));
  if (hs.abort) {
    set_error("triangular solve: a device-side wait exceeded its bound");
    return GMRESIR_EINTERNAL;
  }
  return 0;
}

int gmresir_errors(gmresir_ctx* h, const double* b, const double* x, const double* x_true,
                   double* out, void* stream) {
  if (!h || !b || !x || !out) {
    set_error("invalid errors arguments");
    return GMRESIR_EINVAL;
  }
  if (h->status == GMRESIR_ERANGE) return GMRESIR_ERANGE;
  if (stream) h->stream = reinterpret_cast<hipStream_t>(stream);
  hipStream_t s = h->stream;
  const int n = (int)h->n;
  // the caller's vectors are copied into the handle's aligned scratch first
  gir::launch_copy_i32(reinterpret_cast<int*>(h->y64), reinterpret_cast<const int*>(b), 2 * n, s);
  gir::launch_copy_i32(reinterpret_cast<int*>(h->t64), reinterpret_cast<const int*>(x), 2 * n, s);
  gir::launch_maxabs(h->y64, n, h->norms + 2, s);
  gir::launch_residual_dd(h->A64, h->ld, n, h->y64, h->t64, h->r64, h->norms, s);
  GIR_HIP(hipGetLastError());
  unsigned long long nb[gir::kNormCw + 1];
  GIR_TRY(download(h, nb, h->norms, sizeof(nb)));
  double rmax, xmax, bmax, etac;
  std::memcpy(&rmax, &nb[0], 8);
  std::memcpy(&xmax, &nb[1], 8);
  std::memcpy(&bmax, &nb[2], 8);
  std::memcpy(&etac, &nb[gir::kNormCw], 8);
  const double den = h->norm_a * xmax + bmax;
  out[0] = (rmax == 0.0) ? 0.0 : (den > 0.0 ? rmax / den : INFINITY);
  out[1] = etac;
  out[2] = NAN;
  if (x_true) {
    gir::launch_copy_i32(reinterpret_cast<int*>(h->y64), reinterpret_cast<const int*>(x_true),
                         2 * n, s);
    gir::launch_ferr(h->t64, h->y64, n, h->norms + 2, s);
    GIR_HIP(hipGetLastError());
    unsigned long long fb[2];
    GIR_TRY(download(h, fb, h->norms + 2, sizeof(fb)));
    double dmax, tmax;
    std::memcpy(&dmax, &fb[0], 8);
    std::memcpy(&tmax, &fb[1], 8);
    out[2] = (dmax == 0.0) ? 0.0 : (tmax > 0.0 ? dmax / tmax : INFINITY);
  }
  return 0;
}

int gmresir_kernel_stats(gmresir_ctx* h, gmresir_kernel_stat* out, int32_t cap,
                         int32_t* count) {
  if (!h || !count || cap < 0 || (cap > 0 && !out)) {
    set_error("invalid handle or output");
    return GMRESIR_EINVAL;
  }
  if (!h->o.timing) {
    set_error("the handle was created with timing = 0");
    return GMRESIR_EINVAL;
  }
  GIR_TRY(flush_timing(h));
  int32_t c = 0;
  for (int k = 0; k < kKcCount; ++k) {
    if (h->kstat[k].launches == 0) continue;
    if (c < cap) {
      gmresir_kernel_stat& r = out[c];
      std::memset(&r, 0, sizeof(r));
      std::strncpy(r.name, kKcName[k], sizeof(r.name) - 1);
      r.launches = (int32_t)h->kstat[k].launches;
      r.bound = kKcFlops[k] ? 1 : 0;
      r.total_ms = h->kstat[k].ms;
      r.work = h->kstat[k].work;
    }
    ++c;
  }
  *count = std::min(c, cap);
  return 0;
}

int gmresir_query(gmresir_ctx* h, int64_t* n, int32_t* abi) {
  if (abi) *abi = GMRESIR_ABI_VERSION;
  if (!h) return GMRESIR_EINVAL;
  if (n) *n = h->n;
  return 0;
}

}  // extern "C"
