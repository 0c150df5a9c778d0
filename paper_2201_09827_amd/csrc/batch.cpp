// Batched solves: many independent systems of uneven size, each with its own
// right-hand sides, factored and solved concurrently.
//
// Every system runs the same path as gmresir_factor + gmresir_solve
// (Algorithm 3, or Algorithm 2 with k = 0), so a system's result does not
// depend on the batch it is part of.  A system of n <= 2048 leaves most of
// the GPU idle (its block columns use at most four workgroups, its triangular
// solves n / 128), so the batch keeps several of them in flight: worker
// threads, each with its own HIP stream, take systems largest first from a
// shared counter.  The host-side parts of a solve (the harmonic Ritz problem,
// the Givens least-squares update, the refinement test) of one system then
// overlap the device work of the others.
//
// Handles stay alive until every worker has finished: freeing device memory
// synchronises the device, which would stall the other workers' streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "gmresir.h"

namespace {

constexpr int kDefaultWorkers = 8;
constexpr int kMaxWorkers = 64;

struct Worker {
  std::vector<gmresir_ctx*> handles;
  int rc = 0;  // a failure of the worker itself (stream creation)
};

void work(int device, gmresir_batch_item* items, const std::vector<int64_t>* order,
          std::atomic<int64_t>* next, const gmresir_opts* opts, Worker* w) {
  if (hipSetDevice(device) != hipSuccess) {
    w->rc = GMRESIR_EHIP;
    return;
  }
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    w->rc = GMRESIR_EHIP;
    return;
  }
  for (;;) {
    const int64_t i = next->fetch_add(1);
    if (i >= (int64_t)order->size()) break;
    gmresir_batch_item& it = items[(*order)[i]];
    gmresir_ctx* h = nullptr;
    int rc = gmresir_factor(it.A, it.n, it.lda, opts, s, &h);
    if (rc < 0 || h == nullptr) {
      it.status = rc < 0 ? rc : GMRESIR_EINTERNAL;
      continue;
    }
    w->handles.push_back(h);
    // one solve per right-hand side, each with its own record; a singular
    // or out-of-range factorisation is reported by the solves as well
    int st = rc;
    for (int64_t j = 0; j < it.nrhs; ++j) {
      gmresir_info local;
      gmresir_info* info = it.info ? it.info + j : &local;
      const int rs = gmresir_solve(h, it.b + j * it.ldb, it.x + j * it.ldb, 1, it.ldb, s, info);
      if (rs < 0) {
        st = rs;
        break;
      }
      if (st == 0) st = rs;
    }
    it.status = st;
  }
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
}

// no exception may leave a thread (it would end the process)
void run_worker(int device, gmresir_batch_item* items, const std::vector<int64_t>* order,
                std::atomic<int64_t>* next, const gmresir_opts* opts, Worker* w) {
  try {
    work(device, items, order, next, opts, w);
  } catch (...) {
    w->rc = GMRESIR_ENOMEM;
  }
}

}  // namespace

extern "C" int gmresir_solve_batched(gmresir_batch_item* items, int64_t count,
                                     const gmresir_opts* opts, int32_t workers, void* stream) {
  if (count < 0 || (count > 0 && items == nullptr)) return GMRESIR_EINVAL;
  for (int64_t i = 0; i < count; ++i) {
    const gmresir_batch_item& it = items[i];
    if (it.A == nullptr || it.b == nullptr || it.x == nullptr || it.n <= 0 || it.lda < it.n ||
        it.nrhs <= 0 || it.ldb < it.n)
      return GMRESIR_EINVAL;
  }
  if (count == 0) return 0;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return GMRESIR_EHIP;
  // inputs produced on the caller's stream are complete before any worker
  // reads them
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return GMRESIR_EHIP;
  for (int64_t i = 0; i < count; ++i) items[i].status = GMRESIR_EINTERNAL;
  // largest first (n^3 work per factorisation, n^2 per right-hand side)
  std::vector<int64_t> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return items[a].n != items[b].n ? items[a].n > items[b].n : items[a].nrhs > items[b].nrhs;
  });
  int nw = workers <= 0 ? kDefaultWorkers : std::min(workers, kMaxWorkers);
  nw = (int)std::min<int64_t>(nw, count);
  std::atomic<int64_t> next{0};
  std::vector<Worker> ws((size_t)nw);
  std::vector<std::thread> th;
  th.reserve((size_t)nw);
  try {
    for (int w = 0; w < nw; ++w)
      th.emplace_back(run_worker, device, items, &order, &next, opts, &ws[(size_t)w]);
  } catch (...) {
    // a thread could not be started: the ones running finish the batch
  }
  for (auto& t : th) t.join();
  if (th.empty()) return GMRESIR_ENOMEM;
  int rc = 0;
  for (auto& w : ws) {
    for (gmresir_ctx* h : w.handles) gmresir_free(h);
    if (w.rc != 0 && rc == 0) rc = w.rc;
  }
  if (rc != 0) return rc;
  for (int64_t i = 0; i < count; ++i)
    if (items[i].status < 0) return items[i].status;
  return 0;
}
