// Batches of independent ROKS systems: a host-side work queue over contexts,
// longest (estimated) first, drained by a pool of threads.  Each worker
// thread has a stream of its own, created together at batch creation so
// that they spread evenly over the device's few hardware queues (streams
// are bound to queues as they are created, so the contexts' own streams,
// created one per context and at no particular time, may pile onto the same
// queue); while a worker runs a context, that context's launches go to the
// worker's stream, and the launches of different systems overlap on the GPU.
// Each context is driven by one thread at a time, which keeps its host-side
// state single-threaded.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "roks_internal.h"

struct roks_batch_s {
  std::vector<roks_ctx> ctxs;
  std::vector<int> order;  // queue: decreasing cost
  int workers = 1;
  int device = 0;                    // device of the worker streams
  std::vector<hipStream_t> streams;  // one per worker
  ~roks_batch_s() {
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
  }
};

namespace {

double cost_estimate(const roks::Ctx& c) {
  const double n3 = (double)c.ntot;
  return (double)c.nb * n3 * std::log2(std::max(2.0, n3)) + (double)c.nproj * c.nb * c.npw;
}

// job(idx) -> roks_status; the context runs on worker w's stream when it is
// on the batch's device, its own stream otherwise
template <typename F>
void run_queue(roks_batch b, roks_status* status, F&& job) {
  const int n = (int)b->ctxs.size();
  std::atomic<int> next{0};
  auto worker = [&](int w) {
    for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
      const int idx = b->order[i];
      roks::Ctx& c = b->ctxs[idx]->c;
      roks_status st = hipSetDevice(c.device) == hipSuccess ? ROKS_OK : ROKS_ERR_HIP;
      const hipStream_t own = c.stream;
      const bool swap = c.device == b->device && w < (int)b->streams.size();
      if (st == ROKS_OK && swap) {
        // the context's own stream is idle before its launches move
        if (hipStreamSynchronize(own) != hipSuccess) st = ROKS_ERR_HIP;
        c.stream = b->streams[w];
      }
      if (st == ROKS_OK) st = job(idx);
      if (swap) {
        // and the worker's stream is drained before they move back
        if (hipStreamSynchronize(c.stream) != hipSuccess && st == ROKS_OK) st = ROKS_ERR_HIP;
        c.stream = own;
      }
      if (status) status[idx] = st;
    }
  };
  const int nw = std::max(1, std::min(b->workers, n));
  std::vector<std::thread> pool;
  pool.reserve(nw - 1);
  for (int t = 1; t < nw; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

roks_status roks_batch_create(const roks_ctx* ctxs, int32_t n, int32_t workers, roks_batch* out) {
  if (!out || !ctxs || n <= 0 || workers <= 0) return ROKS_ERR_ARG;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return ROKS_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return ROKS_ERR_ARG;  // one thread per context
  }
  roks_batch b = new (std::nothrow) roks_batch_s;
  if (!b) return ROKS_ERR_OOM;
  b->ctxs.assign(ctxs, ctxs + n);
  b->workers = workers;
  b->device = ctxs[0]->c.device;
  int prev = 0;
  bool ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(b->device) == hipSuccess;
  const int nw = std::min(workers, n);
  for (int w = 0; ok && w < nw; ++w) {
    hipStream_t st = nullptr;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (ok) b->streams.push_back(st);
  }
  (void)hipSetDevice(prev);
  if (!ok) {
    delete b;
    return ROKS_ERR_HIP;
  }
  b->order.resize(n);
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    b->order[i] = i;
    cost[i] = cost_estimate(ctxs[i]->c);
  }
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return cost[x] > cost[y]; });
  *out = b;
  return ROKS_OK;
}

roks_status roks_batch_destroy(roks_batch b) {
  if (!b) return ROKS_ERR_ARG;
  delete b;
  return ROKS_OK;
}

roks_status roks_batch_solve(roks_batch b, double tol, int32_t maxiter, double switch_tol,
                             roks_status* status, int32_t* iterations, roks_step_info* last) {
  if (!b || !(tol > 0) || maxiter <= 0 || switch_tol < 0) return ROKS_ERR_ARG;
  run_queue(b, status, [&](int i) {
    roks_ctx ctx = b->ctxs[i];
    roks_step_info info{};
    int32_t it = 0, it2 = 0;
    roks_status st = ROKS_OK;
    if (switch_tol > 0 && ctx->c.prec == ROKS_FP32) {
      st = roks_solve(ctx, switch_tol, maxiter, &info, &it);
      // a search that stalls in the FP32 tier above its resolution moves to
      // FP64 all the same (the orbitals are those of the last accepted step)
      if (st == ROKS_OK || st == ROKS_ERR_LINESEARCH) st = roks_set_precision(ctx, ROKS_FP64);
    }
    if (st == ROKS_OK) st = roks_solve(ctx, tol, maxiter, &info, &it2);
    if (iterations) iterations[i] = it + it2;
    if (last) last[i] = info;
    return st;
  });
  return ROKS_OK;
}

roks_status roks_batch_steps(roks_batch b, int32_t steps, roks_status* status) {
  if (!b || steps < 0) return ROKS_ERR_ARG;
  run_queue(b, status, [&](int i) {
    roks_status st = ROKS_OK;
    for (int k = 0; k < steps && st == ROKS_OK; ++k) st = roks_pcg_step(b->ctxs[i], nullptr);
    return st;
  });
  return ROKS_OK;
}

roks_status roks_batch_graph_steps(roks_batch b, int32_t k, roks_status* status, int32_t* accepted) {
  if (!b || k < 1) return ROKS_ERR_ARG;
  run_queue(b, status, [&](int i) {
    int32_t a = 0;
    const roks_status st = roks_graph_steps(b->ctxs[i], k, nullptr, &a);
    if (accepted) accepted[i] = a;
    return st;
  });
  return ROKS_OK;
}

}  // extern "C"
