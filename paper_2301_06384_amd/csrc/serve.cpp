// Serving loop: continuous admission of kernel-machine requests by device
// memory footprint, concurrent execution on a pool of streams.
//
// A request is admitted as soon as a worker slot is free and the sum of the
// footprints of running requests plus its own fits the budget (the basis
// storage of Table 2 dominates the footprint).  Requests are admitted in
// arrival order; a request larger than the whole budget fails with
// GK_ENOMEM.  Each admitted request runs the same kernel sequence on its own
// stream as it would alone, so its result is bitwise identical alone and in
// any mix; the device overlaps the kernels of concurrent requests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "gk_internal.h"

namespace gk {

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket;
  gk_request r;
  std::vector<int64_t> samples;
  std::vector<double> y;
  std::vector<double> poly;
  uint64_t foot;
  gk_result res{};
};

struct Server {
  std::mutex mu;
  std::condition_variable cv;       // scheduler / worker wakeups
  std::condition_variable done_cv;  // completions
  std::deque<Req*> pending;
  std::map<uint64_t, Req*> done;
  std::map<uint64_t, Req*> inflight;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  int max_active = 0;
  int active = 0;
  uint64_t budget = 0;
  uint64_t used = 0;
  uint64_t next_ticket = 1;
  bool running = false;
  bool stopping = false;
  Clock::time_point t0;
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
};

Server& srv() {
  static Server* s = new Server();
  return *s;
}

// Pop the next admissible request (FIFO); returns null when none fits now.
Req* admit_locked(Server& S) {
  if (S.pending.empty() || S.active >= S.max_active) return nullptr;
  Req* q = S.pending.front();
  if (q->foot > S.budget) {
    // can never run: fail it
    S.pending.pop_front();
    q->res.status = GK_ENOMEM;
    q->res.t_start_ms = q->res.t_complete_ms = S.now_ms();
    S.inflight.erase(q->ticket);
    S.done[q->ticket] = q;
    S.done_cv.notify_all();
    return admit_locked(S);
  }
  if (S.used + q->foot > S.budget) return nullptr;
  S.pending.pop_front();
  S.used += q->foot;
  S.active++;
  return q;
}

void worker_main(int idx) {
  Server& S = srv();
  hipStream_t st = S.streams[idx % S.streams.size()];
  set_thread_stream(st);
  for (;;) {
    Req* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv.wait(lk, [&] {
        if (S.stopping && S.pending.empty()) return true;
        if (S.pending.empty() || S.active >= S.max_active) return false;
        Req* f = S.pending.front();
        return f->foot > S.budget || S.used + f->foot <= S.budget;
      });
      if (S.stopping && S.pending.empty()) return;
      q = admit_locked(S);
      if (!q) continue;
      q->res.t_start_ms = S.now_ms();
    }
    gk_stats stats{};
    gk_phi phi = q->r.phi;
    if (phi.kind == GK_PHI_POLYNOMIAL) phi.poly = q->poly.data();
    CallArgs a{q->r.graph, q->samples.data(), q->r.s, &phi, q->r.m, q->r.variant, q->r.precision,
               q->r.flags & ~GK_IO_DEVICE, q->y.data(), q->r.gamma, nullptr, nullptr, q->r.coef_out,
               q->r.pred_out, &stats, true};
    int rc;
    try {
      rc = run_call(a, st);
    } catch (const Error& e) {
      set_detail(e.msg);
      rc = e.code;
    } catch (...) {
      rc = GK_EDEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(S.mu);
      q->res.status = rc;
      q->res.stats = stats;
      q->res.t_complete_ms = S.now_ms();
      S.used -= q->foot;
      S.active--;
      S.inflight.erase(q->ticket);
      S.done[q->ticket] = q;
    }
    S.done_cv.notify_all();
    S.cv.notify_all();
  }
}

}  // namespace
}  // namespace gk

extern "C" {

int gk_serve_start(int32_t max_active, uint64_t hbm_budget_bytes, int32_t n_streams) {
  using namespace gk;
  Server& S = srv();
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.running) return GK_OK;
  if (max_active < 1 || max_active > 64 || n_streams < 1 || n_streams > 16) return GK_EINVAL;
  try {
    uint64_t budget = hbm_budget_bytes;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      GK_HIP(hipMemGetInfo(&fr, &tot));
      budget = (uint64_t)(0.9 * (double)fr);
    }
    S.streams.clear();
    for (int i = 0; i < n_streams; ++i) {
      hipStream_t st;
      GK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      S.streams.push_back(st);
    }
    S.budget = budget;
    S.used = 0;
    S.max_active = max_active;
    S.active = 0;
    S.stopping = false;
    S.running = true;
    S.t0 = Clock::now();
    for (int i = 0; i < max_active; ++i) S.workers.emplace_back(worker_main, i);
    return GK_OK;
  } catch (const Error& e) {
    set_detail(e.msg);
    return e.code;
  }
}

int gk_submit(const gk_request* r, uint64_t* ticket) {
  using namespace gk;
  if (!r || !ticket) return GK_EINVAL;
  Server& S = srv();
  if (r->flags & GK_IO_DEVICE) {
    set_detail("serving requests take host buffers");
    return GK_EINVAL;
  }
  if (!r->graph || !r->samples || !r->y || r->s < 1 || r->s > 1024 || r->m < 1 || r->m > 4096) return GK_EINVAL;
  if (r->phi.kind == GK_PHI_POLYNOMIAL && (!r->phi.poly || r->phi.poly_len < 1)) return GK_EINVAL;
  Req* q = new Req();
  q->r = *r;
  q->samples.assign(r->samples, r->samples + r->s);
  q->y.assign(r->y, r->y + r->s);
  if (r->phi.kind == GK_PHI_POLYNOMIAL) q->poly.assign(r->phi.poly, r->phi.poly + r->phi.poly_len);
  q->foot = footprint_bytes(r->graph->n, r->s, r->m, r->variant, r->precision, r->flags);
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.running || S.stopping) {
      delete q;
      return GK_ESHUTDOWN;
    }
    q->ticket = S.next_ticket++;
    q->res.t_submit_ms = S.now_ms();
    S.inflight[q->ticket] = q;
    S.pending.push_back(q);
    *ticket = q->ticket;
  }
  S.cv.notify_all();
  return GK_OK;
}

int gk_poll(uint64_t ticket, int64_t timeout_us, gk_result* res) {
  using namespace gk;
  Server& S = srv();
  std::unique_lock<std::mutex> lk(S.mu);
  auto ready = [&] { return S.done.count(ticket) > 0; };
  if (!ready()) {
    if (!S.inflight.count(ticket)) return GK_EINVAL;
    if (timeout_us == 0) return GK_EAGAIN;
    if (timeout_us < 0) S.done_cv.wait(lk, ready);
    else if (!S.done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return GK_EAGAIN;
  }
  Req* q = S.done[ticket];
  S.done.erase(ticket);
  if (res) *res = q->res;
  delete q;
  return GK_OK;
}

int gk_serve_stop(void) {
  using namespace gk;
  Server& S = srv();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.running) return GK_OK;
    S.stopping = true;
  }
  S.cv.notify_all();
  for (auto& t : S.workers) t.join();
  std::lock_guard<std::mutex> lk(S.mu);
  S.workers.clear();
  for (auto st : S.streams) (void)hipStreamSynchronize(st);
  cache_settle();
  for (auto st : S.streams) (void)hipStreamDestroy(st);
  S.streams.clear();
  S.running = false;
  S.stopping = false;
  return GK_OK;
}

}  // extern "C"
