// Serving loop: continuous batching of kernel-machine requests with
// admission by device memory footprint.
//
// A request is admitted as soon as a slot is free and the sum of the
// footprints of running requests plus its own fits the budget (the basis
// storage of Table 2 dominates the footprint); requests are admitted in
// arrival order, and one larger than the whole budget fails with GK_ENOMEM.
//
// Classical block Lanczos requests are batched at the iteration level: a
// stepper thread advances every admitted request by one Lanczos step per
// round, with one grouped SpMM launch per graph over the requests' blocks
// and one batched launch of their CholQR factors per pass; a request that
// arrives joins at the next round, and one that has taken its m steps leaves
// for its phi stage, fit and predictor on a second stream while the others
// go on.  A completion thread copies results back as they finish.  The other
// variants run whole on a worker of their own.  Every request executes the
// kernels of a lone call on the same operands in the same order, so its
// result is bitwise identical alone and in any mix.
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
  gk_phi phi{};
  gk_stats stats{};
  uint64_t foot;
  gk_result res{};
  BatchCall* B = nullptr;
  CallArgs args() {
    phi = r.phi;
    if (phi.kind == GK_PHI_POLYNOMIAL) phi.poly = poly.data();
    return CallArgs{r.graph, samples.data(), r.s, &phi, r.m, r.variant, r.precision, r.flags & ~GK_IO_DEVICE,
                    y.data(), r.gamma, nullptr, nullptr, r.coef_out, r.pred_out, &stats, true};
  }
};

struct Server {
  std::mutex mu;
  std::condition_variable cv;       // stepper / worker wakeups
  std::condition_variable done_cv;  // completions
  std::condition_variable fin_cv;   // completion-thread wakeups
  std::deque<Req*> pending;         // submitted, not admitted
  std::deque<Req*> admitted;        // admitted lockstep requests, not begun
  std::deque<Req*> solo;            // admitted requests of the other variants
  std::deque<Req*> finishing;       // lockstep requests whose outputs are enqueued
  std::map<uint64_t, Req*> done;
  std::map<uint64_t, Req*> inflight;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;   // [0], [1] phi stage and outputs, [2] other variants, [3..] the
                                      // per-graph lockstep groups (all shared when there are fewer)
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

void finish_locked(Server& S, Req* q, int rc) {
  q->res.status = rc;
  q->res.stats = q->stats;
  q->res.t_complete_ms = S.now_ms();
  S.used -= q->foot;
  S.active--;
  S.inflight.erase(q->ticket);
  S.done[q->ticket] = q;
}

// Admit pending requests in arrival order while slots and memory allow.
void admit_locked(Server& S) {
  while (!S.pending.empty() && S.active < S.max_active) {
    Req* q = S.pending.front();
    if (q->foot > S.budget) {
      // can never run: fail it
      S.pending.pop_front();
      q->res.status = GK_ENOMEM;
      q->res.t_start_ms = q->res.t_complete_ms = S.now_ms();
      S.inflight.erase(q->ticket);
      S.done[q->ticket] = q;
      S.done_cv.notify_all();
      continue;
    }
    if (S.used + q->foot > S.budget) break;
    S.pending.pop_front();
    S.used += q->foot;
    S.active++;
    q->res.t_start_ms = S.now_ms();
    CallArgs a = q->args();
    if (batch_eligible(a)) {
      S.admitted.push_back(q);
    } else {
      S.solo.push_back(q);
      S.cv.notify_all();   // the other thread waiting on cv may be the one to take it
    }
  }
}

// Requests on one graph advance together: one round enqueues one Lanczos
// step of each of them on the group's stream.  Groups of different graphs
// advance independently (a small graph's requests never wait for a large
// graph's step), each at most kAhead rounds ahead of the device, so that a
// request admitted now joins its group's next rounds on the device rather
// than queueing behind rounds enqueued long in advance.
struct Group {
  hipStream_t st = nullptr;
  std::vector<Req*> live;           // in admission order
  std::deque<hipEvent_t> rounds;    // completion events of enqueued rounds
};

void stepper_main() {
  Server& S = srv();
  // finishing streams: [0] and [1], taken in turn
  size_t next_fin = 0;
  constexpr size_t kAhead = 2;
  std::map<const gk_graph*, Group> groups;
  size_t next_stream = 0;
  auto group_of = [&](const gk_graph* g) -> Group& {
    Group& G = groups[g];
    if (!G.st) {
      // group streams: the pool beyond the finishing and other-variant streams
      const size_t first = std::min<size_t>(3, S.streams.size() - 1);
      const size_t span = S.streams.size() - first;
      G.st = S.streams[first + (next_stream++ % span)];
    }
    return G;
  };
  auto any_live = [&]() {
    for (auto& kv : groups)
      if (!kv.second.live.empty()) return true;
    return false;
  };
  for (;;) {
    std::vector<Req*> fresh;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      const bool busy = any_live();
      S.cv.wait(lk, [&] {
        admit_locked(S);
        if (!S.admitted.empty() || busy) return true;
        return S.stopping && S.pending.empty() && S.active == 0;
      });
      if (S.admitted.empty() && !busy) {
        S.cv.notify_all();   // wake the worker to let it see the stop too
        for (auto& kv : groups)
          for (hipEvent_t e : kv.second.rounds) (void)hipEventDestroy(e);
        return;
      }
      while (!S.admitted.empty()) {
        fresh.push_back(S.admitted.front());
        S.admitted.pop_front();
      }
    }
    // begin the newly admitted requests (validation, start block) on their
    // graph's stream
    for (Req* q : fresh) {
      Group& G = group_of(q->r.graph);
      set_thread_stream(G.st);
      try {
        q->B = batch_begin(q->args(), G.st);
        G.live.push_back(q);
      } catch (const Error& e) {
        set_detail(e.msg);
        std::lock_guard<std::mutex> lk(S.mu);
        finish_locked(S, q, e.code);
        S.done_cv.notify_all();
      } catch (...) {
        std::lock_guard<std::mutex> lk(S.mu);
        finish_locked(S, q, GK_EDEVICE);
        S.done_cv.notify_all();
      }
    }
    // one round for every group that is not kAhead rounds ahead
    bool progressed = false;
    Group* oldest = nullptr;
    for (auto& kv : groups) {
      Group& G = kv.second;
      while (!G.rounds.empty() && hipEventQuery(G.rounds.front()) == hipSuccess) {
        (void)hipEventDestroy(G.rounds.front());
        G.rounds.pop_front();
      }
      (void)hipGetLastError();
      if (G.live.empty()) continue;
      if (G.rounds.size() >= kAhead) {
        if (!oldest) oldest = &G;
        continue;
      }
      set_thread_stream(G.st);
      std::vector<BatchCall*> calls;
      for (Req* q : G.live) calls.push_back(q->B);
      std::vector<Req*> ended;
      try {
        batch_step(calls, G.st);
        hipEvent_t ev;
        GK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        GK_HIP(hipEventRecord(ev, G.st));
        G.rounds.push_back(ev);
        std::vector<Req*> keep;
        for (Req* q : G.live) (batch_stepping(q->B) ? keep : ended).push_back(q);
        G.live.swap(keep);
      } catch (...) {
        // a launch failed: every request of the group ends with a device error
        std::lock_guard<std::mutex> lk(S.mu);
        for (Req* q : G.live) {
          batch_free(q->B);
          q->B = nullptr;
          finish_locked(S, q, GK_EDEVICE);
        }
        G.live.clear();
        S.done_cv.notify_all();
        continue;
      }
      progressed = true;
      // requests that took their last step: phi stage, fit and predictor on
      // a finishing stream, then to the completion thread
      for (Req* q : ended) {
        hipStream_t fin = S.streams[(next_fin++ % 2) % S.streams.size()];
        set_thread_stream(fin);
        int rc = GK_OK;
        try {
          batch_finish(q->B, G.st, fin);
        } catch (const Error& e) {
          set_detail(e.msg);
          rc = e.code;
        } catch (...) {
          rc = GK_EDEVICE;
        }
        std::lock_guard<std::mutex> lk(S.mu);
        if (rc != GK_OK) {
          batch_free(q->B);
          q->B = nullptr;
          finish_locked(S, q, rc);
          S.done_cv.notify_all();
        } else {
          S.finishing.push_back(q);
          S.fin_cv.notify_all();
        }
      }
    }
    // every group is kAhead rounds ahead: wait for the oldest round of one
    if (!progressed && oldest) {
      (void)hipEventSynchronize(oldest->rounds.front());
      (void)hipGetLastError();
    }
  }
}

void completion_main() {
  Server& S = srv();
  set_thread_stream(S.streams[1 % S.streams.size()]);
  for (;;) {
    Req* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.fin_cv.wait(lk, [&] { return !S.finishing.empty() || (S.stopping && S.active == 0); });
      if (S.finishing.empty()) return;
      q = S.finishing.front();
      S.finishing.pop_front();
    }
    int rc;
    try {
      rc = batch_complete(q->B);
    } catch (const Error& e) {
      set_detail(e.msg);
      rc = e.code;
    } catch (...) {
      rc = GK_EDEVICE;
    }
    batch_free(q->B);
    q->B = nullptr;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      finish_locked(S, q, rc);
    }
    S.done_cv.notify_all();
    S.cv.notify_all();
  }
}

// requests of the other variants, whole, one after another
void solo_main() {
  Server& S = srv();
  hipStream_t st = S.streams[2 % S.streams.size()];
  set_thread_stream(st);
  for (;;) {
    Req* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv.wait(lk, [&] {
        admit_locked(S);
        return !S.solo.empty() || (S.stopping && S.pending.empty() && S.active == 0);
      });
      if (S.solo.empty()) {
        S.cv.notify_all();
        return;
      }
      q = S.solo.front();
      S.solo.pop_front();
    }
    CallArgs a = q->args();
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
      finish_locked(S, q, rc);
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
    S.threads.emplace_back(stepper_main);
    S.threads.emplace_back(completion_main);
    S.threads.emplace_back(solo_main);
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
  S.fin_cv.notify_all();
  for (auto& t : S.threads) {
    // the completion thread waits for the active count to drop to zero
    t.join();
    S.fin_cv.notify_all();
    S.cv.notify_all();
  }
  std::lock_guard<std::mutex> lk(S.mu);
  S.threads.clear();
  for (auto st : S.streams) (void)hipStreamSynchronize(st);
  cache_settle();
  for (auto st : S.streams) (void)hipStreamDestroy(st);
  S.streams.clear();
  S.running = false;
  S.stopping = false;
  return GK_OK;
}

}  // extern "C"
