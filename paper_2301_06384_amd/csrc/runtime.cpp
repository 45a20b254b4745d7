// ABI plumbing: error reporting, device memory (caching allocator or a
// caller-installed one), per-thread stream, phase timers, version.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>

#include "gk_internal.h"

namespace gk {

static thread_local std::string t_detail;
void set_detail(const std::string& msg) { t_detail = msg; }

// ------------------------------------------------------------ allocator
// Default: a size-keyed cache over hipMalloc.  A block returned to the cache
// carries an event recorded on the stream that last used it; a later
// allocation on another stream waits for that event before reuse.  Cached
// blocks go back to HIP when an allocation fails (the cache is released and
// the allocation retried once), on gk_trim, or at process exit.
namespace {
struct CachedBlock {
  void* p;
  size_t bytes;
  hipEvent_t ev;
};
struct Cache {
  std::mutex mu;
  std::multimap<size_t, CachedBlock> free_blocks;
  std::map<void*, size_t> live;
  uint64_t live_bytes = 0;
  uint64_t cached_bytes = 0;
};
Cache& cache() {
  static Cache* c = new Cache();   // never destroyed: blocks may outlive static destruction order
  return *c;
}
// the installed allocator hooks, read and written as one triple
std::mutex g_hook_mu;
void* (*g_alloc_fn)(size_t, void*) = nullptr;
void (*g_free_fn)(void*, void*) = nullptr;
void* g_alloc_ctx = nullptr;
thread_local hipStream_t t_stream = nullptr;
}  // namespace

hipStream_t current_stream() { return t_stream; }

void* dev_alloc(size_t bytes, FreeHook* made_by) {
  void* (*afn)(size_t, void*);
  FreeHook h;
  {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    afn = g_alloc_fn;
    h.fn = g_free_fn;
    h.ctx = g_alloc_ctx;
  }
  *made_by = h;
  if (afn) return afn(bytes, h.ctx);
  made_by->fn = nullptr;
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.free_blocks.lower_bound(bytes);
  if (it != c.free_blocks.end() && it->first <= bytes * 2 + (64u << 20)) {
    CachedBlock b = it->second;
    c.free_blocks.erase(it);
    c.cached_bytes -= b.bytes;
    if (b.ev) {
      if (hipEventQuery(b.ev) != hipSuccess) (void)hipStreamWaitEvent(t_stream, b.ev, 0);
      (void)hipEventDestroy(b.ev);
      // best-effort calls: do not leave their status behind for the next
      // launch check (the event's stream may have been destroyed since)
      (void)hipGetLastError();
    }
    c.live[b.p] = b.bytes;
    c.live_bytes += b.bytes;
    return b.p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once
    for (auto& kv : c.free_blocks) {
      if (kv.second.ev) {
        (void)hipEventSynchronize(kv.second.ev);
        (void)hipEventDestroy(kv.second.ev);
      }
      (void)hipFree(kv.second.p);
    }
    c.free_blocks.clear();
    c.cached_bytes = 0;
    (void)hipGetLastError();
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  c.live[p] = bytes;
  c.live_bytes += bytes;
  return p;
}

void dev_free(void* p, const FreeHook& made_by, bool settled) {
  if (!p) return;
  if (made_by.fn) {
    made_by.fn(p, made_by.ctx);
    return;
  }
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  const size_t b = it->second;
  c.live.erase(it);
  c.live_bytes -= b;
  hipEvent_t ev = nullptr;
  if (!settled && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
    if (hipEventRecord(ev, t_stream) != hipSuccess) {
      (void)hipEventDestroy(ev);
      ev = nullptr;
    }
  }
  (void)hipGetLastError();
  c.free_blocks.emplace(b, CachedBlock{p, b, ev});
  c.cached_bytes += b;
}

void set_thread_stream(hipStream_t s) { t_stream = s; }

uint64_t cache_trim() {
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  uint64_t released = 0;
  for (auto& kv : c.free_blocks) {
    if (kv.second.ev) {
      (void)hipEventSynchronize(kv.second.ev);
      (void)hipEventDestroy(kv.second.ev);
    }
    (void)hipFree(kv.second.p);
    released += kv.second.bytes;
  }
  c.free_blocks.clear();
  c.cached_bytes = 0;
  (void)hipGetLastError();
  return released;
}

void cache_settle() {
  Cache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto& kv : c.free_blocks) {
    if (kv.second.ev) {
      (void)hipEventSynchronize(kv.second.ev);
      (void)hipEventDestroy(kv.second.ev);
      kv.second.ev = nullptr;
    }
  }
  (void)hipGetLastError();
}

// ------------------------------------------------------------ timers
void PhaseTimer::begin(int phase) {
  if (!on) return;
  end();
  hipEvent_t a;
  GK_HIP(hipEventCreate(&a));
  GK_HIP(hipEventRecord(a, st));
  cur = phase;
  cur_start = a;
}
void PhaseTimer::end() {
  if (!on || cur < 0) return;
  hipEvent_t b;
  GK_HIP(hipEventCreate(&b));
  GK_HIP(hipEventRecord(b, st));
  ev.push_back({cur, {cur_start, b}});
  cur = -1;
  cur_start = nullptr;
}
void PhaseTimer::collect(gk_stats* s) {
  if (!on) return;
  end();
  if (!s) return;
  double t[PH_TOTAL + 1] = {0};
  double nspmm = 0;
  for (auto& e : ev) {
    GK_HIP(hipEventSynchronize(e.second.second));
    float ms = 0;
    GK_HIP(hipEventElapsedTime(&ms, e.second.first, e.second.second));
    t[e.first] += ms;
    if (e.first == PH_SPMM) nspmm += 1;
  }
  s->t_spmm_ms = t[PH_SPMM];
  s->t_orth_ms = t[PH_ORTH];
  s->t_reorth_ms = t[PH_REORTH];
  s->t_phi_ms = t[PH_PHI];
  s->t_asm_ms = t[PH_ASM];
  s->t_fit_ms = t[PH_FIT];
  s->t_total_ms = t[PH_TOTAL];
  s->spmm_launches = nspmm;
}
// ------------------------------------------------------------ kernel timer
namespace {
const char* const kKernelClassName[KC_COUNT] = {
    "spmm_diff",          "panel_gramv",     "panel_update_self", "panel_apply_self", "panel_apply_write",
    "gram",               "tsgemm",          "arch_gram",         "arch_update",
    "reduce_parts",       "cholqr",          "omega",             "banded_factor",    "banded_solve",
    "cheb_step",          "jacobi_eig",      "assemble",          "predict"};
struct KtRec {
  int cls;
  hipEvent_t a, b;
  double bytes, flops;
  const int* flag;   // device flag of a flag-gated launch (work only when *flag != 0)
};
struct KtState {
  bool on = false;
  std::vector<KtRec> recs;
  int cur = -1;
  hipEvent_t cur_a = nullptr;
  gk_kernel_timing agg[KC_COUNT];
  int nagg = 0;
};
thread_local KtState t_kt;
}  // namespace

void kt_start(bool on) {
  for (auto& r : t_kt.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (t_kt.cur_a) (void)hipEventDestroy(t_kt.cur_a);
  t_kt.cur_a = nullptr;
  t_kt.on = on;
  t_kt.recs.clear();
  t_kt.cur = -1;
}
void kt_begin(int cls, hipStream_t st) {
  if (!t_kt.on) return;
  hipEvent_t a;
  GK_HIP(hipEventCreate(&a));
  GK_HIP(hipEventRecord(a, st));
  t_kt.cur = cls;
  t_kt.cur_a = a;
}
void kt_end(hipStream_t st, double bytes, double flops, const int* flag) {
  if (!t_kt.on || t_kt.cur < 0) return;
  hipEvent_t b;
  GK_HIP(hipEventCreate(&b));
  GK_HIP(hipEventRecord(b, st));
  t_kt.recs.push_back({t_kt.cur, t_kt.cur_a, b, bytes, flops, flag});
  t_kt.cur = -1;
  t_kt.cur_a = nullptr;
}
void kt_finish() {
  if (!t_kt.on) return;
  for (int c = 0; c < KC_COUNT; ++c) {
    gk_kernel_timing& g = t_kt.agg[c];
    std::memset(&g, 0, sizeof(g));
    std::strncpy(g.name, kKernelClassName[c], sizeof(g.name) - 1);
  }
  for (auto& r : t_kt.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      int active = 1;
      if (r.flag && hipMemcpy(&active, r.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) active = 1;
      gk_kernel_timing& g = t_kt.agg[r.cls];
      g.launches += 1;
      g.total_ms += ms;
      if (active) {
        g.alg_bytes += r.bytes;
        g.alg_flops += r.flops;
      }
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  t_kt.recs.clear();
  t_kt.nagg = KC_COUNT;
  t_kt.on = false;
}

PhaseTimer::~PhaseTimer() {
  for (auto& e : ev) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  if (cur_start) (void)hipEventDestroy(cur_start);
}

}  // namespace gk

// ------------------------------------------------------------------ ABI
extern "C" {

const char* gk_strerror(int code) {
  switch (code) {
    case GK_OK: return "ok";
    case GK_EINVAL: return "invalid argument";
    case GK_ENOTSYM: return "Laplacian not symmetric";
    case GK_ENOTLAP: return "not a graph Laplacian (positive off-diagonal or negative diagonal excess)";
    case GK_EDUPSAMPLE: return "duplicate sample nodes";
    case GK_ERANGE: return "sample node out of range";
    case GK_ENOMEM: return "out of device memory or refused by admission";
    case GK_ENOTSPD: return "kernel system not solvable";
    case GK_EDEVICE: return "HIP device error";
    case GK_EUNSUPPORTED: return "unsupported combination";
    case GK_EAGAIN: return "not finished";
    case GK_ESHUTDOWN: return "serving loop stopped";
    default: return "unknown error";
  }
}

const char* gk_last_error_detail(void) { return gk::t_detail.c_str(); }

int gk_set_allocator(void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return GK_EINVAL;
  std::lock_guard<std::mutex> lk(gk::g_hook_mu);
  gk::g_alloc_fn = alloc_fn;
  gk::g_free_fn = free_fn;
  gk::g_alloc_ctx = ctx;
  return GK_OK;
}

int gk_trim(uint64_t* released_bytes) {
  const uint64_t r = gk::cache_trim();
  if (released_bytes) *released_bytes = r;
  return GK_OK;
}

int gk_set_stream(void* hip_stream) {
  gk::t_stream = static_cast<hipStream_t>(hip_stream);
  return GK_OK;
}

const char* gk_version(void) { return "gk 0.1 gfx950"; }

}  // extern "C"

extern "C" int gk_kernel_timings(gk_kernel_timing* out, int32_t cap, int32_t* count) {
  using namespace gk;
  if (!count || cap < 0 || (cap > 0 && !out)) return GK_EINVAL;
  const int n = std::min<int>(cap, t_kt.nagg);
  for (int i = 0; i < n; ++i) out[i] = t_kt.agg[i];
  *count = t_kt.nagg;
  return GK_OK;
}
