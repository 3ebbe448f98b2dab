// C-ABI entry points of the t-SGNE library (declared in include/tsgne.h):
// argument validation, the graph handle and its device memory, the step
// workspace, and the sequencing of the kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace tsgne {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

tsgne_status fail(tsgne_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

tsgne_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? TSGNE_E_NOMEM : TSGNE_E_DEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
std::mutex g_pool_mutex;
std::map<int, hipMemPool_t> g_pools;  // one per device, kept until the process ends
}  // namespace

hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    auto it = g_pools.find(dev);
    if (it == g_pools.end()) {
      hipMemPoolProps props{};
      props.allocType = hipMemAllocationTypePinned;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      e = hipMemPoolCreate(&pool, &props);
      if (e != hipSuccess) return e;
      uint64_t keep = (uint64_t)1 << 30;  // cached bytes kept across synchronisations
      e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return e;
      }
      g_pools[dev] = pool;
    } else {
      pool = it->second;
    }
  }
  return hipMallocFromPoolAsync(p, bytes ? bytes : 1, pool, s);
}

void scratch_free(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

namespace {

void free_workspace(Workspace& ws) {
  dfree(ws.items);
  dfree(ws.part);
  dfree(ws.zpart);
  dfree(ws.zpart32);
  dfree(ws.Z);
  dfree(ws.attract);
  dfree(ws.klpart);
  dfree(ws.klout);
  dfree(ws.tstep);
  if (ws.pinned) (void)hipHostFree(ws.pinned);
  ws.pinned = nullptr;
  ws.plan = RepulsionPlan{};
}

void timer_destroy(PhaseTimer& t);

}  // namespace

void free_graph(tsgne_graph* g) {
  if (!g) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  free_workspace(g->ws);
  timer_destroy(g->timer);
  dfree(g->row_ptr);
  dfree(g->col);
  dfree(g->mirror);
  dfree(g->row_of);
  dfree(g->P);
  dfree(g->beta);
  dfree(g->heavy);
  (void)hipSetDevice(cur);
  delete g;
}

namespace {


// --- phase timing -----------------------------------------------------------

hipEvent_t timer_event(PhaseTimer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a timed launch; returns the index to close, or -1.
int timer_begin(tsgne_graph* g, int phase, hipStream_t s) {
  PhaseTimer& t = g->timer;
  if (!t.enabled) return -1;
  hipEvent_t a = timer_event(t), b = timer_event(t);
  if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
    if (a) t.pool.push_back(a);
    if (b) t.pool.push_back(b);
    return -1;
  }
  t.pending.push_back({phase, a, b});
  return (int)t.pending.size() - 1;
}

void timer_end(tsgne_graph* g, int idx, hipStream_t s) {
  if (idx < 0) return;
  (void)hipEventRecord(g->timer.pending[(size_t)idx].stop, s);
}

// Folds completed event pairs into the totals (waits for each stop event).
hipError_t timer_resolve(tsgne_graph* g) {
  PhaseTimer& t = g->timer;
  hipError_t err = hipSuccess;
  for (auto& p : t.pending) {
    hipError_t e = hipEventSynchronize(p.stop);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e == hipSuccess) {
      t.ms[p.phase] += ms;
      t.launches[p.phase] += 1;
    } else if (err == hipSuccess) {
      err = e;
    }
    t.pool.push_back(p.start);
    t.pool.push_back(p.stop);
  }
  t.pending.clear();
  return err;
}

void timer_destroy(PhaseTimer& t) {
  for (auto& p : t.pending) {
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
  t.pending.clear();
  t.pool.clear();
}

struct Timed {
  tsgne_graph* g;
  int idx;
  hipStream_t s;
  Timed(tsgne_graph* g_, int phase, hipStream_t s_) : g(g_), idx(timer_begin(g_, phase, s_)), s(s_) {}
  ~Timed() { timer_end(g, idx, s); }
};

}  // namespace

tsgne_status graph_structure(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d, hipStream_t s,
                             tsgne_graph** out) {
  *out = nullptr;
  tsgne_graph* g = new (std::nothrow) tsgne_graph();
  if (!g) return fail(TSGNE_E_NOMEM, "host allocation failed");
  g->n = n;
  g->nnz = nnz;
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return fail(TSGNE_E_DEVICE, "no HIP device");
  }
  struct Cleanup {
    tsgne_graph* g;
    ~Cleanup() { free_graph(g); }
  } guard{g};

  // temporaries from the stream-ordered pool (freeing them does not wait for
  // other streams' work, unlike hipFree)
  ScratchBlock tmp;
  tmp.s = s;
  const size_t o_counters = 256, o_partial = 512;
  TSGNE_HIP(scratch_alloc(&tmp.p, o_partial + sizeof(int2) * (size_t)row_check_blocks(n), s), "allocate CSR checks");
  uint32_t* err = static_cast<uint32_t*>(tmp.p);
  int32_t* counters = reinterpret_cast<int32_t*>(static_cast<char*>(tmp.p) + o_counters);
  int2* partial = reinterpret_cast<int2*>(static_cast<char*>(tmp.p) + o_partial);

  const int32_t heavy_cap = (int32_t)std::min<int64_t>(n, nnz / (kHeavyDegree + 1) + 1);
  TSGNE_HIP(dalloc(&g->row_ptr, (size_t)n + 1), "allocate row_ptr");
  TSGNE_HIP(dalloc(&g->col, (size_t)nnz), "allocate col");
  TSGNE_HIP(dalloc(&g->mirror, (size_t)nnz), "allocate mirror");
  TSGNE_HIP(dalloc(&g->row_of, (size_t)nnz), "allocate row_of");
  TSGNE_HIP(dalloc(&g->P, (size_t)nnz), "allocate P");
  TSGNE_HIP(dalloc(&g->beta, (size_t)n), "allocate beta");
  TSGNE_HIP(dalloc(&g->heavy, (size_t)heavy_cap), "allocate heavy rows");

  TSGNE_HIP(hipMemcpyAsync(g->row_ptr, row_ptr_d, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s),
            "copy row_ptr");
  if (nnz > 0)
    TSGNE_HIP(hipMemcpyAsync(g->col, col_d, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s), "copy col");
  TSGNE_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s), "clear error word");
  TSGNE_HIP(hipMemsetAsync(counters, 0, 2 * sizeof(int32_t), s), "clear counters");

  // 1. row_ptr must be valid before any kernel indexes col with it.
  TSGNE_HIP(launch_check_rows(g->row_ptr, n, nnz, kHeavyDegree, err, counters, partial, g->heavy, nullptr, heavy_cap, s),
            "launch row check");
  uint32_t host_err = 0;
  int32_t host_counters[2] = {0, 0};
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipMemcpyAsync(host_counters, counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s), "read counters");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise row check");
  if (host_err) return fail(TSGNE_E_GRAPH, "row_ptr is not nondecreasing from 0 to nnz");
  g->nonisolated = host_counters[0];
  g->n_heavy = std::min(host_counters[1], heavy_cap);

  // 2. Column checks, symmetry, mirror index.
  TSGNE_HIP(launch_mirror(g->row_ptr, g->col, n, nnz, g->mirror, g->row_of, err, s), "launch mirror");
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise CSR check");
  if (host_err) {
    std::string why = "CSR is not canonical/symmetric:";
    if (host_err & kErrColRange) why += " column outside [0, n);";
    if (host_err & kErrSelfLoop) why += " self-loop;";
    if (host_err & kErrOrder) why += " columns not strictly ascending;";
    if (host_err & kErrAsym) why += " entry (i,j) without (j,i);";
    return fail(TSGNE_E_GRAPH, why);
  }
  guard.g = nullptr;
  *out = g;
  return TSGNE_OK;
}

tsgne_status validate_params(const tsgne_params* p) {
  if (!std::isfinite(p->early_exaggeration) || p->early_exaggeration <= 0.f)
    return fail(TSGNE_E_INVAL, "early_exaggeration must be finite and > 0");
  if (p->exaggeration_iters < 0) return fail(TSGNE_E_INVAL, "exaggeration_iters must be >= 0");
  if (!std::isfinite(p->learning_rate)) return fail(TSGNE_E_INVAL, "learning_rate must be finite");
  if (!std::isfinite(p->momentum_early) || !std::isfinite(p->momentum_late) || p->momentum_early < 0.f ||
      p->momentum_late < 0.f || p->momentum_early >= 1.f || p->momentum_late >= 1.f)
    return fail(TSGNE_E_INVAL, "momentum must lie in [0, 1)");
  if (!std::isfinite(p->min_gain) || p->min_gain < 0.f) return fail(TSGNE_E_INVAL, "min_gain must be >= 0");
  if (p->precision != TSGNE_PREC_SPLIT && p->precision != TSGNE_PREC_FP32)
    return fail(TSGNE_E_INVAL, "precision must be TSGNE_PREC_SPLIT or TSGNE_PREC_FP32");
  if (p->kl_every < 0) return fail(TSGNE_E_INVAL, "kl_every must be >= 0");
  if (p->repulsion < TSGNE_REPULSION_AUTO || p->repulsion > TSGNE_REPULSION_SYMMETRIC)
    return fail(TSGNE_E_INVAL, "unknown repulsion variant");
  if (p->tile_rows != 0 && !tile_rows_supported(p->tile_rows))
    return fail(TSGNE_E_INVAL, "tile_rows must be 0, 1, 2, 4, 8, 12, 14, 15 or 16");
  return TSGNE_OK;
}

float effective_eta(const tsgne_graph* g, const tsgne_params* p) {
  if (p->learning_rate > 0.f) return p->learning_rate;
  return std::max((float)g->n / (4.0f * p->early_exaggeration), 50.0f);
}

// Allocates (or re-plans) the per-step buffers for the requested tiling.
tsgne_status ensure_workspace(tsgne_graph* g, const tsgne_params* p) {
  Workspace& ws = g->ws;
  const RepulsionPlan want = make_plan(g->n, p->tile_rows, p->repulsion);
  const bool same = ws.part && ws.plan.R == want.R && ws.plan.variant == want.variant;
  if (same) return TSGNE_OK;
  if (ws.part) {
    // Buffers may still be in use by queued work on any stream.
    TSGNE_HIP(hipDeviceSynchronize(), "synchronise before re-planning");
  }
  free_workspace(ws);
  ws.plan = want;
  const RepulsionPlan& pl = ws.plan;
  // Symmetric plans dispatch the diagonal tiles (one resident row per lane
  // per pass, the slower kind) first, then the off-diagonal tiles row by row,
  // and last the tiles against the last block (a, nb - 1), which is partly
  // filled when T does not divide n: the launch's tail is made of its
  // shortest tiles.  A tile's position in this list is also its Z partial's
  // slot, i.e. Z's summation order.
  std::vector<int2> items;
  items.reserve((size_t)pl.items);
  if (pl.variant == TSGNE_REPULSION_DIRECT) {
    for (int32_t a = 0; a < pl.nb; ++a)
      for (int32_t b = 0; b < pl.nb; ++b) items.push_back(make_int2(a, b));
  } else {
    for (int32_t a = 0; a < pl.nb; ++a) items.push_back(make_int2(a, a));
    for (int32_t a = 0; a < pl.nb; ++a)
      for (int32_t b = a + 1; b < pl.nb - 1; ++b) items.push_back(make_int2(a, b));
    for (int32_t a = 0; a < pl.nb - 1; ++a) items.push_back(make_int2(a, pl.nb - 1));
  }
  const size_t part_len = (size_t)pl.nb * pl.nb * pl.T;
  ws.kl_blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(1024, (g->nnz + 255) / 256));
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dalloc(&ws.items, items.size());
  if (e == hipSuccess) e = dalloc(&ws.part, part_len);
  if (e == hipSuccess) e = dalloc(&ws.zpart, (size_t)pl.items);
  if (e == hipSuccess) e = dalloc(&ws.zpart32, (size_t)pl.items);
  if (e == hipSuccess) e = dalloc(&ws.Z, 1);
  if (e == hipSuccess) e = dalloc(&ws.attract, (size_t)g->n);
  if (e == hipSuccess) e = dalloc(&ws.klpart, (size_t)ws.kl_blocks);
  if (e == hipSuccess) e = dalloc(&ws.klout, 1);
  if (e == hipSuccess) e = dalloc(&ws.tstep, 2);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ws.pinned), 64 * sizeof(double), 0);
  if (e == hipSuccess)
    e = hipMemcpy(ws.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_workspace(ws);
    return hip_fail(e, "allocate step workspace");
  }
  return TSGNE_OK;
}

namespace {

// Repulsion partials, Z, attraction: everything the gradient needs at Y.
// Inside a run (tstep set) the Z sum also advances the device step counter,
// and with a trace the step's input layout is sampled for KL when due (with
// the Z just summed at it, before the update moves it).
tsgne_status enqueue_forces(tsgne_graph* g, const float* Y, int precision, hipStream_t s, int32_t* tstep = nullptr,
                            int32_t kl_every = 0, double* trace = nullptr) {
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  {
    Timed tm(g, TSGNE_PHASE_REPULSION, s);
    TSGNE_HIP(launch_repulsion(g->ws, g->n, Y2, precision, s), "launch repulsion");
  }
  {
    Timed tm(g, TSGNE_PHASE_ZSUM, s);
    TSGNE_HIP(launch_zsum(g->ws, precision, s, tstep), "launch Z reduction");
  }
  if (trace) {
    Timed tm(g, TSGNE_PHASE_KL, s);
    TSGNE_HIP(launch_kl(g, Y2, s, tstep, kl_every, trace), "launch KL sample");
  }
  {
    Timed tm(g, TSGNE_PHASE_ATTRACT, s);
    TSGNE_HIP(launch_attract(g, Y2, precision, g->ws.attract, s), "launch attraction");
  }
  return TSGNE_OK;
}

tsgne_status check_graph(const tsgne_graph* g) {
  if (!g) return fail(TSGNE_E_INVAL, "graph is NULL");
  return TSGNE_OK;
}

tsgne_status step_impl(tsgne_graph* g, float* Y, float* U, float* G, int32_t t, const tsgne_params* p, float* grad_out,
                       double* Z_out, hipStream_t s) {
  const bool early = t < p->exaggeration_iters;
  const float alpha = early ? p->early_exaggeration : 1.0f;
  const float mom = early ? p->momentum_early : p->momentum_late;
  tsgne_status st = enqueue_forces(g, Y, p->precision, s);
  if (st != TSGNE_OK) return st;
  Timed tm(g, TSGNE_PHASE_UPDATE, s);
  TSGNE_HIP(launch_update(g, reinterpret_cast<float2*>(Y), reinterpret_cast<float2*>(U), reinterpret_cast<float2*>(G),
                          alpha, mom, effective_eta(g, p), p->min_gain, p->precision, true,
                          reinterpret_cast<float2*>(grad_out), Z_out, s),
            "launch update");
  return TSGNE_OK;
}

// KL at Y (eq. (5), unexaggerated P): Z from a pass over the repulsion's tiles
// that forms only the weights (in the split precision, bitwise the Z a step at
// Y sums), then the FP64 sum over the stored entries.  trace (nullable)
// receives the value on the device as well.
tsgne_status enqueue_kl(tsgne_graph* g, const float* Y, hipStream_t s, double* trace = nullptr) {
  const float2* Y2 = reinterpret_cast<const float2*>(Y);
  Timed tm(g, TSGNE_PHASE_KL, s);
  TSGNE_HIP(launch_zonly(g->ws, g->n, Y2, TSGNE_PREC_SPLIT, s), "launch Z pass");
  TSGNE_HIP(launch_zsum(g->ws, TSGNE_PREC_SPLIT, s), "launch Z reduction");
  TSGNE_HIP(launch_kl(g, Y2, s, nullptr, 0, trace), "launch KL");
  return TSGNE_OK;
}

tsgne_status kl_impl(tsgne_graph* g, const float* Y, double* kl_h, hipStream_t s) {
  if (tsgne_status st = enqueue_kl(g, Y, s)) return st;
  TSGNE_HIP(hipMemcpyAsync(g->ws.pinned, g->ws.klout, sizeof(double), hipMemcpyDeviceToHost, s), "copy KL");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise KL");
  *kl_h = g->ws.pinned[0];
  return TSGNE_OK;
}

// Steps per captured HIP graph of a run (when sampling KL, the smallest
// multiple of kl_every at or above it, so that every replay samples at the
// same positions).
constexpr int32_t kRunChunk = 32;

// One step of a run on the device step counter: alpha and the momentum are
// read on the device, so the same launches serve every step.
tsgne_status enqueue_run_step(tsgne_graph* g, float* Y, float* U, float* G, const tsgne_params* p, float eta,
                              double* trace, hipStream_t s) {
  int32_t* tstep = g->ws.tstep;
  if (tsgne_status st = enqueue_forces(g, Y, p->precision, s, tstep, p->kl_every, trace)) return st;
  StepSchedule sched;
  sched.tstep = tstep;
  sched.exaggeration_iters = p->exaggeration_iters;
  sched.early_exaggeration = p->early_exaggeration;
  sched.momentum_early = p->momentum_early;
  sched.momentum_late = p->momentum_late;
  Timed tm(g, TSGNE_PHASE_UPDATE, s);
  TSGNE_HIP(launch_update(g, reinterpret_cast<float2*>(Y), reinterpret_cast<float2*>(U), reinterpret_cast<float2*>(G),
                          1.0f, 0.0f, eta, p->min_gain, p->precision, true, nullptr, nullptr, s, sched),
            "launch update");
  return TSGNE_OK;
}

tsgne_status run_impl(tsgne_graph* g, float* Y, int32_t n_iter, const tsgne_params* p, double* kl_trace_h,
                      hipStream_t s) {
  const int32_t n_samples = (kl_trace_h && p->kl_every > 0) ? n_iter / p->kl_every : 0;
  const size_t len = 2 * (size_t)g->n;
  ScratchBlock sb_state, sb_misc;
  sb_state.s = sb_misc.s = s;
  TSGNE_HIP(scratch_alloc(&sb_state.p, 2 * len * sizeof(float), s), "allocate optimiser state");
  TSGNE_HIP(scratch_alloc(&sb_misc.p, 256 + sizeof(double) * (size_t)std::max(n_samples, 1), s), "allocate run scratch");
  float* U = static_cast<float*>(sb_state.p);
  float* G = U + len;
  uint32_t* flag = static_cast<uint32_t*>(sb_misc.p);
  double* trace = n_samples > 0 ? reinterpret_cast<double*>(static_cast<char*>(sb_misc.p) + 256) : nullptr;
  {
    std::vector<float> ones(len, 1.0f);
    TSGNE_HIP(hipMemsetAsync(U, 0, len * sizeof(float), s), "clear update buffer");
    TSGNE_HIP(hipMemcpyAsync(G, ones.data(), len * sizeof(float), hipMemcpyHostToDevice, s), "set gains");
    TSGNE_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t), s), "clear flag");
    TSGNE_HIP(hipMemsetAsync(g->ws.tstep, 0, 2 * sizeof(int32_t), s), "reset step counter");
    TSGNE_HIP(hipStreamSynchronize(s), "synchronise run set-up");
  }
  const float eta = effective_eta(g, p);
  int32_t chunk = kRunChunk;
  if (trace) chunk = (std::max(kRunChunk, p->kl_every) + p->kl_every - 1) / p->kl_every * p->kl_every;
  // With phase timing on, every launch is bracketed by its own pair of events
  // on s, so the steps are launched one by one (HIP events recorded during
  // stream capture order the graph's nodes but cannot be timed).
  const int32_t replays = g->timer.enabled ? 0 : n_iter / chunk;
  int32_t done = 0;
  if (replays > 0) {
    // Capture on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is launched on s.
    hipStream_t cs = nullptr;
    TSGNE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "create capture stream");
    struct CS {
      hipStream_t s;
      ~CS() { (void)hipStreamDestroy(s); }
    } cs_guard{cs};
    TSGNE_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    tsgne_status st = TSGNE_OK;
    for (int32_t k = 0; k < chunk && st == TSGNE_OK; ++k)
      st = enqueue_run_step(g, Y, U, G, p, eta, (trace && k % p->kl_every == 0) ? trace : nullptr, cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    struct GG {
      hipGraph_t g;
      hipGraphExec_t x = nullptr;
      ~GG() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
      }
    } gg{graph};
    if (st != TSGNE_OK) return st;
    TSGNE_HIP(ce, "end capture");
    TSGNE_HIP(hipGraphInstantiate(&gg.x, graph, nullptr, nullptr, 0), "instantiate run graph");
    for (int32_t r = 0; r < replays; ++r) TSGNE_HIP(hipGraphLaunch(gg.x, s), "launch run graph");
    done = replays * chunk;
  }
  for (int32_t t = done; t < n_iter; ++t) {
    const bool sample = trace && (t - done) % p->kl_every == 0;
    if (tsgne_status st = enqueue_run_step(g, Y, U, G, p, eta, sample ? trace : nullptr, s)) return st;
  }
  // the layout after the last step: no step follows to sum Z at it
  if (n_samples > 0 && n_iter % p->kl_every == 0)
    if (tsgne_status st = enqueue_kl(g, Y, s, trace + (n_samples - 1))) return st;
  TSGNE_HIP(launch_nonfinite_check(reinterpret_cast<const float2*>(Y), g->n, flag, s), "launch finiteness check");
  uint32_t host_flag = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read flag");
  if (n_samples > 0)
    TSGNE_HIP(hipMemcpyAsync(kl_trace_h, trace, sizeof(double) * (size_t)n_samples, hipMemcpyDeviceToHost, s),
              "read KL trace");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise run");
  if (host_flag) return fail(TSGNE_E_NONFINITE, "layout holds a NaN or infinity");
  return TSGNE_OK;
}

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_repulsion_plan(int32_t n, int32_t tile_rows, int32_t repulsion, int32_t* tile_rows_out,
                                  int64_t* tiles_out, int64_t* partial_bytes_out) {
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (tile_rows != 0 && !tile_rows_supported(tile_rows))
    return fail(TSGNE_E_INVAL, "tile_rows must be 0, 1, 2, 4, 8, 12, 14, 15 or 16");
  const RepulsionPlan pl = make_plan(n, tile_rows, repulsion);
  if (tile_rows_out) *tile_rows_out = pl.R;
  if (tiles_out) *tiles_out = pl.items;
  if (partial_bytes_out) *partial_bytes_out = (int64_t)pl.nb * pl.nb * pl.T * (int64_t)sizeof(float2);
  return TSGNE_OK;
}

void tsgne_params_default(tsgne_params* p) {
  if (!p) return;
  p->early_exaggeration = 12.0f;
  p->exaggeration_iters = 250;
  p->learning_rate = 0.0f;
  p->momentum_early = 0.5f;
  p->momentum_late = 0.8f;
  p->min_gain = 0.01f;
  p->precision = TSGNE_PREC_SPLIT;
  p->kl_every = 0;
  p->repulsion = TSGNE_REPULSION_AUTO;
  p->tile_rows = 0;
}

const char* tsgne_last_error(void) { return g_error.c_str(); }

const char* tsgne_status_string(tsgne_status s) {
  switch (s) {
    case TSGNE_OK: return "TSGNE_OK";
    case TSGNE_E_INVAL: return "TSGNE_E_INVAL";
    case TSGNE_E_GRAPH: return "TSGNE_E_GRAPH";
    case TSGNE_E_NOMEM: return "TSGNE_E_NOMEM";
    case TSGNE_E_DEVICE: return "TSGNE_E_DEVICE";
    case TSGNE_E_NONFINITE: return "TSGNE_E_NONFINITE";
    case TSGNE_E_BUSY: return "TSGNE_E_BUSY";
    default: return "TSGNE_E_UNKNOWN";
  }
}

// Counting sort by row, then per-row sort and de-duplication.
tsgne_status tsgne_csr_from_edges(int32_t n, int64_t m, const int32_t* uv_h, int32_t* row_ptr_h, int32_t* col_h,
                                  int64_t* nnz_out) {
  if (n < 0 || m < 0) return fail(TSGNE_E_INVAL, "n and m must be >= 0");
  if (!row_ptr_h || !nnz_out || (m > 0 && (!uv_h || !col_h))) return fail(TSGNE_E_INVAL, "null pointer");
  std::vector<int64_t> count((size_t)n + 1, 0);
  for (int64_t t = 0; t < m; ++t) {
    const int32_t u = uv_h[2 * t], v = uv_h[2 * t + 1];
    if (u < 0 || v < 0 || u >= n || v >= n) return fail(TSGNE_E_INVAL, "edge endpoint outside [0, n)");
    if (u == v) continue;
    ++count[(size_t)u + 1];
    ++count[(size_t)v + 1];
  }
  for (int32_t i = 0; i < n; ++i) count[(size_t)i + 1] += count[i];
  if (count[n] >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "graph has 2^31 or more stored entries");
  std::vector<int64_t> fill(count.begin(), count.end() - 1);
  std::vector<int32_t> tmp((size_t)count[n]);
  for (int64_t t = 0; t < m; ++t) {
    const int32_t u = uv_h[2 * t], v = uv_h[2 * t + 1];
    if (u == v) continue;
    tmp[(size_t)fill[u]++] = v;
    tmp[(size_t)fill[v]++] = u;
  }
  int64_t w = 0;
  row_ptr_h[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    auto first = tmp.begin() + count[i], last = tmp.begin() + count[(size_t)i + 1];
    std::sort(first, last);
    auto end = std::unique(first, last);
    for (auto it = first; it != end; ++it) col_h[w++] = *it;
    row_ptr_h[i + 1] = (int32_t)w;
  }
  *nnz_out = w;
  return TSGNE_OK;
}

tsgne_status tsgne_build_P(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d, const float* X_d,
                           int32_t d, float perplexity, void* stream, tsgne_graph** out) {
  if (!out) return fail(TSGNE_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (d < 1) return fail(TSGNE_E_INVAL, "d must be >= 1");
  if (!std::isfinite(perplexity) || perplexity <= 1.0f) return fail(TSGNE_E_INVAL, "perplexity must be > 1");
  if (!row_ptr_d || !X_d || (nnz > 0 && !col_d)) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  tsgne_graph* g = nullptr;
  if (tsgne_status st = graph_structure(n, nnz, row_ptr_d, col_d, s, &g)) return st;
  struct Cleanup {
    tsgne_graph* g;
    ~Cleanup() { free_graph(g); }
  } guard{g};
  g->d = d;
  g->perplexity = perplexity;

  ScratchBlock tmp;
  tmp.s = s;
  const size_t o_pcond = ((size_t)std::max<int64_t>(nnz, 1) * sizeof(double) + 255) & ~(size_t)255;
  TSGNE_HIP(scratch_alloc(&tmp.p, 2 * o_pcond, s), "allocate distances and conditional affinities");
  double* D = static_cast<double*>(tmp.p);
  double* pcond = reinterpret_cast<double*>(static_cast<char*>(tmp.p) + o_pcond);

  // Distances, calibration, symmetrisation.
  TSGNE_HIP(launch_sqdist(g->row_of, g->col, nnz, X_d, d, D, s), "launch distances");
  TSGNE_HIP(launch_calibrate(g->row_ptr, n, g->heavy, g->n_heavy, D, (double)perplexity, pcond, g->beta, s),
            "launch calibration");
  const double S = 2.0 * (double)g->nonisolated;
  TSGNE_HIP(launch_symmetrise(g->mirror, nnz, pcond, S, g->P, s), "launch symmetrisation");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise build_P");
  guard.g = nullptr;
  *out = g;
  return TSGNE_OK;
}

tsgne_status tsgne_graph_from_host_P(int32_t n, int64_t nnz, const int32_t* row_ptr_h, const int32_t* col_h,
                                     const float* P_h, void* stream, tsgne_graph** out) {
  if (!out) return fail(TSGNE_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (!row_ptr_h || (nnz > 0 && (!col_h || !P_h))) return fail(TSGNE_E_INVAL, "null pointer");
  if (row_ptr_h[0] != 0 || row_ptr_h[n] != nnz) return fail(TSGNE_E_GRAPH, "row_ptr must span [0, nnz]");
  for (int64_t e = 0; e < nnz; ++e)
    if (!std::isfinite(P_h[e]) || P_h[e] < 0.f) return fail(TSGNE_E_INVAL, "P must be finite and >= 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int32_t* rp_d = nullptr;
  int32_t* col_d = nullptr;
  struct Upload {
    int32_t*& rp;
    int32_t*& col;
    ~Upload() {
      dfree(rp);
      dfree(col);
    }
  } upload{rp_d, col_d};
  TSGNE_HIP(dalloc(&rp_d, (size_t)n + 1), "allocate row_ptr");
  TSGNE_HIP(dalloc(&col_d, (size_t)nnz), "allocate col");
  TSGNE_HIP(hipMemcpyAsync(rp_d, row_ptr_h, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s),
            "upload row_ptr");
  if (nnz > 0)
    TSGNE_HIP(hipMemcpyAsync(col_d, col_h, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s), "upload col");
  tsgne_graph* g = nullptr;
  if (tsgne_status st = graph_structure(n, nnz, rp_d, col_d, s, &g)) return st;
  struct Cleanup {
    tsgne_graph* g;
    ~Cleanup() { free_graph(g); }
  } guard{g};
  // the CSR is canonical and symmetric now: P must be too (p_ij = p_ji)
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t e = row_ptr_h[i]; e < row_ptr_h[i + 1]; ++e) {
      const int32_t j = col_h[e];
      const int32_t* first = col_h + row_ptr_h[j];
      const int32_t* hit = std::lower_bound(first, col_h + row_ptr_h[j + 1], i);
      if (P_h[e] != P_h[row_ptr_h[j] + (hit - first)]) return fail(TSGNE_E_INVAL, "P must be symmetric");
    }
  }
  if (nnz > 0)
    TSGNE_HIP(hipMemcpyAsync(g->P, P_h, sizeof(float) * (size_t)nnz, hipMemcpyHostToDevice, s), "upload P");
  TSGNE_HIP(hipMemsetAsync(g->beta, 0, sizeof(double) * (size_t)n, s), "clear beta");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise graph_from_host_P");
  guard.g = nullptr;
  *out = g;
  return TSGNE_OK;
}

tsgne_status tsgne_graph_free(tsgne_graph* g) {
  free_graph(g);
  return TSGNE_OK;
}

tsgne_status tsgne_graph_info(const tsgne_graph* g, int32_t* n, int64_t* nnz) {
  if (tsgne_status st = check_graph(g)) return st;
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  return TSGNE_OK;
}

tsgne_status tsgne_graph_export(const tsgne_graph* g, int32_t* row_ptr_h, int32_t* col_h, int32_t* mirror_h,
                                float* P_h, double* beta_h) {
  if (tsgne_status st = check_graph(g)) return st;
  DeviceGuard dg(g->device);
  TSGNE_HIP(hipDeviceSynchronize(), "synchronise before export");
  if (row_ptr_h)
    TSGNE_HIP(hipMemcpy(row_ptr_h, g->row_ptr, sizeof(int32_t) * ((size_t)g->n + 1), hipMemcpyDeviceToHost),
              "export row_ptr");
  if (g->nnz > 0) {
    if (col_h) TSGNE_HIP(hipMemcpy(col_h, g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost), "export col");
    if (mirror_h)
      TSGNE_HIP(hipMemcpy(mirror_h, g->mirror, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost), "export mirror");
    if (P_h) TSGNE_HIP(hipMemcpy(P_h, g->P, sizeof(float) * g->nnz, hipMemcpyDeviceToHost), "export P");
  }
  if (beta_h) TSGNE_HIP(hipMemcpy(beta_h, g->beta, sizeof(double) * g->n, hipMemcpyDeviceToHost), "export beta");
  return TSGNE_OK;
}

tsgne_status tsgne_gradient(tsgne_graph* g, const float* Y_d, float alpha, const tsgne_params* p, float* grad_d,
                            double* Z_d, void* stream) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!Y_d || !grad_d) return fail(TSGNE_E_INVAL, "null pointer");
  if (!std::isfinite(alpha)) return fail(TSGNE_E_INVAL, "alpha must be finite");
  tsgne_params def;
  tsgne_params_default(&def);
  if (!p) p = &def;
  if (tsgne_status st = validate_params(p)) return st;
  DeviceGuard dg(g->device);
  if (tsgne_status st = ensure_workspace(g, p)) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (tsgne_status st = enqueue_forces(g, Y_d, p->precision, s)) return st;
  TSGNE_HIP(launch_update(g, nullptr, nullptr, nullptr, alpha, 0.f, 0.f, 0.f, p->precision, false,
                          reinterpret_cast<float2*>(grad_d), Z_d, s),
            "launch gradient");
  return TSGNE_OK;
}

tsgne_status tsgne_attraction(tsgne_graph* g, const float* Y_d, int32_t precision, double* A_d, void* stream) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!Y_d || !A_d) return fail(TSGNE_E_INVAL, "null pointer");
  if (precision != TSGNE_PREC_SPLIT && precision != TSGNE_PREC_FP32)
    return fail(TSGNE_E_INVAL, "precision must be TSGNE_PREC_SPLIT or TSGNE_PREC_FP32");
  DeviceGuard dg(g->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Timed tm(g, TSGNE_PHASE_ATTRACT, s);
  TSGNE_HIP(launch_attract(g, reinterpret_cast<const float2*>(Y_d), precision, reinterpret_cast<double2*>(A_d), s),
            "launch attraction");
  return TSGNE_OK;
}

tsgne_status tsgne_step(tsgne_graph* g, float* Y_d, float* upd_d, float* gains_d, int32_t t, const tsgne_params* p,
                        float* grad_out_d, double* Z_out_d, void* stream) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!Y_d || !upd_d || !gains_d || !p) return fail(TSGNE_E_INVAL, "null pointer");
  if (t < 0) return fail(TSGNE_E_INVAL, "t must be >= 0");
  if (tsgne_status st = validate_params(p)) return st;
  DeviceGuard dg(g->device);
  if (tsgne_status st = ensure_workspace(g, p)) return st;
  return step_impl(g, Y_d, upd_d, gains_d, t, p, grad_out_d, Z_out_d, reinterpret_cast<hipStream_t>(stream));
}

tsgne_status tsgne_run(tsgne_graph* g, float* Y_d, int32_t n_iter, const tsgne_params* p, double* kl_trace_h,
                       void* stream) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!Y_d || !p) return fail(TSGNE_E_INVAL, "null pointer");
  if (n_iter < 0) return fail(TSGNE_E_INVAL, "n_iter must be >= 0");
  if (tsgne_status st = validate_params(p)) return st;
  DeviceGuard dg(g->device);
  if (tsgne_status st = ensure_workspace(g, p)) return st;
  return run_impl(g, Y_d, n_iter, p, kl_trace_h, reinterpret_cast<hipStream_t>(stream));
}

tsgne_status tsgne_kl(tsgne_graph* g, const float* Y_d, double* kl_h, void* stream) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!Y_d || !kl_h) return fail(TSGNE_E_INVAL, "null pointer");
  tsgne_params def;
  tsgne_params_default(&def);
  DeviceGuard dg(g->device);
  if (!g->ws.part)
    if (tsgne_status st = ensure_workspace(g, &def)) return st;
  return kl_impl(g, Y_d, kl_h, reinterpret_cast<hipStream_t>(stream));
}

tsgne_status tsgne_graph_set_timing(tsgne_graph* g, int32_t enable) {
  if (tsgne_status st = check_graph(g)) return st;
  DeviceGuard dg(g->device);
  TSGNE_HIP(timer_resolve(g), "resolve timing events");
  PhaseTimer& t = g->timer;
  t.enabled = enable != 0;
  for (int k = 0; k < TSGNE_NUM_PHASES; ++k) {
    t.ms[k] = 0.0;
    t.launches[k] = 0;
  }
  return TSGNE_OK;
}

tsgne_status tsgne_graph_timing(tsgne_graph* g, tsgne_timing* out) {
  if (tsgne_status st = check_graph(g)) return st;
  if (!out) return fail(TSGNE_E_INVAL, "out is NULL");
  DeviceGuard dg(g->device);
  TSGNE_HIP(timer_resolve(g), "resolve timing events");
  for (int k = 0; k < TSGNE_NUM_PHASES; ++k) {
    out->ms[k] = g->timer.ms[k];
    out->launches[k] = g->timer.launches[k];
  }
  return TSGNE_OK;
}

}  // extern "C"
