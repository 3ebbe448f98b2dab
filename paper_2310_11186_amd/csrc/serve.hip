// Layout server: continuous batching of t-SGNE requests on one GPU.
//
// Requests are copied in at submission and queued.  A worker thread owns all
// device work: between rounds it admits queued requests while their estimated
// device footprint fits the budget (building their affinities), then advances
// every active request by its share of the round (at most `steps_per_round`
// steps) in one captured batched sequence (each request at its own step
// index), and completes the requests that reached n_iter (layout copied out,
// memory released).  Requests are grouped by tile size, one batched plan per
// group, the groups running on parallel branches of each captured round, each
// branch as long as its own group's largest share.  Every request's arithmetic and
// reduction order depend only on itself and its tile size (a function of its
// size, or the server's fixed choice), so its layout is the same alone or in
// any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace tsgne {
namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double>(t - t0).count();
}

struct Request {
  uint64_t ticket = 0;
  int32_t n = 0, d = 0, n_iter = 0;
  int32_t R = 8;  // repulsion tile rows of this request
  float perplexity = 30.f;
  // canonical CSR, built on the submitting thread (prep != OK: the edge list
  // was refused, and the request fails with that status when admitted)
  std::vector<int32_t> row_ptr, col;
  int64_t nnz = 0;
  tsgne_status prep = TSGNE_OK;
  std::string prep_error;
  std::vector<float> X, Y0, Y;
  size_t footprint = 0;
  Clock::time_point t_submit, t_admit, t_done;
  bool admitted = false;
  bool done = false, cancel = false;
  tsgne_status status = TSGNE_OK;
  std::string error;
};

struct Slot {
  std::shared_ptr<Request> req;
  tsgne_graph* g = nullptr;
  float* state = nullptr;  // Y, U, gains: float32[3][n][2]
  int32_t* t = nullptr;
  int32_t progress = 0;    // steps already run (host view)
};

// Tile rows of a request when the server does not fix them: graphs with
// enough tiles to fill the GPU by themselves (kLargeRequest nodes: 128 blocks
// of 1024), and every request of a server that runs one at a time, take the
// single-graph plan's choice; smaller ones sharing rounds take 8, whose tiles
// keep a shared round's steps short.
constexpr int32_t kLargeRequest = 131072;
int32_t request_tile_rows(int32_t n, int32_t max_active) {
  return (n >= kLargeRequest || max_active == 1) ? make_plan(n, 0, TSGNE_REPULSION_SYMMETRIC).R : 8;
}

// Device bytes a request holds while active (graph, workspace, state) plus the
// transient build buffers, for tile rows R.
size_t footprint_bytes(int32_t n, int64_t m, int32_t d, int32_t R) {
  const int64_t nnz = 2 * m;
  const int64_t T = (int64_t)kWave * R, nb = (n + T - 1) / T;
  const int64_t items = nb * (nb + 1) / 2;
  const int64_t graph = 4 * (n + 1) + 16 * nnz + 8 * (int64_t)n + 4 * (int64_t)n;
  const int64_t work = 8 * nb * nb * T + 12 * items + 16 * (int64_t)n + 8 * 1024 + 4096;
  const int64_t state = 24 * (int64_t)n + 4;
  const int64_t build = 4 * (int64_t)n * d + 16 * nnz + 4 * (n + 1) + 4 * nnz;
  return (size_t)(graph + work + state + build);
}

}  // namespace
}  // namespace tsgne

using namespace tsgne;

struct tsgne_server {
  tsgne_server_config cfg{};
  int device = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<Slot> active;
  bool stop = false;
  int32_t n_active = 0;  // active.size(), published under mu for other threads
  uint64_t next_ticket = 1;
  size_t hbm_used = 0;
  // statistics
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, rounds = 0;
  std::vector<double> latencies_ms;
  bool have_first = false;
  Clock::time_point t_first, t_last_done;
  double busy_s = 0.0;

  void run();
  void admit(hipStream_t s);
  void finish(Slot& sl, tsgne_status st, const std::string& why, bool copy_out, hipStream_t s);
};

namespace {

void free_slot(Slot& sl) {
  if (sl.g) tsgne_graph_free(sl.g);
  dfree(sl.state);
  dfree(sl.t);
  sl.g = nullptr;
}

// Uploads one request and builds its graph; on failure frees what it made.
tsgne_status build_slot(const Request& r, int32_t R, hipStream_t s, Slot& out) {
  if (r.prep != TSGNE_OK) return fail(r.prep, r.prep_error);
  const std::vector<int32_t>& rp = r.row_ptr;
  const std::vector<int32_t>& col = r.col;
  const int64_t nnz = r.nnz;
  int32_t* d_rp = nullptr;
  int32_t* d_col = nullptr;
  float* d_X = nullptr;
  struct Tmp {
    int32_t*& a;
    int32_t*& b;
    float*& c;
    ~Tmp() {
      dfree(a);
      dfree(b);
      dfree(c);
    }
  } tmp{d_rp, d_col, d_X};
  TSGNE_HIP(dalloc(&d_rp, rp.size()), "allocate request CSR");
  TSGNE_HIP(dalloc(&d_col, (size_t)std::max<int64_t>(nnz, 1)), "allocate request CSR");
  TSGNE_HIP(dalloc(&d_X, (size_t)r.n * r.d), "allocate request embedding");
  TSGNE_HIP(hipMemcpyAsync(d_rp, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice, s), "upload CSR");
  if (nnz) TSGNE_HIP(hipMemcpyAsync(d_col, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s), "upload CSR");
  TSGNE_HIP(hipMemcpyAsync(d_X, r.X.data(), sizeof(float) * r.X.size(), hipMemcpyHostToDevice, s), "upload X");
  tsgne_graph* g = nullptr;
  if (tsgne_status st = tsgne_build_P(r.n, nnz, d_rp, d_col, d_X, r.d, r.perplexity, s, &g)) return st;
  out.g = g;
  const size_t len = 2 * (size_t)r.n;
  std::vector<float> init(3 * len, 0.0f);
  std::copy(r.Y0.begin(), r.Y0.end(), init.begin());
  std::fill(init.begin() + 2 * len, init.end(), 1.0f);
  const int32_t zero = 0;
  hipError_t e = dalloc(&out.state, 3 * len);
  if (e == hipSuccess) e = dalloc(&out.t, 1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out.state, init.data(), sizeof(float) * init.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out.t, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_slot(out);
    return hip_fail(e, "set up request state");
  }
  tsgne_params pr{};
  tsgne_params_default(&pr);
  pr.tile_rows = R;
  pr.repulsion = TSGNE_REPULSION_SYMMETRIC;
  if (tsgne_status st = ensure_workspace(g, &pr)) {
    free_slot(out);
    return st;
  }
  return TSGNE_OK;
}

}  // namespace

void tsgne_server::finish(Slot& sl, tsgne_status st, const std::string& why, bool copy_out, hipStream_t s) {
  Request& r = *sl.req;
  if (copy_out) {
    r.Y.resize(2 * (size_t)r.n);
    hipError_t e = hipMemcpyAsync(r.Y.data(), sl.state, sizeof(float) * r.Y.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = TSGNE_E_DEVICE;
    } else {
      for (float v : r.Y)
        if (!std::isfinite(v)) {
          st = TSGNE_E_NONFINITE;
          break;
        }
    }
  }
  free_slot(sl);
  std::lock_guard<std::mutex> lk(mu);
  hbm_used -= r.footprint;
  r.t_done = Clock::now();
  r.status = st;
  r.error = why;
  r.done = true;
  if (st == TSGNE_OK) {
    ++completed;
    latencies_ms.push_back(1e3 * seconds_since(r.t_submit, r.t_done));
    t_last_done = r.t_done;
  } else if (r.cancel) {
    ++cancelled;
  } else {
    ++failed;
  }
  cv_done.notify_all();
}

void tsgne_server::admit(hipStream_t s) {
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (queue.empty() || (int32_t)active.size() >= cfg.max_active) return;  // only this thread changes active
      if (hbm_used + queue.front()->footprint > (size_t)cfg.hbm_budget) return;  // wait for memory
      r = queue.front();
      queue.pop_front();
      hbm_used += r->footprint;
      r->t_admit = Clock::now();
      r->admitted = true;
    }
    Slot sl;
    sl.req = r;
    tsgne_status st = build_slot(*r, r->R, s, sl);
    if (st != TSGNE_OK) {
      finish(sl, st, tsgne_last_error(), false, s);
      continue;
    }
    active.push_back(sl);
  }
}

void tsgne_server::run() {
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
  int32_t* limits = nullptr;  // per-member pause step of the current round
  if (dalloc(&limits, (size_t)cfg.max_active) != hipSuccess) limits = nullptr;
  // Requests are grouped by tile size, one batched plan per group.  With
  // several groups a round forks one branch per group (its own stream) from
  // the main stream and joins them at the end, so the groups run together.
  std::map<int32_t, BatchRun> groups;
  bool plan_valid = false;
  constexpr int kMaxGroups = 6;  // the supported tile sizes
  hipStream_t branch[kMaxGroups] = {};
  hipEvent_t fork = nullptr, join[kMaxGroups] = {};
  bool branches_ok = hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < kMaxGroups && branches_ok; ++k)
    branches_ok = hipStreamCreateWithFlags(&branch[k], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&join[k], hipEventDisableTiming) == hipSuccess;
  // Captured rounds for the current membership, keyed by the number of steps
  // each group's branch launches (groups in ascending tile size).
  std::map<std::vector<int32_t>, hipGraphExec_t> execs;
  constexpr size_t kMaxExecs = 32;
  auto clear_execs = [&]() {
    for (auto& kv : execs) (void)hipGraphExecDestroy(kv.second);
    execs.clear();
  };
  auto drop_execs = [&]() {
    clear_execs();
    plan_valid = false;
  };
  // ordered pairs evaluated per second, refined from measured rounds
  double pair_rate = 5e12;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop) break;
    }
    const size_t before = active.size();
    admit(s);
    // cancelled active requests leave at a round boundary
    bool changed = active.size() != before;
    for (size_t k = 0; k < active.size();) {
      bool c;
      {
        std::lock_guard<std::mutex> lk(mu);
        c = active[k].req->cancel;
      }
      if (c) {
        finish(active[k], TSGNE_E_CANCELLED, "cancelled", false, s);
        active.erase(active.begin() + (long)k);
        changed = true;
      } else {
        ++k;
      }
    }
    if (changed) drop_execs();
    {
      std::lock_guard<std::mutex> lk(mu);
      n_active = (int32_t)active.size();
    }
    if (active.empty()) continue;
    const Clock::time_point t0 = Clock::now();
    tsgne_status st = limits ? TSGNE_OK : fail(TSGNE_E_NOMEM, "allocate round limits");
    if (st == TSGNE_OK && !plan_valid) {
      std::map<int32_t, std::vector<BatchMember>> members;
      for (size_t k = 0; k < active.size(); ++k) {
        Slot& sl = active[k];
        const size_t len = 2 * (size_t)sl.req->n;
        members[sl.req->R].push_back(BatchMember{sl.g, sl.state, sl.state + len, sl.state + 2 * len, sl.t,
                                                 limits + k, sl.req->n_iter});
      }
      groups.clear();
      if (members.size() > 1 && !branches_ok) st = fail(TSGNE_E_DEVICE, "create round branches");
      for (auto& kv : members) {
        if (st != TSGNE_OK) break;
        st = groups[kv.first].setup(kv.second.data(), (int32_t)kv.second.size(), kv.first, &cfg.params);
      }
      if (st == TSGNE_OK) plan_valid = true;
    }
    // Steps per request this round: an equal share of the round's target time
    // (small graphs take many steps, large ones few), or the same count for
    // all when no target is set.
    // With oldest_share > 0 the request that has waited longest gets that
    // fraction of the round and the others split the rest.
    std::vector<int32_t> take(active.size()), lim(active.size());
    std::map<int32_t, int32_t> longest;  // per group (tile size): the most steps any member takes
    double pairs = 0.0;
    const double budget = cfg.round_ms > 0.f ? pair_rate * 1e-3 * cfg.round_ms : 0.0;
    size_t oldest = 0;
    for (size_t k = 1; k < active.size(); ++k)
      if (active[k].req->t_submit < active[oldest].req->t_submit) oldest = k;
    const bool favour = cfg.oldest_share > 0.f && active.size() > 1;
    auto per_step_of = [&](size_t k) { return (double)active[k].req->n * (double)(active[k].req->n - 1) + 1.0; };
    // Smallest-first: the time left after the oldest request's part goes to
    // the requests with the least remaining work, each as much as a round
    // allows, until it runs out (the others still take one step).
    std::vector<double> share_of(active.size(), 0.0);
    if (cfg.rest_policy == TSGNE_SHARE_SMALLEST_FIRST && budget > 0.0) {
      std::vector<size_t> rest;
      for (size_t k = 0; k < active.size(); ++k)
        if (!(favour && k == oldest)) rest.push_back(k);
      auto remaining = [&](size_t k) { return per_step_of(k) * (double)(active[k].req->n_iter - active[k].progress); };
      std::stable_sort(rest.begin(), rest.end(), [&](size_t a, size_t b) { return remaining(a) < remaining(b); });
      double left = favour ? budget * (1.0 - cfg.oldest_share) : budget;
      for (size_t k : rest) {
        const double want = per_step_of(k) * (double)std::min(cfg.steps_per_round, active[k].req->n_iter - active[k].progress);
        share_of[k] = std::min(want, left);
        left -= share_of[k];
      }
      if (favour) share_of[oldest] = budget * cfg.oldest_share;
    }
    for (size_t k = 0; k < active.size(); ++k) {
      const Slot& sl = active[k];
      const double per_step = per_step_of(k);
      const double share = cfg.rest_policy == TSGNE_SHARE_SMALLEST_FIRST ? share_of[k]
                           : !favour ? budget / (double)active.size()
                           : k == oldest ? budget * cfg.oldest_share
                                         : budget * (1.0 - cfg.oldest_share) / (double)(active.size() - 1);
      int32_t steps = cfg.steps_per_round;
      if (budget > 0.0) steps = (int32_t)std::max(1.0, std::min((double)cfg.steps_per_round, std::floor(share / per_step)));
      steps = std::max(0, std::min(steps, sl.req->n_iter - sl.progress));
      take[k] = steps;
      lim[k] = sl.progress + steps;
      int32_t& most = longest[sl.req->R];
      most = std::max(most, steps);
      pairs += per_step * steps;
    }
    // Each group's branch launches the power of two at or above its own
    // longest allotment (members pause at their limit on the device), so a
    // group of large graphs that take one step in a round does not launch
    // the many steps a group of small ones takes beside it.
    std::vector<int32_t> lens;
    for (const auto& kv : groups) {
      int32_t len = 1;
      while (len < longest[kv.first]) len *= 2;
      lens.push_back(std::min(len, cfg.steps_per_round));
    }
    if (st == TSGNE_OK) {
      hipError_t e = hipMemcpyAsync(limits, lim.data(), sizeof(int32_t) * lim.size(), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) st = hip_fail(e, "upload round limits");
    }
    if (st == TSGNE_OK && !execs.count(lens)) {
      if (execs.size() >= kMaxExecs) clear_execs();
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      hipError_t le = hipSuccess;
      if (groups.size() == 1) {
        const BatchRun& br = groups.begin()->second;
        for (int32_t k = 0; e == hipSuccess && k < lens[0] && le == hipSuccess; ++k)
          le = launch_batch_step(br.plan(), cfg.params, s);
      } else if (e == hipSuccess) {
        le = hipEventRecord(fork, s);
        int gi = 0;
        for (auto it = groups.begin(); it != groups.end() && le == hipSuccess; ++it, ++gi) {
          le = hipStreamWaitEvent(branch[gi], fork, 0);
          for (int32_t k = 0; k < lens[gi] && le == hipSuccess; ++k)
            le = launch_batch_step(it->second.plan(), cfg.params, branch[gi]);
          if (le == hipSuccess) le = hipEventRecord(join[gi], branch[gi]);
        }
        for (int k = 0; k < gi && le == hipSuccess; ++k) le = hipStreamWaitEvent(s, join[k], 0);
      }
      if (e == hipSuccess) e = hipStreamEndCapture(s, &graph);
      if (e == hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) st = hip_fail(e, "capture a serving round");
      else execs[lens] = exec;
    }
    if (st == TSGNE_OK) {
      hipError_t e = hipGraphLaunch(execs[lens], s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = hip_fail(e, "run a serving round");
    }
    if (st != TSGNE_OK) {
      // a device failure ends every active request with that status
      const std::string why = tsgne_last_error();
      for (Slot& sl : active) finish(sl, st, why, false, s);
      active.clear();
      drop_execs();
      continue;
    }
    const double dt = seconds_since(t0, Clock::now());
    if (dt > 0.0 && pairs > 1e9) pair_rate = 0.5 * pair_rate + 0.5 * pairs / dt;
    {
      std::lock_guard<std::mutex> lk(mu);
      ++rounds;
      busy_s += dt;
    }
    bool left = false;
    for (size_t k = 0, j = 0; k < active.size(); ++j) {
      Slot& sl = active[k];
      sl.progress += take[j];
      if (sl.progress >= sl.req->n_iter) {
        finish(sl, TSGNE_OK, "", true, s);
        active.erase(active.begin() + (long)k);
        left = true;
      } else {
        ++k;
      }
    }
    if (left) drop_execs();
    {
      std::lock_guard<std::mutex> lk(mu);
      n_active = (int32_t)active.size();
    }
  }
  drop_execs();
  for (Slot& sl : active) {
    sl.req->cancel = true;
    finish(sl, TSGNE_E_CANCELLED, "server destroyed", false, s);
  }
  active.clear();
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& r : queue) {
      r->cancel = true;
      r->done = true;
      r->status = TSGNE_E_CANCELLED;
      ++cancelled;
    }
    queue.clear();
    n_active = 0;
    cv_done.notify_all();
  }
  groups.clear();
  dfree(limits);
  for (int k = 0; k < kMaxGroups; ++k) {
    if (branch[k]) (void)hipStreamDestroy(branch[k]);
    if (join[k]) (void)hipEventDestroy(join[k]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (s) (void)hipStreamDestroy(s);
}

extern "C" {

void tsgne_server_config_default(tsgne_server_config* c) {
  if (!c) return;
  c->hbm_budget = 0;
  c->max_active = 64;
  c->max_queue = 1 << 20;
  c->steps_per_round = 64;
  c->round_ms = 25.0f;
  c->oldest_share = 0.5f;
  c->rest_policy = TSGNE_SHARE_EQUAL;
  c->tile_rows = 0;
  tsgne_params_default(&c->params);
}

tsgne_status tsgne_server_create(const tsgne_server_config* cfg, tsgne_server** out) {
  if (!cfg || !out) return fail(TSGNE_E_INVAL, "null pointer");
  *out = nullptr;
  if (tsgne_status st = validate_params(&cfg->params)) return st;
  if (!std::isfinite(cfg->round_ms)) return fail(TSGNE_E_INVAL, "round_ms must be finite");
  if (!(cfg->oldest_share >= 0.f && cfg->oldest_share < 1.f))
    return fail(TSGNE_E_INVAL, "oldest_share must lie in [0, 1)");
  if (cfg->rest_policy != TSGNE_SHARE_EQUAL && cfg->rest_policy != TSGNE_SHARE_SMALLEST_FIRST)
    return fail(TSGNE_E_INVAL, "rest_policy must be TSGNE_SHARE_EQUAL or TSGNE_SHARE_SMALLEST_FIRST");
  if (cfg->max_active < 1 || cfg->max_queue < 1 || cfg->steps_per_round < 1)
    return fail(TSGNE_E_INVAL, "max_active, max_queue and steps_per_round must be >= 1");
  if (cfg->tile_rows != 0 && !tile_rows_supported(cfg->tile_rows))
    return fail(TSGNE_E_INVAL, "tile_rows must be 0 (per request), 1, 2, 4, 8, 12, 14, 15 or 16");
  if (cfg->hbm_budget < 0) return fail(TSGNE_E_INVAL, "hbm_budget must be >= 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TSGNE_E_DEVICE, "no HIP device");
  tsgne_server* srv = new (std::nothrow) tsgne_server();
  if (!srv) return fail(TSGNE_E_NOMEM, "host allocation failed");
  srv->cfg = *cfg;
  srv->device = dev;
  if (srv->cfg.hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete srv;
      return fail(TSGNE_E_DEVICE, "cannot query device memory");
    }
    srv->cfg.hbm_budget = (int64_t)(0.8 * (double)free_b);
  }
  srv->worker = std::thread([srv] { srv->run(); });
  *out = srv;
  return TSGNE_OK;
}

tsgne_status tsgne_server_submit(tsgne_server* srv, const tsgne_request* rq, uint64_t* ticket) {
  const Clock::time_point t_call = Clock::now();
  if (!srv || !rq || !ticket) return fail(TSGNE_E_INVAL, "null pointer");
  if (rq->n < 1 || rq->m < 0 || rq->d < 1 || rq->n_iter < 0) return fail(TSGNE_E_INVAL, "bad request sizes");
  if (!std::isfinite(rq->perplexity) || rq->perplexity <= 1.0f) return fail(TSGNE_E_INVAL, "perplexity must be > 1");
  if (!rq->X_h || !rq->Y0_h || (rq->m > 0 && !rq->edges_h)) return fail(TSGNE_E_INVAL, "null request buffer");
  auto r = std::make_shared<Request>();
  r->n = rq->n;
  r->d = rq->d;
  r->n_iter = rq->n_iter;
  r->perplexity = rq->perplexity;
  r->R = srv->cfg.tile_rows ? srv->cfg.tile_rows : request_tile_rows(rq->n, srv->cfg.max_active);
  r->footprint = footprint_bytes(rq->n, rq->m, rq->d, r->R);
  if (r->footprint > (size_t)srv->cfg.hbm_budget)
    return fail(TSGNE_E_NOMEM, "request needs more device memory than the server's budget");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if ((int64_t)srv->queue.size() >= srv->cfg.max_queue) return fail(TSGNE_E_BUSY, "request queue is full");
  }
  // The canonical CSR is built here, on the caller's thread, so that the
  // server's worker (which keeps the GPU busy) only uploads and builds P.
  r->row_ptr.resize((size_t)rq->n + 1);
  r->col.resize((size_t)std::max<int64_t>(2 * rq->m, 1));
  r->prep = tsgne_csr_from_edges(rq->n, rq->m, rq->edges_h, r->row_ptr.data(), r->col.data(), &r->nnz);
  if (r->prep != TSGNE_OK) r->prep_error = tsgne_last_error();
  r->col.resize((size_t)std::max<int64_t>(r->nnz, 1));
  r->X.assign(rq->X_h, rq->X_h + (size_t)rq->n * rq->d);
  r->Y0.assign(rq->Y0_h, rq->Y0_h + 2 * (size_t)rq->n);
  std::lock_guard<std::mutex> lk(srv->mu);
  if ((int64_t)srv->queue.size() >= srv->cfg.max_queue) return fail(TSGNE_E_BUSY, "request queue is full");
  r->ticket = srv->next_ticket++;
  r->t_submit = t_call;
  if (!srv->have_first) {
    srv->have_first = true;
    srv->t_first = r->t_submit;
  }
  srv->queue.push_back(r);
  srv->all[r->ticket] = r;
  ++srv->submitted;
  *ticket = r->ticket;
  srv->cv_work.notify_one();
  return TSGNE_OK;
}

tsgne_status tsgne_server_poll(tsgne_server* srv, uint64_t ticket, float* Y_h, int32_t* done, tsgne_status* result) {
  if (!srv || !done) return fail(TSGNE_E_INVAL, "null pointer");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  Request& r = *it->second;
  *done = r.done ? 1 : 0;
  if (r.done) {
    if (result) *result = r.status;
    if (Y_h && r.status == TSGNE_OK) std::copy(r.Y.begin(), r.Y.end(), Y_h);
  }
  return TSGNE_OK;
}

tsgne_status tsgne_server_wait(tsgne_server* srv, uint64_t ticket, float* Y_h, tsgne_status* result) {
  if (!srv) return fail(TSGNE_E_INVAL, "null pointer");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  std::shared_ptr<Request> r = it->second;
  srv->cv_done.wait(lk, [&] { return r->done; });
  if (result) *result = r->status;
  if (Y_h && r->status == TSGNE_OK) std::copy(r->Y.begin(), r->Y.end(), Y_h);
  return TSGNE_OK;
}

tsgne_status tsgne_server_latency(tsgne_server* srv, uint64_t ticket, double* latency_ms, double* queued_ms) {
  if (!srv) return fail(TSGNE_E_INVAL, "null pointer");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  const Request& r = *it->second;
  if (!r.done) return fail(TSGNE_E_BUSY, "request still queued or running");
  if (latency_ms) *latency_ms = 1e3 * seconds_since(r.t_submit, r.t_done);
  if (queued_ms) *queued_ms = 1e3 * seconds_since(r.t_submit, r.admitted ? r.t_admit : r.t_done);
  return TSGNE_OK;
}

tsgne_status tsgne_server_release(tsgne_server* srv, uint64_t ticket) {
  if (!srv) return fail(TSGNE_E_INVAL, "null pointer");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  if (!it->second->done) return fail(TSGNE_E_BUSY, "request still running");
  srv->all.erase(it);
  return TSGNE_OK;
}

tsgne_status tsgne_server_cancel(tsgne_server* srv, uint64_t ticket) {
  if (!srv) return fail(TSGNE_E_INVAL, "null pointer");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  Request& r = *it->second;
  if (r.done) return TSGNE_OK;
  r.cancel = true;
  for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q) {
    if ((*q)->ticket == ticket) {
      srv->queue.erase(q);
      r.done = true;
      r.status = TSGNE_E_CANCELLED;
      r.t_done = Clock::now();
      ++srv->cancelled;
      srv->cv_done.notify_all();
      break;
    }
  }
  srv->cv_work.notify_one();
  return TSGNE_OK;
}

tsgne_status tsgne_server_get_stats(tsgne_server* srv, tsgne_server_stats* out) {
  if (!srv || !out) return fail(TSGNE_E_INVAL, "null pointer");
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->failed = srv->failed;
  out->cancelled = srv->cancelled;
  out->queued = (int32_t)srv->queue.size();
  out->active = srv->n_active;
  out->hbm_in_use = (int64_t)srv->hbm_used;
  out->hbm_budget = srv->cfg.hbm_budget;
  out->rounds = srv->rounds;
  out->busy_s = srv->busy_s;
  std::vector<double> l = srv->latencies_ms;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    const size_t k = (size_t)std::min<double>((double)l.size() - 1, std::ceil(q * (double)l.size()) - 1);
    return l[k];
  };
  out->latency_p50_ms = pct(0.50);
  out->latency_p99_ms = pct(0.99);
  double sum = 0.0;
  for (double v : l) sum += v;
  out->latency_mean_ms = l.empty() ? 0.0 : sum / (double)l.size();
  const double span = (srv->completed > 0) ? seconds_since(srv->t_first, srv->t_last_done) : 0.0;
  out->layouts_per_s = span > 0.0 ? (double)srv->completed / span : 0.0;
  return TSGNE_OK;
}

tsgne_status tsgne_server_destroy(tsgne_server* srv) {
  if (!srv) return TSGNE_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  delete srv;
  return TSGNE_OK;
}

}  // extern "C"
