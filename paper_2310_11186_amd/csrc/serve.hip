// Layout server: continuous batching of t-SGNE requests on one GPU.
//
// Requests are copied in at submission and queued.  A worker thread owns all
// device work.  It runs rounds: each active request is given a number of
// steps (its share of the round's target time, by the share policy; by
// default short requests first and long ones one at a time in submission
// order), and every group of requests with the same tile size replays a
// captured chunk of batched steps (each request at its own step index,
// pausing on the device at its allotment) on its own branch stream, the
// groups running together.  While a round runs, queued requests are admitted
// as their estimated device footprint fits the budget (their affinities built
// on a stream of their own); they join the next round.  Requests that reached
// n_iter complete at the round's end (layout copied out, memory released).
// Every request's arithmetic and reduction order depend only on itself and
// its tile size (a function of its size, or the server's fixed choice), so
// its layout is the same alone or in any mix.
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
  // when this request would finish if every request ran alone in submission
  // order (estimated at admission, in that order; see tsgne_server::fifo_due)
  Clock::time_point fifo_due;
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
  int32_t id = -1;         // index of this slot's pause limit in the round's limit array (kept while active)
  int32_t progress = 0;    // steps already run (host view)
};

// Tile rows of a request when the server does not fix them: the single-graph
// plan's choice, whose step is the shortest for the request's size (1 or 2
// rows for the smallest graphs, whose steps are a few microseconds, up to
// 14-16 for those that fill the GPU by themselves).  The layout therefore
// equals the request's own tsgne_run with the automatic tile.
int32_t request_tile_rows(int32_t n) { return make_plan(n, 0, TSGNE_REPULSION_SYMMETRIC).R; }

// Distinct tile sizes, hence the most batched groups of short requests a
// round can hold (the running long request's group comes on top).
constexpr int kMaxGroups = 8;
// Group key of the running long request: kHeadKey + its tile rows.
constexpr int32_t kHeadKey = 1000;

// Shortest time of one step of the smallest graphs (a few dependent kernel
// launches), below which a step does not get faster however few pairs it has.
constexpr double kStepFloorSeconds = 15e-6;

// Estimated GPU time of n_iter steps of an n-node graph alone.
double alone_seconds(int32_t n, int32_t n_iter, double pair_rate) {
  const double pairs = (double)n * (double)(n - 1);
  return (double)n_iter * std::max(pairs / pair_rate, kStepFloorSeconds);
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
  std::thread worker, admitter;
  std::mutex mu;
  // Held while the worker captures a chunk and while the admitter builds a
  // request: a build's synchronous HIP calls (hipMalloc, hipMemcpy on the null
  // stream) must not run while a stream is being captured.
  std::mutex capture_mu;
  std::condition_variable cv_work, cv_done, cv_admit;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<Slot> active;
  std::vector<Slot> incoming;      // built by the admitter; active from the next round
  std::vector<int32_t> free_ids;   // limit-array indices not held by a slot
  int32_t building = 0;            // requests the admitter is building
  bool admitter_done = false;      // the admitter has left its loop (it touches incoming no more)
  bool stop = false;
  int32_t n_active = 0;  // active.size(), published under mu for other threads
  uint64_t next_ticket = 1;
  size_t hbm_used = 0;
  // statistics
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, rounds = 0;
  std::vector<double> latencies_ms;
  bool have_first = false;
  Clock::time_point t_first, t_last_done;
  double busy_s = 0.0, admit_s = 0.0, plan_s = 0.0;
  // ordered pairs evaluated per second, refined from measured rounds
  double pair_rate = 5e12;
  // the one-at-a-time schedule's clock: the estimated finish of the last
  // request admitted, had every request run alone in submission order
  Clock::time_point fifo_clock;
  bool fifo_started = false;

  void run();
  void admit_loop();
  bool can_admit() const;
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
  // uploads in stream-ordered pool memory, released once the graph is built
  ScratchBlock tmp;
  tmp.s = s;
  const size_t b_rp = (sizeof(int32_t) * rp.size() + 255) & ~(size_t)255;
  const size_t b_col = (sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1) + 255) & ~(size_t)255;
  TSGNE_HIP(scratch_alloc(&tmp.p, b_rp + b_col + sizeof(float) * r.X.size(), s), "allocate request uploads");
  int32_t* d_rp = static_cast<int32_t*>(tmp.p);
  int32_t* d_col = reinterpret_cast<int32_t*>(static_cast<char*>(tmp.p) + b_rp);
  float* d_X = reinterpret_cast<float*>(static_cast<char*>(tmp.p) + b_rp + b_col);
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
  if (sl.id >= 0) free_ids.push_back(sl.id);
  sl.id = -1;
  hbm_used -= r.footprint;
  cv_admit.notify_one();
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

// Under mu: the next queued request can be admitted (a slot and its memory).
bool tsgne_server::can_admit() const {
  if (queue.empty() || free_ids.empty()) return false;
  if (n_active + (int32_t)incoming.size() + building >= cfg.max_active) return false;
  return hbm_used + queue.front()->footprint <= (size_t)cfg.hbm_budget;  // else wait for memory
}

// The admitter thread: takes queued requests in submission order as slots and
// memory allow, uploads them and builds their affinities on a stream of its
// own (overlapping the rounds the worker runs), and hands the built slots to
// the worker, which adds them at its next round boundary.
void tsgne_server::admit_loop() {
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  const bool stream_ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    std::shared_ptr<Request> r;
    Slot sl;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_admit.wait(lk, [&] { return stop || can_admit(); });
      if (stop) break;
      r = queue.front();
      queue.pop_front();
      hbm_used += r->footprint;
      r->t_admit = Clock::now();
      r->admitted = true;
      // its finish in the one-at-a-time schedule: after the previous
      // request's and its own estimated time alone
      const Clock::time_point start = (!fifo_started || r->t_submit > fifo_clock) ? r->t_submit : fifo_clock;
      r->fifo_due = start + std::chrono::duration_cast<Clock::duration>(
                                std::chrono::duration<double>(alone_seconds(r->n, r->n_iter, pair_rate)));
      fifo_clock = r->fifo_due;
      fifo_started = true;
      sl.req = r;
      sl.id = free_ids.back();
      free_ids.pop_back();
      building = 1;
    }
    const Clock::time_point t0 = Clock::now();
    tsgne_status st;
    {
      std::lock_guard<std::mutex> cl(capture_mu);
      st = stream_ok ? build_slot(*r, r->R, s, sl) : fail(TSGNE_E_DEVICE, "create the admission stream");
    }
    const std::string why = st == TSGNE_OK ? std::string() : std::string(tsgne_last_error());
    if (st != TSGNE_OK) finish(sl, st, why, false, s);
    std::lock_guard<std::mutex> lk(mu);
    building = 0;
    admit_s += seconds_since(t0, Clock::now());
    if (st == TSGNE_OK) {
      incoming.push_back(sl);
      cv_work.notify_one();
    }
  }
  if (s) (void)hipStreamDestroy(s);
  std::lock_guard<std::mutex> lk(mu);
  admitter_done = true;
  cv_work.notify_all();
}

namespace {

// Steps of one captured chunk of a group (replayed as often as a round needs).
constexpr int32_t kChunkSteps = 64;

// The active requests of one tile size: their batched plan, the members'
// tickets in plan order, and the captured chunks of that plan by length.
struct Group {
  BatchRun run;
  std::vector<uint64_t> tickets;
  std::map<int32_t, hipGraphExec_t> chunks;
  ~Group() { clear(); }
  void clear() {
    for (auto& kv : chunks) (void)hipGraphExecDestroy(kv.second);
    chunks.clear();
  }
};

// A captured chunk of `len` batched steps of a group's plan.
tsgne_status chunk_exec(Group& gr, int32_t len, const tsgne_params& p, hipStream_t cap, hipGraphExec_t* out) {
  auto it = gr.chunks.find(len);
  if (it != gr.chunks.end()) {
    *out = it->second;
    return TSGNE_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  TSGNE_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t le = hipSuccess;
  for (int32_t k = 0; k < len && le == hipSuccess; ++k) le = launch_batch_step(gr.run.plan(), p, cap);
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (e == hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "capture a serving chunk");
  gr.chunks[len] = exec;
  *out = exec;
  return TSGNE_OK;
}

}  // namespace

void tsgne_server::run() {
  (void)hipSetDevice(device);
  hipStream_t s = nullptr, cap = nullptr;
  bool streams_ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
                    hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
  int32_t* limits = nullptr;  // per-slot pause step of the current round, indexed by slot id
  if (dalloc(&limits, (size_t)cfg.max_active) != hipSuccess) limits = nullptr;
  std::vector<int32_t> lim_host((size_t)cfg.max_active, 0);
  // Requests are grouped by tile size, one batched plan per group.  With
  // several groups a round forks one branch per group (its own stream) from
  // the main stream and joins them at the end, so the groups run together.
  std::map<int32_t, Group> groups;
  hipStream_t branch[kMaxGroups] = {};
  hipEvent_t fork = nullptr, join[kMaxGroups] = {};
  bool branches_ok = hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < kMaxGroups && branches_ok; ++k)
    branches_ok = hipStreamCreateWithFlags(&branch[k], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&join[k], hipEventDisableTiming) == hipSuccess;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !active.empty() || !incoming.empty(); });
      if (stop) break;
      // requests the admitter built during the last round join now
      for (Slot& sl : incoming) active.push_back(sl);
      incoming.clear();
      n_active = (int32_t)active.size();
      cv_admit.notify_one();  // slots may have come free
    }
    // cancelled active requests leave at a round boundary
    for (size_t k = 0; k < active.size();) {
      bool c;
      {
        std::lock_guard<std::mutex> lk(mu);
        c = active[k].req->cancel;
      }
      if (c) {
        finish(active[k], TSGNE_E_CANCELLED, "cancelled", false, s);
        active.erase(active.begin() + (long)k);
      } else {
        ++k;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      n_active = (int32_t)active.size();
      cv_admit.notify_one();  // slots may have come free
    }
    if (active.empty()) continue;
    const Clock::time_point t_plan = Clock::now();
    tsgne_status st = (limits && streams_ok) ? TSGNE_OK : fail(TSGNE_E_NOMEM, "allocate server state");
    // Steps per request this round: an equal share of the round's target time
    // (small graphs take many steps, large ones few), or the same count for
    // all when no target is set.
    // With oldest_share > 0 the request that has waited longest gets that
    // fraction of the round and the others split the rest.
    std::vector<int32_t> take(active.size());
    std::map<int32_t, int32_t> longest;  // per group (tile size): the most steps any member takes
    double pairs = 0.0;
    const double budget = cfg.round_ms > 0.f ? pair_rate * 1e-3 * cfg.round_ms : 0.0;
    size_t oldest = 0;
    for (size_t k = 1; k < active.size(); ++k)
      if (active[k].req->t_submit < active[oldest].req->t_submit) oldest = k;
    const bool favour = cfg.oldest_share > 0.f && active.size() > 1;
    auto per_step_of = [&](size_t k) { return (double)active[k].req->n * (double)(active[k].req->n - 1) + 1.0; };
    auto remaining = [&](size_t k) { return per_step_of(k) * (double)(active[k].req->n_iter - active[k].progress); };
    std::vector<double> share_of(active.size(), 0.0);
    // Short-first: requests with at most long_ms of GPU time left are short;
    // they take what they need first, least remaining first.  Long requests
    // run one at a time in submission order (the oldest, the head, takes the
    // rest of the round; the others are paused), so a long request never
    // shares the GPU with another long one.  While a head runs, the short
    // requests take at most short_share of a round, and only out of the
    // head's slack: the time by which it is ahead of its finish in the
    // one-at-a-time schedule (fifo_due), after the work of every active
    // request due before it (short requests due before it take what they
    // need).  So short requests overtake a long one only as far as it would
    // otherwise have waited for them, and no request is meant to finish later
    // than it would one at a time.
    std::vector<char> paused(active.size(), 0);
    size_t head = active.size();  // the running long request (short-first), if any
    const double long_pairs = pair_rate * 1e-3 * (double)cfg.long_ms;
    const bool short_first = cfg.rest_policy == TSGNE_SHARE_SHORT_FIRST && budget > 0.0;
    if (short_first) {
      std::vector<size_t> shorts;
      for (size_t k = 0; k < active.size(); ++k) {
        if (remaining(k) <= long_pairs) {
          shorts.push_back(k);
        } else if (head == active.size() || active[k].req->t_submit < active[head].req->t_submit) {
          head = k;
        }
      }
      for (size_t k = 0; k < active.size(); ++k)
        if (k != head && remaining(k) > long_pairs) paused[k] = 1;
      std::stable_sort(shorts.begin(), shorts.end(), [&](size_t a, size_t b) { return remaining(a) < remaining(b); });
      double left = budget;
      if (head < active.size()) {
        // seconds of GPU work due no later than the head, the head's own included
        double ahead = 0.0;
        for (size_t k = 0; k < active.size(); ++k)
          if (active[k].req->fifo_due <= active[head].req->fifo_due)
            ahead += alone_seconds(active[k].req->n, active[k].req->n_iter - active[k].progress, pair_rate);
        const double slack = std::chrono::duration<double>(active[head].req->fifo_due - Clock::now()).count() -
                             ahead - 1e-3 * (double)cfg.round_ms;
        left = std::min(budget * (double)cfg.short_share, std::max(0.0, slack) * pair_rate);
      }
      double used = 0.0;
      for (size_t k : shorts) {
        const double want =
            per_step_of(k) * (double)std::min(cfg.steps_per_round, active[k].req->n_iter - active[k].progress);
        // a short request due before the head is ahead of it in the
        // one-at-a-time order too: it takes what it needs
        const bool ahead_of_head = head < active.size() && active[k].req->fifo_due <= active[head].req->fifo_due;
        const double give = ahead_of_head ? want : std::min(want, left);
        if (give < per_step_of(k)) {  // no room for one step this round
          paused[k] = 1;
          continue;
        }
        share_of[k] = give;
        if (!ahead_of_head) left -= give;
        used += give;
      }
      if (head < active.size()) share_of[head] = std::max(budget - used, budget * (1.0 - (double)cfg.short_share));
    } else if (cfg.rest_policy == TSGNE_SHARE_SMALLEST_FIRST && budget > 0.0) {
      // Smallest-first: the time left after the oldest request's part goes to
      // the requests with the least remaining work, each as much as a round
      // allows, until it runs out (the others still take one step).
      std::vector<size_t> rest;
      for (size_t k = 0; k < active.size(); ++k)
        if (!(favour && k == oldest)) rest.push_back(k);
      std::stable_sort(rest.begin(), rest.end(), [&](size_t a, size_t b) { return remaining(a) < remaining(b); });
      double left = favour ? budget * (1.0 - cfg.oldest_share) : budget;
      for (size_t k : rest) {
        const double want =
            per_step_of(k) * (double)std::min(cfg.steps_per_round, active[k].req->n_iter - active[k].progress);
        share_of[k] = std::min(want, left);
        left -= share_of[k];
      }
      if (favour) share_of[oldest] = budget * cfg.oldest_share;
    }
    for (size_t k = 0; k < active.size(); ++k) {
      const Slot& sl = active[k];
      const double per_step = per_step_of(k);
      const bool by_share =
          cfg.rest_policy == TSGNE_SHARE_SMALLEST_FIRST || cfg.rest_policy == TSGNE_SHARE_SHORT_FIRST;
      const double share = by_share ? share_of[k]
                           : !favour ? budget / (double)active.size()
                           : k == oldest ? budget * cfg.oldest_share
                                         : budget * (1.0 - cfg.oldest_share) / (double)(active.size() - 1);
      int32_t steps = cfg.steps_per_round;
      if (budget > 0.0)
        steps = (int32_t)std::max(1.0, std::min((double)cfg.steps_per_round, std::floor(share / per_step)));
      if (paused[k]) steps = 0;
      steps = std::max(0, std::min(steps, sl.req->n_iter - sl.progress));
      take[k] = steps;
    }
    // Batched groups: one per tile size; under short-first the running long
    // request has a group of its own (run after the others, see below) and
    // the paused long requests are in none, so that no launch carries the
    // tiles of graphs that wait.
    std::vector<int32_t> key(active.size());
    for (size_t k = 0; k < active.size(); ++k) {
      const int32_t R = active[k].req->R;
      key[k] = !short_first ? R : k == head ? kHeadKey + R : remaining(k) > long_pairs ? -1 : R;
    }
    // a round always advances someone: if every request was paused (no long
    // request, and no short one with room for a step), the one with the least
    // remaining work takes one step
    if (std::all_of(take.begin(), take.end(), [](int32_t v) { return v == 0; })) {
      size_t k0 = active.size();
      for (size_t k = 0; k < active.size(); ++k)
        if (key[k] >= 0 && (k0 == active.size() || remaining(k) < remaining(k0))) k0 = k;
      if (k0 < active.size()) take[k0] = std::min(1, active[k0].req->n_iter - active[k0].progress);
    }
    for (size_t k = 0; k < active.size(); ++k) {
      const Slot& sl = active[k];
      if (key[k] < 0) take[k] = 0;
      lim_host[(size_t)sl.id] = sl.progress + take[k];
      if (key[k] >= 0) {
        int32_t& most = longest[key[k]];
        most = std::max(most, take[k]);
      }
      pairs += per_step_of(k) * take[k];
    }
    // Re-plan the groups whose membership changed (the others keep their
    // plans and captured chunks).
    if (st == TSGNE_OK) {
      std::map<int32_t, std::vector<size_t>> by_tile;
      for (size_t k = 0; k < active.size(); ++k)
        if (key[k] >= 0) by_tile[key[k]].push_back(k);
      if (by_tile.size() > (size_t)kMaxGroups + 1) st = fail(TSGNE_E_INVAL, "more tile sizes than round branches");
      if (by_tile.size() > 1 && !branches_ok) st = fail(TSGNE_E_DEVICE, "create round branches");
      for (auto it = groups.begin(); it != groups.end();) {
        if (!by_tile.count(it->first)) it = groups.erase(it);
        else ++it;
      }
      for (auto& kv : by_tile) {
        if (st != TSGNE_OK) break;
        std::vector<uint64_t> tickets;
        for (size_t k : kv.second) tickets.push_back(active[k].req->ticket);
        Group& gr = groups[kv.first];
        if (gr.tickets == tickets) continue;
        gr.clear();
        gr.tickets.clear();
        std::vector<BatchMember> members;
        for (size_t k : kv.second) {
          Slot& sl = active[k];
          const size_t len = 2 * (size_t)sl.req->n;
          members.push_back(BatchMember{sl.g, sl.state, sl.state + len, sl.state + 2 * len, sl.t,
                                        limits + sl.id, sl.req->n_iter});
        }
        st = gr.run.setup(members.data(), (int32_t)members.size(), kv.first % kHeadKey, &cfg.params);
        if (st == TSGNE_OK) gr.tickets = tickets;
      }
    }

    // Each group replays a captured chunk of its own length (the power of two
    // at or above its longest allotment, at most kChunkSteps) as often as that
    // allotment needs; members pause at their limit on the device, so a group
    // of large graphs that take one step in a round does not launch the many
    // steps a group of small ones takes beside it.
    // The groups run together, except the running long request's group,
    // which runs after them: the long request fills the GPU by itself, and
    // small graphs' steps beside its kernels cost it more than they gain;
    // the small requests, batched together, take about the time one of them
    // takes alone.
    struct Launch {
      hipGraphExec_t exec;
      int32_t reps;
      bool after;
    };
    std::vector<Launch> launches;
    for (auto& kv : groups) {
      if (st != TSGNE_OK) break;
      const int32_t most = longest[kv.first];
      if (most <= 0) continue;  // every member pauses: nothing to launch
      int32_t len = 1;
      while (len < most && len < kChunkSteps) len *= 2;
      hipGraphExec_t exec = nullptr;
      {
        std::lock_guard<std::mutex> cl(capture_mu);
        st = chunk_exec(kv.second, len, cfg.params, cap, &exec);
      }
      launches.push_back(Launch{exec, (most + len - 1) / len, kv.first >= kHeadKey});
    }
    if (st == TSGNE_OK) {
      hipError_t e = hipMemcpyAsync(limits, lim_host.data(), sizeof(int32_t) * lim_host.size(),
                                    hipMemcpyHostToDevice, s);
      if (e != hipSuccess) st = hip_fail(e, "upload round limits");
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      plan_s += seconds_since(t_plan, Clock::now());
    }
    const Clock::time_point t0 = Clock::now();
    if (st == TSGNE_OK) {
      hipError_t e = hipSuccess;
      std::vector<const Launch*> together, after;
      for (const Launch& l : launches) (l.after ? after : together).push_back(&l);
      if (together.size() == 1) {
        for (int32_t r = 0; r < together[0]->reps && e == hipSuccess; ++r) e = hipGraphLaunch(together[0]->exec, s);
      } else if (together.size() > 1) {
        e = hipEventRecord(fork, s);
        for (size_t gi = 0; gi < together.size() && e == hipSuccess; ++gi) {
          e = hipStreamWaitEvent(branch[gi], fork, 0);
          for (int32_t r = 0; r < together[gi]->reps && e == hipSuccess; ++r)
            e = hipGraphLaunch(together[gi]->exec, branch[gi]);
          if (e == hipSuccess) e = hipEventRecord(join[gi], branch[gi]);
          if (e == hipSuccess) e = hipStreamWaitEvent(s, join[gi], 0);
        }
      }
      for (const Launch* l : after)
        for (int32_t r = 0; r < l->reps && e == hipSuccess; ++r) e = hipGraphLaunch(l->exec, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = hip_fail(e, "run a serving round");
    }
    if (st != TSGNE_OK) {
      // a device failure ends every active request with that status
      const std::string why = tsgne_last_error();
      for (Slot& sl : active) finish(sl, st, why, false, s);
      active.clear();
      groups.clear();
      continue;
    }
    const double dt = seconds_since(t0, Clock::now());
    {
      std::lock_guard<std::mutex> lk(mu);
      if (dt > 0.0 && pairs > 1e9) pair_rate = 0.5 * pair_rate + 0.5 * pairs / dt;
      ++rounds;
      busy_s += dt;
    }
    for (size_t k = 0, j = 0; k < active.size(); ++j) {
      Slot& sl = active[k];
      sl.progress += take[j];
      if (sl.progress >= sl.req->n_iter) {
        finish(sl, TSGNE_OK, "", true, s);
        active.erase(active.begin() + (long)k);
      } else {
        ++k;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      n_active = (int32_t)active.size();
      cv_admit.notify_one();  // slots may have come free
    }
  }
  groups.clear();
  {
    // wait for the admitter to leave its loop: nothing else touches these then
    std::unique_lock<std::mutex> lk(mu);
    cv_work.wait(lk, [&] { return admitter_done; });
  }
  for (std::vector<Slot>* v : {&active, &incoming}) {
    for (Slot& sl : *v) {
      sl.req->cancel = true;
      finish(sl, TSGNE_E_CANCELLED, "server destroyed", false, s);
    }
    v->clear();
  }
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
  dfree(limits);
  for (int k = 0; k < kMaxGroups; ++k) {
    if (branch[k]) (void)hipStreamDestroy(branch[k]);
    if (join[k]) (void)hipEventDestroy(join[k]);
  }
  if (fork) (void)hipEventDestroy(fork);
  for (hipStream_t q : {s, cap})
    if (q) (void)hipStreamDestroy(q);
}

extern "C" {

void tsgne_server_config_default(tsgne_server_config* c) {
  if (!c) return;
  c->hbm_budget = 0;
  c->max_active = 64;
  c->max_queue = 1 << 20;
  c->steps_per_round = 512;
  c->round_ms = 25.0f;
  c->oldest_share = 0.5f;
  c->rest_policy = TSGNE_SHARE_SHORT_FIRST;
  c->tile_rows = 0;
  tsgne_params_default(&c->params);
  c->long_ms = 150.0f;
  c->short_share = 0.3f;
}

tsgne_status tsgne_server_create(const tsgne_server_config* cfg, tsgne_server** out) {
  if (!cfg || !out) return fail(TSGNE_E_INVAL, "null pointer");
  *out = nullptr;
  if (tsgne_status st = validate_params(&cfg->params)) return st;
  if (!std::isfinite(cfg->round_ms)) return fail(TSGNE_E_INVAL, "round_ms must be finite");
  if (!(cfg->oldest_share >= 0.f && cfg->oldest_share < 1.f))
    return fail(TSGNE_E_INVAL, "oldest_share must lie in [0, 1)");
  if (cfg->rest_policy != TSGNE_SHARE_EQUAL && cfg->rest_policy != TSGNE_SHARE_SMALLEST_FIRST &&
      cfg->rest_policy != TSGNE_SHARE_SHORT_FIRST)
    return fail(TSGNE_E_INVAL, "rest_policy must be TSGNE_SHARE_EQUAL, _SMALLEST_FIRST or _SHORT_FIRST");
  if (!(cfg->long_ms >= 0.f) || !std::isfinite(cfg->long_ms)) return fail(TSGNE_E_INVAL, "long_ms must be >= 0");
  if (!(cfg->short_share > 0.f && cfg->short_share < 1.f))
    return fail(TSGNE_E_INVAL, "short_share must lie in (0, 1)");
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
  for (int32_t k = srv->cfg.max_active - 1; k >= 0; --k) srv->free_ids.push_back(k);
  srv->worker = std::thread([srv] { srv->run(); });
  srv->admitter = std::thread([srv] { srv->admit_loop(); });
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
  r->R = srv->cfg.tile_rows ? srv->cfg.tile_rows : request_tile_rows(rq->n);
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
  srv->cv_admit.notify_one();
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

tsgne_status tsgne_server_error(tsgne_server* srv, uint64_t ticket, char* buf, int32_t len) {
  if (!srv || !buf || len < 1) return fail(TSGNE_E_INVAL, "null pointer or empty buffer");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return fail(TSGNE_E_INVAL, "unknown ticket");
  const Request& r = *it->second;
  if (!r.done) return fail(TSGNE_E_BUSY, "request still queued or running");
  const size_t n = std::min(r.error.size(), (size_t)len - 1);
  std::copy(r.error.begin(), r.error.begin() + (long)n, buf);
  buf[n] = 0;
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
  out->admit_s = srv->admit_s;
  out->plan_s = srv->plan_s;
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
    srv->cv_admit.notify_all();
  }
  // the admitter first: once it has stopped, only the worker holds slots
  if (srv->admitter.joinable()) srv->admitter.join();
  if (srv->worker.joinable()) srv->worker.join();
  delete srv;
  return TSGNE_OK;
}

}  // extern "C"
