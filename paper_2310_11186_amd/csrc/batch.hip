// Batched optimisation of many independent graphs: one set of fused launches
// per step for the whole batch, captured once as a HIP graph and replayed, and
// the autotuner that picks the repulsion tile for a batch by timing it.
#include <algorithm>
#include <cctype>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

namespace tsgne {

constexpr int kBatchBlockRows = 256;  // rows per update block
constexpr int kBatchAttractRows = 256 / kAttractRowLanes;  // rows per attraction block

BatchRun::~BatchRun() {
  if (tables_) (void)hipFree(tables_);
}

tsgne_status BatchRun::setup(const BatchMember* m, int32_t count, int32_t R, const tsgne_params* p) {
  tsgne_params pr = *p;
  pr.tile_rows = R;
  pr.repulsion = TSGNE_REPULSION_SYMMETRIC;
  for (int32_t k = 0; k < count; ++k)
    if (tsgne_status st = ensure_workspace(m[k].g, &pr)) return st;
  bp_ = BatchPlan{};
  bp_.count = count;
  bp_.R = R;
  bp_.T = kWave * R;
  std::vector<BatchDesc> descs((size_t)count);
  std::vector<int4> diag_items, items, last_items;
  std::vector<int2> chunks, heavy, blocks;
  for (int32_t k = 0; k < count; ++k) {
    tsgne_graph* g = m[k].g;
    const Workspace& ws = g->ws;
    BatchDesc& d = descs[(size_t)k];
    d.Y = reinterpret_cast<float2*>(m[k].Y);
    d.U = reinterpret_cast<float2*>(m[k].U);
    d.G = reinterpret_cast<float2*>(m[k].G);
    d.row_ptr = g->row_ptr;
    d.col = g->col;
    d.P = g->P;
    d.part = ws.part;
    d.zpart = ws.zpart;
    d.zpart32 = ws.zpart32;
    d.Z = ws.Z;
    d.attract = ws.attract;
    d.t = m[k].t;
    d.limit = m[k].limit;
    d.n_items = ws.plan.items;
    d.n = g->n;
    d.nb = ws.plan.nb;
    d.n_iter = m[k].n_iter;
    d.eta = effective_eta(g, p);
    // each tile's Z partial slot is its index in the graph's own list
    // (diagonal tiles first, then the off-diagonal ones row by row, the tiles
    // against the last block last)
    const int32_t nb = ws.plan.nb;
    int64_t li = nb;
    for (int32_t a = 0; a < nb; ++a) {
      diag_items.push_back(make_int4(k, a, a, a));
      for (int32_t b = a + 1; b < nb - 1; ++b, ++li) items.push_back(make_int4(k, a, b, (int)li));
    }
    for (int32_t a = 0; a < nb - 1; ++a, ++li) last_items.push_back(make_int4(k, a, nb - 1, (int)li));
    for (int32_t r = 0; r < g->n; r += kBatchAttractRows) chunks.push_back(make_int2(k, r));
    for (int32_t r = 0; r < g->n; r += kBatchBlockRows) blocks.push_back(make_int2(k, r));
    if (g->n_heavy > 0) {
      std::vector<int32_t> h((size_t)g->n_heavy);
      TSGNE_HIP(hipMemcpy(h.data(), g->heavy, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost), "read heavy rows");
      for (int32_t r : h) heavy.push_back(make_int2(k, r));
    }
  }
  // diagonal tiles (one row per lane per pass, the slower kind) go first,
  // the tiles against each graph's partly filled last block last
  diag_items.insert(diag_items.end(), items.begin(), items.end());
  diag_items.insert(diag_items.end(), last_items.begin(), last_items.end());
  bp_.n_items = (int64_t)diag_items.size();
  bp_.n_light_chunks = (int32_t)chunks.size();
  bp_.n_heavy = (int32_t)heavy.size();
  bp_.n_row_blocks = (int32_t)blocks.size();

  const size_t b_descs = sizeof(BatchDesc) * descs.size();
  const size_t b_items = sizeof(int4) * diag_items.size();
  const size_t b_chunks = sizeof(int2) * chunks.size();
  const size_t b_heavy = sizeof(int2) * heavy.size();
  const size_t b_blocks = sizeof(int2) * blocks.size();
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t total = up(b_descs) + up(b_items) + up(b_chunks) + up(b_heavy) + up(b_blocks);
  if (tables_) (void)hipFree(tables_);
  tables_ = nullptr;
  TSGNE_HIP(hipMalloc(&tables_, total), "allocate batch tables");
  char* base = static_cast<char*>(tables_);
  size_t at = 0;
  auto place = [&](size_t bytes) {
    char* q = base + at;
    at += up(bytes);
    return q;
  };
  bp_.descs = reinterpret_cast<BatchDesc*>(place(b_descs));
  bp_.items = reinterpret_cast<int4*>(place(b_items));
  bp_.light_chunks = reinterpret_cast<int2*>(place(b_chunks));
  bp_.heavy = reinterpret_cast<int2*>(place(b_heavy));
  bp_.row_blocks = reinterpret_cast<int2*>(place(b_blocks));
  TSGNE_HIP(hipMemcpy(bp_.descs, descs.data(), b_descs, hipMemcpyHostToDevice), "upload batch descriptors");
  if (b_items) TSGNE_HIP(hipMemcpy(bp_.items, diag_items.data(), b_items, hipMemcpyHostToDevice), "upload items");
  if (b_chunks) TSGNE_HIP(hipMemcpy(bp_.light_chunks, chunks.data(), b_chunks, hipMemcpyHostToDevice), "upload rows");
  if (b_heavy) TSGNE_HIP(hipMemcpy(bp_.heavy, heavy.data(), b_heavy, hipMemcpyHostToDevice), "upload heavy rows");
  if (b_blocks) TSGNE_HIP(hipMemcpy(bp_.row_blocks, blocks.data(), b_blocks, hipMemcpyHostToDevice), "upload blocks");
  return TSGNE_OK;
}

tsgne_status run_batch_steps(const BatchRun& br, const tsgne_params* p, int32_t n_steps, int32_t chunk,
                             hipStream_t s) {
  if (n_steps <= 0) return TSGNE_OK;
  chunk = std::max(1, std::min(chunk, n_steps));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  TSGNE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t le = hipSuccess;
  for (int32_t k = 0; k < chunk && le == hipSuccess; ++k) le = launch_batch_step(br.plan(), *p, s);
  hipError_t ce = hipStreamEndCapture(s, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(le, "launch batched step during capture");
  }
  TSGNE_HIP(ce, "end capture");
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "instantiate batch graph");
  }
  const int32_t replays = (n_steps + chunk - 1) / chunk;
  for (int32_t r = 0; r < replays && e == hipSuccess; ++r) e = hipGraphLaunch(exec, s);
  hipError_t se = hipStreamSynchronize(s);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  TSGNE_HIP(e, "launch batch graph");
  TSGNE_HIP(se, "synchronise batch");
  return TSGNE_OK;
}

// Streams and events to run several batched plans side by side.
struct Branches {
  hipStream_t stream[kMaxTileKinds] = {};
  hipEvent_t fork = nullptr, join[kMaxTileKinds] = {};
  bool ok = false;
  Branches() {
    ok = hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < kMaxTileKinds && ok; ++k)
      ok = hipStreamCreateWithFlags(&stream[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&join[k], hipEventDisableTiming) == hipSuccess;
  }
  ~Branches() {
    for (int k = 0; k < kMaxTileKinds; ++k) {
      if (stream[k]) (void)hipStreamDestroy(stream[k]);
      if (join[k]) (void)hipEventDestroy(join[k]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
};

// One batched step of every plan: with one plan on s itself, with several
// each on its own branch stream, forked from s and joined back into it.
hipError_t launch_groups_step(const std::vector<const BatchRun*>& runs, const tsgne_params& p, const Branches& br,
                              hipStream_t s) {
  if (runs.size() == 1) return launch_batch_step(runs[0]->plan(), p, s);
  hipError_t e = hipEventRecord(br.fork, s);
  for (size_t k = 0; k < runs.size() && e == hipSuccess; ++k) {
    e = hipStreamWaitEvent(br.stream[k], br.fork, 0);
    if (e == hipSuccess) e = launch_batch_step(runs[k]->plan(), p, br.stream[k]);
    if (e == hipSuccess) e = hipEventRecord(br.join[k], br.stream[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, br.join[k], 0);
  }
  return e;
}

namespace {

constexpr int kCaptureSteps = 25;  // steps per captured HIP graph

// Optimiser state (U = 0, gains = 1, t = 0, no pause limit) for a list of
// graphs, contiguous.
struct PooledState {
  float* f = nullptr;
  int32_t* t = nullptr;  // [count] step indices, then [count] limits
  ~PooledState() {
    dfree(f);
    dfree(t);
  }
  tsgne_status make(tsgne_graph* const* gs, float* const* Ys, const int32_t* n_iter, int32_t count,
                    std::vector<BatchMember>& out, hipStream_t s) {
    int64_t total = 0;
    for (int32_t k = 0; k < count; ++k) total += gs[k]->n;
    TSGNE_HIP(dalloc(&f, (size_t)4 * total), "allocate batch state");
    TSGNE_HIP(dalloc(&t, 2 * (size_t)count), "allocate step indices");
    std::vector<float> init((size_t)4 * total, 0.0f);
    std::fill(init.begin() + 2 * total, init.end(), 1.0f);
    std::vector<int32_t> ti(2 * (size_t)count, 0);
    std::fill(ti.begin() + count, ti.end(), INT32_MAX);
    TSGNE_HIP(hipMemcpyAsync(f, init.data(), sizeof(float) * init.size(), hipMemcpyHostToDevice, s),
              "initialise batch state");
    TSGNE_HIP(hipMemcpyAsync(t, ti.data(), sizeof(int32_t) * ti.size(), hipMemcpyHostToDevice, s),
              "reset step indices");
    TSGNE_HIP(hipStreamSynchronize(s), "synchronise batch set-up");
    out.resize((size_t)count);
    int64_t off = 0;
    for (int32_t k = 0; k < count; ++k) {
      out[(size_t)k] = BatchMember{gs[k], Ys[k], f + 2 * off, f + 2 * total + 2 * off, t + k, t + count + k,
                                   n_iter[k]};
      off += gs[k]->n;
    }
    return TSGNE_OK;
  }
};

tsgne_status check_batch_args(tsgne_graph* const* gs, const float* const* Ys, int32_t count, const tsgne_params* p) {
  if (!gs || !Ys || !p) return fail(TSGNE_E_INVAL, "null pointer");
  if (count < 1) return fail(TSGNE_E_INVAL, "count must be >= 1");
  if (tsgne_status st = validate_params(p)) return st;
  std::set<const void*> seen_g, seen_y;
  for (int32_t k = 0; k < count; ++k) {
    if (!gs[k] || !Ys[k]) return fail(TSGNE_E_INVAL, "null graph or layout in the batch");
    if (gs[k]->device != gs[0]->device) return fail(TSGNE_E_INVAL, "all graphs of a batch must be on one device");
    if (!seen_g.insert(gs[k]).second) return fail(TSGNE_E_INVAL, "a graph appears twice in the batch");
    if (!seen_y.insert(Ys[k]).second) return fail(TSGNE_E_INVAL, "two graphs share a layout buffer");
  }
  return TSGNE_OK;
}

// Tile chosen without timing: the largest R leaving ~8 waves of tiles per SIMD.
int32_t default_batch_R(tsgne_graph* const* gs, int32_t count) {
  for (int32_t R : {16, 8}) {
    int64_t items = 0;
    for (int32_t k = 0; k < count; ++k) {
      const int64_t nb = (gs[k]->n + kWave * R - 1) / (kWave * R);
      items += nb * (nb + 1) / 2;
    }
    if (items >= 8192) return R;
  }
  return 4;
}

// A stream that can be captured: the caller's, or a private one for NULL.
struct CaptureStream {
  hipStream_t s = nullptr;
  bool owned = false;
  explicit CaptureStream(void* user) {
    s = reinterpret_cast<hipStream_t>(user);
    if (!s) {
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess) owned = true;
      else s = nullptr;
    }
  }
  ~CaptureStream() {
    if (owned) (void)hipStreamDestroy(s);
  }
};

// Graphs grouped by tile rows over one pooled optimiser state: one batched
// plan per group (ascending tile rows).
struct TiledBatch {
  PooledState ps;
  std::vector<BatchMember> members;
  std::map<int32_t, BatchRun> runs;
  std::vector<const BatchRun*> order;
  tsgne_status setup(tsgne_graph* const* gs, float* const* Ys, const int32_t* n_iter, const int32_t* tiles,
                     int32_t count, const tsgne_params* p, hipStream_t s) {
    if (tsgne_status st = ps.make(gs, Ys, n_iter, count, members, s)) return st;
    std::map<int32_t, std::vector<BatchMember>> by_tile;
    for (int32_t k = 0; k < count; ++k) by_tile[tiles[k]].push_back(members[(size_t)k]);
    for (auto& kv : by_tile)
      if (tsgne_status st = runs[kv.first].setup(kv.second.data(), (int32_t)kv.second.size(), kv.first, p)) return st;
    order.clear();
    for (auto& kv : runs) order.push_back(&kv.second);
    return TSGNE_OK;
  }
};

// Runs n_steps steps of several plans side by side: `chunk` steps captured
// once (fork and join included) and replayed.  Synchronises s.
tsgne_status run_groups(const std::vector<const BatchRun*>& runs, const tsgne_params* p, int32_t n_steps,
                        int32_t chunk, const Branches& br, hipStream_t s) {
  if (n_steps <= 0) return TSGNE_OK;
  chunk = std::max(1, std::min(chunk, n_steps));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  TSGNE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t le = hipSuccess;
  for (int32_t k = 0; k < chunk && le == hipSuccess; ++k) le = launch_groups_step(runs, *p, br, s);
  hipError_t ce = hipStreamEndCapture(s, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(le, "launch batched step during capture");
  }
  TSGNE_HIP(ce, "end capture");
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(e, "instantiate batch graph");
  }
  const int32_t replays = (n_steps + chunk - 1) / chunk;
  for (int32_t r = 0; r < replays && e == hipSuccess; ++r) e = hipGraphLaunch(exec, s);
  hipError_t se = hipStreamSynchronize(s);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  TSGNE_HIP(e, "launch batch graph");
  TSGNE_HIP(se, "synchronise batch");
  return TSGNE_OK;
}

// Finiteness of the final layouts.
tsgne_status check_layouts(tsgne_graph* const* graphs, float* const* Y_d, int32_t count, hipStream_t s) {
  ScratchBlock flag;
  flag.s = s;
  TSGNE_HIP(scratch_alloc(&flag.p, sizeof(uint32_t), s), "allocate flag");
  uint32_t* f = static_cast<uint32_t*>(flag.p);
  TSGNE_HIP(hipMemsetAsync(f, 0, sizeof(uint32_t), s), "clear flag");
  for (int32_t k = 0; k < count; ++k)
    TSGNE_HIP(launch_nonfinite_check(reinterpret_cast<const float2*>(Y_d[k]), graphs[k]->n, f, s),
              "launch finiteness check");
  uint32_t host_flag = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_flag, f, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read flag");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise batch");
  if (host_flag) return fail(TSGNE_E_NONFINITE, "a layout holds a NaN or infinity");
  return TSGNE_OK;
}

// Size bucket of a graph for the tile table: floor(log2(n)).
int32_t size_bucket(int32_t n) {
  int32_t b = 0;
  while (b < TSGNE_TILE_BUCKETS - 1 && ((int64_t)1 << (b + 1)) <= n) ++b;
  return b;
}

// The device's architecture name without feature suffixes ("gfx950").
std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// The tile cache file: a JSON object of architectures, each an object of
// size buckets (as strings) to tile rows, e.g. {"gfx950": {"13": 8, "14": 12}}.
// Read leniently: anything that is not that shape is ignored.
using TileCache = std::map<std::string, std::map<int32_t, int32_t>>;

TileCache read_tile_cache(const char* path) {
  TileCache out;
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  size_t i = 0;
  auto skip = [&]() {
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
  };
  auto string_at = [&](std::string* v) {
    skip();
    if (i >= text.size() || text[i] != '"') return false;
    const size_t e = text.find('"', i + 1);
    if (e == std::string::npos) return false;
    *v = text.substr(i + 1, e - i - 1);
    i = e + 1;
    return true;
  };
  auto expect = [&](char c) {
    skip();
    if (i < text.size() && text[i] == c) {
      ++i;
      return true;
    }
    return false;
  };
  if (!expect('{')) return out;
  while (true) {
    std::string arch;
    if (!string_at(&arch) || !expect(':') || !expect('{')) break;
    while (true) {
      std::string key;
      if (!string_at(&key) || !expect(':')) break;
      skip();
      char* end = nullptr;
      const long v = std::strtol(text.c_str() + i, &end, 10);
      if (end == text.c_str() + i) break;
      i = (size_t)(end - text.c_str());
      const long b = std::strtol(key.c_str(), nullptr, 10);
      if (tile_rows_supported((int32_t)v) && b >= 0 && b < TSGNE_TILE_BUCKETS) out[arch][(int32_t)b] = (int32_t)v;
      if (!expect(',')) break;
    }
    if (!expect('}') || !expect(',')) break;
  }
  return out;
}

bool write_tile_cache(const char* path, const TileCache& cache) {
  const std::string tmp = std::string(path) + ".tmp";
  std::FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{");
  bool first_arch = true;
  for (const auto& a : cache) {
    std::fprintf(f, "%s\n \"%s\": {", first_arch ? "" : ",", a.first.c_str());
    bool first = true;
    for (const auto& kv : a.second) {
      std::fprintf(f, "%s\"%d\": %d", first ? "" : ", ", kv.first, kv.second);
      first = false;
    }
    std::fprintf(f, "}");
    first_arch = false;
  }
  std::fprintf(f, "\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_batch_run(tsgne_graph* const* graphs, float* const* Y_d, const int32_t* n_iter, int32_t count,
                             const tsgne_params* p, void* stream) {
  if (tsgne_status st = check_batch_args(graphs, const_cast<const float* const*>(Y_d), count, p)) return st;
  if (!n_iter) return fail(TSGNE_E_INVAL, "n_iter is NULL");
  int32_t max_iter = 0;
  for (int32_t k = 0; k < count; ++k) {
    if (n_iter[k] < 0) return fail(TSGNE_E_INVAL, "n_iter must be >= 0");
    max_iter = std::max(max_iter, n_iter[k]);
  }
  DeviceGuard dg(graphs[0]->device);
  CaptureStream cs(stream);
  if (!cs.s) return fail(TSGNE_E_DEVICE, "cannot create a stream");
  const int32_t R = p->tile_rows ? p->tile_rows : default_batch_R(graphs, count);
  PooledState ps;
  std::vector<BatchMember> members;
  if (tsgne_status st = ps.make(graphs, Y_d, n_iter, count, members, cs.s)) return st;
  BatchRun br;
  if (tsgne_status st = br.setup(members.data(), count, R, p)) return st;
  if (tsgne_status st = run_batch_steps(br, p, max_iter, kCaptureSteps, cs.s)) return st;
  uint32_t* flag = nullptr;
  TSGNE_HIP(dalloc(&flag, 1), "allocate flag");
  struct F {
    uint32_t*& f;
    ~F() { dfree(f); }
  } ff{flag};
  TSGNE_HIP(hipMemsetAsync(flag, 0, sizeof(uint32_t), cs.s), "clear flag");
  for (int32_t k = 0; k < count; ++k)
    TSGNE_HIP(launch_nonfinite_check(reinterpret_cast<const float2*>(Y_d[k]), graphs[k]->n, flag, cs.s),
              "launch finiteness check");
  uint32_t host_flag = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, cs.s), "read flag");
  TSGNE_HIP(hipStreamSynchronize(cs.s), "synchronise batch");
  if (host_flag) return fail(TSGNE_E_NONFINITE, "a layout holds a NaN or infinity");
  return TSGNE_OK;
}

tsgne_status tsgne_autotune(tsgne_graph* const* graphs, const float* const* Y_d, int32_t count,
                            const tsgne_params* p, int32_t steps, int32_t* best_tile_rows, double* ms_per_step,
                            void* stream) {
  if (!best_tile_rows) return fail(TSGNE_E_INVAL, "null pointer");
  if (steps < 1) return fail(TSGNE_E_INVAL, "steps must be >= 1");
  if (tsgne_status st = check_batch_args(graphs, Y_d, count, p)) return st;
  DeviceGuard dg(graphs[0]->device);
  CaptureStream cs(stream);
  if (!cs.s) return fail(TSGNE_E_DEVICE, "cannot create a stream");
  std::vector<float*> scratch((size_t)count, nullptr);
  struct Scratch {
    std::vector<float*>& v;
    ~Scratch() {
      for (float*& q : v) dfree(q);
    }
  } sc{scratch};
  for (int32_t k = 0; k < count; ++k)
    TSGNE_HIP(dalloc(&scratch[(size_t)k], 2 * (size_t)graphs[k]->n), "allocate scratch layout");
  std::vector<int32_t> iters((size_t)count, steps + 1);
  const int32_t candidates[TSGNE_AUTOTUNE_TILES] = {4, 8, 12, 16};
  double best = INFINITY;
  int32_t best_R = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TSGNE_HIP(hipEventCreate(&e0), "create event");
  TSGNE_HIP(hipEventCreate(&e1), "create event");
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  for (int c = 0; c < TSGNE_AUTOTUNE_TILES; ++c) {
    const int32_t R = candidates[c];
    for (int32_t k = 0; k < count; ++k)
      TSGNE_HIP(hipMemcpyAsync(scratch[(size_t)k], Y_d[k], sizeof(float) * 2 * graphs[k]->n,
                               hipMemcpyDeviceToDevice, cs.s),
                "copy layout");
    PooledState ps;
    std::vector<BatchMember> members;
    if (tsgne_status st = ps.make(graphs, scratch.data(), iters.data(), count, members, cs.s)) return st;
    BatchRun br;
    if (tsgne_status st = br.setup(members.data(), count, R, p)) return st;
    TSGNE_HIP(launch_batch_step(br.plan(), *p, cs.s), "warm-up step");
    TSGNE_HIP(hipEventRecord(e0, cs.s), "record event");
    for (int32_t k = 0; k < steps; ++k) TSGNE_HIP(launch_batch_step(br.plan(), *p, cs.s), "timed step");
    TSGNE_HIP(hipEventRecord(e1, cs.s), "record event");
    TSGNE_HIP(hipEventSynchronize(e1), "synchronise autotune");
    float ms = 0.f;
    TSGNE_HIP(hipEventElapsedTime(&ms, e0, e1), "read event time");
    const double per = ms / steps;
    if (ms_per_step) ms_per_step[c] = per;
    if (per < best) {
      best = per;
      best_R = R;
    }
  }
  *best_tile_rows = best_R;
  return TSGNE_OK;
}

tsgne_status tsgne_batch_run_tiles(tsgne_graph* const* graphs, float* const* Y_d, const int32_t* n_iter,
                                   const int32_t* tile_rows, int32_t count, const tsgne_params* p, void* stream) {
  if (tsgne_status st = check_batch_args(graphs, const_cast<const float* const*>(Y_d), count, p)) return st;
  if (!n_iter || !tile_rows) return fail(TSGNE_E_INVAL, "n_iter or tile_rows is NULL");
  int32_t max_iter = 0;
  std::vector<int32_t> tiles((size_t)count);
  for (int32_t k = 0; k < count; ++k) {
    if (n_iter[k] < 0) return fail(TSGNE_E_INVAL, "n_iter must be >= 0");
    if (tile_rows[k] != 0 && !tile_rows_supported(tile_rows[k]))
      return fail(TSGNE_E_INVAL, "tile_rows must be 0, 1, 2, 4, 8, 12, 14, 15 or 16");
    tiles[(size_t)k] = tile_rows[k] ? tile_rows[k] : make_plan(graphs[k]->n, 0, TSGNE_REPULSION_SYMMETRIC).R;
    max_iter = std::max(max_iter, n_iter[k]);
  }
  DeviceGuard dg(graphs[0]->device);
  CaptureStream cs(stream);
  if (!cs.s) return fail(TSGNE_E_DEVICE, "cannot create a stream");
  Branches br;
  if (!br.ok) return fail(TSGNE_E_DEVICE, "cannot create branch streams");
  TiledBatch tb;
  if (tsgne_status st = tb.setup(graphs, Y_d, n_iter, tiles.data(), count, p, cs.s)) return st;
  if (tsgne_status st = run_groups(tb.order, p, max_iter, kCaptureSteps, br, cs.s)) return st;
  return check_layouts(graphs, Y_d, count, cs.s);
}

tsgne_status tsgne_autotune_tiles(tsgne_graph* const* graphs, const float* const* Y_d, int32_t count,
                                  const tsgne_params* p, int32_t steps, const char* cache_path,
                                  int32_t* tile_rows_out, double* ms_uniform, double* ms_tuned, void* stream) {
  if (!tile_rows_out) return fail(TSGNE_E_INVAL, "null pointer");
  if (steps < 1) return fail(TSGNE_E_INVAL, "steps must be >= 1");
  if (tsgne_status st = check_batch_args(graphs, Y_d, count, p)) return st;
  DeviceGuard dg(graphs[0]->device);
  CaptureStream cs(stream);
  if (!cs.s) return fail(TSGNE_E_DEVICE, "cannot create a stream");
  Branches br;
  if (!br.ok) return fail(TSGNE_E_DEVICE, "cannot create branch streams");
  const std::string arch = device_arch();
  TileCache cache = cache_path ? read_tile_cache(cache_path) : TileCache{};
  std::map<int32_t, int32_t>& known = cache[arch];
  // buckets present, heaviest (sum of n^2) first
  std::map<int32_t, double> work;
  std::vector<int32_t> bucket((size_t)count);
  for (int32_t k = 0; k < count; ++k) {
    bucket[(size_t)k] = size_bucket(graphs[k]->n);
    work[bucket[(size_t)k]] += (double)graphs[k]->n * (double)graphs[k]->n;
  }
  std::vector<int32_t> open;  // buckets the cache does not fix
  for (auto& kv : work)
    if (!known.count(kv.first)) open.push_back(kv.first);
  std::stable_sort(open.begin(), open.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });

  std::vector<float*> scratch((size_t)count, nullptr);
  struct Scratch {
    std::vector<float*>& v;
    ~Scratch() {
      for (float*& q : v) dfree(q);
    }
  } sc{scratch};
  for (int32_t k = 0; k < count; ++k)
    TSGNE_HIP(dalloc(&scratch[(size_t)k], 2 * (size_t)graphs[k]->n), "allocate scratch layout");
  std::vector<int32_t> iters((size_t)count, steps + 1);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TSGNE_HIP(hipEventCreate(&e0), "create event");
  TSGNE_HIP(hipEventCreate(&e1), "create event");
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  // ms per batched step with the tile of each bucket from `rows`
  auto time_rows = [&](const std::map<int32_t, int32_t>& rows, double* ms) -> tsgne_status {
    std::vector<int32_t> tiles((size_t)count);
    for (int32_t k = 0; k < count; ++k) tiles[(size_t)k] = rows.at(bucket[(size_t)k]);
    for (int32_t k = 0; k < count; ++k)
      TSGNE_HIP(hipMemcpyAsync(scratch[(size_t)k], Y_d[k], sizeof(float) * 2 * graphs[k]->n,
                               hipMemcpyDeviceToDevice, cs.s),
                "copy layout");
    TiledBatch tb;
    if (tsgne_status st = tb.setup(graphs, scratch.data(), iters.data(), tiles.data(), count, p, cs.s)) return st;
    TSGNE_HIP(launch_groups_step(tb.order, *p, br, cs.s), "warm-up step");
    TSGNE_HIP(hipEventRecord(e0, cs.s), "record event");
    for (int32_t k = 0; k < steps; ++k) TSGNE_HIP(launch_groups_step(tb.order, *p, br, cs.s), "timed step");
    TSGNE_HIP(hipEventRecord(e1, cs.s), "record event");
    TSGNE_HIP(hipEventSynchronize(e1), "synchronise autotune");
    float t = 0.f;
    TSGNE_HIP(hipEventElapsedTime(&t, e0, e1), "read event time");
    *ms = t / steps;
    return TSGNE_OK;
  };
  const int32_t candidates[] = {2, 4, 8, 12, 16};
  std::map<int32_t, int32_t> rows = known;
  // 1. one tile for every open bucket
  double best = INFINITY;
  int32_t best_R = 8;
  for (int32_t R : candidates) {
    if (open.empty()) break;
    for (int32_t b : open) rows[b] = R;
    double ms = 0.0;
    if (tsgne_status st = time_rows(rows, &ms)) return st;
    if (ms < best) {
      best = ms;
      best_R = R;
    }
  }
  for (int32_t b : open) rows[b] = best_R;
  if (open.empty()) {
    if (tsgne_status st = time_rows(rows, &best)) return st;
  }
  if (ms_uniform) *ms_uniform = best;
  // 2. each open bucket in turn, heaviest first: the tile that makes the whole
  // batch fastest with the others fixed (kept only if at least 0.5 % faster)
  for (int32_t b : open) {
    const int32_t keep = rows[b];
    int32_t pick = keep;
    for (int32_t R : candidates) {
      if (R == keep) continue;
      rows[b] = R;
      double ms = 0.0;
      if (tsgne_status st = time_rows(rows, &ms)) return st;
      if (ms < 0.995 * best) {
        best = ms;
        pick = R;
      }
    }
    rows[b] = pick;
  }
  if (ms_tuned) *ms_tuned = best;
  for (int32_t k = 0; k < count; ++k) tile_rows_out[k] = rows[bucket[(size_t)k]];
  if (cache_path && !open.empty()) {
    for (int32_t b : open) known[b] = rows[b];
    if (!write_tile_cache(cache_path, cache)) return fail(TSGNE_E_INVAL, std::string("cannot write ") + cache_path);
  }
  return TSGNE_OK;
}

}  // extern "C"
