// Internal declarations of the t-SGNE HIP library: the graph handle, the
// repulsion tiling plan and the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tsgne.h"

namespace tsgne {

// Rows per wave lane in the repulsion tile: a tile spans 64 * R positions.
constexpr int kWave = 64;

// Degree above which a row is handled by a whole wave (calibration, attraction).
constexpr int32_t kHeavyDegree = 64;
// Lanes per row in the attraction of rows up to kHeavyDegree entries (the
// single-graph and batched kernels must agree: it fixes the summation order).
constexpr int kAttractRowLanes = 8;

// Bits of the device error word written by the CSR check.
enum : uint32_t {
  kErrRowPtr = 1u << 0,   // row_ptr not monotone or not spanning [0, nnz]
  kErrColRange = 1u << 1, // column outside [0, n)
  kErrSelfLoop = 1u << 2,
  kErrOrder = 1u << 3,    // columns not strictly ascending in a row
  kErrAsym = 1u << 4,     // (i, j) stored without (j, i)
};

// All-pairs repulsion plan: positions are cut into nb blocks of T = 64 * R;
// tile (a, b) covers rows of block a against columns of block b.
struct RepulsionPlan {
  int32_t R = 0;        // rows per lane
  int32_t T = 0;        // block length = 64 * R
  int32_t nb = 0;       // number of blocks, the last one possibly partial
  int32_t variant = 0;  // TSGNE_REPULSION_DIRECT or _SYMMETRIC
  int64_t items = 0;    // work items (one wave each)
};

struct Workspace {
  RepulsionPlan plan;
  int2* items = nullptr;        // (a, b) per work item
  float2* part = nullptr;       // [nb][nb][T] force partials: part[k][o] = sum over block o acting on block k
  double* zpart = nullptr;      // [items] Z partial of each item (ordered pairs)
  double* Z = nullptr;          // [1] normaliser
  float* zpart32 = nullptr;     // [items] FP32-mode partials
  double2* attract = nullptr;   // [n] sum_j P_ij w_ij (y_i - y_j) (unscaled by alpha)
  double* klpart = nullptr;     // [kl_blocks] KL partial sums
  double* klout = nullptr;      // [1]
  int32_t* tstep = nullptr;     // [2] device step counter of a run: next step, step being run
  double* pinned = nullptr;     // host-pinned scratch for read-backs
  int32_t kl_blocks = 0;
};

// The early-exaggeration schedule read on the device by a replayed step
// (tstep == nullptr: the host passes alpha and the momentum instead).
struct StepSchedule {
  const int32_t* tstep = nullptr;
  int32_t exaggeration_iters = 0;
  float early_exaggeration = 1.f;
  float momentum_early = 0.f;
  float momentum_late = 0.f;
};

// Per-graph view used by the batched kernels (device memory, one per graph).
struct BatchDesc {
  float2* Y;
  float2* U;
  float2* G;
  const int32_t* row_ptr;
  const int32_t* col;
  const float* P;
  float2* part;
  double* zpart;
  float* zpart32;
  double* Z;
  double2* attract;
  int32_t* t;        // this graph's step index (advanced after every step)
  const int32_t* limit;  // steps run only while t < limit (a round's allotment)
  int64_t n_items;
  int32_t n;
  int32_t nb;
  int32_t n_iter;
  float eta;
};

// Launch tables of a batch (all device pointers).
struct BatchPlan {
  BatchDesc* descs = nullptr;
  int4* items = nullptr;          // (graph, a, b, item index within the graph)
  int2* light_chunks = nullptr;   // (graph, first row) per 32-row block
  int2* heavy = nullptr;          // (graph, row) per heavy row
  int2* row_blocks = nullptr;     // (graph, first row) per 256-row block
  int64_t n_items = 0;
  int32_t n_light_chunks = 0;
  int32_t n_heavy = 0;
  int32_t n_row_blocks = 0;
  int32_t count = 0;
  int32_t R = 0;
  int32_t T = 0;
};

// One graph of a batch with its own optimiser state (device pointers).
struct BatchMember {
  tsgne_graph* g;
  float* Y;        // float32[n][2]
  float* U;        // float32[n][2]
  float* G;        // float32[n][2] gains
  int32_t* t;      // step index
  const int32_t* limit;  // step index at which this graph pauses (device int)
  int32_t n_iter;
};

// Launch tables for a set of members, all tiled with the same R.
class BatchRun {
 public:
  ~BatchRun();
  tsgne_status setup(const BatchMember* m, int32_t count, int32_t R, const tsgne_params* p);
  const BatchPlan& plan() const { return bp_; }

 private:
  BatchPlan bp_;
  void* tables_ = nullptr;
};

// Runs n_steps batched steps: one captured sequence of up to `chunk` steps,
// replayed (graphs past their n_iter skip their work).  Synchronises s.
tsgne_status run_batch_steps(const BatchRun& br, const tsgne_params* p, int32_t n_steps, int32_t chunk,
                             hipStream_t s);

// Distinct repulsion tile sizes (1, 2, 4, 8, 12, 14, 15, 16).
constexpr int kMaxTileKinds = 8;

// Event-pair timing of kernel phases (see tsgne_graph_set_timing).
struct PhaseTimer {
  struct Pending {
    int phase;
    hipEvent_t start, stop;
  };
  bool enabled = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[TSGNE_NUM_PHASES] = {};
  int64_t launches[TSGNE_NUM_PHASES] = {};
};

}  // namespace tsgne

struct tsgne_graph {
  int device = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t d = 0;
  float perplexity = 0.f;
  int32_t* row_ptr = nullptr;   // [n+1]
  int32_t* col = nullptr;       // [nnz]
  int32_t* mirror = nullptr;    // [nnz]
  int32_t* row_of = nullptr;    // [nnz] row of each entry
  float* P = nullptr;           // [nnz]
  double* beta = nullptr;       // [n]
  int32_t* heavy = nullptr;     // rows with degree > kHeavyDegree
  int32_t n_heavy = 0;
  int64_t nonisolated = 0;
  tsgne::Workspace ws;
  tsgne::PhaseTimer timer;
};

namespace tsgne {

// Thread-local error message.
void set_error(const std::string& msg);
tsgne_status fail(tsgne_status code, const std::string& msg);
tsgne_status hip_fail(hipError_t e, const char* what);

#define TSGNE_HIP(call, what)                        \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Per-call scratch from a library-owned stream-ordered pool on the current
// device: up to 1 GiB of freed blocks stays cached in the pool, so repeated
// calls do not pay for hipMalloc/hipFree.  Usable in stream order on s.
hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s);
void scratch_free(void* p, hipStream_t s);

// Owns one scratch allocation until the end of a scope.
struct ScratchBlock {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~ScratchBlock() {
    if (p) scratch_free(p, s);
  }
};

// Makes a device current for the duration of a scope.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

tsgne_status validate_params(const tsgne_params* p);
// A graph with its CSR copied from the caller's device buffers, checked
// (canonical and symmetric, E_GRAPH otherwise), with mirror, row_of, the
// heavy-row list and the non-isolated count; P and beta allocated, not
// filled.  Synchronising.
tsgne_status graph_structure(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d, hipStream_t s,
                             tsgne_graph** out);
void free_graph(tsgne_graph* g);
// Checks on the device that (row_ptr, col) is a canonical symmetric CSR
// (synchronising; E_GRAPH otherwise).
tsgne_status validate_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, hipStream_t s);
// The same in caller-provided device scratch of validate_csr_bytes(n, nnz);
// *row_of_out (nullable) then points at the row of every entry, inside the
// scratch.
size_t validate_csr_bytes(int32_t n, int64_t nnz);
tsgne_status validate_csr_in(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, void* scratch,
                             hipStream_t s, int32_t** row_of_out = nullptr);
float effective_eta(const tsgne_graph* g, const tsgne_params* p);
tsgne_status ensure_workspace(tsgne_graph* g, const tsgne_params* p);

// Launchers (return hipSuccess or the first HIP error).
// Checks row_ptr (err |= row bit) and selects, in ascending order, the rows
// of degree above `threshold` into ids (int32) and/or recs (row, first,
// end, 0), at most cap of them.  counters[0] = rows with entries,
// counters[1] = selected rows.  partial: int2[row_check_blocks(n)] scratch.
int64_t row_check_blocks(int32_t n);
hipError_t launch_check_rows(const int32_t* row_ptr, int32_t n, int64_t nnz, int32_t threshold, uint32_t* err,
                             int32_t* counters, int2* partial, int32_t* ids, int4* recs, int32_t cap,
                             hipStream_t s);
// Fills row_of (the row of every entry) and checks columns and symmetry
// (err |= column bits); mirror[e] = position of the reverse entry.
hipError_t launch_mirror(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz, int32_t* mirror,
                         int32_t* row_of, uint32_t* err, hipStream_t s);
hipError_t launch_sqdist(const int32_t* row_of, const int32_t* col, int64_t nnz, const float* X, int32_t d,
                         double* D, hipStream_t s);
hipError_t launch_calibrate(const int32_t* row_ptr, int32_t n, const int32_t* heavy, int32_t n_heavy, const double* D,
                            double perplexity, double* pcond, double* beta, hipStream_t s);
hipError_t launch_symmetrise(const int32_t* mirror, int64_t nnz, const double* pcond, double S, float* P,
                             hipStream_t s);

hipError_t launch_repulsion(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s);
// Z partials only (the repulsion's tiles without forces): bitwise the Z the
// force pass gives at the same Y and plan; partial forces untouched.
hipError_t launch_zonly(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s);
// tstep (nullable): advance a run's device step counter (see Workspace::tstep).
hipError_t launch_zsum(const Workspace& ws, int precision, hipStream_t s, int32_t* tstep = nullptr);
hipError_t launch_attract(const tsgne_graph* g, const float2* Y, int precision, double2* out, hipStream_t s);
hipError_t launch_update(const tsgne_graph* g, float2* Y, float2* U, float2* gains, float alpha, float momentum,
                         float eta, float min_gain, int precision, bool do_update, float2* grad_out, double* Z_out,
                         hipStream_t s, const StepSchedule& sched = StepSchedule{});
// KL at Y with the Z in the workspace into klout; inside a run (tstep set)
// only on sampled steps, also into trace (see k_kl_final); with tstep null and
// trace set, also into trace[0].
hipError_t launch_kl(const tsgne_graph* g, const float2* Y, hipStream_t s, const int32_t* tstep = nullptr,
                     int32_t kl_every = 0, double* trace = nullptr);
// KL of g's P at Y with the Z, partials and output of a given workspace view
// (ws.Z, ws.klpart[ws.kl_blocks], ws.klout).
hipError_t launch_kl_ws(const tsgne_graph* g, const Workspace& ws, const float2* Y, hipStream_t s);
hipError_t launch_nonfinite_check(const float2* Y, int32_t n, uint32_t* flag, hipStream_t s);
hipError_t launch_batch_step(const BatchPlan& bp, const tsgne_params& p, hipStream_t s);

// Rows per lane for which the repulsion kernels are compiled.
inline bool tile_rows_supported(int32_t R) {
  return R == 1 || R == 2 || R == 4 || R == 8 || R == 12 || R == 14 || R == 15 || R == 16;
}

// Repulsion plan for n positions (R = 0 picks automatically).
RepulsionPlan make_plan(int32_t n, int32_t R, int32_t variant);

}  // namespace tsgne
