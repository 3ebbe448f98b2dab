// One GPU's share of a sharded all-pairs repulsion.  The symmetric tiles of
// the block triangle (tile (a, b), a <= b, covers the pairs between row block
// a and row block b) are dealt to shards by pairs of row blocks: row blocks a
// and nb-1-a form pair p = min(a, nb-1-a), which together hold nb+1 tiles,
// and pair p goes to shard p mod n_shards.  A shard runs the same tile kernels
// as the single-GPU step on its own tile list, then sums, for every row, the
// partials its tiles left for that row (as row block and as column block) in
// FP64.  Summed over the shards, the force sums and the Z partials are the
// full repulsive term and Z of eq. (4).  In a multi-GPU run each GPU holds a
// replica of Y, calls this for its shard, and the force sums are reduced
// across GPUs (a reduce-scatter of 16 bytes per node, an all-reduce of one
// double for Z).
#include <algorithm>
#include <utility>
#include <vector>

#include "internal.h"

using namespace tsgne;

struct tsgne_shard {
  int device = 0;
  int32_t n = 0;
  int32_t shard = 0;
  int32_t n_shards = 1;
  int64_t pairs = 0;  // ordered pairs (i, j), i != j, of this shard's tiles
  Workspace ws;       // plan, tile list, partial buffers (ws.Z unused)
  // the shard's row blocks in ascending order, and for every row block k the
  // number of them below k (nb + 1 counts), for the per-row sums
  int32_t* owned = nullptr;
  int32_t* below = nullptr;
  int32_t n_owned = 0;
  // event-pair timing of the tile kernel (tsgne_shard_set_timing)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double tile_ms = 0.0;
  int64_t tile_launches = 0;
};

namespace {

constexpr int kReduceBlock = 256;

__device__ __forceinline__ int32_t block_owner(int32_t a, int32_t nb, int32_t n_shards) {
  return min(a, nb - 1 - a) % n_shards;
}

// F_i = sum over the shard's tiles touching row i of their partial for i.
// The partials of row block k that this shard wrote are those of its own row
// blocks below k (tiles (o, k)) and, if it owns k, those of every block from k
// on (tiles (k, o)): a list of blocks in ascending order.  A workgroup takes
// 64 rows of one row block; its kReduceWaves waves split that list into
// contiguous quarters, each summing its quarter in block order, and the
// quarters are added in order (FP64 in split mode, FP32 stored as FP64
// otherwise), so the result is deterministic.  The loads of a batch carry no
// guard (a guarded load sits behind its own branch and is waited for before
// the next one is issued): past the quarter's end a list index is clamped to
// its last entry, an in-bounds re-read that adds +0.  Rows past n read the
// partial buffer inside their own row block and store nothing.
constexpr int kReduceWaves = 4;

template <bool SPLIT>
__global__ __launch_bounds__(kReduceBlock) void k_shard_reduce(const float2* __restrict__ part, int32_t nb, int32_t T,
                                                              int32_t n, int32_t shard, int32_t n_shards,
                                                              const int32_t* __restrict__ owned,
                                                              const int32_t* __restrict__ below, int32_t n_owned,
                                                              double2* __restrict__ F) {
  __shared__ double2 acc[kReduceWaves][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int32_t row0 = blockIdx.x * kWave;  // T is a multiple of 64: one row block per workgroup
  const int32_t k = row0 / T;
  const int32_t i = row0 + lane;
  const float2* __restrict__ pp = part + (int64_t)k * nb * T + (i - k * T);
  const int32_t b_k = below[k];
  const int32_t m = b_k + (block_owner(k, nb, n_shards) == shard ? nb - k : 0);
  const int32_t q = (m + kReduceWaves - 1) / kReduceWaves;
  const int32_t t_begin = w * q, t_end = min(m, t_begin + q);
  double rx = 0.0, ry = 0.0;
  float sx = 0.f, sy = 0.f;
  constexpr int kBatchLoads = 16;
  for (int32_t t0 = t_begin; t0 < t_end; t0 += kBatchLoads) {
    float2 v[kBatchLoads];
#pragma unroll
    for (int u = 0; u < kBatchLoads; ++u) {
      const int32_t t = min(t0 + u, t_end - 1);
      const int32_t o = t < b_k ? owned[min(t, n_owned - 1)] : k + (t - b_k);
      v[u] = pp[(int64_t)o * T];
    }
    const int32_t count = t_end - t0;
#pragma unroll
    for (int u = 0; u < kBatchLoads; ++u) {
      const bool in = u < count;
      if (SPLIT) {
        rx += in ? (double)v[u].x : 0.0;
        ry += in ? (double)v[u].y : 0.0;
      } else {
        sx += in ? v[u].x : 0.f;
        sy += in ? v[u].y : 0.f;
      }
    }
  }
  acc[w][lane] = SPLIT ? make_double2(rx, ry) : make_double2((double)sx, (double)sy);
  __syncthreads();
  if (w != 0 || i >= n) return;
  if (SPLIT) {
    double2 t = acc[0][lane];
    for (int u = 1; u < kReduceWaves; ++u) {
      t.x += acc[u][lane].x;
      t.y += acc[u][lane].y;
    }
    F[i] = t;
  } else {
    float tx = (float)acc[0][lane].x, ty = (float)acc[0][lane].y;
    for (int u = 1; u < kReduceWaves; ++u) {
      tx += (float)acc[u][lane].x;
      ty += (float)acc[u][lane].y;
    }
    F[i] = make_double2((double)tx, (double)ty);
  }
}

// A shard with no tile: nothing acts on any row.  (A kernel rather than a
// memset, so that the call can be captured in a graph.)
__global__ __launch_bounds__(kReduceBlock) void k_shard_zero(int32_t n, double2* __restrict__ F, double* __restrict__ Z) {
  const int32_t i = blockIdx.x * kReduceBlock + threadIdx.x;
  if (i < n) F[i] = make_double2(0.0, 0.0);
  if (i == 0) *Z = 0.0;
}

int32_t owner_host(int32_t a, int32_t nb, int32_t n_shards) { return std::min(a, nb - 1 - a) % n_shards; }

// Tiles of the shard for tile rows R, a ascending then b ascending.
std::vector<int2> shard_tiles(int32_t n, int32_t R, int32_t shard, int32_t n_shards, int64_t* pairs) {
  const int64_t T = (int64_t)kWave * R;
  const int32_t nb = (int32_t)((n + T - 1) / T);
  std::vector<int2> items;
  int64_t pr = 0;
  for (int32_t a = 0; a < nb; ++a) {
    if (owner_host(a, nb, n_shards) != shard) continue;
    const int64_t va = std::min<int64_t>(T, (int64_t)n - a * T);
    for (int32_t b = a; b < nb; ++b) {
      items.push_back(make_int2(a, b));
      const int64_t vb = std::min<int64_t>(T, (int64_t)n - b * T);
      pr += a == b ? va * (va - 1) : 2 * va * vb;
    }
  }
  *pairs = pr;
  return items;
}

// Tile rows for a shard: the single-graph cost model applied to the largest
// shard's tile count (its tiles over the chip's 1024 SIMDs rounded up, at
// least the 64 / R a SIMD needs to hide latency, times the tile area, over
// the tile's per-pair efficiency relative to R = 16, the values the
// single-graph plan uses: measured on MI355X at 200K-500K nodes).
int32_t shard_tile_rows(int32_t n, int32_t n_shards) {
  const int32_t rs[6] = {16, 15, 14, 12, 8, 4};
  const double eff[6] = {1.0, 1.004, 0.996, 0.997, 0.969, 0.827};
  constexpr int64_t kSimds = 1024;
  double best = 0.0;
  int32_t R = 8;
  for (int k = 0; k < 6; ++k) {
    const int64_t T = (int64_t)kWave * rs[k], nb = (n + T - 1) / T;
    // a pair of row blocks holds nb + 1 tiles; the largest shard has the most pairs
    const int64_t pairs = (nb + 1) / 2;
    const int64_t per_shard = (pairs + n_shards - 1) / n_shards * (nb + 1);
    const int64_t per_simd = std::max<int64_t>((per_shard + kSimds - 1) / kSimds, kWave / rs[k]);
    const double cost = (double)per_simd * (double)(T * T) / eff[k];
    if (best == 0.0 || cost < best) {
      best = cost;
      R = rs[k];
    }
  }
  return R;
}

// Adds the elapsed time of every recorded event pair (waiting for each).
hipError_t resolve_timing(tsgne_shard* sh) {
  hipError_t first = hipSuccess;
  for (auto& pr : sh->pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e == hipSuccess) {
      sh->tile_ms += ms;
      sh->tile_launches += 1;
    } else if (first == hipSuccess) {
      first = e;
    }
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  sh->pending.clear();
  return first;
}

void free_shard_buffers(tsgne_shard* sh) {
  dfree(sh->ws.items);
  dfree(sh->ws.part);
  dfree(sh->ws.zpart);
  dfree(sh->ws.zpart32);
  dfree(sh->owned);
  dfree(sh->below);
}

}  // namespace

extern "C" {

tsgne_status tsgne_shard_create(int32_t n, int32_t shard, int32_t n_shards, int32_t tile_rows, tsgne_shard** out) {
  if (!out) return fail(TSGNE_E_INVAL, "null pointer");
  *out = nullptr;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (n_shards < 1 || n_shards > 65536) return fail(TSGNE_E_INVAL, "n_shards must lie in [1, 65536]");
  if (shard < 0 || shard >= n_shards) return fail(TSGNE_E_INVAL, "shard must lie in [0, n_shards)");
  if (tile_rows != 0 && !tile_rows_supported(tile_rows))
    return fail(TSGNE_E_INVAL, "tile_rows must be 0 (chosen for the shard), 1, 2, 4, 8, 12, 14, 15 or 16");
  const int32_t R = tile_rows ? tile_rows : shard_tile_rows(n, n_shards);
  const int64_t T = (int64_t)kWave * R, nb = (n + T - 1) / T;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TSGNE_E_DEVICE, "no HIP device");
  tsgne_shard* sh = new tsgne_shard();
  sh->device = dev;
  sh->n = n;
  sh->shard = shard;
  sh->n_shards = n_shards;
  std::vector<int2> items = shard_tiles(n, R, shard, n_shards, &sh->pairs);
  Workspace& ws = sh->ws;
  ws.plan.R = R;
  ws.plan.T = (int32_t)T;
  ws.plan.nb = (int32_t)nb;
  ws.plan.variant = TSGNE_REPULSION_SYMMETRIC;
  ws.plan.items = (int64_t)items.size();
  std::vector<int32_t> owned, below((size_t)nb + 1, 0);
  for (int32_t a = 0; a < (int32_t)nb; ++a) {
    below[(size_t)a + 1] = below[(size_t)a];
    if (owner_host(a, (int32_t)nb, n_shards) == shard) {
      owned.push_back(a);
      below[(size_t)a + 1] += 1;
    }
  }
  sh->n_owned = (int32_t)owned.size();
  hipError_t e = hipSuccess;
  if (!items.empty()) {
    e = dalloc(&ws.items, items.size());
    if (e == hipSuccess) e = dalloc(&ws.part, (size_t)(nb * nb * T));
    if (e == hipSuccess) e = dalloc(&ws.zpart, items.size());
    if (e == hipSuccess) e = dalloc(&ws.zpart32, items.size());
    if (e == hipSuccess) e = dalloc(&sh->owned, owned.size());
    if (e == hipSuccess) e = dalloc(&sh->below, below.size());
    if (e == hipSuccess) e = hipMemcpy(ws.items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sh->owned, owned.data(), owned.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sh->below, below.data(), below.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    free_shard_buffers(sh);
    delete sh;
    if (e == hipErrorOutOfMemory)
      return fail(TSGNE_E_NOMEM, "shard workspace (partials of nb * nb tiles) does not fit in device memory");
    return hip_fail(e, "allocate shard workspace");
  }
  *out = sh;
  return TSGNE_OK;
}

tsgne_status tsgne_shard_info(const tsgne_shard* sh, int32_t* tile_rows, int64_t* tiles, int64_t* pairs) {
  if (!sh) return fail(TSGNE_E_INVAL, "shard is NULL");
  if (tile_rows) *tile_rows = sh->ws.plan.R;
  if (tiles) *tiles = sh->ws.plan.items;
  if (pairs) *pairs = sh->pairs;
  return TSGNE_OK;
}

tsgne_status tsgne_shard_repulsion(tsgne_shard* sh, const float* Y_d, int32_t precision, double* F_d, double* Z_d,
                                   void* stream) {
  if (!sh) return fail(TSGNE_E_INVAL, "shard is NULL");
  if (!Y_d || !F_d || !Z_d) return fail(TSGNE_E_INVAL, "null pointer");
  if (precision != TSGNE_PREC_SPLIT && precision != TSGNE_PREC_FP32)
    return fail(TSGNE_E_INVAL, "precision must be TSGNE_PREC_SPLIT or TSGNE_PREC_FP32");
  DeviceGuard dg(sh->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool split = precision != TSGNE_PREC_FP32;
  if (sh->ws.plan.items == 0) {
    const dim3 zgrid((unsigned)((sh->n + kReduceBlock - 1) / kReduceBlock));
    hipLaunchKernelGGL(k_shard_zero, zgrid, dim3(kReduceBlock), 0, s, sh->n, reinterpret_cast<double2*>(F_d), Z_d);
    TSGNE_HIP(hipGetLastError(), "launch shard clear");
    return TSGNE_OK;
  }
  Workspace ws = sh->ws;
  ws.Z = Z_d;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (sh->timing) {
    TSGNE_HIP(hipEventCreate(&ev[0]), "create timing event");
    if (hipEventCreate(&ev[1]) != hipSuccess || hipEventRecord(ev[0], s) != hipSuccess) {
      (void)hipEventDestroy(ev[0]);
      if (ev[1]) (void)hipEventDestroy(ev[1]);
      return fail(TSGNE_E_DEVICE, "record timing event");
    }
  }
  const hipError_t le = launch_repulsion(ws, sh->n, reinterpret_cast<const float2*>(Y_d), precision, s);
  if (sh->timing) {
    if (le == hipSuccess && hipEventRecord(ev[1], s) == hipSuccess) {
      sh->pending.emplace_back(ev[0], ev[1]);
    } else {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
    }
  }
  TSGNE_HIP(le, "launch repulsion");
  TSGNE_HIP(launch_zsum(ws, precision, s), "launch Z reduction");
  static_assert(kReduceBlock == kReduceWaves * kWave, "one wave per quarter of the blocks");
  const dim3 grid((unsigned)((sh->n + kWave - 1) / kWave));
  if (split)
    hipLaunchKernelGGL((k_shard_reduce<true>), grid, dim3(kReduceBlock), 0, s, ws.part, ws.plan.nb, ws.plan.T, sh->n,
                       sh->shard, sh->n_shards, sh->owned, sh->below, sh->n_owned, reinterpret_cast<double2*>(F_d));
  else
    hipLaunchKernelGGL((k_shard_reduce<false>), grid, dim3(kReduceBlock), 0, s, ws.part, ws.plan.nb, ws.plan.T, sh->n,
                       sh->shard, sh->n_shards, sh->owned, sh->below, sh->n_owned, reinterpret_cast<double2*>(F_d));
  TSGNE_HIP(hipGetLastError(), "launch shard reduction");
  return TSGNE_OK;
}

tsgne_status tsgne_shard_set_timing(tsgne_shard* sh, int32_t enable) {
  if (!sh) return fail(TSGNE_E_INVAL, "shard is NULL");
  DeviceGuard dg(sh->device);
  const hipError_t e = resolve_timing(sh);
  sh->timing = enable != 0;
  sh->tile_ms = 0.0;
  sh->tile_launches = 0;
  TSGNE_HIP(e, "resolve timing events");
  return TSGNE_OK;
}

tsgne_status tsgne_shard_timing(tsgne_shard* sh, double* tile_ms, int64_t* launches) {
  if (!sh) return fail(TSGNE_E_INVAL, "shard is NULL");
  DeviceGuard dg(sh->device);
  TSGNE_HIP(resolve_timing(sh), "resolve timing events");
  if (tile_ms) *tile_ms = sh->tile_ms;
  if (launches) *launches = sh->tile_launches;
  return TSGNE_OK;
}

tsgne_status tsgne_shard_free(tsgne_shard* sh) {
  if (!sh) return TSGNE_OK;
  DeviceGuard dg(sh->device);
  // buffers may still be in use by queued work
  (void)hipDeviceSynchronize();
  (void)resolve_timing(sh);
  free_shard_buffers(sh);
  delete sh;
  return TSGNE_OK;
}

}  // extern "C"
