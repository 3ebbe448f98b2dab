// KL of a layout without any device allocation (tsgne_kl_noalloc): the same
// kernels as tsgne_kl, with their scratch (the repulsion's tile list and Z
// partials, the KL partials) in one file-scope device array of fixed size.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace tsgne {

// Bytes of the device array: tile list (8 B) and Z partial (8 B) per tile of
// the repulsion's plan, Z, and up to 1024 KL partials.
constexpr size_t kNoAllocBytes = (size_t)32 << 20;

// Every GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kKLMaxBlocks = 1024;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's array, looked up once per device.  The
// array's name in host code is a host-side stand-in, never a device address.
hipError_t scratch_address(int dev, char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return hipSuccess;
}

constexpr int kFillThreads = 256;

// Tile list of a plan, in the order of the host's list: direct plans row by
// row over the square; symmetric plans the nb diagonal tiles (a, a) first,
// then the tiles (a, a < b < nb - 1) row by row, then the tiles (a, nb - 1).
// Row block a (one workgroup) writes its own tiles.
__global__ __launch_bounds__(kFillThreads) void k_fill_items(int32_t nb, int symmetric, int2* __restrict__ items) {
  const int32_t a = blockIdx.x;
  if (!symmetric) {
    for (int32_t b = (int32_t)threadIdx.x; b < nb; b += kFillThreads) items[(int64_t)a * nb + b] = make_int2(a, b);
    return;
  }
  if (threadIdx.x == 0) {
    items[a] = make_int2(a, a);
    // after the nb diagonal and the (nb - 1)(nb - 2) / 2 inner tiles
    if (a < nb - 1) items[nb + (int64_t)(nb - 1) * (nb - 2) / 2 + a] = make_int2(a, nb - 1);
  }
  // rows before a hold (nb - 2 - 0) + ... + (nb - 2 - (a - 1)) inner tiles
  const int64_t first = nb + (int64_t)a * (nb - 2) - (int64_t)a * (a - 1) / 2;
  for (int32_t b = a + 1 + (int32_t)threadIdx.x; b < nb - 1; b += kFillThreads)
    items[first + (b - a - 1)] = make_int2(a, b);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_kl_noalloc(tsgne_graph* g, const float* Y_d, double* kl_d, void* stream) {
  if (!g) return fail(TSGNE_E_INVAL, "graph is NULL");
  if (!Y_d || !kl_d) return fail(TSGNE_E_INVAL, "null pointer");
  DeviceGuard dg(g->device);
  // the plan the graph's own KL would use: its workspace's, or the automatic one
  const RepulsionPlan plan = g->ws.part ? g->ws.plan : make_plan(g->n, 0, TSGNE_REPULSION_AUTO);
  const int32_t kl_blocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kKLMaxBlocks, (g->nnz + 255) / 256));
  size_t o = 0;
  const size_t o_items = o;
  o = align256(o + sizeof(int2) * (size_t)plan.items);
  const size_t o_zpart = o;
  o = align256(o + sizeof(double) * (size_t)plan.items);
  const size_t o_Z = o;
  o = align256(o + sizeof(double));
  const size_t o_kl = o;
  o = align256(o + sizeof(double) * (size_t)kl_blocks);
  if (o > kNoAllocBytes)
    return fail(TSGNE_E_INVAL, "graph too large for tsgne_kl_noalloc: its " + std::to_string(plan.items) +
                                   " repulsion tiles need " + std::to_string(o) + " bytes of scratch, the maximum is " +
                                   std::to_string(kNoAllocBytes) + " (about 2 million nodes)");
  char* base = nullptr;
  TSGNE_HIP(scratch_address(g->device, &base), "look up the no-allocation scratch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace ws;
  ws.plan = plan;
  ws.items = reinterpret_cast<int2*>(base + o_items);
  ws.zpart = reinterpret_cast<double*>(base + o_zpart);
  ws.Z = reinterpret_cast<double*>(base + o_Z);
  ws.klpart = reinterpret_cast<double*>(base + o_kl);
  ws.klout = kl_d;
  ws.kl_blocks = kl_blocks;
  // every slot read below is written first in this call: nothing to clear
  hipLaunchKernelGGL(k_fill_items, dim3((unsigned)plan.nb), dim3(kFillThreads), 0, s, plan.nb,
                     plan.variant == TSGNE_REPULSION_SYMMETRIC ? 1 : 0, ws.items);
  TSGNE_HIP(hipGetLastError(), "launch tile list");
  const float2* Y2 = reinterpret_cast<const float2*>(Y_d);
  TSGNE_HIP(launch_zonly(ws, g->n, Y2, TSGNE_PREC_SPLIT, s), "launch Z pass");
  TSGNE_HIP(launch_zsum(ws, TSGNE_PREC_SPLIT, s), "launch Z reduction");
  TSGNE_HIP(launch_kl_ws(g, ws, Y2, s), "launch KL");
  return TSGNE_OK;
}

}  // extern "C"
