// The t-SGNE neighbourhood graph G_knn,G (section 2.2, eq. (7)): nodes i and
// j are joined when one is among the first k nearest neighbours of the other
// on G, nearest by breadth-first search.  The first k neighbours of i are the
// k smallest nodes j != i under (hop distance from i, node id).
//
// One wave per source node.  Each BFS level is enumerated in ascending id
// order by a wave-wide k-way merge of the frontier's adjacency rows (CSR rows
// are sorted): every lane owns up to kPerLane frontier rows with a cursor, the
// wave takes the minimum head, advances every cursor holding it (duplicates),
// and keeps it if it is not yet visited.  The visited set and the frontier are
// striped over the lanes' registers (membership is one ballot), so nothing is
// shared through memory inside a wave.  The directed lists are then made
// symmetric and canonical with a radix sort and a unique pass.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>

#include <algorithm>
#include <climits>
#include <vector>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPerLane = 4;                 // frontier rows per lane
constexpr int kMaxK = kWave * kPerLane;     // 256
constexpr int kVisPerLane = kPerLane + 1;   // visited: k + 1 entries

__device__ __forceinline__ int32_t wave_min(int32_t v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}

__global__ __launch_bounds__(kBlock) void k_knn_bfs(const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, int32_t n, int32_t k,
                                                    int32_t* __restrict__ out, int32_t* __restrict__ out_count) {
  const int32_t i = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  if (i >= n) return;
  const int lane = threadIdx.x & (kWave - 1);
  int32_t vis[kVisPerLane];  // visited node at index lane + 64 u
  int32_t fcur[kPerLane], fend[kPerLane], fhead[kPerLane];
  int32_t nfront[kPerLane];  // the level being taken (next frontier)
#pragma unroll
  for (int u = 0; u < kVisPerLane; ++u) vis[u] = -1;
  if (lane == 0) vis[0] = i;
  int32_t n_vis = 1;
  // frontier = {i}, owned by lane 0
#pragma unroll
  for (int u = 0; u < kPerLane; ++u) {
    fcur[u] = 0;
    fend[u] = 0;
    fhead[u] = INT_MAX;
  }
  if (lane == 0) {
    fcur[0] = row_ptr[i];
    fend[0] = row_ptr[i + 1];
    fhead[0] = fcur[0] < fend[0] ? col[fcur[0]] : INT_MAX;
  }
  int32_t found = 0;
  while (found < k) {
    int32_t taken = 0;
    for (;;) {
      int32_t h = INT_MAX;
#pragma unroll
      for (int u = 0; u < kPerLane; ++u) h = min(h, fhead[u]);
      const int32_t m = wave_min(h);
      if (m == INT_MAX) break;  // level exhausted
#pragma unroll
      for (int u = 0; u < kPerLane; ++u) {
        if (fhead[u] == m) {
          ++fcur[u];
          fhead[u] = fcur[u] < fend[u] ? col[fcur[u]] : INT_MAX;
        }
      }
      bool mine = false;
#pragma unroll
      for (int u = 0; u < kVisPerLane; ++u) mine |= (vis[u] == m);
      if (__ballot(mine) != 0) continue;  // visited (an earlier level or the source)
      // take m: output, visited, next frontier (striped by index)
      if (lane == 0) out[(int64_t)i * k + found] = m;
#pragma unroll
      for (int u = 0; u < kVisPerLane; ++u)
        if (n_vis == u * kWave + lane) vis[u] = m;
#pragma unroll
      for (int u = 0; u < kPerLane; ++u)
        if (taken == u * kWave + lane) nfront[u] = m;
      ++n_vis;
      ++taken;
      ++found;
      if (found == k) break;
    }
    if (taken == 0 || found == k) break;  // component exhausted, or done
    // the level just taken becomes the frontier
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      if (u * kWave + lane < taken) {
        const int32_t v = nfront[u];
        fcur[u] = row_ptr[v];
        fend[u] = row_ptr[v + 1];
        fhead[u] = fcur[u] < fend[u] ? col[fcur[u]] : INT_MAX;
      } else {
        fcur[u] = fend[u] = 0;
        fhead[u] = INT_MAX;
      }
    }
  }
  if (lane == 0) out_count[i] = found;
}

// Both directions of every chosen pair as (row << 32 | col); empty slots get
// the largest key, which sorts last.
__global__ __launch_bounds__(kBlock) void k_knn_keys(const int32_t* __restrict__ out,
                                                     const int32_t* __restrict__ count, int32_t n, int32_t k,
                                                     uint64_t* __restrict__ keys) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= (int64_t)n * k) return;
  const int32_t i = (int32_t)(s / k), t = (int32_t)(s - (int64_t)i * k);
  uint64_t a = ~0ull, b = ~0ull;
  if (t < count[i]) {
    const uint64_t j = (uint32_t)out[s];
    a = ((uint64_t)(uint32_t)i << 32) | j;
    b = (j << 32) | (uint32_t)i;
  }
  keys[2 * s] = a;
  keys[2 * s + 1] = b;
}

__global__ __launch_bounds__(kBlock) void k_knn_csr(const uint64_t* __restrict__ keys, int64_t nnz, int32_t n,
                                                    int32_t* __restrict__ row_ptr, int32_t* __restrict__ col) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < nnz) col[t] = (int32_t)(keys[t] & 0xffffffffull);
  if (t <= n) {
    // first entry whose row is >= t
    int64_t lo = 0, hi = nnz;
    const uint64_t target = (uint64_t)t << 32;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    row_ptr[t] = (int32_t)lo;
  }
}

unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

}  // namespace

size_t validate_csr_bytes(int32_t n, int64_t nnz) {
  return sizeof(int32_t) * (4 + 2 * (size_t)row_check_blocks(n) + 2 * (size_t)nnz);
}

tsgne_status validate_csr(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, hipStream_t s) {
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, validate_csr_bytes(n, nnz), s), "allocate CSR check buffers");
  return validate_csr_in(n, nnz, row_ptr, col, tmp.p, s);
}

// Checks that (row_ptr, col) is a canonical symmetric CSR, in scratch of
// validate_csr_bytes(n, nnz): error word, counters, per-block row counts,
// mirror, row index.
tsgne_status validate_csr_in(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, void* scratch,
                             hipStream_t s, int32_t** row_of_out) {
  const int64_t blocks = row_check_blocks(n);
  int32_t* const buf = static_cast<int32_t*>(scratch);
  uint32_t* const err = reinterpret_cast<uint32_t*>(buf);
  int32_t* const counters = buf + 1;
  int2* const partial = reinterpret_cast<int2*>(buf + 4);
  int32_t* const mirror = buf + 4 + 2 * blocks;
  int32_t* const row_of = mirror + nnz;
  TSGNE_HIP(hipMemsetAsync(buf, 0, 4 * sizeof(int32_t), s), "clear error word and counters");
  TSGNE_HIP(launch_check_rows(row_ptr, n, nnz, INT32_MAX, err, counters, partial, nullptr, nullptr, 0, s),
            "launch row check");
  // the column checks skip themselves when the row check failed
  TSGNE_HIP(launch_mirror(row_ptr, col, n, nnz, mirror, row_of, err, s), "launch CSR check");
  uint32_t host_err = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise CSR check");
  if (host_err & kErrRowPtr) return fail(TSGNE_E_GRAPH, "row_ptr is not nondecreasing from 0 to nnz");
  if (host_err) return fail(TSGNE_E_GRAPH, "CSR is not canonical and symmetric");
  if (row_of_out) *row_of_out = row_of;
  return TSGNE_OK;
}

}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_knn_graph(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d, int32_t k,
                             int32_t* knn_row_ptr_d, int32_t* knn_col_d, int64_t knn_capacity, int64_t* knn_nnz,
                             void* stream) {
  if (!knn_nnz) return fail(TSGNE_E_INVAL, "knn_nnz is NULL");
  *knn_nnz = 0;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (k < 1 || k > kMaxK) return fail(TSGNE_E_INVAL, "k must lie in [1, 256]");
  if (!row_ptr_d || (nnz > 0 && !col_d) || !knn_row_ptr_d || (knn_capacity > 0 && !knn_col_d))
    return fail(TSGNE_E_INVAL, "null pointer");
  if ((int64_t)n * k * 2 >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "n * k too large");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (tsgne_status st = validate_csr(n, nnz, row_ptr_d, col_d, s)) return st;

  const int64_t slots = (int64_t)n * k;
  int32_t* out = nullptr;
  int32_t* count = nullptr;
  uint64_t* keys = nullptr;
  uint64_t* sorted = nullptr;
  int64_t* n_unique = nullptr;
  void* temp = nullptr;
  struct Tmp {
    int32_t*& o;
    int32_t*& c;
    uint64_t*& k1;
    uint64_t*& k2;
    int64_t*& u;
    void*& t;
    ~Tmp() {
      dfree(o);
      dfree(c);
      dfree(k1);
      dfree(k2);
      dfree(u);
      if (t) (void)hipFree(t);
    }
  } tmp{out, count, keys, sorted, n_unique, temp};
  TSGNE_HIP(dalloc(&out, (size_t)slots), "allocate neighbour lists");
  TSGNE_HIP(dalloc(&count, (size_t)n), "allocate counts");
  TSGNE_HIP(dalloc(&keys, 2 * (size_t)slots), "allocate keys");
  TSGNE_HIP(dalloc(&sorted, 2 * (size_t)slots), "allocate keys");
  TSGNE_HIP(dalloc(&n_unique, 1), "allocate count");

  hipLaunchKernelGGL(k_knn_bfs, dim3((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock)), dim3(kBlock), 0, s,
                     row_ptr_d, col_d, n, k, out, count);
  TSGNE_HIP(hipGetLastError(), "launch BFS");
  hipLaunchKernelGGL(k_knn_keys, dim3(blocks_for(slots)), dim3(kBlock), 0, s, out, count, n, k, keys);
  TSGNE_HIP(hipGetLastError(), "launch key build");
  // keys below 2^(32 + bits(n)) except the sentinel; sort all 64 bits
  size_t sort_bytes = 0, uniq_bytes = 0;
  const int n_keys = (int)(2 * slots);
  TSGNE_HIP(rocprim::radix_sort_keys(nullptr, sort_bytes, keys, sorted, n_keys, 0, 64, s), "size sort");
  TSGNE_HIP(rocprim::unique(nullptr, uniq_bytes, sorted, keys, n_unique, (size_t)n_keys, rocprim::equal_to<uint64_t>(), s), "size unique");
  TSGNE_HIP(hipMalloc(&temp, std::max<size_t>(std::max(sort_bytes, uniq_bytes), 1)), "allocate sort scratch");
  TSGNE_HIP(rocprim::radix_sort_keys(temp, sort_bytes, keys, sorted, n_keys, 0, 64, s), "sort keys");
  TSGNE_HIP(rocprim::unique(temp, uniq_bytes, sorted, keys, n_unique, (size_t)n_keys, rocprim::equal_to<uint64_t>(), s), "unique keys");
  int64_t host_unique = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_unique, n_unique, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read count");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise unique");
  uint64_t last = 0;
  if (host_unique > 0)
    TSGNE_HIP(hipMemcpy(&last, keys + host_unique - 1, sizeof(uint64_t), hipMemcpyDeviceToHost), "read last key");
  const int64_t total = host_unique - ((host_unique > 0 && last == ~0ull) ? 1 : 0);
  *knn_nnz = total;
  if (total > knn_capacity) return fail(TSGNE_E_INVAL, "knn_col capacity is smaller than the result (see *knn_nnz)");
  hipLaunchKernelGGL(k_knn_csr, dim3(blocks_for(std::max<int64_t>(total, (int64_t)n + 1))), dim3(kBlock), 0, s, keys,
                     total, n, knn_row_ptr_d, knn_col_d);
  TSGNE_HIP(hipGetLastError(), "launch CSR build");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise kNN graph");
  return TSGNE_OK;
}

}  // extern "C"
