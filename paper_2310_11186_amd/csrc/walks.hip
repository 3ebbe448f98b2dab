// P from random walks (section 2.1): each node starts `walks` walks of
// `length` steps on the graph; a step from u goes to the neighbour v with
// probability proportional to exp(-||x_u - x_v||^2); p_{j|i} is the fraction
// of i's walks that end at j != i, and symmetrising as in eq. (3) (the total
// mass as normaliser) gives P_ij = (c_ij + c_ji) / (2 M) on the support of
// the walks, M the walks that do not end where they started.
//
// The random numbers are Philox4x32-10 (Salmon et al., SC 2011) for counter
// (node, walk, step, 0) and the 64-bit seed as key, so every walk is a pure
// function of its indices.  One thread per walk; the next node is found by
// binary search in the row's running transition weights, which are summed
// per row in CSR order in FP64 (distances without contraction, in coordinate
// order).  The endpoints become 64-bit keys i*n + j and j*n + i; a radix
// sort over the bits those need and a run-length encoding give the canonical
// symmetric CSR and the counts.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_run_length_encode.hpp>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// 53 uniform bits in [0, 1) for step s of walk w from node i.
__device__ __forceinline__ double walk_uniform(uint64_t seed, int32_t i, int32_t w, int32_t s) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)w, (uint32_t)s, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((double)c[0] * 2097152.0 + (double)(c[1] >> 11)) * 0x1p-53;  // exact
}

// D_e = ||x_u - x_v||^2 in FP64, one thread per entry, the coordinates
// summed in order without contraction (float4 loads when d is a multiple of
// 4, several in flight).
template <bool VEC4>
__global__ __launch_bounds__(kBlock) void k_walk_dist(const int32_t* __restrict__ row_of,
                                                      const int32_t* __restrict__ col, int64_t nnz,
                                                      const float* __restrict__ X, int32_t d,
                                                      double* __restrict__ D) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  const float* xu = X + (int64_t)row_of[e] * d;
  const float* xv = X + (int64_t)col[e] * d;
  double acc = 0;
  if constexpr (VEC4) {
#pragma unroll 8
    for (int32_t k = 0; k < d; k += 4) {
#pragma clang fp contract(off)
      const float4 p = *reinterpret_cast<const float4*>(xu + k);
      const float4 q = *reinterpret_cast<const float4*>(xv + k);
      const double t0 = (double)p.x - (double)q.x, t1 = (double)p.y - (double)q.y;
      const double t2 = (double)p.z - (double)q.z, t3 = (double)p.w - (double)q.w;
      acc = acc + t0 * t0;
      acc = acc + t1 * t1;
      acc = acc + t2 * t2;
      acc = acc + t3 * t3;
    }
  } else {
    for (int32_t k = 0; k < d; ++k) {
#pragma clang fp contract(off)
      const double t = (double)xu[k] - (double)xv[k];
      acc = acc + t * t;
    }
  }
  D[e] = acc;
}

// Running transition weights, one wave per row u, in CSR order:
// C_e = sum over the row's entries up to e of exp(-(D - D_min)), in place
// over D.  Lanes take 64 entries at a time; the running sum is carried
// through the lanes one by one, so it is the sequential sum.
__global__ __launch_bounds__(kBlock) void k_walk_weights(const int32_t* __restrict__ row_ptr, int32_t n,
                                                         double* __restrict__ C) {
  const int32_t u = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (u >= n) return;  // whole wave
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t a = row_ptr[u], b = row_ptr[u + 1];
  double dmin = INFINITY;
  for (int32_t e = a + lane; e < b; e += kWave) dmin = fmin(dmin, C[e]);
  for (int off = kWave / 2; off > 0; off >>= 1) dmin = fmin(dmin, __shfl_xor(dmin, off, kWave));
  double run = 0;  // the same in every lane
  for (int32_t c0 = a; c0 < b; c0 += kWave) {
    const int32_t e = c0 + lane;
    const double w = e < b ? exp(-(C[e] - dmin)) : 0.0;
    const int cnt = min(kWave, b - c0);
    double mine = 0;
    for (int j = 0; j < cnt; ++j) {
      run = run + __shfl(w, j, kWave);
      if (lane == j) mine = run;
    }
    if (e < b) C[e] = mine;
  }
}

// One thread per walk: its endpoint as the keys i*n + j and j*n + i, or two
// n*n (after every pair) when it ends at its start.
__global__ __launch_bounds__(kBlock) void k_walks(const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ C,
                                                  int32_t n, int32_t walks, int32_t length, uint64_t seed,
                                                  uint64_t* __restrict__ keys) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)n * walks) return;
  const int32_t i = (int32_t)(t / walks), w = (int32_t)(t % walks);
  int32_t u = i;
  for (int32_t s = 0; s < length; ++s) {
    const int32_t a = row_ptr[u], b = row_ptr[u + 1];
    if (a == b) break;
    const double r = walk_uniform(seed, i, w, s) * C[b - 1];
    int32_t lo = a, hi = b - 1;  // first entry with C > r, else the last
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (C[mid] > r) hi = mid;
      else lo = mid + 1;
    }
    u = col[lo];
  }
  uint64_t k0 = (uint64_t)n * n, k1 = k0;
  if (u != i) {
    k0 = (uint64_t)i * n + u;
    k1 = (uint64_t)u * n + i;
  }
  keys[2 * t] = k0;
  keys[2 * t + 1] = k1;
}

// CSR and P from the distinct sorted keys (i*n + j) and their counts; total
// keys of non-returning walks = 2 M.
__global__ __launch_bounds__(kBlock) void k_walk_csr(const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ counts, int64_t total, int32_t n,
                                                     double two_m, int32_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ col, float* __restrict__ P) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < total) {
    col[t] = (int32_t)(keys[t] % (uint64_t)n);
    P[t] = (float)((double)counts[t] / two_m);
  }
  if (t <= n) {  // row_ptr[t] = first key with row >= t
    int64_t lo = 0, hi = total;
    const uint64_t target = (uint64_t)t * n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (keys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[t] = (int32_t)lo;
  }
}

unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_build_P_walks(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                 const float* X_d, int32_t d, int32_t walks, int32_t length, uint64_t seed,
                                 void* stream, tsgne_graph** out) {
  if (!out) return fail(TSGNE_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (d < 1) return fail(TSGNE_E_INVAL, "d must be >= 1");
  if (walks < 1 || length < 1 || length > 4096) return fail(TSGNE_E_INVAL, "need walks >= 1 and 1 <= length <= 4096");
  if (2 * (int64_t)n * walks >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "2 * n * walks must be below 2^31");
  if (!row_ptr_d || !X_d || (nnz > 0 && !col_d)) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  const int64_t n_keys = 2 * (int64_t)n * walks;
  const uint64_t no_key = (uint64_t)n * n;  // a walk that ended where it started
  int end_bit = 1;
  while (end_bit < 64 && (no_key >> end_bit) != 0) ++end_bit;  // keys are at most n*n
  size_t sort_bytes = 0, rle_bytes = 0;
  TSGNE_HIP(rocprim::radix_sort_keys(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (int)n_keys, 0,
                                    end_bit, s),
            "size sort");
  TSGNE_HIP(rocprim::run_length_encode(nullptr, rle_bytes, (uint64_t*)nullptr, (unsigned int)n_keys, (uint64_t*)nullptr,
                                      (int32_t*)nullptr, (int64_t*)nullptr, s),
            "size run-length encoding");
  // one allocation: CSR check | C | keys | sorted keys | run keys | run counts
  //                 | run count | new row_ptr | new col | new P | sort scratch
  size_t o = 0;
  const size_t o_chk = o;
  o = align256(o + validate_csr_bytes(n, nnz));
  const size_t o_C = o;
  o = align256(o + sizeof(double) * (size_t)std::max<int64_t>(nnz, 1));
  const size_t o_keys = o;
  o = align256(o + sizeof(uint64_t) * (size_t)n_keys);
  const size_t o_sorted = o;
  o = align256(o + sizeof(uint64_t) * (size_t)n_keys);
  const size_t o_runs = o;
  o = align256(o + sizeof(uint64_t) * (size_t)n_keys);
  const size_t o_cnt = o;
  o = align256(o + sizeof(int32_t) * (size_t)n_keys);
  const size_t o_nruns = o;
  o = align256(o + sizeof(int64_t));
  const size_t o_rp = o;
  o = align256(o + sizeof(int32_t) * ((size_t)n + 1));
  const size_t o_col = o;
  o = align256(o + sizeof(int32_t) * (size_t)n_keys);
  const size_t o_P = o;
  o = align256(o + sizeof(float) * (size_t)n_keys);
  const size_t o_tmp = o;
  o = align256(o + std::max<size_t>(std::max(sort_bytes, rle_bytes), 1));
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate walk buffers");
  char* const base = static_cast<char*>(tmp.p);
  int32_t* row_of = nullptr;
  if (tsgne_status st = validate_csr_in(n, nnz, row_ptr_d, col_d, base + o_chk, s, &row_of)) return st;

  double* const C = reinterpret_cast<double*>(base + o_C);
  uint64_t* const keys = reinterpret_cast<uint64_t*>(base + o_keys);
  uint64_t* const sorted = reinterpret_cast<uint64_t*>(base + o_sorted);
  uint64_t* const runs = reinterpret_cast<uint64_t*>(base + o_runs);
  int32_t* const counts = reinterpret_cast<int32_t*>(base + o_cnt);
  int64_t* const n_runs = reinterpret_cast<int64_t*>(base + o_nruns);
  int32_t* const new_rp = reinterpret_cast<int32_t*>(base + o_rp);
  int32_t* const new_col = reinterpret_cast<int32_t*>(base + o_col);
  float* const new_P = reinterpret_cast<float*>(base + o_P);
  void* const sort_tmp = base + o_tmp;

  if (nnz > 0) {
    if (d % 4 == 0)
      hipLaunchKernelGGL(k_walk_dist<true>, dim3(blocks_for(nnz)), dim3(kBlock), 0, s, row_of, col_d, nnz, X_d, d, C);
    else
      hipLaunchKernelGGL(k_walk_dist<false>, dim3(blocks_for(nnz)), dim3(kBlock), 0, s, row_of, col_d, nnz, X_d, d, C);
    hipLaunchKernelGGL(k_walk_weights, dim3((unsigned)(((int64_t)n + kWavesPerBlock - 1) / kWavesPerBlock)),
                       dim3(kBlock), 0, s, row_ptr_d, n, C);
  }
  hipLaunchKernelGGL(k_walks, dim3(blocks_for((int64_t)n * walks)), dim3(kBlock), 0, s, row_ptr_d, col_d, C, n, walks,
                     length, seed, keys);
  TSGNE_HIP(hipGetLastError(), "launch walks");
  size_t bytes = sort_bytes;
  TSGNE_HIP(rocprim::radix_sort_keys(sort_tmp, bytes, keys, sorted, (int)n_keys, 0, end_bit, s),
            "sort endpoints");
  bytes = rle_bytes;
  TSGNE_HIP(rocprim::run_length_encode(sort_tmp, bytes, sorted, (unsigned int)n_keys, runs, counts, n_runs, s),
            "count endpoints");
  int64_t host_runs = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_runs, n_runs, sizeof(int64_t), hipMemcpyDeviceToHost, s), "read run count");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise endpoint count");
  uint64_t last_key = 0;
  int32_t last_count = 0;
  if (host_runs > 0) {
    TSGNE_HIP(hipMemcpy(&last_key, runs + host_runs - 1, sizeof(uint64_t), hipMemcpyDeviceToHost), "read last key");
    TSGNE_HIP(hipMemcpy(&last_count, counts + host_runs - 1, sizeof(int32_t), hipMemcpyDeviceToHost),
              "read last count");
  }
  const bool has_returns = host_runs > 0 && last_key == no_key;
  const int64_t total = host_runs - (has_returns ? 1 : 0);
  const int64_t two_m = n_keys - (has_returns ? last_count : 0);
  hipLaunchKernelGGL(k_walk_csr, dim3(blocks_for(std::max<int64_t>(total, (int64_t)n + 1))), dim3(kBlock), 0, s, runs,
                     counts, total, n, (double)std::max<int64_t>(two_m, 1), new_rp, new_col, new_P);
  TSGNE_HIP(hipGetLastError(), "launch CSR build");

  tsgne_graph* g = nullptr;
  if (tsgne_status st = graph_structure(n, total, new_rp, new_col, s, &g)) return st;
  struct Cleanup {
    tsgne_graph* g;
    ~Cleanup() { free_graph(g); }
  } guard{g};
  g->d = d;
  g->perplexity = 0.f;
  if (total > 0)
    TSGNE_HIP(hipMemcpyAsync(g->P, new_P, sizeof(float) * (size_t)total, hipMemcpyDeviceToDevice, s), "copy P");
  TSGNE_HIP(hipMemsetAsync(g->beta, 0, sizeof(double) * (size_t)n, s), "clear beta");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise walk P");
  guard.g = nullptr;
  *out = g;
  return TSGNE_OK;
}

}  // extern "C"
