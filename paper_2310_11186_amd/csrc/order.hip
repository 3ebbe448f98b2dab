// Node renumbering for memory locality.
//
// tsgne_locality_order: a node order along a Morton (Z-order) curve of the
// leading coordinates of the embedding.  By the premise of t-SGNE (section
// 2.2) nodes that are close in the graph are close in R^d, so this order puts
// most graph neighbours at nearby ids, and the position gathers of the
// attraction then stay within a small window of Y.
// tsgne_permute_graph / tsgne_permute_rows apply such an order to a CSR and
// to row-major node arrays (and map results back).
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kFinal = 1024;
constexpr int kMaxCoords = 8;
constexpr uint32_t kErrFinite = 1u, kErrPerm = 2u;

// Per-block min/max of the leading m coordinates.
__global__ __launch_bounds__(kBlock) void k_coord_box(const float* __restrict__ X, int32_t n, int32_t d, int m,
                                                      float2* __restrict__ part, uint32_t* __restrict__ err) {
  __shared__ float2 s[kBlock / kWave][kMaxCoords];
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  for (int c = 0; c < m; ++c) {
    float lo = INFINITY, hi = -INFINITY;
    if (i < n) {
      const float v = X[(int64_t)i * d + c];
      if (!isfinite(v)) atomicOr(err, kErrFinite);
      lo = hi = v;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off, kWave));
      hi = fmaxf(hi, __shfl_xor(hi, off, kWave));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x >> 6][c] = make_float2(lo, hi);
  }
  __syncthreads();
  if (threadIdx.x < m) {
    float2 b = s[0][threadIdx.x];
    for (int w = 1; w < kBlock / kWave; ++w) {
      b.x = fminf(b.x, s[w][threadIdx.x].x);
      b.y = fmaxf(b.y, s[w][threadIdx.x].y);
    }
    part[(int64_t)blockIdx.x * kMaxCoords + threadIdx.x] = b;
  }
}

// box[c] = (lo, hi) of coordinate c as doubles.
__global__ __launch_bounds__(kFinal) void k_coord_box_final(const float2* __restrict__ part, int32_t blocks, int m,
                                                            double2* __restrict__ box) {
  __shared__ float2 s[kFinal / kWave];
  for (int c = 0; c < m; ++c) {
    float lo = INFINITY, hi = -INFINITY;
    for (int32_t b = threadIdx.x; b < blocks; b += kFinal) {
      const float2 p = part[(int64_t)b * kMaxCoords + c];
      lo = fminf(lo, p.x);
      hi = fmaxf(hi, p.y);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off, kWave));
      hi = fmaxf(hi, __shfl_xor(hi, off, kWave));
    }
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x >> 6] = make_float2(lo, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kFinal / kWave; ++w) {
        lo = fminf(lo, s[w].x);
        hi = fmaxf(hi, s[w].y);
      }
      box[c] = make_double2(lo, hi);
    }
  }
}

// Morton key of node i: b bits of each of the m coordinates, quantised over
// their ranges (q = min(floor((x - lo) / (hi - lo) * 2^b), 2^b - 1), 0 on a
// flat axis), interleaved from the top bit down, coordinate 0 first.
__global__ __launch_bounds__(kBlock) void k_morton(const float* __restrict__ X, int32_t n, int32_t d, int m, int b,
                                                   const double2* __restrict__ box, uint64_t* __restrict__ key,
                                                   int32_t* __restrict__ id) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t q[kMaxCoords];
  const double scale = ldexp(1.0, b);
  const uint64_t top = (b == 64) ? ~0ull : ((1ull << b) - 1);
  for (int c = 0; c < m; ++c) {
#pragma clang fp contract(off)
    const double lo = box[c].x, span = box[c].y - box[c].x;
    uint64_t u = 0;
    if (span > 0) {
      const double t = floor(((double)X[(int64_t)i * d + c] - lo) / span * scale);
      u = t >= (double)top ? top : (uint64_t)t;
    }
    q[c] = u;
  }
  uint64_t k = 0;
  for (int t = b - 1; t >= 0; --t)
    for (int c = 0; c < m; ++c) k = (k << 1) | ((q[c] >> t) & 1u);
  key[i] = k;
  id[i] = i;
}

// inv[perm[r]] = r, with a count of how often each id occurs.
__global__ __launch_bounds__(kBlock) void k_invert(const int32_t* __restrict__ perm, int32_t n,
                                                   int32_t* __restrict__ inv, int32_t* __restrict__ seen,
                                                   uint32_t* __restrict__ err) {
  const int32_t r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int32_t v = perm[r];
  if (v < 0 || v >= n) {
    atomicOr(err, kErrPerm);
    return;
  }
  inv[v] = r;
  if (atomicAdd(&seen[v], 1) != 0) atomicOr(err, kErrPerm);  // a repeat (then some id is missing too)
}

// Keys inv[i] * n + inv[j] of every entry (i, j), one thread per row.
__global__ __launch_bounds__(kBlock) void k_relabel_keys(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, int32_t n,
                                                         const int32_t* __restrict__ inv,
                                                         uint64_t* __restrict__ key) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint64_t r = (uint64_t)inv[i] * n;
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) key[e] = r + inv[col[e]];
}

// CSR from sorted keys r * n + c.
__global__ __launch_bounds__(kBlock) void k_keys_csr(const uint64_t* __restrict__ key, int64_t nnz, int32_t n,
                                                     int32_t* __restrict__ row_ptr, int32_t* __restrict__ col) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < nnz) col[t] = (int32_t)(key[t] % (uint64_t)n);
  if (t <= n) {  // first key of row t
    int64_t lo = 0, hi = nnz;
    const uint64_t target = (uint64_t)t * n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (key[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    row_ptr[t] = (int32_t)lo;
  }
}

// dst row r = src row perm[r] (gather), or dst row perm[r] = src row r
// (scatter), rows of `words` 32-bit words.
__global__ __launch_bounds__(kBlock) void k_permute_rows(const uint32_t* __restrict__ src,
                                                         const int32_t* __restrict__ perm, int32_t n, int32_t words,
                                                         int inverse, uint32_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)n * words) return;
  const int32_t r = (int32_t)(t / words), w = (int32_t)(t % words);
  const int32_t p = perm[r];
  if (inverse) dst[(int64_t)p * words + w] = src[t];
  else dst[t] = src[(int64_t)p * words + w];
}

unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_locality_order(int32_t n, const float* X_d, int32_t d, int32_t* perm_d, void* stream) {
  if (n < 1 || d < 1) return fail(TSGNE_E_INVAL, "need n >= 1 and d >= 1");
  if (!X_d || !perm_d) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int m = std::min(d, kMaxCoords);
  const int b = 64 / m;
  const unsigned blocks = blocks_for(n);
  size_t sort_bytes = 0;
  TSGNE_HIP(rocprim::radix_sort_pairs(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                     (int32_t*)nullptr, (int32_t*)nullptr, n, 0, 64, s),
            "size sort");
  size_t o = 0;
  const size_t o_err = o;
  o = align256(o + sizeof(uint32_t));
  const size_t o_part = o;
  o = align256(o + sizeof(float2) * kMaxCoords * blocks);
  const size_t o_box = o;
  o = align256(o + sizeof(double2) * kMaxCoords);
  const size_t o_key = o;
  o = align256(o + sizeof(uint64_t) * (size_t)n);
  const size_t o_key2 = o;
  o = align256(o + sizeof(uint64_t) * (size_t)n);
  const size_t o_id = o;
  o = align256(o + sizeof(int32_t) * (size_t)n);
  const size_t o_tmp = o;
  o = align256(o + std::max<size_t>(sort_bytes, 1));
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate order buffers");
  char* const base = static_cast<char*>(tmp.p);
  uint32_t* const err = reinterpret_cast<uint32_t*>(base + o_err);
  double2* const box = reinterpret_cast<double2*>(base + o_box);
  uint64_t* const key = reinterpret_cast<uint64_t*>(base + o_key);
  uint64_t* const key2 = reinterpret_cast<uint64_t*>(base + o_key2);
  int32_t* const id = reinterpret_cast<int32_t*>(base + o_id);
  TSGNE_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s), "clear error word");
  hipLaunchKernelGGL(k_coord_box, dim3(blocks), dim3(kBlock), 0, s, X_d, n, d, m,
                     reinterpret_cast<float2*>(base + o_part), err);
  hipLaunchKernelGGL(k_coord_box_final, dim3(1), dim3(kFinal), 0, s, reinterpret_cast<float2*>(base + o_part),
                     (int32_t)blocks, m, box);
  hipLaunchKernelGGL(k_morton, dim3(blocks), dim3(kBlock), 0, s, X_d, n, d, m, b, box, key, id);
  TSGNE_HIP(hipGetLastError(), "launch keys");
  size_t bytes = sort_bytes;
  // ids enter in ascending order and the sort is stable: ties stay by id
  TSGNE_HIP(rocprim::radix_sort_pairs(base + o_tmp, bytes, key, key2, id, perm_d, n, 0, 64, s),
            "sort keys");
  uint32_t host_err = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise order");
  if (host_err) return fail(TSGNE_E_NONFINITE, "embedding has a non-finite coordinate");
  return TSGNE_OK;
}

tsgne_status tsgne_permute_graph(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                 const int32_t* perm_d, int32_t* out_row_ptr_d, int32_t* out_col_d, void* stream) {
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (!row_ptr_d || (nnz > 0 && (!col_d || !out_col_d)) || !perm_d || !out_row_ptr_d)
    return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int end_bit = bits_for((uint64_t)n * n);
  size_t sort_bytes = 0;
  TSGNE_HIP(rocprim::radix_sort_keys(nullptr, sort_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                    (int)std::max<int64_t>(nnz, 1), 0, end_bit, s),
            "size sort");
  size_t o = 0;
  const size_t o_chk = o;
  o = align256(o + validate_csr_bytes(n, nnz));
  const size_t o_err = o;
  o = align256(o + sizeof(uint32_t));
  const size_t o_inv = o;
  o = align256(o + sizeof(int32_t) * (size_t)n);
  const size_t o_seen = o;
  o = align256(o + sizeof(int32_t) * (size_t)n);
  const size_t o_key = o;
  o = align256(o + sizeof(uint64_t) * (size_t)std::max<int64_t>(nnz, 1));
  const size_t o_key2 = o;
  o = align256(o + sizeof(uint64_t) * (size_t)std::max<int64_t>(nnz, 1));
  const size_t o_tmp = o;
  o = align256(o + std::max<size_t>(sort_bytes, 1));
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate permutation buffers");
  char* const base = static_cast<char*>(tmp.p);
  if (tsgne_status st = validate_csr_in(n, nnz, row_ptr_d, col_d, base + o_chk, s)) return st;
  uint32_t* const err = reinterpret_cast<uint32_t*>(base + o_err);
  int32_t* const inv = reinterpret_cast<int32_t*>(base + o_inv);
  int32_t* const seen = reinterpret_cast<int32_t*>(base + o_seen);
  uint64_t* const key = reinterpret_cast<uint64_t*>(base + o_key);
  uint64_t* const key2 = reinterpret_cast<uint64_t*>(base + o_key2);
  TSGNE_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s), "clear error word");
  TSGNE_HIP(hipMemsetAsync(seen, 0, sizeof(int32_t) * (size_t)n, s), "clear counts");
  hipLaunchKernelGGL(k_invert, dim3(blocks_for(n)), dim3(kBlock), 0, s, perm_d, n, inv, seen, err);
  uint32_t host_err = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise permutation check");
  if (host_err) return fail(TSGNE_E_INVAL, "perm is not a permutation of [0, n)");
  if (nnz > 0) {
    hipLaunchKernelGGL(k_relabel_keys, dim3(blocks_for(n)), dim3(kBlock), 0, s, row_ptr_d, col_d, n, inv, key);
    size_t bytes = sort_bytes;
    TSGNE_HIP(rocprim::radix_sort_keys(base + o_tmp, bytes, key, key2, (int)nnz, 0, end_bit, s),
              "sort entries");
  }
  hipLaunchKernelGGL(k_keys_csr, dim3(blocks_for(std::max<int64_t>(nnz, (int64_t)n + 1))), dim3(kBlock), 0, s, key2,
                     nnz, n, out_row_ptr_d, out_col_d);
  TSGNE_HIP(hipGetLastError(), "launch CSR build");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise permuted graph");
  return TSGNE_OK;
}

tsgne_status tsgne_permute_rows(int32_t n, int32_t row_bytes, const void* src_d, const int32_t* perm_d,
                                int32_t inverse, void* dst_d, void* stream) {
  if (n < 1 || row_bytes < 4 || row_bytes % 4 != 0) return fail(TSGNE_E_INVAL, "need n >= 1 and row_bytes a positive multiple of 4");
  if (!src_d || !perm_d || !dst_d) return fail(TSGNE_E_INVAL, "null pointer");
  if (src_d == dst_d) return fail(TSGNE_E_INVAL, "src and dst must not be the same buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int32_t words = row_bytes / 4;
  hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for((int64_t)n * words)), dim3(kBlock), 0, s,
                     static_cast<const uint32_t*>(src_d), perm_d, n, words, inverse ? 1 : 0,
                     static_cast<uint32_t*>(dst_d));
  TSGNE_HIP(hipGetLastError(), "launch row permutation");
  return TSGNE_OK;
}

}  // extern "C"
