// Layout quality on the device: k-means on the layout (the layout
// clustering of section 2.5), NMI of two labelings (section 2.5, eq. (11))
// and aesthetic quality (section 2.6, eqs. (12)-(14)).
//
// Every integer decision (a label, a grid cell, a good cell) is taken by the
// same IEEE double operations, in the same order and without contraction,
// as the definition: the layout box is an exact min/max, the clustering runs
// on the layout mapped to a 2^24 grid over that box with exact integer sums
// per cluster, and centres are one division.  So labels, cells and counts are
// reproducible bit for bit; only the NMI's final sums are order-dependent.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kFinal = 1024;          // threads of the one-block kernels
constexpr int kMaxClusters = 1024;    // k-means centres held in LDS
constexpr int kIterChunk = 8;         // k-means passes queued between checks
constexpr int kLdsContingency = 4096; // contingency tables up to this size are counted in LDS first
constexpr uint32_t kErrFinite = 1u, kErrSeed = 2u, kErrLabel = 4u;

// ---- layout box -----------------------------------------------------------

// Per-block min/max of both axes; err |= kErrFinite on a non-finite value.
__global__ __launch_bounds__(kBlock) void k_box_partial(const float2* __restrict__ Y, int32_t n,
                                                        float4* __restrict__ part, uint32_t* __restrict__ err) {
  __shared__ float4 s[kBlock / kWave];
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);  // xlo, xhi, ylo, yhi
  if (i < n) {
    const float2 y = Y[i];
    if (!isfinite(y.x) || !isfinite(y.y)) atomicOr(err, kErrFinite);
    b = make_float4(y.x, y.x, y.y, y.y);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    b.x = fminf(b.x, __shfl_xor(b.x, off, kWave));
    b.y = fmaxf(b.y, __shfl_xor(b.y, off, kWave));
    b.z = fminf(b.z, __shfl_xor(b.z, off, kWave));
    b.w = fmaxf(b.w, __shfl_xor(b.w, off, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      b.x = fminf(b.x, s[w].x);
      b.y = fmaxf(b.y, s[w].y);
      b.z = fminf(b.z, s[w].z);
      b.w = fmaxf(b.w, s[w].w);
    }
    part[blockIdx.x] = b;
  }
}

// box = (xlo, xhi, ylo, yhi) as doubles (exact: min and max of floats).
__global__ __launch_bounds__(kFinal) void k_box_final(const float4* __restrict__ part, int32_t blocks,
                                                      double* __restrict__ box) {
  __shared__ float4 s[kFinal / kWave];
  float4 b = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  for (int32_t i = threadIdx.x; i < blocks; i += kFinal) {
    const float4 p = part[i];
    b.x = fminf(b.x, p.x);
    b.y = fmaxf(b.y, p.y);
    b.z = fminf(b.z, p.z);
    b.w = fmaxf(b.w, p.w);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    b.x = fminf(b.x, __shfl_xor(b.x, off, kWave));
    b.y = fmaxf(b.y, __shfl_xor(b.y, off, kWave));
    b.z = fminf(b.z, __shfl_xor(b.z, off, kWave));
    b.w = fmaxf(b.w, __shfl_xor(b.w, off, kWave));
  }
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kFinal / kWave; ++w) {
      b.x = fminf(b.x, s[w].x);
      b.y = fmaxf(b.y, s[w].y);
      b.z = fminf(b.z, s[w].z);
      b.w = fmaxf(b.w, s[w].w);
    }
    box[0] = b.x;
    box[1] = b.y;
    box[2] = b.z;
    box[3] = b.w;
  }
}

// ---- k-means ----------------------------------------------------------------

// q = min(floor((y - lo) / (hi - lo) * 2^24), 2^24 - 1), 0 on a flat axis.
__device__ __forceinline__ int32_t quantise(float y, double lo, double hi) {
#pragma clang fp contract(off)
  const double span = hi - lo;
  if (!(span > 0)) return 0;
  const double t = floor(((double)y - lo) / span * 16777216.0);
  return t > 16777215.0 ? 16777215 : (int32_t)t;
}

__global__ __launch_bounds__(kBlock) void k_quantise(const float2* __restrict__ Y, int32_t n,
                                                     const double* __restrict__ box, int2* __restrict__ q) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float2 y = Y[i];
  q[i] = make_int2(quantise(y.x, box[0], box[1]), quantise(y.y, box[2], box[3]));
}

// Centres from the seed points; labels start at -1 (every point changes in
// the first pass).
__global__ __launch_bounds__(kBlock) void k_km_init(const int2* __restrict__ q, int32_t n,
                                                    const int32_t* __restrict__ seeds, int32_t k,
                                                    double2* __restrict__ centre, int32_t* __restrict__ labels,
                                                    uint32_t* __restrict__ err) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < k) {
    const int32_t s = seeds[i];
    if (s < 0 || s >= n) {
      atomicOr(err, kErrSeed);
      centre[i] = make_double2(0.0, 0.0);
    } else {
      centre[i] = make_double2((double)q[s].x, (double)q[s].y);
    }
  }
  if (i < n) labels[i] = -1;
}

struct KmState {
  double2* centre;          // [k]
  unsigned long long* sum;  // [k][2] exact integer sums of the members
  int32_t* count;           // [k]
  int32_t* changed;         // [blocks] labels changed per block in this pass
  int32_t* done;            // [0] converged, [1] passes made when converged
};

// One assignment pass: nearest centre (squared distance in FP64, no
// contraction, ties to the lower index), per-block change count, and the
// members' exact integer sums added to the cluster totals.
__global__ __launch_bounds__(kBlock) void k_km_assign(const int2* __restrict__ q, int32_t n, int32_t k,
                                                      int32_t* __restrict__ labels, KmState st) {
  __shared__ double2 s_c[kMaxClusters];
  __shared__ unsigned long long s_sum[2 * kMaxClusters];
  __shared__ int32_t s_cnt[kMaxClusters];
  if (st.done[0]) return;  // converged in an earlier pass of this chunk (uniform)
  for (int c = threadIdx.x; c < k; c += kBlock) {
    s_c[c] = st.centre[c];
    s_sum[2 * c] = 0;
    s_sum[2 * c + 1] = 0;
    s_cnt[c] = 0;
  }
  __syncthreads();
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  bool moved = false;
  if (i < n) {
#pragma clang fp contract(off)
    const int2 p = q[i];
    const double px = (double)p.x, py = (double)p.y;
    int32_t best = 0;
    double bd = INFINITY;
    for (int32_t c = 0; c < k; ++c) {
      const double dx = px - s_c[c].x, dy = py - s_c[c].y;
      const double dist = dx * dx + dy * dy;
      if (dist < bd) {
        bd = dist;
        best = c;
      }
    }
    moved = labels[i] != best;
    labels[i] = best;
    atomicAdd(&s_sum[2 * best], (unsigned long long)p.x);
    atomicAdd(&s_sum[2 * best + 1], (unsigned long long)p.y);
    atomicAdd(&s_cnt[best], 1);
  }
  const int n_moved = __syncthreads_count(moved);
  if (threadIdx.x == 0) st.changed[blockIdx.x] = n_moved;
  for (int c = threadIdx.x; c < k; c += kBlock) {
    if (s_cnt[c] > 0) {
      atomicAdd(&st.sum[2 * c], s_sum[2 * c]);
      atomicAdd(&st.sum[2 * c + 1], s_sum[2 * c + 1]);
      atomicAdd(&st.count[c], s_cnt[c]);
    }
  }
}

// One block: if no label changed in the pass, mark convergence (and the pass
// number); otherwise move each non-empty cluster's centre to its mean.  The
// sums are cleared for the next pass either way.
__global__ __launch_bounds__(kFinal) void k_km_update(int32_t k, int32_t blocks, int32_t pass, KmState st) {
  __shared__ int32_t s_tot[kFinal / kWave];
  if (st.done[0]) return;
  int32_t moved = 0;
  for (int32_t b = threadIdx.x; b < blocks; b += kFinal) moved += st.changed[b];
  for (int off = kWave / 2; off > 0; off >>= 1) moved += __shfl_xor(moved, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) s_tot[threadIdx.x >> 6] = moved;
  __syncthreads();
  int32_t total = 0;
  for (int w = 0; w < kFinal / kWave; ++w) total += s_tot[w];
  for (int c = threadIdx.x; c < k; c += kFinal) {
    if (total > 0 && st.count[c] > 0) {
      const double cnt = (double)st.count[c];
      st.centre[c] = make_double2((double)st.sum[2 * c] / cnt, (double)st.sum[2 * c + 1] / cnt);
    }
    st.sum[2 * c] = 0;
    st.sum[2 * c + 1] = 0;
    st.count[c] = 0;
  }
  if (threadIdx.x == 0 && total == 0) {
    st.done[0] = 1;
    st.done[1] = pass;
  }
}

// ---- NMI ----------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_contingency(const int32_t* __restrict__ a, int32_t ka,
                                                        const int32_t* __restrict__ b, int32_t kb, int32_t n,
                                                        int32_t* __restrict__ table, uint32_t* __restrict__ err) {
  __shared__ int32_t s_t[kLdsContingency];
  const int32_t cells = ka * kb;
  const bool local = cells <= kLdsContingency;
  if (local) {
    for (int c = threadIdx.x; c < cells; c += kBlock) s_t[c] = 0;
    __syncthreads();
  }
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const int32_t x = a[i], y = b[i];
    if (x < 0 || x >= ka || y < 0 || y >= kb) {
      atomicOr(err, kErrLabel);
    } else if (local) {
      atomicAdd(&s_t[x * kb + y], 1);
    } else {
      atomicAdd(&table[(int64_t)x * kb + y], 1);
    }
  }
  if (local) {
    __syncthreads();
    for (int c = threadIdx.x; c < cells; c += kBlock)
      if (s_t[c]) atomicAdd(&table[c], s_t[c]);
  }
}

__device__ double block_sum(double v, double* s) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < kFinal / kWave; ++w) t += s[w];
  return t;
}

// One block: marginals, entropies, mutual information, NMI (eq. (11)).
__global__ __launch_bounds__(kFinal) void k_nmi_final(const int32_t* __restrict__ table, int32_t ka, int32_t kb,
                                                      int32_t n, int64_t* __restrict__ na, int64_t* __restrict__ nb,
                                                      double* __restrict__ out) {
  __shared__ double s[kFinal / kWave];
  for (int32_t x = threadIdx.x; x < ka; x += kFinal) {
    int64_t r = 0;
    for (int32_t y = 0; y < kb; ++y) r += table[(int64_t)x * kb + y];
    na[x] = r;
  }
  for (int32_t y = threadIdx.x; y < kb; y += kFinal) {
    int64_t c = 0;
    for (int32_t x = 0; x < ka; ++x) c += table[(int64_t)x * kb + y];
    nb[y] = c;
  }
  __syncthreads();
  const double N = (double)n;
  double ha = 0, hb = 0, mi = 0;
  for (int32_t x = threadIdx.x; x < ka; x += kFinal)
    if (na[x] > 0) ha -= ((double)na[x] / N) * log((double)na[x] / N);
  for (int32_t y = threadIdx.x; y < kb; y += kFinal)
    if (nb[y] > 0) hb -= ((double)nb[y] / N) * log((double)nb[y] / N);
  const int64_t cells = (int64_t)ka * kb;
  for (int64_t c = threadIdx.x; c < cells; c += kFinal) {
    const int32_t v = table[c];
    if (v > 0) {
      const int32_t x = (int32_t)(c / kb), y = (int32_t)(c % kb);
      mi += ((double)v / N) * log(N * (double)v / ((double)na[x] * (double)nb[y]));
    }
  }
  ha = block_sum(ha, s);
  hb = block_sum(hb, s);
  mi = block_sum(mi, s);
  if (threadIdx.x == 0) out[0] = (ha + hb > 0) ? 2.0 * mi / (ha + hb) : 1.0;
}

// ---- AQ -------------------------------------------------------------------------

// The grid cell of a coordinate: floor((y - lo) / w), w = (hi - lo) / grid,
// upper edge into the last cell, a flat axis into the first.
__device__ __forceinline__ int32_t grid_cell(float y, double lo, double hi, int32_t grid) {
#pragma clang fp contract(off)
  const double w = (hi - lo) / grid;
  if (!(w > 0)) return 0;
  const double t = floor(((double)y - lo) / w);
  return t > grid - 1 ? grid - 1 : (int32_t)t;
}

__global__ __launch_bounds__(kBlock) void k_aq_count(const float2* __restrict__ Y, const int32_t* __restrict__ labels,
                                                     int32_t n, int32_t n_labels, int32_t grid,
                                                     const double* __restrict__ box, int32_t* __restrict__ count,
                                                     uint32_t* __restrict__ err) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t l = labels[i];
  if (l < 0 || l >= n_labels) {
    atomicOr(err, kErrLabel);
    return;
  }
  const float2 y = Y[i];
  const int32_t cx = grid_cell(y.x, box[0], box[1], grid), cy = grid_cell(y.y, box[2], box[3], grid);
  atomicAdd(&count[((int64_t)cy * grid + cx) * n_labels + l], 1);
}

// Per block of cells: how many are good (largest label fraction > p).
__global__ __launch_bounds__(kBlock) void k_aq_cells(const int32_t* __restrict__ count, int64_t cells,
                                                     int32_t n_labels, double p, int32_t* __restrict__ good) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool ok = false;
  if (c < cells) {
    int64_t total = 0, best = 0;
    for (int32_t l = 0; l < n_labels; ++l) {
      const int64_t v = count[c * n_labels + l];
      total += v;
      best = v > best ? v : best;
    }
    ok = total > 0 && (double)best / (double)total > p;
  }
  const int g = __syncthreads_count(ok);
  if (threadIdx.x == 0) good[blockIdx.x] = g;
}

unsigned blocks_of(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

// The layout box into box_d[4] (device); err_d must be cleared.
hipError_t launch_box(const float2* Y, int32_t n, float4* part, double* box, uint32_t* err, hipStream_t s) {
  const unsigned blocks = blocks_of(n);
  hipLaunchKernelGGL(k_box_partial, dim3(blocks), dim3(kBlock), 0, s, Y, n, part, err);
  hipLaunchKernelGGL(k_box_final, dim3(1), dim3(kFinal), 0, s, part, (int32_t)blocks, box);
  return hipGetLastError();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_kmeans(int32_t n, const float* Y_d, int32_t k, const int32_t* seeds_d, int32_t max_iter,
                          int32_t* labels_d, int32_t* iters_out, void* stream) {
  if (iters_out) *iters_out = 0;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (k < 1 || k > kMaxClusters) return fail(TSGNE_E_INVAL, "k must lie in [1, 1024]");
  if (max_iter < 1) return fail(TSGNE_E_INVAL, "max_iter must be >= 1");
  if (!Y_d || !seeds_d || !labels_d) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const unsigned blocks = blocks_of(n);
  // scratch: err + done | box | box partials | q | centres | sums | counts | changed
  size_t o = 0;
  const size_t o_err = o;
  o = align256(o + 4 * sizeof(int32_t));
  const size_t o_box = o;
  o = align256(o + 4 * sizeof(double));
  const size_t o_part = o;
  o = align256(o + sizeof(float4) * blocks);
  const size_t o_q = o;
  o = align256(o + sizeof(int2) * (size_t)n);
  const size_t o_c = o;
  o = align256(o + sizeof(double2) * (size_t)k);
  const size_t o_sum = o;
  o = align256(o + 2 * sizeof(unsigned long long) * (size_t)k);
  const size_t o_cnt = o;
  o = align256(o + sizeof(int32_t) * (size_t)k);
  const size_t o_chg = o;
  o = align256(o + sizeof(int32_t) * blocks);
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate k-means state");
  char* const base = static_cast<char*>(tmp.p);
  uint32_t* const err = reinterpret_cast<uint32_t*>(base + o_err);
  int32_t* const done = reinterpret_cast<int32_t*>(base + o_err) + 2;
  double* const box = reinterpret_cast<double*>(base + o_box);
  KmState st{reinterpret_cast<double2*>(base + o_c), reinterpret_cast<unsigned long long*>(base + o_sum),
             reinterpret_cast<int32_t*>(base + o_cnt), reinterpret_cast<int32_t*>(base + o_chg), done};
  TSGNE_HIP(hipMemsetAsync(base + o_err, 0, 4 * sizeof(int32_t), s), "clear flags");
  TSGNE_HIP(hipMemsetAsync(base + o_sum, 0, o_chg - o_sum, s), "clear sums");
  const float2* Y = reinterpret_cast<const float2*>(Y_d);
  int2* const q = reinterpret_cast<int2*>(base + o_q);
  TSGNE_HIP(launch_box(Y, n, reinterpret_cast<float4*>(base + o_part), box, err, s), "launch layout box");
  hipLaunchKernelGGL(k_quantise, dim3(blocks), dim3(kBlock), 0, s, Y, n, box, q);
  hipLaunchKernelGGL(k_km_init, dim3(blocks_of(std::max(n, k))), dim3(kBlock), 0, s, q, n, seeds_d, k, st.centre,
                     labels_d, err);
  TSGNE_HIP(hipGetLastError(), "launch k-means set-up");
  uint32_t host_err = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise k-means set-up");
  if (host_err & kErrFinite) return fail(TSGNE_E_NONFINITE, "layout has a non-finite coordinate");
  if (host_err & kErrSeed) return fail(TSGNE_E_INVAL, "a seed index lies outside [0, n)");

  int32_t host_done[2] = {0, 0};
  int32_t pass = 0;
  while (pass < max_iter) {
    const int32_t last = std::min(max_iter, pass + kIterChunk);
    for (int32_t it = pass + 1; it <= last; ++it) {
      hipLaunchKernelGGL(k_km_assign, dim3(blocks), dim3(kBlock), 0, s, q, n, k, labels_d, st);
      hipLaunchKernelGGL(k_km_update, dim3(1), dim3(kFinal), 0, s, k, (int32_t)blocks, it, st);
    }
    TSGNE_HIP(hipGetLastError(), "launch k-means passes");
    TSGNE_HIP(hipMemcpyAsync(host_done, done, sizeof(host_done), hipMemcpyDeviceToHost, s), "read convergence");
    TSGNE_HIP(hipStreamSynchronize(s), "synchronise k-means passes");
    pass = last;
    if (host_done[0]) break;
  }
  if (iters_out) *iters_out = host_done[0] ? host_done[1] : max_iter;
  return TSGNE_OK;
}

tsgne_status tsgne_nmi(int32_t n, const int32_t* a_d, int32_t ka, const int32_t* b_d, int32_t kb, double* nmi_out,
                       void* stream) {
  if (!nmi_out) return fail(TSGNE_E_INVAL, "nmi_out is NULL");
  *nmi_out = NAN;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (ka < 1 || kb < 1 || (int64_t)ka * kb > ((int64_t)1 << 26))
    return fail(TSGNE_E_INVAL, "label counts must be >= 1 with ka * kb <= 2^26");
  if (!a_d || !b_d) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t cells = (int64_t)ka * kb;
  size_t o = 0;
  const size_t o_err = o;
  o = align256(o + sizeof(uint32_t));
  const size_t o_out = o;
  o = align256(o + sizeof(double));
  const size_t o_tab = o;
  o = align256(o + sizeof(int32_t) * (size_t)cells);
  const size_t o_na = o;
  o = align256(o + sizeof(int64_t) * (size_t)ka);
  const size_t o_nb = o;
  o = align256(o + sizeof(int64_t) * (size_t)kb);
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate contingency table");
  char* const base = static_cast<char*>(tmp.p);
  uint32_t* const err = reinterpret_cast<uint32_t*>(base + o_err);
  int32_t* const table = reinterpret_cast<int32_t*>(base + o_tab);
  TSGNE_HIP(hipMemsetAsync(base, 0, o_na, s), "clear contingency table");
  hipLaunchKernelGGL(k_contingency, dim3(blocks_of(n)), dim3(kBlock), 0, s, a_d, ka, b_d, kb, n, table, err);
  hipLaunchKernelGGL(k_nmi_final, dim3(1), dim3(kFinal), 0, s, table, ka, kb, n,
                     reinterpret_cast<int64_t*>(base + o_na), reinterpret_cast<int64_t*>(base + o_nb),
                     reinterpret_cast<double*>(base + o_out));
  TSGNE_HIP(hipGetLastError(), "launch NMI");
  uint32_t host_err = 0;
  double result = NAN;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipMemcpyAsync(&result, base + o_out, sizeof(double), hipMemcpyDeviceToHost, s), "read NMI");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise NMI");
  if (host_err) return fail(TSGNE_E_INVAL, "a label lies outside its range");
  *nmi_out = result;
  return TSGNE_OK;
}

tsgne_status tsgne_aq(int32_t n, const float* Y_d, const int32_t* labels_d, int32_t n_labels, int32_t grid, double p,
                      double* aq_out, void* stream) {
  if (!aq_out) return fail(TSGNE_E_INVAL, "aq_out is NULL");
  *aq_out = NAN;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (n_labels < 1 || grid < 1 || grid > 4096 || (int64_t)grid * grid * n_labels > ((int64_t)1 << 28))
    return fail(TSGNE_E_INVAL, "need n_labels >= 1, 1 <= grid <= 4096 and grid^2 * n_labels <= 2^28");
  if (std::isnan(p)) return fail(TSGNE_E_INVAL, "p is NaN");
  if (!Y_d || !labels_d) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t cells = (int64_t)grid * grid;
  const unsigned blocks = blocks_of(n), cell_blocks = blocks_of(cells);
  size_t o = 0;
  const size_t o_err = o;
  o = align256(o + sizeof(uint32_t));
  const size_t o_cnt = o;
  o = align256(o + sizeof(int32_t) * (size_t)cells * n_labels);
  const size_t o_box = o;
  o = align256(o + 4 * sizeof(double));
  const size_t o_part = o;
  o = align256(o + sizeof(float4) * blocks);
  const size_t o_good = o;
  o = align256(o + sizeof(int32_t) * cell_blocks);
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, o, s), "allocate AQ counts");
  char* const base = static_cast<char*>(tmp.p);
  uint32_t* const err = reinterpret_cast<uint32_t*>(base + o_err);
  double* const box = reinterpret_cast<double*>(base + o_box);
  int32_t* const count = reinterpret_cast<int32_t*>(base + o_cnt);
  int32_t* const good = reinterpret_cast<int32_t*>(base + o_good);
  TSGNE_HIP(hipMemsetAsync(base, 0, o_box, s), "clear AQ counts");
  const float2* Y = reinterpret_cast<const float2*>(Y_d);
  TSGNE_HIP(launch_box(Y, n, reinterpret_cast<float4*>(base + o_part), box, err, s), "launch layout box");
  hipLaunchKernelGGL(k_aq_count, dim3(blocks), dim3(kBlock), 0, s, Y, labels_d, n, n_labels, grid, box, count, err);
  hipLaunchKernelGGL(k_aq_cells, dim3(cell_blocks), dim3(kBlock), 0, s, count, cells, n_labels, p, good);
  TSGNE_HIP(hipGetLastError(), "launch AQ");
  std::vector<int32_t> host_good(cell_blocks);
  uint32_t host_err = 0;
  TSGNE_HIP(hipMemcpyAsync(&host_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "read error word");
  TSGNE_HIP(hipMemcpyAsync(host_good.data(), good, sizeof(int32_t) * cell_blocks, hipMemcpyDeviceToHost, s),
            "read good cells");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise AQ");
  if (host_err & kErrFinite) return fail(TSGNE_E_NONFINITE, "layout has a non-finite coordinate");
  if (host_err) return fail(TSGNE_E_INVAL, "a label lies outside [0, n_labels)");
  int64_t total = 0;
  for (int32_t g : host_good) total += g;
  *aq_out = (double)total / (double)cells;
  return TSGNE_OK;
}

}  // extern "C"
