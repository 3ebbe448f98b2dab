// Affinity construction on the device: CSR check and mirror index, squared
// edge distances, per-row perplexity calibration and symmetrisation
// (section 2.1, eqs. (2)-(3), over graph neighbours as in section 2.2).
#include <cmath>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_check_rows(const int32_t* __restrict__ row_ptr, int32_t n, int64_t nnz,
                                                       uint32_t* __restrict__ err, int32_t* __restrict__ counters,
                                                       int32_t* __restrict__ heavy, int32_t heavy_cap) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t a = row_ptr[i], b = row_ptr[i + 1];
  bool bad = b < a || a < 0 || b > nnz;
  if (i == 0 && a != 0) bad = true;
  if (i == n - 1 && b != nnz) bad = true;
  if (bad) {
    atomicOr(err, kErrRowPtr);
    return;
  }
  const int64_t deg = b - a;
  if (deg > 0) atomicAdd(&counters[0], 1);
  if (deg > kHeavyDegree) {
    const int32_t k = atomicAdd(&counters[1], 1);
    if (k < heavy_cap) heavy[k] = i;
  }
}

// One thread per stored entry e: its row (binary search in row_ptr, which the
// previous kernel validated), the checks on its column, and the position of
// the reverse entry in the column's row.
__global__ __launch_bounds__(kBlock) void k_mirror(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, int32_t n, int64_t nnz,
                                                   int32_t* __restrict__ mirror, int32_t* __restrict__ row_of,
                                                   uint32_t* __restrict__ err) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  int32_t lo = 0, hi = n;  // row_ptr[lo] <= e < row_ptr[hi]
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (row_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  const int32_t i = lo;
  row_of[e] = i;
  const int32_t j = col[e];
  uint32_t bits = 0;
  int32_t pos = -1;
  if (j < 0 || j >= n) {
    bits |= kErrColRange;
  } else {
    if (j == i) bits |= kErrSelfLoop;
    if (e > row_ptr[i] && col[e - 1] >= j) bits |= kErrOrder;
    int64_t l = row_ptr[j], h = (int64_t)row_ptr[j + 1] - 1;
    while (l <= h) {
      const int64_t m = l + (h - l) / 2;
      const int32_t c = col[m];
      if (c == i) {
        pos = (int32_t)m;
        break;
      }
      if (c < i) l = m + 1; else h = m - 1;
    }
    if (pos < 0) bits |= kErrAsym;
  }
  mirror[e] = pos;
  if (bits) atomicOr(err, bits);
}

// D_e = ||x_i - x_j||^2 (the squared distance of eq. (2)) from FP32 rows,
// accumulated in FP64.  Sixteen lanes per entry stride over the d
// coordinates (consecutive lanes read consecutive floats of a row).
constexpr int kDistLanes = 16;

__global__ __launch_bounds__(kBlock) void k_sqdist(const int32_t* __restrict__ row_of, const int32_t* __restrict__ col,
                                                   int64_t nnz, const float* __restrict__ X, int32_t d,
                                                   double* __restrict__ D) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t e = t / kDistLanes;
  const int sub = threadIdx.x & (kDistLanes - 1);
  const bool live = e < nnz;
  double acc = 0.0;
  if (live) {
    const float* xi = X + (int64_t)row_of[e] * d;
    const float* xj = X + (int64_t)col[e] * d;
    for (int32_t k = sub; k < d; k += kDistLanes) {
      const double diff = (double)xi[k] - (double)xj[k];
      acc = fma(diff, diff, acc);
    }
  }
  for (int off = kDistLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kDistLanes);
  if (live && sub == 0) D[e] = acc;
}

// ---------------------------------------------------------------------------
// Per-row calibration.  The same steps run either on one thread (light rows)
// or on a whole wave (heavy rows, elements strided over lanes, sums reduced
// with butterflies so every lane holds the same bits and takes the same
// branch).
// ---------------------------------------------------------------------------

template <bool WAVE>
struct RowReduce {
  int lane;
  __device__ int first() const { return WAVE ? lane : 0; }
  __device__ int stride() const { return WAVE ? kWave : 1; }
  __device__ double sum(double v) const {
    if (WAVE)
      for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
  }
  __device__ double min(double v) const {
    if (WAVE)
      for (int off = kWave / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    return v;
  }
};

// Entropy in nats of p_k = exp(-beta delta_k) / S over the row.
template <bool WAVE>
__device__ double row_entropy(const double* __restrict__ Dr, int64_t deg, double dmin, double beta,
                              const RowReduce<WAVE>& rr) {
  double S = 0.0, T = 0.0;
  for (int64_t k = rr.first(); k < deg; k += rr.stride()) {
    const double dk = Dr[k] - dmin;
    const double ek = exp(-beta * dk);
    S += ek;
    T += dk * ek;
  }
  S = rr.sum(S);
  T = rr.sum(T);
  return log(S) + beta * T / S;
}

// beta_i = 1/(2 sigma_i^2) such that the row's entropy is log(perp): bracket
// from 1/mean(delta) by doubling or halving, then bisection to a relative
// width of 1e-13 (section 2.1: sigma_i is found by binary search).
template <bool WAVE>
__device__ void calibrate_row(const double* __restrict__ Dr, int64_t deg, double perp, double* __restrict__ pc,
                              double* __restrict__ beta_out, const RowReduce<WAVE>& rr) {
  const bool writer = !WAVE || rr.lane == 0;
  if (deg == 0) {
    if (writer) *beta_out = 0.0;
    return;
  }
  if ((double)deg <= perp) {  // target entropy out of reach: uniform row
    const double u = 1.0 / (double)deg;
    for (int64_t k = rr.first(); k < deg; k += rr.stride()) pc[k] = u;
    if (writer) *beta_out = 0.0;
    return;
  }
  double dmin = INFINITY;
  for (int64_t k = rr.first(); k < deg; k += rr.stride()) dmin = fmin(dmin, Dr[k]);
  dmin = rr.min(dmin);
  double ties = 0.0, mean = 0.0;
  for (int64_t k = rr.first(); k < deg; k += rr.stride()) {
    ties += (Dr[k] == dmin) ? 1.0 : 0.0;
    mean += Dr[k] - dmin;
  }
  ties = rr.sum(ties);
  mean = rr.sum(mean) / (double)deg;
  if (ties >= perp) {  // uniform over the nearest neighbours (beta -> infinity)
    const double u = 1.0 / ties;
    for (int64_t k = rr.first(); k < deg; k += rr.stride()) pc[k] = (Dr[k] == dmin) ? u : 0.0;
    if (writer) *beta_out = INFINITY;
    return;
  }
  const double target = log(perp);
  const double b0 = 1.0 / mean;
  double lo, hi;
  if (row_entropy(Dr, deg, dmin, b0, rr) > target) {
    lo = b0;
    hi = 2.0 * b0;
    while (row_entropy(Dr, deg, dmin, hi, rr) > target) {
      lo = hi;
      hi *= 2.0;
    }
  } else {
    hi = b0;
    lo = 0.5 * b0;
    while (row_entropy(Dr, deg, dmin, lo, rr) <= target) {
      hi = lo;
      lo *= 0.5;
    }
  }
  for (int it = 0; it < 200 && (hi - lo) > 1e-13 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (row_entropy(Dr, deg, dmin, mid, rr) > target) lo = mid; else hi = mid;
  }
  const double bt = 0.5 * (lo + hi);
  double S = 0.0;
  for (int64_t k = rr.first(); k < deg; k += rr.stride()) S += exp(-bt * (Dr[k] - dmin));
  S = rr.sum(S);
  for (int64_t k = rr.first(); k < deg; k += rr.stride()) pc[k] = exp(-bt * (Dr[k] - dmin)) / S;
  if (writer) *beta_out = bt;
}

__global__ __launch_bounds__(kBlock) void k_calibrate_light(const int32_t* __restrict__ row_ptr, int32_t n,
                                                            const double* __restrict__ D, double perp,
                                                            double* __restrict__ pcond, double* __restrict__ beta) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t b = row_ptr[i], deg = (int64_t)row_ptr[i + 1] - b;
  if (deg > kHeavyDegree) return;
  RowReduce<false> rr{0};
  calibrate_row<false>(D + b, deg, perp, pcond + b, beta + i, rr);
}

__global__ __launch_bounds__(kBlock) void k_calibrate_heavy(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ heavy, int32_t n_heavy,
                                                            const double* __restrict__ D, double perp,
                                                            double* __restrict__ pcond, double* __restrict__ beta) {
  const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6)));
  if (w >= n_heavy) return;
  const int32_t i = heavy[w];
  const int64_t b = row_ptr[i], deg = (int64_t)row_ptr[i + 1] - b;
  RowReduce<true> rr{(int)(threadIdx.x & (kWave - 1))};
  calibrate_row<true>(D + b, deg, perp, pcond + b, beta + i, rr);
}

// p_ij = (p_{j|i} + p_{i|j}) / S, eq. (3), with S = 2 * (non-isolated nodes).
__global__ __launch_bounds__(kBlock) void k_symmetrise(const int32_t* __restrict__ mirror, int64_t nnz,
                                                       const double* __restrict__ pcond, double S,
                                                       float* __restrict__ P) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  P[e] = (float)((pcond[e] + pcond[mirror[e]]) / S);
}

inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_check_rows(const int32_t* row_ptr, int32_t n, int64_t nnz, uint32_t* err, int32_t* counters,
                             int32_t* heavy, hipStream_t s) {
  const int32_t cap = (int32_t)std::min<int64_t>(n, nnz / (kHeavyDegree + 1) + 1);
  hipLaunchKernelGGL(k_check_rows, dim3(blocks_for(n)), dim3(kBlock), 0, s, row_ptr, n, nnz, err, counters, heavy,
                     cap);
  return hipGetLastError();
}

hipError_t launch_mirror(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz, int32_t* mirror,
                         int32_t* row_of, uint32_t* err, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror, dim3(blocks_for(nnz)), dim3(kBlock), 0, s, row_ptr, col, n, nnz, mirror, row_of, err);
  return hipGetLastError();
}

hipError_t launch_sqdist(const int32_t* row_of, const int32_t* col, int64_t nnz, const float* X, int32_t d, double* D,
                         hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqdist, dim3(blocks_for(nnz * kDistLanes)), dim3(kBlock), 0, s, row_of, col, nnz, X, d, D);
  return hipGetLastError();
}

hipError_t launch_calibrate(const int32_t* row_ptr, int32_t n, const int32_t* heavy, int32_t n_heavy, const double* D,
                            double perplexity, double* pcond, double* beta, hipStream_t s) {
  hipLaunchKernelGGL(k_calibrate_light, dim3(blocks_for(n)), dim3(kBlock), 0, s, row_ptr, n, D, perplexity, pcond,
                     beta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_heavy == 0) return e;
  const unsigned waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_calibrate_heavy, dim3((n_heavy + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, s,
                     row_ptr, heavy, n_heavy, D, perplexity, pcond, beta);
  return hipGetLastError();
}

hipError_t launch_symmetrise(const int32_t* mirror, int64_t nnz, const double* pcond, double S, float* P,
                             hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_symmetrise, dim3(blocks_for(nnz)), dim3(kBlock), 0, s, mirror, nnz, pcond, S, P);
  return hipGetLastError();
}

}  // namespace tsgne
