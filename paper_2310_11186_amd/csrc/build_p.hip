// Affinity construction on the device: CSR check and mirror index, squared
// edge distances, per-row perplexity calibration and symmetrisation
// (section 2.1, eqs. (2)-(3), over graph neighbours as in section 2.2).
#include <cmath>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;

// Row checks and counts without contended atomics (atomics on one address
// serialise across the whole device): per-block counts, one block turns
// them into offsets, then each block writes its selected rows in order.
__device__ __forceinline__ bool row_ok(const int32_t* __restrict__ row_ptr, int32_t i, int32_t n, int64_t nnz,
                                       int64_t* deg) {
  const int64_t a = row_ptr[i], b = row_ptr[i + 1];
  bool bad = b < a || a < 0 || b > nnz;
  if (i == 0 && a != 0) bad = true;
  if (i == n - 1 && b != nnz) bad = true;
  *deg = b - a;
  return !bad;
}

__global__ __launch_bounds__(kBlock) void k_row_counts(const int32_t* __restrict__ row_ptr, int32_t n, int64_t nnz,
                                                       int32_t threshold, uint32_t* __restrict__ err,
                                                       int2* __restrict__ partial) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  bool nonempty = false, sel = false;
  if (i < n) {
    int64_t deg;
    if (!row_ok(row_ptr, i, n, nnz, &deg)) {
      atomicOr(err, kErrRowPtr);
    } else {
      nonempty = deg > 0;
      sel = deg > threshold;
    }
  }
  const int c_ne = __syncthreads_count(nonempty);
  const int c_sel = __syncthreads_count(sel);
  if (threadIdx.x == 0) partial[blockIdx.x] = make_int2(c_ne, c_sel);
}

constexpr int kScanBlock = 1024;
constexpr int kRowOfRun = 8;     // entries per thread in k_row_of
constexpr int kMirrorPer = 4;    // entries per thread in k_mirror

// One block: partial[b].y becomes the number of selected rows in blocks
// before b; counters = (rows with entries, selected rows).
__global__ __launch_bounds__(kScanBlock) void k_row_offsets(int2* __restrict__ partial, int32_t blocks,
                                                            int32_t* __restrict__ counters) {
  __shared__ int32_t s_sel[kScanBlock / kWave], s_ne[kScanBlock / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t >> 6;
  const int32_t per = (blocks + kScanBlock - 1) / kScanBlock;
  const int32_t lo = min(blocks, t * per), hi = min(blocks, lo + per);
  int32_t sel = 0, ne = 0;
  for (int32_t b = lo; b < hi; ++b) {
    sel += partial[b].y;
    ne += partial[b].x;
  }
  int32_t inc = sel;
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += y;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) ne += __shfl_xor(ne, off, kWave);
  if (lane == kWave - 1) s_sel[wv] = inc;
  if (lane == 0) s_ne[wv] = ne;
  __syncthreads();
  int32_t base = 0, tot_sel = 0, tot_ne = 0;
  for (int w = 0; w < kScanBlock / kWave; ++w) {
    base += (w < wv) ? s_sel[w] : 0;
    tot_sel += s_sel[w];
    tot_ne += s_ne[w];
  }
  int32_t run = base + inc - sel;
  for (int32_t b = lo; b < hi; ++b) {
    const int32_t c = partial[b].y;
    partial[b].y = run;
    run += c;
  }
  if (t == 0) {
    counters[0] = tot_ne;
    counters[1] = tot_sel;
  }
}

__global__ __launch_bounds__(kBlock) void k_row_select(const int32_t* __restrict__ row_ptr, int32_t n, int64_t nnz,
                                                       int32_t threshold, const int2* __restrict__ partial,
                                                       int32_t* __restrict__ ids, int4* __restrict__ recs,
                                                       int32_t cap) {
  __shared__ int32_t s_wave[kBlock / kWave];
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  bool sel = false;
  if (i < n) {
    int64_t deg;
    sel = row_ok(row_ptr, i, n, nnz, &deg) && deg > threshold;
  }
  const unsigned long long m = __ballot(sel);
  if (lane == 0) s_wave[wv] = __popcll(m);
  __syncthreads();
  int32_t pos = partial[blockIdx.x].y + __popcll(m & ((1ull << lane) - 1));
  for (int w = 0; w < wv; ++w) pos += s_wave[w];
  if (sel && pos < cap) {
    if (ids) ids[pos] = i;
    if (recs) recs[pos] = make_int4(i, row_ptr[i], row_ptr[i + 1], 0);
  }
}

// row_of[e] = the row of entry e: one block per kBlock rows shares out the
// entries of its rows.  Does nothing when the row check has failed, so it
// may be queued behind that check without waiting for its result.
__global__ __launch_bounds__(kBlock) void k_row_of(const int32_t* __restrict__ row_ptr, int32_t n,
                                                   int32_t* __restrict__ row_of, const uint32_t* __restrict__ err) {
  __shared__ int32_t s_ptr[kBlock + 1];
  if (*err & kErrRowPtr) return;
  const int32_t r0 = blockIdx.x * kBlock;
  const int32_t rows = min(kBlock, n - r0);
  for (int t = threadIdx.x; t <= rows; t += kBlock) s_ptr[t] = row_ptr[r0 + t];
  __syncthreads();
  const int32_t first = s_ptr[0], end = s_ptr[rows];
  // kRowOfRun consecutive entries per thread: one search, then a walk
  for (int32_t e0 = first + threadIdx.x * kRowOfRun; e0 < end; e0 += kBlock * kRowOfRun) {
    int lo = 0, hi = rows;  // s_ptr[lo] <= e0 < s_ptr[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_ptr[mid] <= e0) lo = mid;
      else hi = mid;
    }
#pragma unroll
    for (int k = 0; k < kRowOfRun; ++k) {
      const int32_t e = e0 + k;
      if (e < end) {
        while (s_ptr[lo + 1] <= e) ++lo;  // stops below rows since e < s_ptr[rows]
        row_of[e] = r0 + lo;
      }
    }
  }
}

// kMirrorPer entries per thread (row from row_of): the checks on each
// entry's column and the position of the reverse entry in the column's row,
// with the binary searches of the entries advancing together so that their
// loads overlap.  Does nothing when the row check has failed.
__global__ __launch_bounds__(kBlock) void k_mirror(const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, int32_t n, int64_t nnz,
                                                   int32_t* __restrict__ mirror, const int32_t* __restrict__ row_of,
                                                   uint32_t* __restrict__ err) {
  if (*err & kErrRowPtr) return;  // row_of is not filled after a failed row check
  const int64_t e0 = (int64_t)blockIdx.x * kBlock * kMirrorPer + threadIdx.x;
  int64_t lo[kMirrorPer], hi[kMirrorPer], mid[kMirrorPer];
  int32_t key[kMirrorPer], pos[kMirrorPer];
  bool live[kMirrorPer];
  uint32_t bits = 0;
#pragma unroll
  for (int k = 0; k < kMirrorPer; ++k) {
    const int64_t e = e0 + (int64_t)k * kBlock;
    live[k] = false;
    pos[k] = -1;
    lo[k] = 0;
    hi[k] = -1;
    key[k] = 0;
    if (e < nnz) {
      const int32_t i = row_of[e];
      const int32_t j = col[e];
      if (j < 0 || j >= n) {
        bits |= kErrColRange;
      } else {
        if (j == i) bits |= kErrSelfLoop;
        if (e > row_ptr[i] && col[e - 1] >= j) bits |= kErrOrder;
        lo[k] = row_ptr[j];
        hi[k] = (int64_t)row_ptr[j + 1] - 1;
        key[k] = i;
        live[k] = lo[k] <= hi[k];
        if (!live[k]) bits |= kErrAsym;
      }
    }
  }
  bool any = true;
  while (any) {
    int32_t c[kMirrorPer];
#pragma unroll
    for (int k = 0; k < kMirrorPer; ++k) {
      if (live[k]) {
        mid[k] = lo[k] + (hi[k] - lo[k]) / 2;
        c[k] = col[mid[k]];
      }
    }
    any = false;
#pragma unroll
    for (int k = 0; k < kMirrorPer; ++k) {
      if (live[k]) {
        if (c[k] == key[k]) {
          pos[k] = (int32_t)mid[k];
          live[k] = false;
        } else {
          if (c[k] < key[k]) lo[k] = mid[k] + 1;
          else hi[k] = mid[k] - 1;
          if (lo[k] > hi[k]) {
            live[k] = false;
            bits |= kErrAsym;
          }
        }
        any |= live[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kMirrorPer; ++k) {
    const int64_t e = e0 + (int64_t)k * kBlock;
    if (e < nnz) mirror[e] = pos[k];
  }
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

int64_t row_check_blocks(int32_t n) { return ((int64_t)n + kBlock - 1) / kBlock; }

hipError_t launch_check_rows(const int32_t* row_ptr, int32_t n, int64_t nnz, int32_t threshold, uint32_t* err,
                             int32_t* counters, int2* partial, int32_t* ids, int4* recs, int32_t cap,
                             hipStream_t s) {
  const int32_t blocks = (int32_t)row_check_blocks(n);
  hipLaunchKernelGGL(k_row_counts, dim3(blocks), dim3(kBlock), 0, s, row_ptr, n, nnz, threshold, err, partial);
  hipLaunchKernelGGL(k_row_offsets, dim3(1), dim3(kScanBlock), 0, s, partial, blocks, counters);
  hipLaunchKernelGGL(k_row_select, dim3(blocks), dim3(kBlock), 0, s, row_ptr, n, nnz, threshold, partial, ids, recs,
                     cap);
  return hipGetLastError();
}

hipError_t launch_mirror(const int32_t* row_ptr, const int32_t* col, int32_t n, int64_t nnz, int32_t* mirror,
                         int32_t* row_of, uint32_t* err, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_of, dim3((unsigned)row_check_blocks(n)), dim3(kBlock), 0, s, row_ptr, n, row_of, err);
  hipLaunchKernelGGL(k_mirror, dim3(blocks_for((nnz + kMirrorPer - 1) / kMirrorPer)), dim3(kBlock), 0, s, row_ptr, col,
                     n, nnz, mirror, row_of, err);
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
