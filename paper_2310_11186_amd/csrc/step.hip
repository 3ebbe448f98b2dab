// Per-step kernels of the t-SGNE loop: all-pairs Student-t repulsion with its
// normaliser Z (eq. (4)), the sparse attraction over graph edges, the gradient
// of eq. (5) and the momentum/gains update, and KL(P || Q).
//
// Repulsion tiling.  Positions are cut into nb blocks of T = 64 * R.  A work
// item is one tile (a, b) processed by one wave; each lane keeps R "resident"
// rows of block a in registers.
//  - Symmetric tiles (a < b): the 64-position sub-blocks of b travel around the
//    wave (a DPP rotation by one lane per step), so every unordered pair
//    (i, j) is met exactly once; w_ij is computed once and its force is added
//    to the resident row (+) and to the travelling column (-).  After 64 steps
//    each travelling position is back in its own lane with its column sum.
//  - Direct tiles (every tile of the direct variant): columns of b are read as
//    wave-uniform values and each ordered pair is computed by the row's lane;
//    the i == j term is masked by index.  Diagonal tiles of the symmetric
//    variant use the same scheme one resident row at a time.
// Each tile writes its row sums to part[a][b] and (symmetric) its column sums
// to part[b][a], so part[k][*] holds every contribution to block k exactly
// once and the update kernel adds them in a fixed order: results do not
// depend on scheduling.  Z partials are per tile.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ float rotate_lanes(float v) {
  // wave_ror:1 -- every lane takes the value of its neighbour on a 64-lane
  // ring.  Every source lane exists, so the "old" operand is never used; passing
  // the value itself lets the move happen in place.
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0x13C, 0xF, 0xF, false));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// The same rotation for a value read once, by the instruction that consumes
// it.  With a constant "old" operand (never used: every source lane exists)
// the compiler folds the move into that instruction as its DPP source, so the
// rotation costs no instruction of its own.
__device__ __forceinline__ float rotate_lanes_once(float v) {
  const int b = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, b, 0x13C, 0xF, 0xF, false));
}

// w = 1 / (1 + dx^2 + dy^2) with the hardware reciprocal (q >= 1, <= 1 ulp).
__device__ __forceinline__ float student_w(float dx, float dy) {
  return __builtin_amdgcn_rcpf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1.0f)));
}

// One step of a symmetric tile: the R resident rows of this lane against the
// travelling column now in it.  The step's Z terms go on the chain zs;
// OPENS starts that chain at the first weight rather than adding it to +0
// (an add the compiler must keep, as -0 + 0 = +0; no weight is -0).
// FORCES = false keeps only the Z terms (the same weights, added in the same
// order, so Z is bitwise the one the force pass gives).
template <int R, bool MASKED, bool OPENS, bool FORCES = true>
__device__ __forceinline__ void sym_step(const float (&yix)[R], const float (&yiy)[R], float (&rix)[R],
                                         float (&riy)[R], float& tx, float& ty, float& fx, float& fy, float& m,
                                         float& zs) {
  float sx = 0.f, sy = 0.f;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float dx = yix[r] - tx, dy = yiy[r] - ty;
    float w = student_w(dx, dy);
    if (MASKED) w *= m;
    zs = (OPENS && r == 0) ? w : zs + w;
    if (FORCES) {
      const float w2 = w * w;
      rix[r] = __builtin_fmaf(w2, dx, rix[r]);
      riy[r] = __builtin_fmaf(w2, dy, riy[r]);
      sx = __builtin_fmaf(w2, dx, sx);
      sy = __builtin_fmaf(w2, dy, sy);
    }
  }
  // the column's travelling force trails it by one lane: carried across
  // and reduced in one instruction
  if (FORCES) {
    fx = rotate_lanes_once(fx) - sx;
    fy = rotate_lanes_once(fy) - sy;
  }
  tx = rotate_lanes(tx);
  ty = rotate_lanes(ty);
  if (MASKED) m = rotate_lanes(m);
}

// A 64-step pass of a symmetric tile (a < b; block a is always full,
// a < nb - 1).  Accumulation is two-level to keep FP32 chains short: the
// travelling sum of one step (R terms) is formed apart and then added, the
// resident sums are folded into a second FP32 sum after every pass, and Z is
// summed in FP32 over two steps (2R terms) before its FP64 sum.
template <int R, bool SPLIT, bool MASKED, bool FORCES = true>
__device__ __forceinline__ void sym_pass(const float (&yix)[R], const float (&yiy)[R], float (&rix)[R],
                                         float (&riy)[R], float& tx, float& ty, float& fx, float& fy, float& m,
                                         double& z64, float& z32) {
  for (int s = 0; s < kWave; s += 2) {
    float zs;
    sym_step<R, MASKED, true, FORCES>(yix, yiy, rix, riy, tx, ty, fx, fy, m, zs);
    sym_step<R, MASKED, false, FORCES>(yix, yiy, rix, riy, tx, ty, fx, fy, m, zs);
    if (SPLIT) z64 += (double)zs; else z32 += zs;
  }
  // after the last step the forces are one lane short of their columns
  if (FORCES) {
    fx = rotate_lanes(fx);
    fy = rotate_lanes(fy);
  }
}

template <int R, bool SPLIT, bool FORCES = true>
__device__ __forceinline__ void tile_symmetric(const float2* __restrict__ Y, int32_t n, int32_t nb, int32_t a, int32_t b,
                               float2* __restrict__ part, double* __restrict__ zpart, float* __restrict__ zpart32,
                               int64_t item, int lane) {
  constexpr int T = kWave * R;
  const int32_t valid_b = min(T, n - b * T);
  float yix[R], yiy[R], rix[R], riy[R], hix[R], hiy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float2 v = Y[(int64_t)a * T + r * kWave + lane];
    yix[r] = v.x;
    yiy[r] = v.y;
    rix[r] = riy[r] = hix[r] = hiy[r] = 0.f;
  }
  double z64 = 0.0;
  float z32 = 0.f;
  for (int q = 0; q < R; ++q) {
    if (q * kWave >= valid_b) break;  // wave-uniform
    const int jl = q * kWave + lane;
    const bool vj = jl < valid_b;
    const float2 v = vj ? Y[(int64_t)b * T + jl] : make_float2(0.f, 0.f);
    float tx = v.x, ty = v.y, fx = 0.f, fy = 0.f;
    // partially valid sub-block (last block only): the mask travels with its position
    float m = vj ? 1.f : 0.f;
    if (q * kWave + kWave <= valid_b)
      sym_pass<R, SPLIT, false, FORCES>(yix, yiy, rix, riy, tx, ty, fx, fy, m, z64, z32);
    else
      sym_pass<R, SPLIT, true, FORCES>(yix, yiy, rix, riy, tx, ty, fx, fy, m, z64, z32);
    if (FORCES) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        hix[r] += rix[r];
        hiy[r] += riy[r];
        rix[r] = riy[r] = 0.f;
      }
      if (vj) part[((int64_t)b * nb + a) * T + jl] = make_float2(fx, fy);
    }
  }
  if (FORCES) {
#pragma unroll
    for (int r = 0; r < R; ++r) part[((int64_t)a * nb + b) * T + r * kWave + lane] = make_float2(hix[r], hiy[r]);
  }
  // every unordered pair stands for the two ordered pairs of Z
  if (SPLIT) {
    const double z = wave_sum(z64);
    if (lane == 0) zpart[item] = 2.0 * z;
  } else {
    const float z = wave_sum(z32);
    if (lane == 0) zpart32[item] = 2.0f * z;
  }
}

// Direct tile: rows of block a against every valid column of block b.
// SELF (a == b) masks the i == j term by index; MASK_I masks rows past n
// (only the last block is partial).  Full off-diagonal tiles run unmasked.
template <int R, bool SPLIT, bool SELF, bool MASK_I, bool FORCES>
__device__ __forceinline__ void tile_direct_body(const float2* __restrict__ Y, int32_t n, int32_t nb, int32_t a, int32_t b,
                                 float2* __restrict__ part, double* __restrict__ zpart, float* __restrict__ zpart32,
                                 int64_t item, int lane) {
  constexpr int T = kWave * R;
  const int32_t valid_a = min(T, n - a * T);
  const int32_t valid_b = min(T, n - b * T);
  float yix[R], yiy[R], rix[R], riy[R], hix[R], hiy[R];
  bool vi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int il = r * kWave + lane;
    vi[r] = !MASK_I || il < valid_a;
    const float2 v = vi[r] ? Y[(int64_t)a * T + il] : make_float2(0.f, 0.f);
    yix[r] = v.x;
    yiy[r] = v.y;
    rix[r] = riy[r] = hix[r] = hiy[r] = 0.f;
  }
  const float2* __restrict__ Yb = Y + (int64_t)b * T;
  double z64 = 0.0;
  float z32 = 0.f;
  // columns in chunks of 64, each chunk's row sums folded into a second sum
  for (int j0 = 0; j0 < valid_b; j0 += kWave) {
    const int j1 = min(j0 + kWave, valid_b);
    for (int jl = j0; jl < j1; ++jl) {
      const float2 v = Yb[jl];
      float zs = 0.f;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float dx = yix[r] - v.x, dy = yiy[r] - v.y;
        float w = student_w(dx, dy);
        if (SELF || MASK_I) {
          const bool keep = vi[r] && !(SELF && jl == r * kWave + lane);
          w = keep ? w : 0.f;
        }
        zs += w;
        if (FORCES) {
          const float w2 = w * w;
          rix[r] = __builtin_fmaf(w2, dx, rix[r]);
          riy[r] = __builtin_fmaf(w2, dy, riy[r]);
        }
      }
      if (SPLIT) z64 += (double)zs; else z32 += zs;
    }
    if (FORCES) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        hix[r] += rix[r];
        hiy[r] += riy[r];
        rix[r] = riy[r] = 0.f;
      }
    }
  }
  if (FORCES) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (vi[r]) part[((int64_t)a * nb + b) * T + r * kWave + lane] = make_float2(hix[r], hiy[r]);
  }
  if (SPLIT) {
    const double z = wave_sum(z64);
    if (lane == 0) zpart[item] = z;
  } else {
    const float z = wave_sum(z32);
    if (lane == 0) zpart32[item] = z;
  }
}

template <int R, bool SPLIT, bool FORCES = true>
__device__ __forceinline__ void tile_direct(const float2* __restrict__ Y, int32_t n, int32_t nb, int32_t a, int32_t b,
                            float2* __restrict__ part, double* __restrict__ zpart, float* __restrict__ zpart32,
                            int64_t item, int lane) {
  const bool partial_a = (int64_t)(a + 1) * (kWave * R) > n;
  if (a == b) {
    if (partial_a) tile_direct_body<R, SPLIT, true, true, FORCES>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
    else tile_direct_body<R, SPLIT, true, false, FORCES>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
  } else {
    if (partial_a) tile_direct_body<R, SPLIT, false, true, FORCES>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
    else tile_direct_body<R, SPLIT, false, false, FORCES>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
  }
}

// Diagonal tile (a, a) inside the symmetric kernel: one resident row per lane
// per pass (few registers, so the symmetric path keeps its occupancy), every
// ordered pair i != j, four interleaved partial sums per coordinate.
template <int R, bool SPLIT, bool FORCES = true>
__device__ __forceinline__ void tile_diag_light(const float2* __restrict__ Y, int32_t n, int32_t nb, int32_t a,
                                float2* __restrict__ part, double* __restrict__ zpart, float* __restrict__ zpart32,
                                int64_t item, int lane) {
  constexpr int T = kWave * R;
  const int32_t valid = min(T, n - a * T);
  const float2* __restrict__ Ya = Y + (int64_t)a * T;
  double z64 = 0.0;
  float z32 = 0.f;
  for (int r = 0; r < R; ++r) {
    const int il = r * kWave + lane;
    if (r * kWave >= valid) break;  // wave-uniform
    const bool vi = il < valid;
    const float2 yi = vi ? Ya[il] : make_float2(0.f, 0.f);
    float hx = 0.f, hy = 0.f;
    for (int j0 = 0; j0 < valid; j0 += kWave) {
      const int j1 = min(j0 + kWave, valid);
      float ax[4] = {0.f, 0.f, 0.f, 0.f}, ay[4] = {0.f, 0.f, 0.f, 0.f}, az[4] = {0.f, 0.f, 0.f, 0.f};
      int jl = j0;
      for (; jl + 4 <= j1; jl += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float2 v = Ya[jl + k];
          const float dx = yi.x - v.x, dy = yi.y - v.y;
          float w = student_w(dx, dy);
          w = (vi && jl + k != il) ? w : 0.f;
          az[k] += w;
          if (FORCES) {
            const float w2 = w * w;
            ax[k] = __builtin_fmaf(w2, dx, ax[k]);
            ay[k] = __builtin_fmaf(w2, dy, ay[k]);
          }
        }
      }
      for (; jl < j1; ++jl) {
        const float2 v = Ya[jl];
        const float dx = yi.x - v.x, dy = yi.y - v.y;
        float w = student_w(dx, dy);
        w = (vi && jl != il) ? w : 0.f;
        az[0] += w;
        if (FORCES) {
          const float w2 = w * w;
          ax[0] = __builtin_fmaf(w2, dx, ax[0]);
          ay[0] = __builtin_fmaf(w2, dy, ay[0]);
        }
      }
      if (FORCES) {
        hx += (ax[0] + ax[1]) + (ax[2] + ax[3]);
        hy += (ay[0] + ay[1]) + (ay[2] + ay[3]);
      }
      const float zc = (az[0] + az[1]) + (az[2] + az[3]);
      if (SPLIT) z64 += (double)zc; else z32 += zc;
    }
    if (FORCES && vi) part[((int64_t)a * nb + a) * T + il] = make_float2(hx, hy);
  }
  if (SPLIT) {
    const double z = wave_sum(z64);
    if (lane == 0) zpart[item] = z;
  } else {
    const float z = wave_sum(z32);
    if (lane == 0) zpart32[item] = z;
  }
}

// Waves per SIMD the repulsion kernels must allow.  With few rows per lane a
// step holds too few independent pairs to hide the dependent-issue latency
// at the 4 waves per SIMD the compiler's default register budget gives
// (measured with R = 8: 37 % more cycles waiting on dependencies than R = 16
// for 4 % more VALU instructions).  Asking for 6 keeps R = 8 at 69 VGPRs
// (7 waves per SIMD) and 5 keeps R = 12 at 93 (5 waves), both without
// spills; R >= 14 would spill below 4 waves and keeps the default.
template <int R>
constexpr int repulse_min_waves() {
  return R <= 8 ? 6 : R <= 12 ? 5 : 1;
}

template <int R, bool SPLIT, bool SYM>
__global__ __launch_bounds__(kBlock, repulse_min_waves<R>()) void k_repulse(const float2* __restrict__ Y, int32_t n, int32_t nb,
                                                    const int2* __restrict__ items, int64_t n_items,
                                                    float2* __restrict__ part, double* __restrict__ zpart,
                                                    float* __restrict__ zpart32) {
  const int64_t item =
      (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (item >= n_items) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int2 ab = items[item];
  const int32_t a = __builtin_amdgcn_readfirstlane(ab.x), b = __builtin_amdgcn_readfirstlane(ab.y);
  if (SYM) {
    if (a != b) tile_symmetric<R, SPLIT>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
    else tile_diag_light<R, SPLIT>(Y, n, nb, a, part, zpart, zpart32, item, lane);
  } else {
    tile_direct<R, SPLIT>(Y, n, nb, a, b, part, zpart, zpart32, item, lane);
  }
}

// Z alone (no forces, no partials written): the weights and their sums in the
// order k_repulse uses, so the Z partials are bitwise those of the force pass.
template <int R, bool SPLIT, bool SYM>
__global__ __launch_bounds__(kBlock, repulse_min_waves<R>()) void k_zonly(const float2* __restrict__ Y, int32_t n,
                                                                          int32_t nb, const int2* __restrict__ items,
                                                                          int64_t n_items, double* __restrict__ zpart,
                                                                          float* __restrict__ zpart32) {
  const int64_t item =
      (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (item >= n_items) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int2 ab = items[item];
  const int32_t a = __builtin_amdgcn_readfirstlane(ab.x), b = __builtin_amdgcn_readfirstlane(ab.y);
  if (SYM) {
    if (a != b) tile_symmetric<R, SPLIT, false>(Y, n, nb, a, b, nullptr, zpart, zpart32, item, lane);
    else tile_diag_light<R, SPLIT, false>(Y, n, nb, a, nullptr, zpart, zpart32, item, lane);
  } else {
    tile_direct<R, SPLIT, false>(Y, n, nb, a, b, nullptr, zpart, zpart32, item, lane);
  }
}

template <int R>
hipError_t launch_zonly_r(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s) {
  const RepulsionPlan& p = ws.plan;
  const dim3 grid((unsigned)((p.items + kWavesPerBlock - 1) / kWavesPerBlock));
  const bool split = precision != TSGNE_PREC_FP32;
  const bool sym = p.variant == TSGNE_REPULSION_SYMMETRIC;
  if (split && sym)
    hipLaunchKernelGGL((k_zonly<R, true, true>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.zpart,
                       ws.zpart32);
  else if (split)
    hipLaunchKernelGGL((k_zonly<R, true, false>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.zpart,
                       ws.zpart32);
  else if (sym)
    hipLaunchKernelGGL((k_zonly<R, false, true>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.zpart,
                       ws.zpart32);
  else
    hipLaunchKernelGGL((k_zonly<R, false, false>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items,
                       ws.zpart, ws.zpart32);
  return hipGetLastError();
}

template <int R>
hipError_t launch_repulsion_r(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s) {
  const RepulsionPlan& p = ws.plan;
  const dim3 grid((unsigned)((p.items + kWavesPerBlock - 1) / kWavesPerBlock));
  const bool split = precision != TSGNE_PREC_FP32;
  const bool sym = p.variant == TSGNE_REPULSION_SYMMETRIC;
  if (split && sym)
    hipLaunchKernelGGL((k_repulse<R, true, true>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.part,
                       ws.zpart, ws.zpart32);
  else if (split)
    hipLaunchKernelGGL((k_repulse<R, true, false>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.part,
                       ws.zpart, ws.zpart32);
  else if (sym)
    hipLaunchKernelGGL((k_repulse<R, false, true>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items, ws.part,
                       ws.zpart, ws.zpart32);
  else
    hipLaunchKernelGGL((k_repulse<R, false, false>), grid, dim3(kBlock), 0, s, Y, n, p.nb, ws.items, p.items,
                       ws.part, ws.zpart, ws.zpart32);
  return hipGetLastError();
}

// Z = sum of the tile partials, one workgroup, fixed order (strided partial
// sums then a tree in LDS).
constexpr int kZThreads = 1024;

template <bool SPLIT>
__device__ __forceinline__ void zsum_block(const double* __restrict__ zpart, const float* __restrict__ zpart32, int64_t n_items,
                           double* __restrict__ Z) {
  __shared__ double sh64[kZThreads];
  __shared__ float sh32[kZThreads];
  const int t = threadIdx.x;
  // Each thread keeps kZLoads independent sums, so that kZLoads loads are in
  // flight at once (a single running sum waits for every load in turn: 25 µs
  // for the 25K tiles of a 200K-node graph), then adds them in a fixed order.
  constexpr int kZLoads = 8;
  const int64_t stride = (int64_t)kZThreads * kZLoads;
  if (SPLIT) {
    double acc[kZLoads] = {};
    int64_t k = t;
    for (; k + (kZLoads - 1) * (int64_t)kZThreads < n_items; k += stride) {
      double v[kZLoads];
#pragma unroll
      for (int u = 0; u < kZLoads; ++u) v[u] = zpart[k + u * kZThreads];
#pragma unroll
      for (int u = 0; u < kZLoads; ++u) acc[u] += v[u];
    }
    for (int u = 0; k < n_items; k += kZThreads, ++u) acc[u] += zpart[k];   // fewer than kZLoads left
    sh64[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  } else {
    float acc[kZLoads] = {};
    int64_t k = t;
    for (; k + (kZLoads - 1) * (int64_t)kZThreads < n_items; k += stride) {
      float v[kZLoads];
#pragma unroll
      for (int u = 0; u < kZLoads; ++u) v[u] = zpart32[k + u * kZThreads];
#pragma unroll
      for (int u = 0; u < kZLoads; ++u) acc[u] += v[u];
    }
    for (int u = 0; k < n_items; k += kZThreads, ++u) acc[u] += zpart32[k];
    sh32[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  static_assert(kZLoads == 8, "the fixed-order combination above adds eight sums");
  __syncthreads();
  for (int w = kZThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      if (SPLIT) sh64[t] += sh64[t + w]; else sh32[t] += sh32[t + w];
    }
    __syncthreads();
  }
  if (t == 0) *Z = SPLIT ? sh64[0] : (double)sh32[0];
}

// tstep (nullable) is the device step counter of a run: {next step, step being
// run}.  The Z sum, the one single-workgroup kernel of a step and the first
// after the repulsion, takes the step's index from it for the kernels after it.
template <bool SPLIT>
__global__ __launch_bounds__(kZThreads) void k_zsum(const double* __restrict__ zpart, const float* __restrict__ zpart32,
                                                    int64_t n_items, double* __restrict__ Z,
                                                    int32_t* __restrict__ tstep) {
  zsum_block<SPLIT>(zpart, zpart32, n_items, Z);
  if (tstep && threadIdx.x == 0) {
    const int32_t t = tstep[0];
    tstep[1] = t;
    tstep[0] = t + 1;
  }
}

// Attraction sum_j p_ij w_ij (y_i - y_j) over the stored entries of row i
// (the p-part of the gradient of eq. (5); alpha is applied in the update).
// Light rows: eight lanes per row.  Heavy rows: one wave per row.
constexpr int kRowLanes = kAttractRowLanes;
constexpr uint32_t kXcds = 8;  // XCDs of an MI355X (gfx950)

template <int LANES, bool SPLIT>
__device__ __forceinline__ void attract_row(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                            const float* __restrict__ P, const float2* __restrict__ Y, int32_t i,
                                            int sub, double2* __restrict__ out) {
  constexpr int U = 4;  // entries per lane whose loads are issued together
  const int32_t b = row_ptr[i], e_end = row_ptr[i + 1];
  const float2 yi = Y[i];
  double ax = 0.0, ay = 0.0;
  float fx = 0.f, fy = 0.f;
  for (int32_t e0 = b + sub; e0 < e_end; e0 += U * LANES) {
    int32_t j[U];
    float p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = e0 + u * LANES;
      j[u] = e < e_end ? col[e] : i;
      p[u] = e < e_end ? P[e] : 0.f;
    }
    float2 yj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) yj[u] = Y[j[u]];
    // entries in increasing order per lane, exactly as a one-at-a-time loop.
    // An entry past the row's end (j = i, p = 0) adds exactly +0, which leaves
    // a sum started at +0 unchanged; with no branch here the gathers of Y are
    // all issued before the first is used (a branch would put each behind its
    // own check and wait).
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float dx = yi.x - yj[u].x, dy = yi.y - yj[u].y;
      const float pw = p[u] * student_w(dx, dy);
      if (SPLIT) {
        ax += (double)(pw * dx);
        ay += (double)(pw * dy);
      } else {
        fx = __builtin_fmaf(pw, dx, fx);
        fy = __builtin_fmaf(pw, dy, fy);
      }
    }
  }
  if (!SPLIT) {
    ax = fx;
    ay = fy;
  }
  for (int off = LANES / 2; off > 0; off >>= 1) {
    if (SPLIT) {
      ax += __shfl_xor(ax, off, LANES);
      ay += __shfl_xor(ay, off, LANES);
    } else {
      fx += __shfl_xor(fx, off, LANES);
      fy += __shfl_xor(fy, off, LANES);
    }
  }
  if (!SPLIT) {
    ax = fx;
    ay = fy;
  }
  if (sub == 0) out[i] = make_double2(ax, ay);
}

template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_attract_light(const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, const float* __restrict__ P,
                                                          const float2* __restrict__ Y, int32_t n,
                                                          double2* __restrict__ out) {
  // Blocks are dealt to the XCDs in turn; renumber them so that each XCD
  // takes one contiguous range of rows, and its L2 sees the neighbours of
  // nearby rows (the grid is a multiple of kXcds).
  const uint32_t per_xcd = gridDim.x / kXcds;
  const uint32_t block = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const int64_t t = (int64_t)block * kBlock + threadIdx.x;
  const int32_t i = (int32_t)min<int64_t>(t / kRowLanes, n - 1);
  const bool live = t / kRowLanes < n && (row_ptr[i + 1] - row_ptr[i]) <= kHeavyDegree;
  // whole 8-lane groups share `live`, so the shuffles inside stay in step
  if (live) attract_row<kRowLanes, SPLIT>(row_ptr, col, P, Y, i, (int)(threadIdx.x & (kRowLanes - 1)), out);
}

template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_attract_heavy(const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col, const float* __restrict__ P,
                                                          const float2* __restrict__ Y,
                                                          const int32_t* __restrict__ heavy, int32_t n_heavy,
                                                          double2* __restrict__ out) {
  const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  if (w >= n_heavy) return;
  attract_row<kWave, SPLIT>(row_ptr, col, P, Y, heavy[w], (int)(threadIdx.x & (kWave - 1)), out);
}

// g_i = 4 (alpha * A_i - R_i / Z), then the momentum/gains update of row i.
template <bool SPLIT>
__device__ __forceinline__ void update_row(const float2* __restrict__ part, int32_t nb, int32_t T,
                                           const double2* __restrict__ attract, double Z, int32_t i,
                                           float2* __restrict__ Y, float2* __restrict__ U, float2* __restrict__ G,
                                           float alpha, float momentum, float eta, float min_gain, bool do_update,
                                           float2* __restrict__ grad_out) {
  const int32_t k = i / T, off = i - k * T;
  const float2* __restrict__ pp = part + (int64_t)k * nb * T + off;
  double rx = 0.0, ry = 0.0;
  float sx = 0.f, sy = 0.f;
  // Partials are read in batches of kBatchLoads whose loads are all issued
  // before the first is added.  The loop body has no branch (a branch around
  // a load makes the compiler wait for it before the next one is issued), so
  // past the last block an index is clamped to it: an in-bounds re-read that
  // adds +0, which leaves a sum started at +0 unchanged.
  constexpr int kBatchLoads = 32;
  for (int32_t o0 = 0; o0 < nb; o0 += kBatchLoads) {
    float2 v[kBatchLoads];
#pragma unroll
    for (int u = 0; u < kBatchLoads; ++u) v[u] = pp[(int64_t)min(o0 + u, nb - 1) * T];
    // added in block order, exactly as a one-at-a-time loop
    const int32_t count = nb - o0;
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
  const double2 A = attract[i];
  float2 g;
  if (SPLIT) {
    const double invZ = Z > 0.0 ? 1.0 / Z : 0.0;
    g.x = (float)(4.0 * ((double)alpha * A.x - rx * invZ));
    g.y = (float)(4.0 * ((double)alpha * A.y - ry * invZ));
  } else {
    const float invZ = Z > 0.0 ? (float)(1.0 / Z) : 0.f;
    g.x = 4.0f * (alpha * (float)A.x - sx * invZ);
    g.y = 4.0f * (alpha * (float)A.y - sy * invZ);
  }
  if (grad_out) grad_out[i] = g;
  if (!do_update) return;
  float2 y = Y[i], u = U[i], gn = G[i];
  gn.x = (g.x * u.x < 0.f) ? gn.x + 0.2f : gn.x * 0.8f;
  gn.y = (g.y * u.y < 0.f) ? gn.y + 0.2f : gn.y * 0.8f;
  gn.x = fmaxf(gn.x, min_gain);
  gn.y = fmaxf(gn.y, min_gain);
  u.x = momentum * u.x - eta * gn.x * g.x;
  u.y = momentum * u.y - eta * gn.y * g.y;
  y.x += u.x;
  y.y += u.y;
  Y[i] = y;
  U[i] = u;
  G[i] = gn;
}

// With sched.tstep set, alpha and the momentum come from the step index on the
// device (early exaggeration while t < t_ee), so that a captured step can be
// replayed; otherwise the host's values are used.
template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_update(const float2* __restrict__ part, int32_t nb, int32_t T,
                                                   const double2* __restrict__ attract, const double* __restrict__ Zp,
                                                   int32_t n, float2* __restrict__ Y, float2* __restrict__ U,
                                                   float2* __restrict__ G, float alpha, float momentum, float eta,
                                                   float min_gain, int do_update, float2* __restrict__ grad_out,
                                                   StepSchedule sched) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (sched.tstep) {
    const bool early = sched.tstep[1] < sched.exaggeration_iters;
    alpha = early ? sched.early_exaggeration : 1.0f;
    momentum = early ? sched.momentum_early : sched.momentum_late;
  }
  update_row<SPLIT>(part, nb, T, attract, *Zp, i, Y, U, G, alpha, momentum, eta, min_gain, do_update != 0, grad_out);
}

// ---------------------------------------------------------------------------
// Batched step over many graphs.  Every graph keeps its own tiling, item
// order, partial buffers and reduction order, so a graph advanced inside a
// batch computes exactly what it computes alone with the same tile size.  Each
// graph's step index lives in device memory (advanced by the last kernel of a
// step), so a captured step can be replayed and graphs at different progress
// can share a launch; graphs with t >= n_iter are skipped.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool batch_live(const BatchDesc& d) {
  const int32_t t = *d.t;
  return t < d.n_iter && t < *d.limit;
}

template <int R, bool SPLIT>
__global__ __launch_bounds__(kBlock, repulse_min_waves<R>()) void k_batch_repulse(const BatchDesc* __restrict__ descs,
                                                          const int4* __restrict__ items, int64_t n_items) {
  const int64_t item =
      (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (item >= n_items) return;
  const int4 it = items[item];
  const int32_t gi = __builtin_amdgcn_readfirstlane(it.x);
  const BatchDesc& d = descs[gi];
  if (!batch_live(d)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t a = __builtin_amdgcn_readfirstlane(it.y), b = __builtin_amdgcn_readfirstlane(it.z);
  const int64_t li = __builtin_amdgcn_readfirstlane(it.w);
  if (a != b) tile_symmetric<R, SPLIT>(d.Y, d.n, d.nb, a, b, d.part, d.zpart, d.zpart32, li, lane);
  else tile_diag_light<R, SPLIT>(d.Y, d.n, d.nb, a, d.part, d.zpart, d.zpart32, li, lane);
}

template <bool SPLIT>
__global__ __launch_bounds__(kZThreads) void k_batch_zsum(const BatchDesc* __restrict__ descs) {
  const BatchDesc& d = descs[blockIdx.x];
  if (!batch_live(d)) return;
  zsum_block<SPLIT>(d.zpart, d.zpart32, d.n_items, d.Z);
}

// One block of 256 threads covers kBlock / kRowLanes light rows of one graph.
template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_batch_attract_light(const BatchDesc* __restrict__ descs,
                                                                const int2* __restrict__ chunks) {
  const int2 ch = chunks[blockIdx.x];
  const BatchDesc& d = descs[ch.x];
  if (!batch_live(d)) return;
  const int32_t i0 = ch.y + (int32_t)(threadIdx.x / kRowLanes);
  const int32_t i = min(i0, d.n - 1);
  const bool live = i0 < d.n && (d.row_ptr[i + 1] - d.row_ptr[i]) <= kHeavyDegree;
  if (live) attract_row<kRowLanes, SPLIT>(d.row_ptr, d.col, d.P, d.Y, i, (int)(threadIdx.x & (kRowLanes - 1)),
                                          d.attract);
}

template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_batch_attract_heavy(const BatchDesc* __restrict__ descs,
                                                                const int2* __restrict__ heavy, int32_t n_heavy) {
  const int32_t w = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  if (w >= n_heavy) return;
  const int2 hr = heavy[w];
  const BatchDesc& d = descs[hr.x];
  if (!batch_live(d)) return;
  attract_row<kWave, SPLIT>(d.row_ptr, d.col, d.P, d.Y, hr.y, (int)(threadIdx.x & (kWave - 1)), d.attract);
}

// One block of 256 threads covers 256 rows of one graph.
template <bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_batch_update(const BatchDesc* __restrict__ descs,
                                                         const int2* __restrict__ blocks, int32_t T, float ee,
                                                         int32_t t_ee, float m_early, float m_late, float min_gain) {
  const int2 bl = blocks[blockIdx.x];
  const BatchDesc& d = descs[bl.x];
  if (!batch_live(d)) return;
  const int32_t t = *d.t;
  const int32_t i = bl.y + (int32_t)threadIdx.x;
  if (i >= d.n) return;
  const bool early = t < t_ee;
  update_row<SPLIT>(d.part, d.nb, T, d.attract, *d.Z, i, d.Y, d.U, d.G, early ? ee : 1.0f, early ? m_early : m_late,
                    d.eta, min_gain, true, nullptr);
}

__global__ __launch_bounds__(kBlock) void k_batch_advance(const BatchDesc* __restrict__ descs, int32_t count) {
  const int32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g < count && batch_live(descs[g])) *descs[g].t += 1;
}

// KL = sum_e P_e log(P_e / q_e), q_e = w_e / Z, in FP64: fixed grid, strided
// per-thread sums, tree per block, then one block over the block sums.
constexpr int kKLThreads = 256;

// KL sampling inside a run (trace != nullptr): the step being run (tstep[1])
// holds the layout after t steps; it is sampled when t is a positive multiple
// of kl_every, into trace[t / kl_every - 1], with the Z this step has just
// summed at that layout.  Other steps return at once.
__device__ __forceinline__ bool kl_skip(const int32_t* tstep, int32_t kl_every) {
  if (!tstep) return false;
  const int32_t t = tstep[1];
  return t <= 0 || t % kl_every != 0;
}

__global__ __launch_bounds__(kKLThreads) void k_kl_edges(const int32_t* __restrict__ row_of,
                                                         const int32_t* __restrict__ col, const float* __restrict__ P,
                                                         const float2* __restrict__ Y, int64_t nnz,
                                                         const double* __restrict__ Zp, double* __restrict__ klpart,
                                                         const int32_t* __restrict__ tstep, int32_t kl_every) {
  if (kl_skip(tstep, kl_every)) return;
  __shared__ double sh[kKLThreads];
  const double logZ = *Zp > 0.0 ? log(*Zp) : 0.0;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kKLThreads;
  for (int64_t e = (int64_t)blockIdx.x * kKLThreads + threadIdx.x; e < nnz; e += stride) {
    const double p = P[e];
    if (p <= 0.0) continue;
    const float2 yi = Y[row_of[e]], yj = Y[col[e]];
    const double dx = (double)yi.x - (double)yj.x, dy = (double)yi.y - (double)yj.y;
    acc += p * (log(p) + logZ + log1p(dx * dx + dy * dy));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kKLThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) klpart[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kKLThreads) void k_kl_final(const double* __restrict__ klpart, int32_t nparts,
                                                         double* __restrict__ out, const int32_t* __restrict__ tstep,
                                                         int32_t kl_every, double* __restrict__ trace) {
  if (kl_skip(tstep, kl_every)) return;
  __shared__ double sh[kKLThreads];
  double acc = 0.0;
  for (int32_t k = threadIdx.x; k < nparts; k += kKLThreads) acc += klpart[k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kKLThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out = sh[0];
    if (trace) trace[tstep ? tstep[1] / kl_every - 1 : 0] = sh[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_nonfinite(const float2* __restrict__ Y, int32_t n,
                                                      uint32_t* __restrict__ flag) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float2 y = Y[i];
  if (!isfinite(y.x) || !isfinite(y.y)) atomicOr(flag, 1u);
}

inline unsigned blocks_for(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

// SIMDs of the chip (256 CUs x 4).
constexpr int64_t kSimds = 1024;
// Largest graphs that take 1 and 2 rows per lane automatically (see make_plan).
constexpr int32_t kOneRowMaxNodes = 3500;
constexpr int32_t kTwoRowMaxNodes = 11000;

RepulsionPlan make_plan(int32_t n, int32_t R, int32_t variant) {
  RepulsionPlan p;
  p.variant = (variant == TSGNE_REPULSION_DIRECT) ? TSGNE_REPULSION_DIRECT : TSGNE_REPULSION_SYMMETRIC;
  auto items_for = [&](int32_t r) {
    const int64_t nb = (n + kWave * r - 1) / (kWave * r);
    return p.variant == TSGNE_REPULSION_DIRECT ? nb * nb : nb * (nb + 1) / 2;
  };
  // Small graphs have too few tiles of 4 or more rows to fill the chip: a
  // layout step is then set by one tile's latency, and smaller tiles win in
  // spite of their lower per-pair efficiency.  Crossovers measured on MI355X
  // over whole layout steps (repulsion, Z sum, update): 1 row per lane up to
  // about 3,500 nodes (2,000 nodes: 17.7 ms for P and 300 steps against 27.8 ms with
  // 4 rows), 2 rows up to about 11,000 (5,000 nodes: 24.3 against 31.0 ms),
  // and from about 11,000 nodes on the cost model below.
  if (!tile_rows_supported(R) && p.variant == TSGNE_REPULSION_SYMMETRIC) {
    if (n <= kOneRowMaxNodes) R = 1;
    else if (n <= kTwoRowMaxNodes) R = 2;
  }
  if (!tile_rows_supported(R)) {
    // Cost model: the tiles (one wave each) of the busiest SIMD, i.e. the
    // tile count over the chip's 1024 SIMDs rounded up, times the tile area,
    // divided by the per-pair efficiency of that tile relative to R = 16
    // (measured on MI355X as tile-pair slots per second of the repulsion at
    // 200K-500K nodes, where every SIMD holds 19 or more tiles: 1.004 for
    // R = 15, 0.996 for 14, 0.997 for 12, 0.969 for 8, 0.827 for 4).  A SIMD
    // needs about 64 / R resident tiles (64 independent pairs per step over
    // its waves) to hide the dependent-issue latency, so fewer tiles than that
    // take as long as that many.  Small graphs get small tiles (every SIMD
    // busy), large graphs the tile whose count divides best over the SIMDs.
    const int32_t rs[6] = {16, 15, 14, 12, 8, 4};
    const double eff[6] = {1.0, 1.004, 0.996, 0.997, 0.969, 0.827};
    double best = 0.0;
    for (int k = 0; k < 6; ++k) {
      const double T = (double)(kWave * rs[k]);
      const int64_t per_simd = std::max<int64_t>((items_for(rs[k]) + kSimds - 1) / kSimds, kWave / rs[k]);
      const double cost = (double)per_simd * T * T / eff[k];
      if (best == 0.0 || cost < best) {
        best = cost;
        R = rs[k];
      }
    }
  }
  p.R = R;
  p.T = kWave * R;
  p.nb = (n + p.T - 1) / p.T;
  p.items = items_for(R);
  return p;
}

hipError_t launch_repulsion(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s) {
  switch (ws.plan.R) {
    case 1: return launch_repulsion_r<1>(ws, n, Y, precision, s);
    case 2: return launch_repulsion_r<2>(ws, n, Y, precision, s);
    case 4: return launch_repulsion_r<4>(ws, n, Y, precision, s);
    case 8: return launch_repulsion_r<8>(ws, n, Y, precision, s);
    case 16: return launch_repulsion_r<16>(ws, n, Y, precision, s);
    case 12: return launch_repulsion_r<12>(ws, n, Y, precision, s);
    case 14: return launch_repulsion_r<14>(ws, n, Y, precision, s);
    case 15: return launch_repulsion_r<15>(ws, n, Y, precision, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zonly(const Workspace& ws, int32_t n, const float2* Y, int precision, hipStream_t s) {
  switch (ws.plan.R) {
    case 1: return launch_zonly_r<1>(ws, n, Y, precision, s);
    case 2: return launch_zonly_r<2>(ws, n, Y, precision, s);
    case 4: return launch_zonly_r<4>(ws, n, Y, precision, s);
    case 8: return launch_zonly_r<8>(ws, n, Y, precision, s);
    case 16: return launch_zonly_r<16>(ws, n, Y, precision, s);
    case 12: return launch_zonly_r<12>(ws, n, Y, precision, s);
    case 14: return launch_zonly_r<14>(ws, n, Y, precision, s);
    case 15: return launch_zonly_r<15>(ws, n, Y, precision, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zsum(const Workspace& ws, int precision, hipStream_t s, int32_t* tstep) {
  if (precision == TSGNE_PREC_FP32)
    hipLaunchKernelGGL(k_zsum<false>, dim3(1), dim3(kZThreads), 0, s, ws.zpart, ws.zpart32, ws.plan.items, ws.Z,
                       tstep);
  else
    hipLaunchKernelGGL(k_zsum<true>, dim3(1), dim3(kZThreads), 0, s, ws.zpart, ws.zpart32, ws.plan.items, ws.Z,
                       tstep);
  return hipGetLastError();
}

hipError_t launch_attract(const tsgne_graph* g, const float2* Y, int precision, double2* out, hipStream_t s) {
  const bool split = precision != TSGNE_PREC_FP32;
  const unsigned lb = blocks_for((int64_t)g->n * kRowLanes, kBlock);
  const unsigned lb8 = (lb + kXcds - 1) / kXcds * kXcds;  // whole rounds over the XCDs
  if (split)
    hipLaunchKernelGGL(k_attract_light<true>, dim3(lb8), dim3(kBlock), 0, s, g->row_ptr, g->col, g->P, Y, g->n, out);
  else
    hipLaunchKernelGGL(k_attract_light<false>, dim3(lb8), dim3(kBlock), 0, s, g->row_ptr, g->col, g->P, Y, g->n, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g->n_heavy == 0) return e;
  const unsigned hb = blocks_for(g->n_heavy, kWavesPerBlock);
  if (split)
    hipLaunchKernelGGL(k_attract_heavy<true>, dim3(hb), dim3(kBlock), 0, s, g->row_ptr, g->col, g->P, Y, g->heavy,
                       g->n_heavy, out);
  else
    hipLaunchKernelGGL(k_attract_heavy<false>, dim3(hb), dim3(kBlock), 0, s, g->row_ptr, g->col, g->P, Y, g->heavy,
                       g->n_heavy, out);
  return hipGetLastError();
}

hipError_t launch_update(const tsgne_graph* g, float2* Y, float2* U, float2* gains, float alpha, float momentum,
                         float eta, float min_gain, int precision, bool do_update, float2* grad_out, double* Z_out,
                         hipStream_t s, const StepSchedule& sched) {
  const Workspace& ws = g->ws;
  const unsigned nbk = blocks_for(g->n, kBlock);
  if (precision == TSGNE_PREC_FP32)
    hipLaunchKernelGGL(k_update<false>, dim3(nbk), dim3(kBlock), 0, s, ws.part, ws.plan.nb, ws.plan.T, ws.attract,
                       ws.Z, g->n, Y, U, gains, alpha, momentum, eta, min_gain, (int)do_update, grad_out, sched);
  else
    hipLaunchKernelGGL(k_update<true>, dim3(nbk), dim3(kBlock), 0, s, ws.part, ws.plan.nb, ws.plan.T, ws.attract,
                       ws.Z, g->n, Y, U, gains, alpha, momentum, eta, min_gain, (int)do_update, grad_out, sched);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !Z_out) return e;
  return hipMemcpyAsync(Z_out, ws.Z, sizeof(double), hipMemcpyDeviceToDevice, s);
}

hipError_t launch_kl(const tsgne_graph* g, const float2* Y, hipStream_t s, const int32_t* tstep, int32_t kl_every,
                     double* trace) {
  const Workspace& ws = g->ws;
  hipLaunchKernelGGL(k_kl_edges, dim3(ws.kl_blocks), dim3(kKLThreads), 0, s, g->row_of, g->col, g->P, Y, g->nnz, ws.Z,
                     ws.klpart, tstep, kl_every);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(kKLThreads), 0, s, ws.klpart, ws.kl_blocks, ws.klout, tstep, kl_every,
                     trace);
  return hipGetLastError();
}

hipError_t launch_kl_ws(const tsgne_graph* g, const Workspace& ws, const float2* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_kl_edges, dim3(ws.kl_blocks), dim3(kKLThreads), 0, s, g->row_of, g->col, g->P, Y, g->nnz, ws.Z,
                     ws.klpart, nullptr, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(kKLThreads), 0, s, ws.klpart, ws.kl_blocks, ws.klout, nullptr, 0,
                     nullptr);
  return hipGetLastError();
}

template <int R>
hipError_t launch_batch_repulse_r(const BatchPlan& bp, bool split, hipStream_t s) {
  const dim3 grid((unsigned)((bp.n_items + kWavesPerBlock - 1) / kWavesPerBlock));
  if (split)
    hipLaunchKernelGGL((k_batch_repulse<R, true>), grid, dim3(kBlock), 0, s, bp.descs, bp.items, bp.n_items);
  else
    hipLaunchKernelGGL((k_batch_repulse<R, false>), grid, dim3(kBlock), 0, s, bp.descs, bp.items, bp.n_items);
  return hipGetLastError();
}

hipError_t launch_batch_step(const BatchPlan& bp, const tsgne_params& p, hipStream_t s) {
  const bool split = p.precision != TSGNE_PREC_FP32;
  hipError_t e = hipSuccess;
  if (bp.n_items > 0) {
    switch (bp.R) {
      case 1: e = launch_batch_repulse_r<1>(bp, split, s); break;
      case 2: e = launch_batch_repulse_r<2>(bp, split, s); break;
      case 4: e = launch_batch_repulse_r<4>(bp, split, s); break;
      case 8: e = launch_batch_repulse_r<8>(bp, split, s); break;
      case 16: e = launch_batch_repulse_r<16>(bp, split, s); break;
      case 12: e = launch_batch_repulse_r<12>(bp, split, s); break;
      case 14: e = launch_batch_repulse_r<14>(bp, split, s); break;
      case 15: e = launch_batch_repulse_r<15>(bp, split, s); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  if (split) hipLaunchKernelGGL(k_batch_zsum<true>, dim3(bp.count), dim3(kZThreads), 0, s, bp.descs);
  else hipLaunchKernelGGL(k_batch_zsum<false>, dim3(bp.count), dim3(kZThreads), 0, s, bp.descs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (bp.n_light_chunks > 0) {
    if (split)
      hipLaunchKernelGGL(k_batch_attract_light<true>, dim3(bp.n_light_chunks), dim3(kBlock), 0, s, bp.descs,
                         bp.light_chunks);
    else
      hipLaunchKernelGGL(k_batch_attract_light<false>, dim3(bp.n_light_chunks), dim3(kBlock), 0, s, bp.descs,
                         bp.light_chunks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (bp.n_heavy > 0) {
    const unsigned hb = blocks_for(bp.n_heavy, kWavesPerBlock);
    if (split)
      hipLaunchKernelGGL(k_batch_attract_heavy<true>, dim3(hb), dim3(kBlock), 0, s, bp.descs, bp.heavy, bp.n_heavy);
    else
      hipLaunchKernelGGL(k_batch_attract_heavy<false>, dim3(hb), dim3(kBlock), 0, s, bp.descs, bp.heavy, bp.n_heavy);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (split)
    hipLaunchKernelGGL(k_batch_update<true>, dim3(bp.n_row_blocks), dim3(kBlock), 0, s, bp.descs, bp.row_blocks, bp.T,
                       p.early_exaggeration, p.exaggeration_iters, p.momentum_early, p.momentum_late, p.min_gain);
  else
    hipLaunchKernelGGL(k_batch_update<false>, dim3(bp.n_row_blocks), dim3(kBlock), 0, s, bp.descs, bp.row_blocks,
                       bp.T, p.early_exaggeration, p.exaggeration_iters, p.momentum_early, p.momentum_late,
                       p.min_gain);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_advance, dim3(blocks_for(bp.count, kBlock)), dim3(kBlock), 0, s, bp.descs, bp.count);
  return hipGetLastError();
}

hipError_t launch_nonfinite_check(const float2* Y, int32_t n, uint32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, Y, n, flag);
  return hipGetLastError();
}

}  // namespace tsgne
