// ShortestPath graph embedding (section 2.3, eq. (8)): X[i][j] is the hop
// distance from node i to target t_j when it is at most l0, otherwise l0 + 1
// (also when t_j cannot be reached).
//
// All d breadth-first searches advance together, level-synchronously, with
// one bit per target.  Per node v the device holds
//   vis[v]    -- targets that have reached v (W words of 32 bits),
//   F[v]      -- targets that reached v at the previous level (the frontier),
//   plane_k[v]-- bit k of the hop distance, for each target (bit-sliced).
// Level L pulls: N = (OR of F[u] over the neighbours u of v) & ~vis[v]; the
// bits of N get distance L, written into the planes where L has a one bit.
// A node every target has reached reads nothing.  The searches stop at
// level floor(l0) or when a level finds nothing.  A final pass decodes the
// planes into X with one coalesced write of every element, so X is written
// once and never read.
//
// Level activity is kept in a ring of three flag sets (levels L-1, L, L+1),
// each spread over 64 cache lines so that the waves reporting activity do
// not all write one line.  Levels are launched in chunks; the host reads the
// last flag set after each chunk, and a launched level whose predecessor
// found nothing returns at once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace tsgne {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLightMax = 256;        // larger degrees are split into chunks
constexpr int kChunk = 2048;          // edges per chunk block
constexpr int kChunkBlock = 1024;     // threads of the chunk-table kernel

// Edges in flight per thread: as many as the registers for their frontier
// words allow.
template <int W>
constexpr int unroll_for() {
  return W <= 4 ? 8 : 4;
}
constexpr int kSlots = 64;            // flags per level
constexpr int kSlotStride = 32;       // ints: one flag per 128-byte line
constexpr int kRing = 3;
constexpr int kFlagInts = kSlots * kSlotStride;
constexpr int kMaxTargets = 256;
constexpr int kLevelsPerCheck = 12;
constexpr uint32_t kErrTarget = 1u;

// Bits of word w that belong to one of the d targets.
__device__ __forceinline__ uint32_t word_mask(int w, int32_t d) {
  const int lo = 32 * w;
  if (d >= lo + 32) return ~0u;
  if (d <= lo) return 0u;
  return (1u << (d - lo)) - 1u;
}

template <int W>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ p, uint32_t (&m)[W]) {
  if constexpr (W >= 4) {
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
      const uint4 v = reinterpret_cast<const uint4*>(p)[q];
      m[4 * q] = v.x;
      m[4 * q + 1] = v.y;
      m[4 * q + 2] = v.z;
      m[4 * q + 3] = v.w;
    }
  } else if constexpr (W == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    m[0] = v.x;
    m[1] = v.y;
  } else {
    m[0] = p[0];
  }
}

template <int W>
__device__ __forceinline__ void store_words(uint32_t* __restrict__ p, const uint32_t (&m)[W]) {
  if constexpr (W >= 4) {
#pragma unroll
    for (int q = 0; q < W / 4; ++q)
      reinterpret_cast<uint4*>(p)[q] = make_uint4(m[4 * q], m[4 * q + 1], m[4 * q + 2], m[4 * q + 3]);
  } else if constexpr (W == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(m[0], m[1]);
  } else {
    p[0] = m[0];
  }
}

// Search state of one level: the previous level's frontier (words and
// activity bytes) is read, this level's is written over the one before.
struct SpState {
  const uint32_t* fcur;  // [n][W] frontier of the previous level
  uint32_t* fnext;       // [n][W] frontier of this level (holds the one two levels back)
  const uint8_t* acur;   // [n] fcur[v] != 0
  uint8_t* anext;        // [n] fnext[v] != 0
  uint32_t* vis;         // [n][W]
  uint32_t* planes;      // [n_planes][n][W]
  int64_t plane_stride;
  int n_planes;
};

// Level 0: every target has reached itself.  vis, F0 and the planes are zero.
__global__ __launch_bounds__(kBlock) void k_sp_init(const int32_t* __restrict__ targets, int32_t d, int32_t n,
                                                    int W, uint32_t* __restrict__ vis, uint32_t* __restrict__ f0,
                                                    uint8_t* __restrict__ a0, int32_t* __restrict__ flags,
                                                    uint32_t* __restrict__ err) {
  const int32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < kRing * kFlagInts) flags[j] = (j == 0) ? 1 : 0;  // level 0 counts as active
  if (j >= d) return;
  const int32_t t = targets[j];
  if (t < 0 || t >= n) {
    atomicOr(err, kErrTarget);
    return;
  }
  const uint32_t bit = 1u << (j & 31);
  atomicOr(&vis[(int64_t)t * W + (j >> 5)], bit);  // targets may repeat
  atomicOr(&f0[(int64_t)t * W + (j >> 5)], bit);
  a0[t] = 1;
}

// The new bits of node v at this level, given the OR of its neighbours'
// frontier words: frontier, activity byte, visited set and distance planes.
// A node without new bits writes its frontier only to clear what was there
// two levels back.  Called by one lane per node.  Returns whether anything
// was new.
template <int W>
__device__ __forceinline__ bool settle(int32_t v, const uint32_t (&acc)[W], const uint32_t (&seen)[W], bool full,
                                       bool was_active, const SpState& st, int32_t level) {
  uint32_t nw[W];
  uint32_t any = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    nw[w] = full ? 0u : (acc[w] & ~seen[w]);
    any |= nw[w];
  }
  if (any == 0) {
    if (was_active) {
      store_words<W>(st.fnext + (int64_t)v * W, nw);
      st.anext[v] = 0;
    }
    return false;
  }
  store_words<W>(st.fnext + (int64_t)v * W, nw);
  st.anext[v] = 1;
  uint32_t nv[W];
#pragma unroll
  for (int w = 0; w < W; ++w) nv[w] = seen[w] | nw[w];
  store_words<W>(st.vis + (int64_t)v * W, nv);
  // planes[k] |= new bits where the level has a one bit; loads in groups
  // of four, ahead of their stores
  for (int k0 = 0; k0 < st.n_planes; k0 += 4) {
    uint32_t pw[4][W];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + q;
      if (k < st.n_planes && ((level >> k) & 1))
        load_words<W>(st.planes + k * st.plane_stride + (int64_t)v * W, pw[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + q;
      if (k < st.n_planes && ((level >> k) & 1)) {
#pragma unroll
        for (int w = 0; w < W; ++w) pw[q][w] |= nw[w];
        store_words<W>(st.planes + k * st.plane_stride + (int64_t)v * W, pw[q]);
      }
    }
  }
  return true;
}

// Exclusive prefix sum over the block (kBlock threads); *total gets the sum.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t x, int32_t* s_wave, int32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  int32_t inc = x;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += y;
  }
  if (lane == kWave - 1) s_wave[wv] = inc;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    const int32_t t = s_wave[w];
    base += (w < wv) ? t : 0;
    tot += t;
  }
  *total = tot;
  return base + inc - x;
}

// One level of all searches.  Blocks [0, light_blocks) take kBlock
// consecutive nodes each (one thread per node for the node's own words) and
// share out the edges of those of degree <= kLightMax over the block: the
// edges are numbered by a prefix sum of the degrees, each thread takes every
// kBlock-th one, and the frontier words of the far ends are ORed into the
// node's word in LDS.  The remaining blocks take one chunk of at most kChunk
// edges of a node of larger degree each; the chunks of one node combine
// their ORs with device atomics, and the last chunk to finish settles the
// node.
template <int W>
__global__ __launch_bounds__(kBlock) void k_sp_level(const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, int32_t n, int32_t d,
                                                     int32_t light_blocks, const int4* __restrict__ chunks,
                                                     uint32_t* __restrict__ heavy_acc, int32_t* __restrict__ heavy_done,
                                                     const SpState st, int32_t level, int32_t* __restrict__ flags) {
  __shared__ int32_t s_pref[kBlock + 1];
  __shared__ int32_t s_start[kBlock];
  __shared__ uint32_t s_acc[W * kBlock];
  __shared__ int32_t s_wave[kWavesPerBlock];
  __shared__ uint32_t s_red[W * kWavesPerBlock];

  int32_t* const prev = flags + ((level - 1) % kRing) * kFlagInts;
  int32_t* const mine = flags + (level % kRing) * kFlagInts;
  int32_t* const next = flags + ((level + 1) % kRing) * kFlagInts;
  if (blockIdx.x == 0 && threadIdx.x < kSlots) next[threadIdx.x * kSlotStride] = 0;
  const int active = threadIdx.x < kSlots ? prev[threadIdx.x * kSlotStride] : 0;
  if (!__syncthreads_or(active)) return;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid >> 6;
  bool found = false;
  if ((int32_t)blockIdx.x < light_blocks) {
    const int32_t v = blockIdx.x * kBlock + tid;
    int32_t a = 0, deg = 0;
    uint32_t seen[W];
    bool full = true, light = false, was_active = false;
#pragma unroll
    for (int w = 0; w < W; ++w) seen[w] = 0u;
    if (v < n) {
      a = row_ptr[v];
      deg = row_ptr[v + 1] - a;
      light = deg <= kLightMax;
      was_active = st.anext[v] != 0;  // the frontier two levels back, overwritten below
      load_words<W>(st.vis + (int64_t)v * W, seen);
#pragma unroll
      for (int w = 0; w < W; ++w) full &= (seen[w] == word_mask(w, d));
    }
    int32_t total;
    const int32_t first = block_exclusive_scan((light && !full) ? deg : 0, s_wave, &total);
    s_pref[tid] = first;
    if (tid == 0) s_pref[kBlock] = total;
    s_start[tid] = a;
#pragma unroll
    for (int w = 0; w < W; ++w) s_acc[w * kBlock + tid] = 0u;
    __syncthreads();
    // Each thread takes kUnroll consecutive edges of the numbering, so that
    // they mostly share one node: their words are ORed in registers and
    // reach LDS once per node rather than once per edge.
    constexpr int kUnroll = unroll_for<W>();
    for (int32_t base = tid * kUnroll; base < total; base += kBlock * kUnroll) {
      int lo = 0, hi = kBlock;  // s_pref[lo] <= base < s_pref[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pref[mid] <= base) lo = mid;
        else hi = mid;
      }
      int32_t u[kUnroll], node[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        const int32_t t = base + k;
        node[k] = -1;
        u[k] = 0;
        if (t < total) {
          while (s_pref[lo + 1] <= t) ++lo;  // stops below kBlock since t < s_pref[kBlock]
          node[k] = lo;
          u[k] = col[s_start[lo] + (t - s_pref[lo])];
        }
      }
      // the frontier words are gathered only from active neighbours
      bool on[kUnroll];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) on[k] = node[k] >= 0 && st.acur[u[k]] != 0;
      uint32_t f[kUnroll][W];
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        if (on[k]) load_words<W>(st.fcur + (int64_t)u[k] * W, f[k]);
      }
      uint32_t run[W];
      int rn = node[0];
#pragma unroll
      for (int w = 0; w < W; ++w) run[w] = 0u;
#pragma unroll
      for (int k = 0; k < kUnroll; ++k) {
        if (node[k] != rn) {  // nodes only increase along the run; -1 marks its end
#pragma unroll
          for (int w = 0; w < W; ++w) {
            if (run[w]) atomicOr(&s_acc[w * kBlock + rn], run[w]);
            run[w] = 0u;
          }
          rn = node[k];
        }
        if (on[k]) {
#pragma unroll
          for (int w = 0; w < W; ++w) run[w] |= f[k][w];
        }
      }
      if (rn >= 0) {
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (run[w]) atomicOr(&s_acc[w * kBlock + rn], run[w]);
      }
    }
    __syncthreads();
    if (v < n && light) {
      uint32_t acc[W];
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] = s_acc[w * kBlock + tid];
      found = settle<W>(v, acc, seen, full, was_active, st, level);
    }
  } else {
    const int4 c = chunks[blockIdx.x - light_blocks];  // node, first edge, end edge, slot (-1: one chunk)
    const int32_t v = c.x;
    uint32_t seen[W], acc[W];
    load_words<W>(st.vis + (int64_t)v * W, seen);
    bool full = true;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      full &= (seen[w] == word_mask(w, d));
      acc[w] = 0u;
    }
    if (!full) {
      constexpr int kUnroll = unroll_for<W>();
      for (int32_t base = c.y; base < c.z; base += kBlock * kUnroll) {
        int32_t u[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const int32_t e = base + k * kBlock + tid;
          u[k] = e < c.z ? col[e] : -1;
        }
        bool on[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) on[k] = u[k] >= 0 && st.acur[u[k]] != 0;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          if (on[k]) {
            uint32_t f[W];
            load_words<W>(st.fcur + (int64_t)u[k] * W, f);
#pragma unroll
            for (int w = 0; w < W; ++w) acc[w] |= f[w];
          }
        }
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) acc[w] |= __shfl_xor(acc[w], off, kWave);
    }
    if (lane == 0) {
#pragma unroll
      for (int w = 0; w < W; ++w) s_red[wv * W + w] = acc[w];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        acc[w] = 0u;
#pragma unroll
        for (int q = 0; q < kWavesPerBlock; ++q) acc[w] |= s_red[q * W + w];
      }
      if (c.w < 0) {
        found = settle<W>(v, acc, seen, full, st.anext[v] != 0, st, level);
      } else {
        uint32_t* const hacc = heavy_acc + (int64_t)c.w * W;
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (acc[w]) atomicOr(&hacc[w], acc[w]);
        __threadfence();
        const int32_t n_chunks = (row_ptr[v + 1] - row_ptr[v] + kChunk - 1) / kChunk;
        if (atomicAdd(&heavy_done[c.w], 1) == n_chunks - 1) {  // every other chunk has added its bits
          __threadfence();
#pragma unroll
          for (int w = 0; w < W; ++w) acc[w] = atomicExch(&hacc[w], 0u);
          atomicExch(&heavy_done[c.w], 0);
          found = settle<W>(v, acc, seen, full, st.anext[v] != 0, st, level);
        }
      }
    }
  }
  if (__ballot(found) != 0 && lane == 0)
    mine[((blockIdx.x * kWavesPerBlock + wv) % kSlots) * kSlotStride] = 1;
}

// X[v][j] from the planes.  Each thread writes VEC consecutive targets of one
// node (VEC divides 32, so they share one word: one load per plane serves
// VEC outputs); a block covers whole rows.
template <int W, int VEC>
__global__ __launch_bounds__(kBlock) void k_sp_decode(int32_t n, int32_t d, const uint32_t* __restrict__ vis,
                                                      const uint32_t* __restrict__ planes, int64_t plane_stride,
                                                      int n_planes, float beyond, float* __restrict__ X) {
  const int per_node = d / VEC;
  const int nodes_per_block = kBlock / per_node;
  const int local = threadIdx.x / per_node;
  if (local >= nodes_per_block) return;
  const int32_t v = blockIdx.x * nodes_per_block + local;
  if (v >= n) return;
  const int j0 = (threadIdx.x - local * per_node) * VEC;
  const int64_t o = (int64_t)v * W + (j0 >> 5);
  const int bit0 = j0 & 31;
  const uint32_t seen = vis[o];
  uint32_t dist[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) dist[c] = 0u;
  for (int k = 0; k < n_planes; ++k) {
    const uint32_t p = planes[k * plane_stride + o] >> bit0;
#pragma unroll
    for (int c = 0; c < VEC; ++c) dist[c] |= ((p >> c) & 1u) << k;
  }
  float x[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) x[c] = ((seen >> (bit0 + c)) & 1u) ? (float)dist[c] : beyond;
  float* const out = X + (int64_t)v * d + j0;
  if constexpr (VEC % 4 == 0) {
#pragma unroll
    for (int q = 0; q < VEC / 4; ++q)
      reinterpret_cast<float4*>(out)[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
  } else {
    out[0] = x[0];
  }
}

// The chunk table, in one block: heavy nodes (ascending) are cut into runs
// of kChunk edges; a node of several runs gets the next accumulator slot.
// counts[1] holds the number of heavy nodes, counts[4] receives the number
// of chunks.
__global__ __launch_bounds__(kChunkBlock) void k_sp_chunks(const int4* __restrict__ heavy, int32_t* __restrict__ counts,
                                                           int32_t heavy_cap, int4* __restrict__ chunks,
                                                           int32_t chunk_cap) {
  __shared__ int32_t s_c[kChunkBlock / kWave], s_s[kChunkBlock / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t >> 6;
  const int32_t nh = min(counts[1], heavy_cap);
  const int32_t per = (nh + kChunkBlock - 1) / kChunkBlock;
  const int32_t lo = min(nh, t * per), hi = min(nh, lo + per);
  int32_t nc = 0, ns = 0;
  for (int32_t h = lo; h < hi; ++h) {
    const int32_t deg = heavy[h].z - heavy[h].y;
    nc += (deg + kChunk - 1) / kChunk;
    ns += deg > kChunk ? 1 : 0;
  }
  int32_t ic = nc, is = ns;
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t yc = __shfl_up(ic, off, kWave), ys = __shfl_up(is, off, kWave);
    if (lane >= off) {
      ic += yc;
      is += ys;
    }
  }
  if (lane == kWave - 1) {
    s_c[wv] = ic;
    s_s[wv] = is;
  }
  __syncthreads();
  int32_t bc = 0, bs = 0, total = 0;
  for (int w = 0; w < kChunkBlock / kWave; ++w) {
    bc += (w < wv) ? s_c[w] : 0;
    bs += (w < wv) ? s_s[w] : 0;
    total += s_c[w];
  }
  int32_t c = bc + ic - nc, slot = bs + is - ns;
  for (int32_t h = lo; h < hi; ++h) {
    const int4 r = heavy[h];
    const bool split = r.z - r.y > kChunk;
    for (int32_t e = r.y; e < r.z; e += kChunk, ++c)
      if (c < chunk_cap) chunks[c] = make_int4(r.x, e, min(r.z, e + kChunk), split ? slot : -1);
    slot += split ? 1 : 0;
  }
  if (t == 0) counts[4] = min(total, chunk_cap);
}

template <int W>
hipError_t launch_level(const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t d, const int4* chunks,
                        int32_t n_chunks, uint32_t* heavy_acc, int32_t* heavy_done, const SpState& st, int32_t level,
                        int32_t* flags, hipStream_t s) {
  const int32_t light_blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_sp_level<W>, dim3((unsigned)(light_blocks + n_chunks)), dim3(kBlock), 0, s, row_ptr, col, n,
                     d, light_blocks, chunks, heavy_acc, heavy_done, st, level, flags);
  return hipGetLastError();
}

template <int W>
hipError_t launch_decode(int32_t n, int32_t d, const uint32_t* vis, const uint32_t* planes, int64_t plane_stride,
                         int n_planes, float beyond, float* X, hipStream_t s) {
  if (d % 16 == 0) {
    const int32_t per_block = kBlock / (d / 16);
    hipLaunchKernelGGL((k_sp_decode<W, 16>), dim3((unsigned)((n + per_block - 1) / per_block)), dim3(kBlock), 0, s,
                       n, d, vis, planes, plane_stride, n_planes, beyond, X);
  } else if (d % 4 == 0) {
    const int32_t per_block = kBlock / (d / 4);
    hipLaunchKernelGGL((k_sp_decode<W, 4>), dim3((unsigned)((n + per_block - 1) / per_block)), dim3(kBlock), 0, s, n,
                       d, vis, planes, plane_stride, n_planes, beyond, X);
  } else {
    const int32_t per_block = kBlock / d;
    hipLaunchKernelGGL((k_sp_decode<W, 1>), dim3((unsigned)((n + per_block - 1) / per_block)), dim3(kBlock), 0, s, n,
                       d, vis, planes, plane_stride, n_planes, beyond, X);
  }
  return hipGetLastError();
}

struct SpKernels {
  hipError_t (*level)(const int32_t*, const int32_t*, int32_t, int32_t, const int4*, int32_t, uint32_t*, int32_t*,
                      const SpState&, int32_t, int32_t*, hipStream_t);
  hipError_t (*decode)(int32_t, int32_t, const uint32_t*, const uint32_t*, int64_t, int, float, float*, hipStream_t);
};

SpKernels kernels_for(int W) {
  switch (W) {
    case 1: return {launch_level<1>, launch_decode<1>};
    case 2: return {launch_level<2>, launch_decode<2>};
    case 4: return {launch_level<4>, launch_decode<4>};
    default: return {launch_level<8>, launch_decode<8>};
  }
}

// Offsets of the per-call buffers inside one device allocation.
struct SpLayout {
  size_t vis, f0, f1, a0, a1, planes, counts, hacc, hdone, zero_end;  // [vis, zero_end) is cleared
  size_t partial, heavy, chunks, flags, total;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

SpLayout make_layout(int32_t n, int64_t words, int n_planes, int64_t blocks, int64_t heavy_cap, int64_t chunk_cap,
                     int W) {
  SpLayout L{};
  size_t o = 0;
  L.vis = o;
  o = align_up(o + 4 * (size_t)words);
  L.f0 = o;
  o = align_up(o + 4 * (size_t)words);
  L.f1 = o;
  o = align_up(o + 4 * (size_t)words);
  L.a0 = o;
  o = align_up(o + (size_t)n);
  L.a1 = o;
  o = align_up(o + (size_t)n);
  L.planes = o;
  o = align_up(o + 4 * (size_t)words * n_planes);
  L.counts = o;
  o = align_up(o + 8 * sizeof(int32_t));
  L.hacc = o;
  o = align_up(o + 4 * (size_t)heavy_cap * W);
  L.hdone = o;
  o = align_up(o + 4 * (size_t)heavy_cap);
  L.zero_end = o;
  L.partial = o;
  o = align_up(o + sizeof(int2) * (size_t)blocks);
  L.heavy = o;
  o = align_up(o + sizeof(int4) * (size_t)heavy_cap);
  L.chunks = o;
  o = align_up(o + sizeof(int4) * (size_t)chunk_cap);
  L.flags = o;
  o = align_up(o + sizeof(int32_t) * kRing * kFlagInts);
  L.total = o;
  return L;
}

}  // namespace
}  // namespace tsgne

using namespace tsgne;

extern "C" {

tsgne_status tsgne_shortest_path_embedding(int32_t n, int64_t nnz, const int32_t* row_ptr_d, const int32_t* col_d,
                                           int32_t d, const int32_t* targets_d, double l0, float* X_d,
                                           int32_t* levels_out, void* stream) {
  if (levels_out) *levels_out = 0;
  if (n < 1) return fail(TSGNE_E_INVAL, "n must be >= 1");
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return fail(TSGNE_E_INVAL, "nnz must lie in [0, 2^31)");
  if (d < 1 || d > kMaxTargets) return fail(TSGNE_E_INVAL, "d must lie in [1, 256]");
  if (std::isnan(l0)) return fail(TSGNE_E_INVAL, "l0 is NaN");
  if (!row_ptr_d || (nnz > 0 && !col_d) || !targets_d || !X_d) return fail(TSGNE_E_INVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (l0 < 0) l0 = std::sqrt((double)(nnz / 2));  // the default threshold sqrt(|E|)
  const float beyond = (float)(l0 + 1.0);
  // Distances beyond n - 1 do not occur, so the searches stop there too.
  const int32_t max_level = (int32_t)std::min<double>(std::floor(l0), (double)(n - 1));
  int n_planes = 0;
  while (n_planes < 31 && (max_level >> n_planes) != 0) ++n_planes;
  const int W = d <= 32 ? 1 : d <= 64 ? 2 : d <= 128 ? 4 : 8;
  const int64_t words = (int64_t)n * W;
  // a valid CSR has at most nnz / (kLightMax + 1) nodes above kLightMax, and
  // they have at most that many plus nnz / kChunk chunks
  const int64_t heavy_cap = std::min<int64_t>(n, nnz / (kLightMax + 1) + 1);
  const int64_t chunk_cap = heavy_cap + nnz / kChunk + 1;
  const SpLayout lay = make_layout(n, words, n_planes, row_check_blocks(n), heavy_cap, chunk_cap, W);

  // one allocation: the CSR check runs in it first, then the search state
  // is laid over it
  ScratchBlock tmp;
  tmp.s = s;
  TSGNE_HIP(scratch_alloc(&tmp.p, std::max(lay.total, validate_csr_bytes(n, nnz)), s), "allocate search state");
  if (tsgne_status st = validate_csr_in(n, nnz, row_ptr_d, col_d, tmp.p, s)) return st;
  char* const base = static_cast<char*>(tmp.p);
  uint32_t* const vis = reinterpret_cast<uint32_t*>(base + lay.vis);
  uint32_t* const f[2] = {reinterpret_cast<uint32_t*>(base + lay.f0), reinterpret_cast<uint32_t*>(base + lay.f1)};
  uint8_t* const act[2] = {reinterpret_cast<uint8_t*>(base + lay.a0), reinterpret_cast<uint8_t*>(base + lay.a1)};
  uint32_t* const planes = reinterpret_cast<uint32_t*>(base + lay.planes);
  // [0] rows with entries, [1] heavy nodes, [2] target error, [3] row error, [4] chunks
  int32_t* const counts = reinterpret_cast<int32_t*>(base + lay.counts);
  int2* const partial = reinterpret_cast<int2*>(base + lay.partial);
  uint32_t* const heavy_acc = reinterpret_cast<uint32_t*>(base + lay.hacc);
  int32_t* const heavy_done = reinterpret_cast<int32_t*>(base + lay.hdone);
  int4* const heavy = reinterpret_cast<int4*>(base + lay.heavy);
  int4* const chunks = reinterpret_cast<int4*>(base + lay.chunks);
  int32_t* const flags = reinterpret_cast<int32_t*>(base + lay.flags);

  TSGNE_HIP(hipMemsetAsync(base, 0, lay.zero_end, s), "clear search state");
  hipLaunchKernelGGL(k_sp_init, dim3((unsigned)((std::max(d, kRing * kFlagInts) + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, targets_d, d, n, W, vis, f[0], act[0], flags,
                     reinterpret_cast<uint32_t*>(counts + 2));
  TSGNE_HIP(hipGetLastError(), "launch target set-up");
  TSGNE_HIP(launch_check_rows(row_ptr_d, n, nnz, kLightMax, reinterpret_cast<uint32_t*>(counts + 3), counts, partial,
                              nullptr, heavy, (int32_t)heavy_cap, s),
            "launch heavy-node list");
  hipLaunchKernelGGL(k_sp_chunks, dim3(1), dim3(kChunkBlock), 0, s, heavy, counts, (int32_t)heavy_cap, chunks,
                     (int32_t)chunk_cap);
  TSGNE_HIP(hipGetLastError(), "launch chunk table");
  int32_t host_counts[8] = {};
  TSGNE_HIP(hipMemcpyAsync(host_counts, counts, sizeof(host_counts), hipMemcpyDeviceToHost, s), "read counters");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise set-up");
  if (host_counts[2] & kErrTarget) return fail(TSGNE_E_INVAL, "a target lies outside [0, n)");
  const int32_t n_chunks = host_counts[4];

  const SpKernels kern = kernels_for(W);
  const int64_t plane_stride = words;
  std::vector<int32_t> host_flags(kFlagInts);
  int32_t level = 1, levels_run = 0;
  while (level <= max_level) {
    const int32_t last = std::min<int32_t>(max_level, level + kLevelsPerCheck - 1);
    for (int32_t L = level; L <= last; ++L) {
      const SpState st{f[(L - 1) & 1], f[L & 1], act[(L - 1) & 1], act[L & 1], vis, planes, plane_stride, n_planes};
      TSGNE_HIP(kern.level(row_ptr_d, col_d, n, d, chunks, n_chunks, heavy_acc, heavy_done, st, L, flags, s),
                "launch search level");
    }
    TSGNE_HIP(hipMemcpyAsync(host_flags.data(), flags + (last % kRing) * kFlagInts, sizeof(int32_t) * kFlagInts,
                             hipMemcpyDeviceToHost, s),
              "read level flags");
    TSGNE_HIP(hipStreamSynchronize(s), "synchronise search levels");
    bool active = false;
    for (int i = 0; i < kSlots; ++i) active |= host_flags[(size_t)i * kSlotStride] != 0;
    levels_run = last;
    if (!active) break;
    level = last + 1;
  }
  TSGNE_HIP(kern.decode(n, d, vis, planes, plane_stride, n_planes, beyond, X_d, s), "launch decode");
  TSGNE_HIP(hipStreamSynchronize(s), "synchronise embedding");
  if (levels_out) *levels_out = levels_run;
  return TSGNE_OK;
}

}  // extern "C"
