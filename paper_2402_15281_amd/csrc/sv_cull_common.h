// Device building blocks of the culled exact passes (per-motion minimum with groups of
// tests skipped that bounding spheres prove to lie above it), shared by the per-call
// pass (sv_cull.hip) and the batched one (sv_batch.hip).
//
// A group is (a wave's 64 P consecutive points of a Morton-sorted cloud, one capsule,
// one block of kCullB consecutive samples).  Its lower bound is
// |c_wave - c_block| - R_wave - R_block; if that exceeds an upper bound G of the
// motion's minimum by more than kCullMargin (which covers the FP32 rounding of the
// bound), every test of the group is larger than the final minimum, so skipping it
// changes neither the minimum nor the lowest index attaining it.
#pragma once

#include "sv_geom_common.h"

namespace sv {
namespace {

constexpr float kCullMargin = 1e-5f;   // m, above the FP32 rounding of the bounds
constexpr int kCullB = 16;            // samples per bounding block
constexpr int kSeedSampleStride = 4;  // the seed bound uses every 4th sample
constexpr int kCullP = 2, kCullNT = 256;  // culled pass: points per lane, threads per block

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ float key_dist(unsigned long long key) {
  return key == kKeyEmpty ? INFINITY : unord_f32((uint32_t)(key >> 32));
}

// Up to 10 bits per axis, interleaved into a Morton code.
__device__ __forceinline__ unsigned spread10(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton cell of point v in a grid of 2^L cells per axis over the bounds bd (bd[0..2]
// minima, bd[3..5] maxima, as order-preserving keys).  Points are binned by cell and
// the cells taken in Morton order, so consecutive points of the sorted cloud are close
// together; the order within a cell is free (every result downstream is a minimum over
// all points, keyed by the caller's point index).
__device__ __forceinline__ unsigned morton_cell(const float v[3], const unsigned* bd, int L) {
  const float cells = (float)(1 << L);
  unsigned q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lo = unord_f32(bd[a]), hi = unord_f32(bd[3 + a]);
    const float sc = hi > lo ? cells / (hi - lo) : 0.f;
    q[a] = (unsigned)fminf(fmaxf((v[a] - lo) * sc, 0.f), cells - 1.f);
  }
  return spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
}

// One culled item for one wave group: the wave's 64 P consecutive sorted points of
// tile `tile` (sx, sy, sz, N; perm maps them to the caller's indices) against one
// capsule of one motion (table entries from e, T samples; sample-block spheres sph,
// nb of them), under the bound G.  Returns, valid in thread 0, the block's smallest
// (distance, index) key of the tests that survive; adds the executed tests to
// `executed`.  Every thread of the block must call it (it contains a barrier).
template <int P, int NT>
__device__ __forceinline__ unsigned long long cull_item(ConstF4Ptr tab, size_t e, int T, ConstF4Ptr sph, int nb,
                                                        const float* __restrict__ sx, const float* __restrict__ sy,
                                                        const float* __restrict__ sz, const int* __restrict__ perm,
                                                        int N, int tile, float G, unsigned long long* wmin,
                                                        unsigned long long& executed) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int base = tile * (NT * P) + wid * (64 * P) + lane;
  float x[P], y[P], z[P], best[P];
  int idx[P];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = base + p * 64;
    const bool ok = j < N;
    idx[p] = ok ? perm[j] : -1;
    x[p] = ok ? sx[j] : 0.f;
    y[p] = ok ? sy[j] : 0.f;
    z[p] = ok ? sz[j] : 0.f;
    best[p] = INFINITY;
    if (ok) {
      lo[0] = fminf(lo[0], x[p]); hi[0] = fmaxf(hi[0], x[p]);
      lo[1] = fminf(lo[1], y[p]); hi[1] = fmaxf(hi[1], y[p]);
      lo[2] = fminf(lo[2], z[p]); hi[2] = fmaxf(hi[2], z[p]);
    }
  }
  if (__builtin_amdgcn_readfirstlane((int)(base < N))) {   // lane 0 holds the wave's first point
    // the wave's sphere
    const float cx = uniform_f(0.5f * (wave_min(lo[0]) + wave_max(hi[0])));
    const float cy = uniform_f(0.5f * (wave_min(lo[1]) + wave_max(hi[1])));
    const float cz = uniform_f(0.5f * (wave_min(lo[2]) + wave_max(hi[2])));
    float r2 = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (idx[p] >= 0) {
        const float dx = x[p] - cx, dy = y[p] - cy, dz = z[p] - cz;
        r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
      }
    const float rw = uniform_f(sqrtf(wave_max(r2)));
    G = uniform_f(G);
    const float r = load_entry(tab, e).r;
    float m2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) m2[p] = INFINITY;
    for (int b = 0; b < nb; ++b) {
      const vf4 sb = sph[b];
      const float dx = sb.x - cx, dy = sb.y - cy, dz = sb.z - cz;
      const float lb = sqrtf(dx * dx + dy * dy + dz * dz) - rw - sb.w;
      if (lb > G + kCullMargin) continue;   // every test of the group exceeds the final minimum
      const int t0 = b * kCullB, t1 = min(t0 + kCullB, T);
      swept_range<P>(tab, e, t0, t1, x, y, z, m2);
      executed += (unsigned long long)(t1 - t0) * (64 * P);
      // tighten the bound with this wave's points
      float wb = INFINITY;
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (idx[p] >= 0) wb = fminf(wb, sqrtf(m2[p]) - r);
      G = uniform_f(fminf(G, wave_min(wb)));
    }
#pragma unroll
    for (int p = 0; p < P; ++p) best[p] = sqrtf(m2[p]) - r;
  }
  return block_min_key<NT>(lane_min_key<P>(best, idx), wmin);
}

}  // namespace
}  // namespace sv
