// Device building blocks of the culled exact passes (per-motion minimum with groups of
// tests skipped that bounding spheres prove to lie above it), shared by the per-call
// pass (sv_cull.hip) and the batched one (sv_batch.hip).
//
// A group is (a wave's 64 P consecutive points of a Morton-sorted cloud, one capsule,
// one block of cull_block_len(T) consecutive samples).  Its lower bound is
// |c_wave - c_block| - R_wave - R_block; if that exceeds an upper bound G of the
// motion's minimum by more than kCullMargin (which covers the FP32 rounding of the
// bound), every test of the group is larger than the final minimum, so skipping it
// changes neither the minimum nor the lowest index attaining it.
#pragma once

#include "sv_geom_common.h"

namespace sv {
namespace {

constexpr float kCullMargin = 1e-5f;   // m, above the FP32 rounding of the bounds
// Samples per bounding block (2 to 16): a block spans about 1/div of a motion, div = 32
// for a linear motion and 64 for a spline (whose path through two via points is several
// times longer), so that its sphere stays tight at every T.  Shorter blocks cost more
// sphere tests, longer ones skip fewer segment tests; these divisors are measured optima
// of the per-call pass (bin-picking workloads, T = 64 to 1024), and the batched pass
// takes them from its launch shape (sv_tile), where an autotuner may choose others
// (kCullDivLinear, kCullDivSpline and the allowed sets are in sv_internal.h).
__host__ __device__ constexpr int cull_block_len_div(int T, int div) {
  return T >= 16 * div ? 16 : T <= 2 * div ? 2 : (T + div - 1) / div;
}
__host__ __device__ constexpr int cull_block_len(int T, int kind, int div_lin = kCullDivLinear,
                                                 int div_spl = kCullDivSpline) {
  return cull_block_len_div(T, kind == SV_SPLINE ? div_spl : div_lin);
}
__host__ __device__ constexpr int cull_block_count(int T, int kind, int div_lin = kCullDivLinear,
                                                   int div_spl = kCullDivSpline) {
  return (T + cull_block_len(T, kind, div_lin, div_spl) - 1) / cull_block_len(T, kind, div_lin, div_spl);
}
// The largest block count of any T <= max_T under any allowed divisor (from T = 16 div on,
// blocks have 16 samples and the count grows with T).
inline int cull_block_count_max(int max_T) {
  int nb = 1;
  for (int d : {16, 32, 64, 128}) {
    for (int T = 1; T <= max_T && T < 16 * d; ++T) {
      const int c = (T + cull_block_len_div(T, d) - 1) / cull_block_len_div(T, d);
      nb = nb > c ? nb : c;
    }
    if (max_T >= 16 * d) nb = nb > (max_T + 15) / 16 ? nb : (max_T + 15) / 16;
  }
  return nb;
}
constexpr int kSeedSamples = 32;      // the seed bound visits about this many samples of a motion
// Sample stride of the seed bound: about kSeedSamples samples whatever T.
__host__ __device__ constexpr int seed_stride(int T) { return T > kSeedSamples ? (T + kSeedSamples - 1) / kSeedSamples : 1; }
constexpr int kCullP = 2, kCullNT = 256;  // culled pass: points per lane, threads per block

// A wave tightens its bound after every kBoundEvery-th sample block it runs: the update
// is a cross-lane reduction whose latency the next block's tests wait for, and a bound a
// few blocks stale skips as much (same-session A/B on bin20k with swept_block's loads,
// bit-identical results and within 0.3% of the executed tests: per culled pass at T =
// 256 / 1,024, updates after every block 0.540 / 1.23 ms, every second 0.533 / 1.19 ms,
// every fourth 0.528 / 1.17 ms; the screened path's exact check of all points 2.95 ->
// 2.63 ms with every second).
constexpr int kBoundEvery = 4;

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

// Spheres of one tile of sorted points [j0, j1) (j1 - j0 <= NT P; all NT threads of a
// block, NT = 256): wave w's group of the culled kernel's points, [j0 + 64 P w, j0 +
// 64 P (w + 1)), into wave_out[w] and the whole tile into *tile_out.  Centres are the
// midpoints of the bounding boxes, radii the largest distance from them (computed in
// FP32; kCullMargin covers the rounding).  An empty group gets radius 0.  part [4][6]
// and pr [4] are LDS scratch; two barriers.
template <int P, int NT>
__device__ void tile_wave_spheres(const float* __restrict__ sx, const float* __restrict__ sy,
                                  const float* __restrict__ sz, int64_t j0, int64_t j1, float4* tile_out,
                                  float4* wave_out, float (*part)[6], float* pr) {
  static_assert(NT == 256, "four wave groups");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float x[P], y[P], z[P];
  bool ok[P];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t j = j0 + wid * (64 * P) + lane + p * 64;
    ok[p] = j < j1;
    x[p] = ok[p] ? sx[j] : 0.f;
    y[p] = ok[p] ? sy[j] : 0.f;
    z[p] = ok[p] ? sz[j] : 0.f;
    if (ok[p]) {
      lo[0] = fminf(lo[0], x[p]); hi[0] = fmaxf(hi[0], x[p]);
      lo[1] = fminf(lo[1], y[p]); hi[1] = fmaxf(hi[1], y[p]);
      lo[2] = fminf(lo[2], z[p]); hi[2] = fmaxf(hi[2], z[p]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min(lo[a]);
    hi[a] = wave_max(hi[a]);
  }
  const bool any = lo[0] <= hi[0];   // the group holds a point
  const float cx = any ? 0.5f * (lo[0] + hi[0]) : 0.f, cy = any ? 0.5f * (lo[1] + hi[1]) : 0.f;
  const float cz = any ? 0.5f * (lo[2] + hi[2]) : 0.f;
  float r2 = 0.f;
#pragma unroll
  for (int p = 0; p < P; ++p)
    if (ok[p]) {
      const float dx = x[p] - cx, dy = y[p] - cy, dz = z[p] - cz;
      r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
    }
  r2 = wave_max(r2);
  if (lane == 0) {
    wave_out[wid] = make_float4(cx, cy, cz, any ? sqrtf(r2) : -INFINITY);   // an empty group never passes
    for (int a = 0; a < 3; ++a) {
      part[wid][a] = lo[a];
      part[wid][3 + a] = hi[a];
    }
  }
  __syncthreads();
  float c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float l = part[0][a], h = part[0][3 + a];
    for (int q = 1; q < 4; ++q) {
      l = fminf(l, part[q][a]);
      h = fmaxf(h, part[q][3 + a]);
    }
    c[a] = 0.5f * (l + h);
  }
  float t2 = 0.f;
#pragma unroll
  for (int p = 0; p < P; ++p)
    if (ok[p]) {
      const float dx = x[p] - c[0], dy = y[p] - c[1], dz = z[p] - c[2];
      t2 = fmaxf(t2, dx * dx + dy * dy + dz * dz);
    }
  t2 = wave_max(t2);
  if (lane == 0) pr[wid] = t2;
  __syncthreads();
  if (threadIdx.x == 0)
    *tile_out = make_float4(c[0], c[1], c[2], sqrtf(fmaxf(fmaxf(pr[0], pr[1]), fmaxf(pr[2], pr[3]))));
}

// Whether the lower bound of the tests between the points in sphere a and the segments
// in sphere b, |c_a - c_b| - R_a - R_b, exceeds G + kCullMargin (tested without the
// square root: with S = G + margin + R_a + R_b, iff S < 0 or |c_a - c_b|^2 > S^2).
__device__ __forceinline__ bool spheres_apart(float4 a, float4 b, float G);

// A sphere around the block spheres sp[b0 .. b1): centred at the midpoint of their
// centres' box, radius to the farthest block sphere's surface, grown by a relative 1e-6
// and 1e-6 m so that it contains them despite the FP32 rounding of its radius.  A
// candidate apart from it (under the bound and kCullMargin) is then apart from each of
// its blocks up to a rounding far below kCullMargin, so no test at or below the bound is
// skipped.
__device__ __forceinline__ float4 group_sphere(const float4* __restrict__ sp, int b0, int b1) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = b0; b < b1; ++b) {
    const float4 s = sp[b];
    lo[0] = fminf(lo[0], s.x); hi[0] = fmaxf(hi[0], s.x);
    lo[1] = fminf(lo[1], s.y); hi[1] = fmaxf(hi[1], s.y);
    lo[2] = fminf(lo[2], s.z); hi[2] = fmaxf(hi[2], s.z);
  }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  float R = 0.f;
  for (int b = b0; b < b1; ++b) {
    const float4 s = sp[b];
    const float dx = s.x - cx, dy = s.y - cy, dz = s.z - cz;
    R = fmaxf(R, sqrtf(dx * dx + dy * dy + dz * dz) + s.w);
  }
  return make_float4(cx, cy, cz, fmaf(R, 1.000001f, 1e-6f));
}

__device__ __forceinline__ bool spheres_apart(float4 a, float4 b, float G) {
  const float dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  const float S = G + kCullMargin + a.w + b.w;
  return S < 0.f || dx * dx + dy * dy + dz * dz > S * S;
}

// Whether a (tile, capsule) item can run any test under the bound G: some sample block
// (spheres sp[0..nb)) within reach of the tile's sphere ts (most candidates fail here),
// and some (wave group, block) pair within reach (the wave groups' spheres ws[0..3]),
// which is what the culled kernel tests.  G only falls, so an item dropped here would
// run no test later either.
// Blocks are tested in groups of kGroupBlocks under a group sphere (gp[i] encloses the
// block spheres sp[8 i .. 8 i + 7]): a group whose sphere is apart skips its blocks, whose
// spheres it contains.  (Scanning every block sphere of a rejected candidate, up to 128 of
// them, had cost 3.4 ms of the 64-request batch's 47 ms.)
__device__ __forceinline__ bool item_may_hit(float4 ts, const float4* __restrict__ ws, const float4* __restrict__ sp,
                                             const float4* __restrict__ gp, int nb, float G) {
  const int ng = cull_group_count(nb);
  bool near_tile = false;
  for (int gi = 0; gi < ng && !near_tile; ++gi) {
    if (spheres_apart(ts, gp[gi], G)) continue;
    const int b1 = min(kGroupBlocks * (gi + 1), nb);
    for (int b = kGroupBlocks * gi; b < b1 && !near_tile; ++b) near_tile = !spheres_apart(ts, sp[b], G);
  }
  if (!near_tile) return false;
  const float4 w0 = ws[0], w1 = ws[1], w2 = ws[2], w3 = ws[3];
  for (int gi = 0; gi < ng; ++gi) {
    const float4 g = gp[gi];
    if (spheres_apart(w0, g, G) && spheres_apart(w1, g, G) && spheres_apart(w2, g, G) && spheres_apart(w3, g, G))
      continue;
    const int b1 = min(kGroupBlocks * (gi + 1), nb);
    for (int b = kGroupBlocks * gi; b < b1; ++b) {
      const float4 s = sp[b];
      if (!spheres_apart(w0, s, G) || !spheres_apart(w1, s, G) || !spheres_apart(w2, s, G) ||
          !spheres_apart(w3, s, G))
        return true;
    }
  }
  return false;
}

// Squared distance from (x, y, z) to the nearest segment of samples 0, ts, 2 ts, ...
// < T of the capsule whose table entries start at e: the per-point part of the seed
// bound, two samples per iteration so that both loads are in flight together.
__device__ __forceinline__ float seed_d2(ConstF4Ptr tab, size_t e, int T, int ts, float x, float y, float z) {
  float m2 = INFINITY;
  int t = 0;
  for (; t + ts < T; t += 2 * ts) {
    const CapEntry a = load_entry(tab, e + t), b = load_entry(tab, e + t + ts);
    m2 = fminf(m2, fminf(seg_d2(a, x, y, z), seg_d2(b, x, y, z)));
  }
  if (t < T) m2 = fminf(m2, seg_d2(load_entry(tab, e + t), x, y, z));
  return m2;
}

// One culled item for one wave group: the wave's 64 P consecutive sorted points of
// tile `tile` (sx, sy, sz, N; perm maps them to the caller's indices; wsph the tile's
// four wave-group spheres) against one capsule of one motion (table entries from e, T
// samples; sample-block spheres sph, nb of them, over blocks of B samples), under the
// bound G.  Returns, valid in thread 0, the block's smallest
// (distance, index) key of the tests that survive; adds the executed tests to
// `executed`.  Every thread of the block must call it (it contains a barrier).
template <int P, int NT>
__device__ __forceinline__ unsigned long long cull_item(ConstF4Ptr tab, size_t e, int T,
                                                        const float4* __restrict__ sph, int nb, int B, ConstF4Ptr wsph, const float* __restrict__ sx,
                                                        const float* __restrict__ sy, const float* __restrict__ sz,
                                                        const int* __restrict__ perm, int N, int tile, float G,
                                                        unsigned long long* wmin, unsigned long long& executed) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int base = tile * (NT * P) + wid * (64 * P) + lane;
  float x[P], y[P], z[P], best[P];
  int idx[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = base + p * 64;
    const bool ok = j < N;
    idx[p] = ok ? perm[j] : -1;
    x[p] = ok ? sx[j] : 0.f;
    y[p] = ok ? sy[j] : 0.f;
    z[p] = ok ? sz[j] : 0.f;
    best[p] = INFINITY;
  }
  if (__builtin_amdgcn_readfirstlane((int)(base < N))) {   // lane 0 holds the wave's first point
    const vf4 ws = wsph[__builtin_amdgcn_readfirstlane(wid)];   // the wave's sphere, from the tile pass
    const float cx = ws.x, cy = ws.y, cz = ws.z, rw = ws.w;
    G = uniform_f(G);
    const float r = load_entry(tab, e).r;
    float m2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) m2[p] = INFINITY;
    // |c_wave - c_block| - R_wave - R_block > G + margin, without the square root:
    // skip iff the centre distance exceeds S = G + margin + R_wave + R_block.  Every test
    // of a skipped group exceeds the final minimum.
    auto skip = [&](float bx, float by, float bz, float br, float g) {
      const float dx = bx - cx, dy = by - cy, dz = bz - cz;
      const float S = g + kCullMargin + rw + br;
      return S < 0.f || dx * dx + dy * dy + dz * dz > S * S;
    };
    int nrun = 0;   // sample blocks run
    for (int b0 = 0; b0 < nb; b0 += 64) {
      // Lane l tests block b0 + l against the bound at the start of the chunk: one vector
      // load and one ballot instead of a chain of dependent scalar loads.  The bound only
      // falls, so a block failing this test fails every later one too.
      const int bl = b0 + lane;
      float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
      bool maybe = false;
      if (bl < nb) {
        q = sph[bl];
        maybe = !skip(q.x, q.y, q.z, q.w, G);
      }
      for (unsigned long long mask = __ballot(maybe); mask; mask &= mask - 1) {
        const int l = __builtin_ctzll(mask);
        const float bx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.x), l));
        const float by = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.y), l));
        const float bz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.z), l));
        const float br = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.w), l));
        if (skip(bx, by, bz, br, G)) continue;   // the bound has tightened since
        const int t0 = (b0 + l) * B, t1 = min(t0 + B, T);
        swept_block<P>(tab, e, t0, t1, x, y, z, m2);
        executed += (unsigned long long)(t1 - t0) * (64 * P);
        if (++nrun % kBoundEvery) continue;
        // Tighten the bound with this wave's points: the square root of the smallest
        // squared distance, minus r (sqrt and - r do not decrease, so this is the
        // smallest sqrt(m2) - r; kCullMargin covers a last-place difference of the
        // hardware square root).  A bound not yet tightened is still an upper bound.
        float mm = INFINITY;
#pragma unroll
        for (int p = 0; p < P; ++p)
          if (idx[p] >= 0) mm = fminf(mm, m2[p]);
        G = uniform_f(fminf(G, sqrtf(wave_min(mm)) - r));
      }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) best[p] = sqrtf(m2[p]) - r;
  }
  return block_min_key<NT>(lane_min_key<P>(best, idx), wmin);
}

}  // namespace
}  // namespace sv
