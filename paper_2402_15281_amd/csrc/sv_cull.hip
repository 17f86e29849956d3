// Exact cloud distance per motion with culling (branch and bound), gfx950.
//
// sv_check_motions needs, per motion, only d(X, m) = min over the cloud of the swept
// distance (Sec. IV-B) and the lowest index attaining it -- not every point's
// distance.  Most (point, capsule, sample) tests of a motion are far above that
// minimum, and whole groups of them can be proven so with two bounding spheres:
//   - a wave's points: the cloud is sorted by Morton cell first (a counting sort), so
//     the 64 P points a wave holds are close together; their sphere is computed once
//     per tile of sorted points (k_tile_spheres) for every item of that tile;
//   - a block of consecutive samples of one capsule (cull_block_len(T) of them): a
//     sphere around all their
//     segment endpoints, grown by the capsule radius (k_block_spheres).
// If |c_wave - c_block| - R_wave - R_block exceeds an upper bound G of d(X, m) (plus
// kCullMargin for FP32 rounding of the bound), every test of that group is larger than
// the final minimum, so skipping it changes neither the minimum nor the lowest index
// attaining it: per-motion results equal the unculled kernels' bit for bit.  G starts
// from an exact check of a stride sample of the sorted cloud (k_exact_seed) and
// tightens as waves finish capsules and as other blocks publish their minima.
// Per-point distances are not produced here (skipped tests would leave them high).
#include "sv_cull_common.h"

namespace sv {
namespace {

// Start values of the pass's counters, in one launch: bounds (minima ~0u, maxima 0),
// the Morton bin counts and the item count and queue head.
__global__ __launch_bounds__(256) void k_cull_init(unsigned* __restrict__ bounds, int* __restrict__ bin_count,
                                                   int64_t nbins, int* __restrict__ list_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbins) bin_count[i] = 0;
  if (i < 6) bounds[i] = i < 3 ? ~0u : 0u;
  if (i < 2) list_count[i] = 0;
}

// Axis-aligned bounds of the cloud as order-preserving keys: bounds[0..2] minima
// (start ~0u), bounds[3..5] maxima (start 0).  One atomic per block and bound.
__global__ __launch_bounds__(256) void k_cloud_bounds(CloudArgs c, unsigned* __restrict__ bounds) {
  __shared__ float part[4][6];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += gridDim.x * blockDim.x) {
    const float v[3] = {c.x[i], c.y[i], c.z[i]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], v[a]);
      hi[a] = fmaxf(hi[a], v[a]);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min(lo[a]);
    hi[a] = wave_max(hi[a]);
    if (lane == 0) {
      part[wid][a] = lo[a];
      part[wid][3 + a] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    float v = part[0][a];
    for (int q = 1; q < 4; ++q) v = a < 3 ? fminf(v, part[q][a]) : fmaxf(v, part[q][a]);
    if (a < 3 && v < INFINITY) atomicMin(bounds + a, ord_f32(v));
    if (a >= 3 && v > -INFINITY) atomicMax(bounds + a, ord_f32(v));
  }
}

// One thread per point: its Morton cell and its slot among the cell's points.
__global__ __launch_bounds__(256) void k_cell_bin(CloudArgs c, const unsigned* __restrict__ bounds, int L,
                                                  int* __restrict__ pbin, int* __restrict__ pslot,
                                                  int* __restrict__ bin_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const float v[3] = {c.x[i], c.y[i], c.z[i]};
  const int b = (int)morton_cell(v, bounds, L);
  pbin[i] = b;
  pslot[i] = atomicAdd(bin_count + b, 1);
}

// One thread per point: the sorted cloud (SoA) and each sorted point's caller index.
__global__ __launch_bounds__(256) void k_cell_scatter(CloudArgs c, const int* __restrict__ pbin,
                                                      const int* __restrict__ pslot,
                                                      const int* __restrict__ bin_start, float* __restrict__ sx,
                                                      float* __restrict__ sy, float* __restrict__ sz,
                                                      int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const int j = bin_start[pbin[i]] + pslot[i];
  sx[j] = c.x[i];
  sy[j] = c.y[i];
  sz[j] = c.z[i];
  perm[j] = i;
}

// ---- exclusive scan of bin counts (three passes over groups of kScanGroup bins) ------
constexpr int kScanGroup = 2048;   // 256 threads x 8 bins
constexpr int kScanTop = 1024;     // threads of the one-block pass over the group sums

// Exclusive scan of v over a 256-thread block; lds: 4 words.  Returns the block total.
__device__ __forceinline__ int block_excl_scan256(int& v, int* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    before += u < wid ? lds[u] : 0;
    total += lds[u];
  }
  v = before + x - v;
  __syncthreads();   // lds free again
  return total;
}

__device__ __forceinline__ int64_t scan_n(int64_t n_host, const int64_t* n_dev) { return n_dev ? *n_dev : n_host; }

// Block-stride over the groups: the count of each group.
__global__ __launch_bounds__(256) void k_scan_up(const int* __restrict__ count, int64_t n_host,
                                                 const int64_t* __restrict__ n_dev, int* __restrict__ group_sum) {
  __shared__ int lds[4];
  const int64_t n = scan_n(n_host, n_dev);
  const int64_t groups = (n + kScanGroup - 1) / kScanGroup;
  for (int64_t gi = blockIdx.x; gi < groups; gi += gridDim.x) {
    const int64_t b0 = gi * kScanGroup + threadIdx.x * 8;
    int v = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) v += b0 + u < n ? count[b0 + u] : 0;
    const int tot = block_excl_scan256(v, lds);
    if (threadIdx.x == 0) group_sum[gi] = tot;
  }
}

// One block: exclusive scan of the group counts into group_off (group_off[groups] =
// total); each thread sums a contiguous run of groups.
__global__ __launch_bounds__(kScanTop) void k_scan_top(const int* __restrict__ group_sum, int64_t n_host,
                                                       const int64_t* __restrict__ n_dev,
                                                       int64_t* __restrict__ group_off) {
  __shared__ int64_t lds[kScanTop];
  const int64_t n = scan_n(n_host, n_dev);
  const int64_t groups = (n + kScanGroup - 1) / kScanGroup;
  const int tid = threadIdx.x;
  const int64_t S = (groups + kScanTop - 1) / kScanTop;
  const int64_t b = min((int64_t)tid * S, groups), e = min(b + S, groups);
  int64_t sum = 0;
  for (int64_t i = b; i < e; ++i) sum += group_sum[i];
  lds[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kScanTop; off <<= 1) {   // Hillis-Steele inclusive scan
    const int64_t y = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += y;
    __syncthreads();
  }
  int64_t run = lds[tid] - sum;
  for (int64_t i = b; i < e; ++i) {
    group_off[i] = run;
    run += group_sum[i];
  }
  if (tid == kScanTop - 1) group_off[groups] = lds[tid];
}

// Block-stride over the groups: the first sorted position of every bin.
__global__ __launch_bounds__(256) void k_scan_down(const int* __restrict__ count, int64_t n_host,
                                                   const int64_t* __restrict__ n_dev,
                                                   const int64_t* __restrict__ group_off, int* __restrict__ start) {
  __shared__ int lds[4];
  const int64_t n = scan_n(n_host, n_dev);
  const int64_t groups = (n + kScanGroup - 1) / kScanGroup;
  for (int64_t gi = blockIdx.x; gi < groups; gi += gridDim.x) {
    const int64_t b0 = gi * kScanGroup + threadIdx.x * 8;
    int c[8], v = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = b0 + u < n ? count[b0 + u] : 0;
      v += c[u];
    }
    block_excl_scan256(v, lds);
    int pos = (int)group_off[gi] + v;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u < n) {
        start[b0 + u] = pos;
        pos += c[u];
      }
  }
}

// One thread per (motion, capsule, block of B samples): centre of the endpoints'
// bounding box and the largest endpoint distance from it plus the capsule radius.
// The segment of every sample in the block lies in the convex hull of its endpoints,
// hence inside that sphere.
__global__ __launch_bounds__(256) void k_block_spheres(const CapEntry* __restrict__ table, int64_t M, int T, int K,
                                                       int nb, int B, float4* __restrict__ spheres) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M * K * nb) return;
  const int64_t mk = g / nb;
  const int b = (int)(g - mk * nb);
  const CapEntry* e = table + mk * T;
  const int t0 = b * B, t1 = min(t0 + B, T);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int t = t0; t < t1; ++t) {
    const CapEntry q = e[t];
    const float a[3] = {q.ax, q.ay, q.az}, d[3] = {q.ax + q.bx, q.ay + q.by, q.az + q.bz};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lo[i] = fminf(lo[i], fminf(a[i], d[i]));
      hi[i] = fmaxf(hi[i], fmaxf(a[i], d[i]));
    }
  }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  float r2 = 0.f;
  for (int t = t0; t < t1; ++t) {
    const CapEntry q = e[t];
    const float ax = q.ax - cx, ay = q.ay - cy, az = q.az - cz;
    const float bx = ax + q.bx, by = ay + q.by, bz = az + q.bz;
    r2 = fmaxf(r2, fmaxf(ax * ax + ay * ay + az * az, bx * bx + by * by + bz * bz));
  }
  spheres[g] = make_float4(cx, cy, cz, sqrtf(r2) + e[t0].r);
}

// The group spheres of every (motion, capsule): group i encloses block spheres 8 i ..
// (group_sphere).  One thread per group.
__global__ __launch_bounds__(256) void k_group_spheres(const float4* __restrict__ spheres, int64_t MK, int nb,
                                                       float4* __restrict__ groups) {
  const int ng = cull_group_count(nb);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= MK * ng) return;
  const int64_t mk = g / ng;
  const int gi = (int)(g - mk * ng);
  groups[g] = group_sphere(spheres + mk * nb, kGroupBlocks * gi, min(kGroupBlocks * (gi + 1), nb));
}

// Upper bound of d(X, m) to start from: the smallest test distance over a stride
// sample of the sorted cloud (thread i: sorted point i * stride) and every tstride-th
// sample of the motion, folded into the motion's key.  Any subset of the tests gives a
// value at or above the minimum, and each value is the distance of a real test, so it
// cannot displace the true minimum or its index.
__global__ __launch_bounds__(256) void k_exact_seed(const CapEntry* __restrict__ table, int T, int K,
                                                    const float* __restrict__ sx, const float* __restrict__ sy,
                                                    const float* __restrict__ sz, const int* __restrict__ perm, int N,
                                                    int stride, int tstride, const int* __restrict__ mlist,
                                                    const int* __restrict__ mcount,
                                                    unsigned long long* __restrict__ keys) {
  const int k = blockIdx.x % K;            // one capsule per block
  const int slot = blockIdx.x / K;
  if (mcount && slot >= *mcount) return;
  const int m = mlist ? mlist[slot] : slot;
  const int j = threadIdx.x * stride;
  const bool ok = j < N;
  const float x = ok ? sx[j] : 0.f, y = ok ? sy[j] : 0.f, z = ok ? sz[j] : 0.f;
  int idx[1] = {ok ? perm[j] : -1};
  const ConstF4Ptr tab = (ConstF4Ptr)table;
  const size_t e = ((size_t)m * K + k) * T;
  const float m2 = seed_d2(tab, e, T, tstride, x, y, z);
  float best[1] = {sqrtf(m2) - load_entry(tab, e).r};
  __shared__ unsigned long long wmin[4];
  const unsigned long long k2 = block_min_key<256>(lane_min_key<1>(best, idx), wmin);
  if (threadIdx.x == 0 && k2 != kKeyEmpty) atomicMin(keys + m, k2);
}

// Bounding sphere of each tile of kTilePts consecutive sorted points: centre of the
// points' bounding box and the largest distance from it.  One block per tile.
__global__ __launch_bounds__(256) void k_tile_spheres(const float* __restrict__ sx, const float* __restrict__ sy,
                                                      const float* __restrict__ sz, int N, float4* __restrict__ tile_out,
                                                      float4* __restrict__ wave_out) {
  __shared__ float part[4][6];
  __shared__ float pr[4];
  const int64_t j0 = (int64_t)blockIdx.x * (kCullNT * kCullP);
  tile_wave_spheres<kCullP, kCullNT>(sx, sy, sz, j0, min(j0 + kCullNT * kCullP, (int64_t)N), tile_out + blockIdx.x,
                                     wave_out + 4 * (size_t)blockIdx.x, part, pr);
}

// Coarse pass: one thread per (motion slot, tile, capsule); the capsule is kept for
// the tile if any of its sample blocks may come within the motion's current bound of
// the tile's sphere and of one of its wave groups' spheres (item_may_hit).  Kept items are appended to (list: slot * tiles + tile, caps:
// capsule, count) -- one atomic per wave.  One capsule per item keeps the items short,
// which balances the persistent blocks, since the surviving work concentrates on the
// few tiles near the robot.
__global__ __launch_bounds__(256) void k_cull_list(const float4* __restrict__ tile_sph,
                                                   const float4* __restrict__ wave_sph,
                                                   const float4* __restrict__ spheres,
                                                   const float4* __restrict__ groups, int K, int nb, int tiles,
                                                   int64_t n_slots, const int* __restrict__ mlist,
                                                   const int* __restrict__ mcount,
                                                   const unsigned long long* __restrict__ keys,
                                                   int* __restrict__ list, int* __restrict__ caps,
                                                   int* __restrict__ count) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slots = mcount ? (int64_t)*mcount : n_slots;
  int mask = 0;
  if (g < slots * tiles * K) {
    const int k = (int)(g % K);
    const int64_t st = g / K;
    const int slot = (int)(st / tiles);
    const int tile = (int)(st - (int64_t)slot * tiles);
    const int m = mlist ? mlist[slot] : slot;
    mask = item_may_hit(tile_sph[tile], wave_sph + 4 * (size_t)tile, spheres + ((size_t)m * K + k) * nb,
                        groups + ((size_t)m * K + k) * cull_group_count(nb), nb,
                        key_dist(keys[m])) ? 1 : 0;
  }
  const bool keep = mask != 0;
  const unsigned long long ballot = __ballot(keep);
  int base = 0;
  if ((threadIdx.x & 63) == 0 && ballot) base = atomicAdd(count, __popcll(ballot));
  base = __shfl(base, 0, 64);
  const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0));
  if (keep) {
    list[base + rank] = (int)(g / K);
    caps[base + rank] = (int)(g % K);
  }
}

// One listed item (motion slot, tile of NT P sorted points, capsule) per block
// iteration; each wave owns 64 P consecutive sorted points and decides per sample
// block whether the group can come below its bound.  Persistent
// blocks take items in list order from a queue (count[1]), which keeps them together
// on neighbouring motions and balances the uneven items.  work (optional) counts the
// executed segment tests.
template <int P, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_exact_cull(const CapEntry* __restrict__ table,
                                                   const float4* __restrict__ spheres,
                                                   const float4* __restrict__ wave_spheres, int T, int K, int nb,
                                                   int B, const float* __restrict__ sx, const float* __restrict__ sy,
                                                   const float* __restrict__ sz, const int* __restrict__ perm, int N,
                                                   int tiles, const int* __restrict__ mlist,
                                                   const int* __restrict__ list, const int* __restrict__ caps,
                                                   int* __restrict__ count,
                                                   unsigned long long* __restrict__ keys,
                                                   unsigned long long* __restrict__ work) {
  __shared__ unsigned long long wexec[NT / 64];
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ int s_next;
  const int n_items = count[0];
  int* head = count + 1;   // queue head, zero on entry
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long executed = 0;
  if (threadIdx.x == 0) s_next = atomicAdd(head, 1);
  __syncthreads();
  for (int it = s_next; it < n_items; it = s_next) {
    int nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(head, 1);   // the next item, requested while this one runs
    const int g = list[it];
    const int k = caps[it];
    const int slot = g / tiles;
    const int tile = g - slot * tiles;
    const int m = mlist ? mlist[slot] : slot;
    const float G = key_dist(__hip_atomic_load(keys + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long k2 =
        cull_item<P, NT>((ConstF4Ptr)table, ((size_t)m * K + k) * T, T, spheres + ((size_t)m * K + k) * nb,
                         nb, B, (ConstF4Ptr)(wave_spheres + 4 * (size_t)tile), sx, sy, sz, perm, N, tile, G, wmin,
                         executed);
    if (threadIdx.x == 0) {
      // publish only a new minimum: most items end above the motion's current key
      if (k2 < __hip_atomic_load(keys + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(keys + m, k2);
      s_next = min(nxt, n_items);
    }
    __syncthreads();   // s_next written; wmin reused by the next item
  }
  // executed tests: one add per block, spread over kWorkSlots counters (same-address
  // atomics from every wave would serialise)
  if (lane == 0) wexec[wid] = executed;
  __syncthreads();
  if (threadIdx.x == 0 && work) {
    unsigned long long ex = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) ex += wexec[q];
    if (ex) atomicAdd(work + blockIdx.x % kWorkSlots, ex);
  }
}

// The exact check of the points a network screen sent (sv_check_motions with a screen):
// per motion, the points of the Morton-sorted cloud listed in plist[m N ..] (sorted
// indices, pcount[m] of them, in sorted order; perm maps them to the caller's).  Block
// (motion, tile of NT P listed points); each wave bounds its 64 P points by a sphere
// (box midpoint, largest distance) and, capsule by capsule, runs the sample blocks that
// the sphere test of cull_item cannot rule out under G.  G starts at the smaller of g0
// and the motion's current key and falls with the wave's own results.  With g0 = +inf
// the result is the minimum over the sent points and its lowest index, bit for bit; with
// g0 = eps - band (certified screening, which only asks whether some sent point lies
// within it) it is that minimum whenever the minimum is <= g0, and a value above g0
// otherwise.  The sorted order keeps a wave's points close together, so that its sphere
// is small.
template <int P, int NT>
__global__ __launch_bounds__(NT) void k_fallback_cull(const CapEntry* __restrict__ table,
                                                      const float4* __restrict__ spheres, int T, int K, int nb, int B,
                                                      const float* __restrict__ sx, const float* __restrict__ sy,
                                                      const float* __restrict__ sz, const int* __restrict__ perm, int N,
                                                      int tiles, const int* __restrict__ plist,
                                                      const int* __restrict__ pcount, float g0,
                                                      unsigned long long* __restrict__ keys,
                                                      unsigned long long* __restrict__ work) {
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ unsigned long long wexec[NT / 64];
  const int m = blockIdx.x / tiles;
  const int tile = blockIdx.x - m * tiles;
  const int n_here = pcount[m];
  if (tile * (NT * P) >= n_here) return;           // block-uniform
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int base = tile * (NT * P) + wid * (64 * P) + lane;
  float x[P], y[P], z[P], best[P];
  int idx[P];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int jj = base + p * 64;
    const bool ok = jj < n_here;
    const int j = ok ? plist[(size_t)m * N + jj] : 0;
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
  unsigned long long executed = 0;
  if (__builtin_amdgcn_readfirstlane((int)(base < n_here))) {   // lane 0 holds the wave's first point
    float c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = uniform_f(0.5f * (wave_min(lo[a]) + wave_max(hi[a])));
    float r2 = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (idx[p] >= 0) {
        const float dx = x[p] - c[0], dy = y[p] - c[1], dz = z[p] - c[2];
        r2 = fmaxf(r2, dx * dx + dy * dy + dz * dz);
      }
    const float rw = uniform_f(sqrtf(wave_max(r2)));
    float G = uniform_f(fminf(g0, key_dist(__hip_atomic_load(keys + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))));
    auto skip = [&](float bx, float by, float bz, float br, float g) {
      const float dx = bx - c[0], dy = by - c[1], dz = bz - c[2];
      const float S = g + kCullMargin + rw + br;
      return S < 0.f || dx * dx + dy * dy + dz * dz > S * S;
    };
    for (int k = 0; k < K; ++k) {
      const size_t e = ((size_t)m * K + k) * T;
      const float4* sph = spheres + ((size_t)m * K + k) * nb;
      const float r = load_entry((ConstF4Ptr)table, e).r;
      float m2[P];
#pragma unroll
      for (int p = 0; p < P; ++p) m2[p] = INFINITY;
      int nrun = 0;
      for (int b0 = 0; b0 < nb; b0 += 64) {
        // lane l tests block b0 + l against the bound at the start of the chunk (the
        // bound only falls, so a block failing here fails every later test too)
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
          swept_block<P>((ConstF4Ptr)table, e, t0, t1, x, y, z, m2);
          executed += (unsigned long long)(t1 - t0) * (64 * P);
          if (++nrun % kBoundEvery) continue;   // as in cull_item
          float mm = INFINITY;
#pragma unroll
          for (int p = 0; p < P; ++p)
            if (idx[p] >= 0) mm = fminf(mm, m2[p]);
          G = uniform_f(fminf(G, sqrtf(wave_min(mm)) - r));
        }
      }
#pragma unroll
      for (int p = 0; p < P; ++p) best[p] = fminf(best[p], sqrtf(m2[p]) - r);
    }
  }
  const unsigned long long k2 = block_min_key<NT>(lane_min_key<P>(best, idx), wmin);
  if (threadIdx.x == 0 && k2 < __hip_atomic_load(keys + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMin(keys + m, k2);
  if (work) {
    if (lane == 0) wexec[wid] = executed;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long ex = 0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) ex += wexec[q];
      if (ex) atomicAdd(work + blockIdx.x % kWorkSlots, ex);
    }
  }
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }
int device_cus_cull() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// Blocks of the persistent culled kernel the device holds at once.
int64_t resident_cull_blocks() {
  static int per_cu[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (per_cu[dev] == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_exact_cull<kCullP, kCullNT>, kCullNT, 0) != hipSuccess ||
        b < 1)
      b = 1;
    per_cu[dev] = b;
  }
  return (int64_t)device_cus_cull() * per_cu[dev];
}

}  // namespace

int64_t bin_scan_groups(int64_t cap) { return (cap + kScanGroup - 1) / kScanGroup; }

hipError_t launch_bin_scan(const int* count, int64_t n_host, const int64_t* n_dev, int64_t cap, int* group_sum,
                           int64_t* group_off, int* start, hipStream_t st) {
  const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(bin_scan_groups(cap), 1), 16384);
  hipLaunchKernelGGL(k_scan_up, dim3(g), dim3(256), 0, st, count, n_host, n_dev, group_sum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, st, group_sum, n_host, n_dev, group_off);
  hipLaunchKernelGGL(k_scan_down, dim3(g), dim3(256), 0, st, count, n_host, n_dev, group_off, start);
  return hipGetLastError();
}

int cull_blocks(int T, int kind) { return cull_block_count(T, kind); }
int cull_tiles(int64_t N) { return (int)((N + kCullNT * kCullP - 1) / (kCullNT * kCullP)); }

hipError_t launch_cull_sort(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                            const CullWs& w, hipStream_t st) {
  if (c.n == 0) return hipSuccess;
  const int K = rb.n_caps, T = mo.T, nb = cull_block_count(T, mo.kind), B = cull_block_len(T, mo.kind);
  hipError_t e;
  const int64_t nbins = (int64_t)1 << (3 * w.level);
  hipLaunchKernelGGL(k_cull_init, dim3(grid_for(std::max<int64_t>(nbins, 6), 256)), dim3(256), 0, st, w.bounds,
                     w.bin_count, nbins, w.list_count);
  hipLaunchKernelGGL(k_cloud_bounds, dim3(std::min<unsigned>(grid_for(c.n, 256), 1024)), dim3(256), 0, st, c,
                     w.bounds);
  hipLaunchKernelGGL(k_cell_bin, dim3(grid_for(c.n, 256)), dim3(256), 0, st, c, w.bounds, w.level, w.pbin, w.pslot,
                     w.bin_count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_bin_scan(w.bin_count, nbins, nullptr, nbins, w.group_sum, w.group_off, w.bin_start, st)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_cell_scatter, dim3(grid_for(c.n, 256)), dim3(256), 0, st, c, w.pbin, w.pslot, w.bin_start,
                     w.sx, w.sy, w.sz, w.perm);
  if (mo.n > 0) {
    hipLaunchKernelGGL(k_block_spheres, dim3(grid_for(mo.n * K * nb, 256)), dim3(256), 0, st, table, mo.n, T, K, nb, B,
                       w.spheres);
    hipLaunchKernelGGL(k_group_spheres, dim3(grid_for(mo.n * K * cull_group_count(nb), 256)), dim3(256), 0, st,
                       w.spheres, mo.n * K, nb, w.group_spheres);
  }
  return hipGetLastError();
}

hipError_t launch_cull_pass(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                            const int* mlist, const int* mcount, int64_t n_slots, unsigned long long* keys,
                            const CullWs& w, bool reset, hipStream_t st) {
  if (n_slots == 0 || c.n == 0) return hipSuccess;
  const int K = rb.n_caps, T = mo.T, nb = cull_block_count(T, mo.kind), B = cull_block_len(T, mo.kind);
  hipError_t e;
  if (reset && (e = launch_fill_i32(w.list_count, 2, 0, st)) != hipSuccess) return e;
  const int stride = std::max(1, c.n / 256);
  hipLaunchKernelGGL(k_exact_seed, dim3((unsigned)(n_slots * K)), dim3(256), 0, st, table, T, K, w.sx, w.sy, w.sz, w.perm,
                     c.n, stride, seed_stride(T), mlist, mcount, keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int tiles = (c.n + kCullNT * kCullP - 1) / (kCullNT * kCullP);
  const int64_t items = n_slots * tiles;
  if (items * K > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_tile_spheres, dim3((unsigned)tiles), dim3(256), 0, st, w.sx, w.sy, w.sz, c.n,
                     w.tile_spheres, w.wave_spheres);
  hipLaunchKernelGGL(k_cull_list, dim3(grid_for(items * K, 256)), dim3(256), 0, st, w.tile_spheres, w.wave_spheres,
                     w.spheres, w.group_spheres, K, nb,
                     tiles, n_slots, mlist, mcount, keys, w.list, w.list_caps, w.list_count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int blocks = (int)std::min<int64_t>(items * K, resident_cull_blocks());
  hipLaunchKernelGGL((k_exact_cull<kCullP, kCullNT>), dim3(blocks), dim3(kCullNT), 0, st, table, w.spheres,
                     w.wave_spheres, T, K, nb, B, w.sx, w.sy, w.sz, w.perm, c.n, tiles, mlist, w.list, w.list_caps,
                     w.list_count, keys, w.work);
  return hipGetLastError();
}

hipError_t launch_exact_culled(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                               const int* mlist, const int* mcount, int64_t n_slots, unsigned long long* keys,
                               const CullWs& w, hipStream_t st) {
  if (n_slots == 0 || c.n == 0) return hipSuccess;
  hipError_t e = launch_cull_sort(rb, table, mo, c, w, st);
  if (e != hipSuccess) return e;
  return launch_cull_pass(rb, table, mo, c, mlist, mcount, n_slots, keys, w, false, st);
}

hipError_t launch_fallback_culled(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, int N,
                                  const int* plist, const int* pcount, float g0, unsigned long long* keys,
                                  const CullWs& w, hipStream_t st) {
  if (mo.n == 0 || N == 0) return hipSuccess;
  const int K = rb.n_caps, T = mo.T, nb = cull_block_count(T, mo.kind), B = cull_block_len(T, mo.kind);
  const int tiles = (N + kCullNT * kCullP - 1) / (kCullNT * kCullP);
  const int64_t blocks = mo.n * tiles;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_fallback_cull<kCullP, kCullNT>), dim3((unsigned)blocks), dim3(kCullNT), 0, st, table, w.spheres,
                     T, K, nb, B, w.sx, w.sy, w.sz, w.perm, N, tiles, plist, pcount, g0, keys, w.work);
  return hipGetLastError();
}

}  // namespace sv
