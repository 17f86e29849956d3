// Exact check of a batch of uneven requests in one fixed launch sequence (gfx950).
//
// A request is the question of Sec. IV-B -- d(X, m) = min over the cloud of the swept
// distance f_d(x, m) of eq. (1)-(4), and "free iff d > eps" (Alg. 1) -- for one set of
// motions against one cloud.  Requests of a batch differ widely in size (a single
// motion against a small cloud next to thousands of motions against a large one), so
// one launch per request leaves the GPU idle on the small ones and queues everything
// behind the large ones.  Here the whole batch is four kernels whose grids depend only
// on capacities:
//   k_batch_plan     one block: validate the request table, order requests by work
//                    (smallest first), per-request offsets and work-item counts;
//   k_batch_tables   capsule table of every (request, motion, sample); key reset;
//   k_batch_exact    persistent blocks drain a work queue of (request, motion, chunk
//                    of point tiles) items; per-point arithmetic is the shared
//                    swept_min, so results equal the per-call kernels' bit for bit;
//                    the block that retires a request's last item finalizes it and
//                    stamps its completion tick;
//   k_batch_fk64 / k_batch_exact64 / k_batch_finalize64: FP64 recheck of the motions
//                    within the certified band of eps, then their requests' stamps.
// No kernel waits on another block: the queue only hands out items, so every block
// exits once the queue is empty, whatever the residency.
#include "sv_cull_common.h"

namespace sv {
namespace {

constexpr int kPlanThreads = 1024;

struct BatchArgs {
  const sv_request* reqs;
  int n_req, max_requests;
  int K;
  int max_T;
  int max_band;
  int64_t max_motions, max_samples, max_points;
  float eps, band;
  int tile_pts;  // points per tile (threads * ppl)
  int tpi;       // tiles per work item
  int culled;    // culled pass (1) or the persistent dense kernel (0)
  int gangs;     // culled pass: queues of the persistent blocks (block index mod gangs)
  int div_lin, div_spl;   // culled pass: sample-block divisors (cull_block_len)
  BatchWs w;
  unsigned long long* done_ticks;
  int* status_out;
};

constexpr int kCullTilePts = kCullNT * kCullP;   // sorted points per tile of the culled pass

// Last index r in [0, n) with off[r] <= g (off[0] = 0 <= g; requests with no entries
// share their offset with the next one, so r is the request that holds g).
__device__ __forceinline__ int find_seg(const int64_t* __restrict__ off, int n, int64_t g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Exclusive prefix sums of get(0..n) into out[0..n] (out[n] = total), one block of
// kPlanThreads threads; lds: kPlanThreads words.  Returns the total in every thread.
template <typename F>
__device__ int64_t plan_scan(int n, F get, int64_t* __restrict__ out, int64_t* lds) {
  const int tid = threadIdx.x;
  const int S = (n + kPlanThreads - 1) / kPlanThreads;
  const int b = min(tid * S, n), e = min(b + S, n);
  int64_t sum = 0;
  for (int i = b; i < e; ++i) sum += get(i);
  lds[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kPlanThreads; off <<= 1) {
    const int64_t v = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += v;
    __syncthreads();
  }
  int64_t run = lds[tid] - sum;
  for (int i = b; i < e; ++i) {
    out[i] = run;
    run += get(i);
  }
  const int64_t total = lds[kPlanThreads - 1];
  if (tid == 0) out[n] = total;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(BatchArgs a) {
  __shared__ int64_t lds[kPlanThreads];
  __shared__ int64_t cost[kMaxBatchRequests];
  __shared__ int s_status;
  const int tid = threadIdx.x, n = a.n_req;
  BatchWs& w = a.w;
  if (tid == 0) s_status = 0;
  if (a.done_ticks && tid == 0) a.done_ticks[n] = wall_clock64();
  __syncthreads();
  for (int r = tid; r < n; r += kPlanThreads) {
    const sv_motions mo = a.reqs[r].motions;
    const sv_cloud cl = a.reqs[r].cloud;
    bool ok = (mo.kind == SV_LINEAR || mo.kind == SV_SPLINE) && mo.T >= 1 && mo.n >= 0 && cl.n >= 0;
    if (ok && mo.n > 0) ok = mo.q0 && mo.q1 && (mo.kind != SV_SPLINE || mo.via);
    if (ok && cl.n > 0) ok = cl.x && cl.y && cl.z;
    bool fits = ok && mo.T <= a.max_T && cl.n <= a.max_points && mo.n <= a.max_motions;
    const int64_t M = fits ? mo.n : 0, N = fits ? cl.n : 0, T = fits ? mo.T : 0;
    const int64_t tiles = (N + a.tile_pts - 1) / a.tile_pts;
    const int64_t chunks = (tiles + a.tpi - 1) / a.tpi;
    const int64_t items = (M > 0 && chunks > 0) ? M * chunks : 1;   // an empty request still retires once
    if (items > 0x7fffffffLL) fits = false;
    if (!ok) atomicOr(&s_status, SV_BATCH_BAD_REQUEST);
    if (ok && !fits) atomicOr(&s_status, SV_BATCH_OVER_CAPACITY);
    w.n_motions[r] = M;
    w.n_samples[r] = M * T;
    w.n_items[r] = items;
    w.tiles[r] = (int)tiles;
    w.chunks[r] = (int)chunks;
    w.remaining[r] = a.culled ? 1 : (int)items;   // culled: a token the list pass releases
    w.n_points[r] = N;
    w.level[r] = morton_level(N);
    const int64_t ctiles = (N + kCullTilePts - 1) / kCullTilePts;
    w.n_cands[r] = M * ctiles * a.K;
    cost[r] = M * N * T;
    if (a.done_ticks) a.done_ticks[r] = 0;
  }
  for (int s = tid; s < a.max_band; s += kPlanThreads) w.keys64[s] = kKeyEmpty;
  for (int s = tid; s < kWorkSlots; s += kPlanThreads) w.work[s] = 0;
  __syncthreads();
  const int64_t tm = plan_scan(n, [&](int i) { return w.n_motions[i]; }, w.motion_off, lds);
  const int64_t ts = plan_scan(n, [&](int i) { return w.n_samples[i]; }, w.sample_off, lds);
  // smallest estimated work first; equal work keeps request order
  for (int r = tid; r < n; r += kPlanThreads) {
    const int64_t c = cost[r];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (cost[j] < c) || (cost[j] == c && j < r);
    w.order[rank] = r;
  }
  __syncthreads();
  const int64_t ti = plan_scan(n, [&](int p) { return w.n_items[w.order[p]]; }, w.item_off, lds);
  const int64_t tp = plan_scan(n, [&](int i) { return w.n_points[i]; }, w.point_off, lds);
  const int64_t tt = plan_scan(n, [&](int i) { return (w.n_points[i] + kCullTilePts - 1) / kCullTilePts; },
                               w.tile_off, lds);
  const int64_t tc = plan_scan(n, [&](int p) { return w.n_cands[w.order[p]]; }, w.cand_off, lds);
  const int64_t tb = plan_scan(n, [&](int i) { return (int64_t)1 << (3 * w.level[i]); }, w.bin_off, lds);
  for (int r = tid; r < n * 6; r += kPlanThreads) w.bounds[r] = (r % 6) < 3 ? 0xffffffffu : 0u;
  for (int p = tid; p < n; p += kPlanThreads) {   // offsets from the scans above (same block)
    const int r = w.order[p];
    BatchReq q;
    q.sample_off = w.sample_off[r];
    q.point_off = (int)w.point_off[r];
    q.motion_off = (int)w.motion_off[r];
    q.n_points = (int)w.n_points[r];
    q.T = a.reqs[r].motions.T;
    q.nb = cull_block_count(q.T, a.reqs[r].motions.kind, a.div_lin, a.div_spl);
    q.blen = cull_block_len(q.T, a.reqs[r].motions.kind, a.div_lin, a.div_spl);
    q.list_off = (int)w.cand_off[p];
    q.tile_off = (int)w.tile_off[r];
    w.req[r] = q;
    w.fill[r] = 0;
  }
  if (tid == 0) {
    int st = s_status;
    if (tm > a.max_motions || ts > a.max_samples || tm > 0x7fffffffLL) st |= SV_BATCH_OVER_CAPACITY;
    if (a.culled && (tp > w.point_cap || tt > w.tile_cap || tc > w.cand_cap || tb > w.bin_cap))
      st |= SV_BATCH_OVER_CAPACITY;
    const bool run = (st & (SV_BATCH_BAD_REQUEST | SV_BATCH_OVER_CAPACITY)) == 0;
    w.plan->status = st;
    w.plan->band_count = 0;
    w.plan->total_items = run ? ti : 0;
    w.plan->total_samples = run ? ts : 0;
    w.plan->next_item = 0;
    w.plan->total_motions = run ? tm : 0;
    w.plan->total_points = run ? tp : 0;
    w.plan->total_tiles = run ? tt : 0;
    w.plan->total_cands = run ? tc : 0;
    w.plan->total_bins = run ? tb : 0;
  }
}

// One thread per (request, motion, sample), grid-stride: capsule entries at
// table[(sample_off[r] + m T) K + k T + t]; sample 0 also resets the motion's key.
__global__ __launch_bounds__(256) void k_batch_tables(Robot32 rb, BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_samples;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_seg(w.sample_off, a.n_req, g);
    const sv_motions mo = a.reqs[r].motions;
    const int64_t local = g - w.sample_off[r];
    const int64_t m = local / mo.T;
    const int t = (int)(local - m * mo.T);
    if (t == 0) w.keys[w.motion_off[r] + m] = kKeyEmpty;
    if (a.reqs[r].cloud.n == 0) continue;
    write_entries(rb, mo.kind, mo.q0 + m * rb.dof, mo.q1 + m * rb.dof, mo.via ? mo.via + m * 2 * rb.dof : nullptr, t,
                  mo.T, w.table + (size_t)(w.sample_off[r] + m * mo.T) * rb.n_caps + t, mo.T);
  }
}

// Results of every motion of request r (all threads of the block); motions within the
// band are queued for the FP64 recheck, and the request is stamped now unless it has
// one (the recheck stamps it then).
template <int NT>
__device__ void finalize_request(const BatchArgs& a, int r, int* s_band) {
  const BatchWs& w = a.w;
  const sv_results out = a.reqs[r].out;
  const int64_t M = w.n_motions[r], g0 = w.motion_off[r];
  for (int64_t m = threadIdx.x; m < M; m += NT) {
    const unsigned long long key = __hip_atomic_load(w.keys + g0 + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    float d;
    int arg;
    decode_key(key, &d, &arg);
    write_result(out, m, d, arg, a.eps);
    if (fabsf(d - a.eps) <= a.band) {
      const int s = atomicAdd(&w.plan->band_count, 1);
      if (s < a.max_band) {
        w.band_list[s] = (int)(g0 + m);
        atomicAdd(s_band, 1);
      } else {
        atomicOr(&w.plan->status, SV_BATCH_BAND_OVERFLOW);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && *s_band == 0 && a.done_ticks) {
    __threadfence();
    a.done_ticks[r] = wall_clock64();
  }
}

// Retires n items of request r (all threads of the block): one release fence and one
// counter update for the run, and the block that retires the request's last item
// finalizes it after an acquire fence.  (A fence per item would write back and
// invalidate the compute unit's L2 once per item.)
template <int NT>
__device__ void retire_run(const BatchArgs& a, int r, int n, int* s_last, int* s_band) {
  if (threadIdx.x == 0) {
    *s_band = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int old = __hip_atomic_fetch_add(a.w.remaining + r, -n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_last = old == n;
    if (old == n) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (*s_last) finalize_request<NT>(a, r, s_band);
  __syncthreads();
}

template <int P, int NT>
__global__ __launch_bounds__(NT) void k_batch_exact(BatchArgs a) {
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ int64_t s_item;
  __shared__ int s_last, s_band;
  const BatchWs& w = a.w;
  const int tid = threadIdx.x;
  const int64_t total = w.plan->total_items;
  const ConstF4Ptr tab = (ConstF4Ptr)w.table;
  int cur = -1, pending = 0;   // request of the current run, items retired in it (block-uniform)
  for (;;) {
    if (tid == 0) s_item = (int64_t)atomicAdd(&w.plan->next_item, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= total) break;
    const int pos = find_seg(w.item_off, a.n_req, item);
    const int r = w.order[pos];
    if (r != cur) {
      if (pending) retire_run<NT>(a, cur, pending, &s_last, &s_band);
      cur = r;
      pending = 0;
    }
    const int64_t local = item - w.item_off[pos];
    const int chunks = w.chunks[r];
    if (w.n_motions[r] > 0 && chunks > 0) {
      const sv_cloud cl = a.reqs[r].cloud;
      const int T = a.reqs[r].motions.T;
      const int N = (int)cl.n, tiles = w.tiles[r];
      const int64_t m = local / chunks;
      const int c = (int)(local - m * chunks);
      const size_t e0 = (size_t)(w.sample_off[r] + m * T) * a.K;
      unsigned long long key = kKeyEmpty;
      const int t1 = min((c + 1) * a.tpi, tiles);
      for (int tile = c * a.tpi; tile < t1; ++tile) {
        const int base = tile * (NT * P) + tid;
        float x[P], y[P], z[P], best[P];
        int idx[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const int j = base + p * NT;
          const bool ok = j < N;
          idx[p] = ok ? j : -1;
          x[p] = ok ? cl.x[j] : 0.f;
          y[p] = ok ? cl.y[j] : 0.f;
          z[p] = ok ? cl.z[j] : 0.f;
        }
        swept_min<P>(tab, e0, T, a.K, x, y, z, best);
        const unsigned long long kk = lane_min_key<P>(best, idx);
        key = kk < key ? kk : key;
      }
      const unsigned long long k2 = block_min_key<NT>(key, wmin);
      if (tid == 0 && k2 != kKeyEmpty) atomicMin(w.keys + w.motion_off[r] + m, k2);
    }
    ++pending;
    __syncthreads();   // s_item and wmin reused by the next item
  }
  if (pending) retire_run<NT>(a, cur, pending, &s_last, &s_band);
}

// ---- culled pass -----------------------------------------------------------------
// All requests' clouds are sorted together by (request, Morton cell within the
// request's bounds), so request r's sorted points occupy [point_off[r], point_off[r] +
// N_r).  Candidates (motion, tile of kCullTilePts sorted points, capsule) are listed in
// work order (smallest request first) when a sample block of the capsule may come
// within the motion's bound of the tile; the persistent kernel then takes the list in
// order, so small requests complete first.  Every request carries a token in
// remaining[] besides its listed items; the last of them to retire finalizes it.

// Per-request bounds of the points (order-preserving keys).  Each block takes one
// contiguous run of the concatenated points, each thread keeps running bounds per
// request, and a block whose final runs share one request reduces them and issues one
// atomic per bound (per wave, the atomics of a 200,000-point request had queued on its six
// words: 0.65 ms of the 64-request batch).
__global__ __launch_bounds__(256) void k_batch_bounds(BatchArgs a) {
  __shared__ unsigned red[4][6];
  __shared__ int rlo[4], rhi[4];
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_points;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // one contiguous run of points per block, so that a block's points mostly share a request
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * chunk, c1 = min(c0 + chunk, total);
  int rc = -1;
  unsigned b[6];
  auto reset = [&]() {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      b[q] = ord_f32(INFINITY);
      b[3 + q] = ord_f32(-INFINITY);
    }
  };
  auto flush = [&]() {
    if (rc < 0) return;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      atomicMin(w.bounds + 6 * rc + q, b[q]);
      atomicMax(w.bounds + 6 * rc + 3 + q, b[3 + q]);
    }
  };
  reset();
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const int r = find_seg(w.point_off, a.n_req, i);
    if (r != rc) {   // a request boundary inside the thread's run
      flush();
      reset();
      rc = r;
    }
    const sv_cloud cl = a.reqs[r].cloud;
    const int64_t j = i - w.point_off[r];
    const float v[3] = {cl.x[j], cl.y[j], cl.z[j]};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      b[q] = min(b[q], ord_f32(v[q]));
      b[3 + q] = max(b[3 + q], ord_f32(v[q]));
    }
  }
  // the block's final runs: one set of atomics if they all belong to one request
  int mn = rc < 0 ? 0x7fffffff : rc, mx = rc;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off, 64));
    mx = max(mx, __shfl_xor(mx, off, 64));
  }
  if (lane == 0) {
    rlo[wid] = mn;
    rhi[wid] = mx;
  }
  __syncthreads();
  const int bmn = min(min(rlo[0], rlo[1]), min(rlo[2], rlo[3]));
  const int bmx = max(max(rhi[0], rhi[1]), max(rhi[2], rhi[3]));
  if (bmx < 0) return;                     // no points in this block
  if (bmn != bmx) {                        // several requests: each thread its own
    flush();
    return;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    unsigned x = b[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned y = __shfl_xor(x, off, 64);
      x = q < 3 ? min(x, y) : max(x, y);
    }
    if (lane == 0) red[wid][q] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      atomicMin(w.bounds + 6 * bmx + q, min(min(red[0][q], red[1][q]), min(red[2][q], red[3][q])));
      atomicMax(w.bounds + 6 * bmx + 3 + q, max(max(red[0][3 + q], red[1][3 + q]), max(red[2][3 + q], red[3][3 + q])));
    }
  }
}

// Counting sort of all requests' points by (request, Morton cell of the request's
// bounds): request r's 8^L_r cells are bins [bin_off[r], bin_off[r+1]).  Points of
// one bin land in the order their atomics were served; nothing downstream depends
// on the order within a bin (every result is a minimum over all points, keyed by the
// caller's point index).

// Grid-stride zero fill of the bin counters in use.
__global__ __launch_bounds__(256) void k_batch_clear_bins(BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_bins;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    w.bin_count[i] = 0;
}

// Grid-stride over the points: bin of each point and its slot within the bin.
__global__ __launch_bounds__(256) void k_batch_bin(BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_points;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_seg(w.point_off, a.n_req, i);
    const sv_cloud cl = a.reqs[r].cloud;
    const int64_t j = i - w.point_off[r];
    const float v[3] = {cl.x[j], cl.y[j], cl.z[j]};
    const int64_t bin = w.bin_off[r] + morton_cell(v, w.bounds + 6 * r, w.level[r]);
    w.pbin[i] = (int)bin;
    w.pslot[i] = atomicAdd(w.bin_count + bin, 1);
  }
}

// Grid-stride over the points: sorted points (SoA) and their index in their
// request's cloud.  Request r's points land in [point_off[r], point_off[r] + N_r).
__global__ __launch_bounds__(256) void k_batch_scatter(BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_points;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_seg(w.point_off, a.n_req, i);
    const sv_cloud cl = a.reqs[r].cloud;
    const int64_t local = i - w.point_off[r];
    const int j = w.bin_start[w.pbin[i]] + w.pslot[i];
    w.sx[j] = cl.x[local];
    w.sy[j] = cl.y[local];
    w.sz[j] = cl.z[local];
    w.sidx[j] = (int)local;
  }
}

// Block-stride over the tiles of all requests: the spheres of each tile's sorted points
// and of its four wave groups.
__global__ __launch_bounds__(256) void k_batch_tile_spheres(BatchArgs a) {
  const BatchWs& w = a.w;
  __shared__ float part[4][6];
  __shared__ float pr[4];
  const int64_t total = w.plan->total_tiles;
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int r = find_seg(w.tile_off, a.n_req, t);
    const int64_t j0 = w.point_off[r] + (t - w.tile_off[r]) * kCullTilePts;
    const int64_t j1 = min(j0 + kCullTilePts, w.point_off[r] + w.n_points[r]);
    tile_wave_spheres<kCullP, kCullNT>(w.sx, w.sy, w.sz, j0, j1, w.tile_sph + t, w.wave_sph + 4 * t, part, pr);
    __syncthreads();   // part, pr reused by the next tile
  }
}

// The sphere of sample block b of capsule k of global motion g (q = (g K + k) nb_max
// + b), at spheres[q]: centred on the block's segment end points, radius to the
// farthest end point plus the capsule radius.
__device__ __forceinline__ void block_sphere(const BatchArgs& a, int64_t q) {
  const BatchWs& w = a.w;
  const int64_t gk = q / w.nb_max;
  const int b = (int)(q - gk * w.nb_max);
  const int64_t g = gk / a.K;
  const int k = (int)(gk - g * a.K);
  const int r = find_seg(w.motion_off, a.n_req, g);
  const int T = a.reqs[r].motions.T, kind = a.reqs[r].motions.kind;
  const int nb = cull_block_count(T, kind, a.div_lin, a.div_spl);
  if (b >= nb || w.n_points[r] == 0) return;
  const int64_t m = g - w.motion_off[r];
  const CapEntry* e = w.table + (size_t)(w.sample_off[r] + m * T) * a.K + (size_t)k * T;
  const int B = cull_block_len(T, kind, a.div_lin, a.div_spl);
  const int t0 = b * B, t1 = min(t0 + B, T);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int t = t0; t < t1; ++t) {
    const CapEntry c = e[t];
    const float p0[3] = {c.ax, c.ay, c.az}, p1[3] = {c.ax + c.bx, c.ay + c.by, c.az + c.bz};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lo[i] = fminf(lo[i], fminf(p0[i], p1[i]));
      hi[i] = fmaxf(hi[i], fmaxf(p0[i], p1[i]));
    }
  }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  float r2 = 0.f;
  for (int t = t0; t < t1; ++t) {
    const CapEntry c = e[t];
    const float ax = c.ax - cx, ay = c.ay - cy, az = c.az - cz;
    const float bx = ax + c.bx, by = ay + c.by, bz = az + c.bz;
    r2 = fmaxf(r2, fmaxf(ax * ax + ay * ay + az * az, bx * bx + by * by + bz * bz));
  }
  w.spheres[(size_t)gk * w.nb_max + b] = make_float4(cx, cy, cz, sqrtf(r2) + e[t0].r);
}

// Grid-stride over (motion, capsule, sample block) of the batch.
__global__ __launch_bounds__(256) void k_batch_block_spheres(BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_motions * a.K * w.nb_max;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x)
    block_sphere(a, q);
}

// Grid-stride over (motion, capsule, group of kGroupBlocks sample blocks): the group
// spheres of the item filter (group_sphere over the request's blocks).
__global__ __launch_bounds__(256) void k_batch_group_spheres(BatchArgs a) {
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_motions * a.K * w.ng_max;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t gk = q / w.ng_max;
    const int gi = (int)(q - gk * w.ng_max);
    const int64_t g = gk / a.K;
    const int r = find_seg(w.motion_off, a.n_req, g);
    const int nb = cull_block_count(a.reqs[r].motions.T, a.reqs[r].motions.kind, a.div_lin, a.div_spl);
    if (kGroupBlocks * gi >= nb || w.n_points[r] == 0) continue;
    w.gspheres[q] = group_sphere(w.spheres + (size_t)gk * w.nb_max, kGroupBlocks * gi,
                                 min(kGroupBlocks * (gi + 1), nb));
  }
}

// The seed bound of (motion g, capsule k) from a stride sample of 256 points of the
// request's sorted cloud and every seed_stride(T)-th sample (a 256-thread block).
__device__ void seed_bound(const BatchArgs& a, int64_t g, int k, unsigned long long* wmin) {
  const BatchWs& w = a.w;
  const int r = find_seg(w.motion_off, a.n_req, g);
  const int64_t N = w.n_points[r];
  if (N == 0) return;   // block-uniform
  const int T = a.reqs[r].motions.T;
  const int64_t m = g - w.motion_off[r];
  const int64_t stride = max((int64_t)1, N / 256);
  const int64_t j = (int64_t)threadIdx.x * stride;
  const bool ok = j < N;
  const int64_t js = w.point_off[r] + (ok ? j : 0);
  const float x = ok ? w.sx[js] : 0.f, y = ok ? w.sy[js] : 0.f, z = ok ? w.sz[js] : 0.f;
  int idx[1] = {ok ? w.sidx[js] : -1};
  const ConstF4Ptr tab = (ConstF4Ptr)w.table;
  const size_t e = (size_t)(w.sample_off[r] + m * T) * a.K + (size_t)k * T;
  const float m2 = seed_d2(tab, e, T, seed_stride(T), x, y, z);
  float best[1] = {sqrtf(m2) - load_entry(tab, e).r};
  const unsigned long long k2 = block_min_key<256>(lane_min_key<1>(best, idx), wmin);
  if (threadIdx.x == 0 && k2 != kKeyEmpty) atomicMin(w.keys + g, k2);
}

// Block-stride over (motion, capsule) of the batch.
__global__ __launch_bounds__(256) void k_batch_seed(BatchArgs a) {
  __shared__ unsigned long long wmin[4];
  const BatchWs& w = a.w;
  const int64_t total = w.plan->total_motions * a.K;
  for (int64_t gk = blockIdx.x; gk < total; gk += gridDim.x) {
    const int64_t g = gk / a.K;
    seed_bound(a, g, (int)(gk - g * a.K), wmin);
    __syncthreads();   // wmin reused by the next pair
  }
}

// One thread per candidate (in work order) up to the capacity: keep the item if any
// of its capsule's sample blocks may come within the motion's bound of the tile and of
// one of its wave groups (item_may_hit).
// Kept items are appended in work order (one atomic per wave); each request's count
// goes to remaining[r], one atomic per wave when its kept items share a request.
__device__ __forceinline__ void cull_list_step(const BatchArgs& a, int64_t c, int64_t total) {
  const BatchWs& w = a.w;
  bool keep = false;
  int r = -1, g32 = 0, tk = 0;
  if (c < total) {
    const int p = find_seg(w.cand_off, a.n_req, c);
    r = w.order[p];
    const int64_t tiles = w.tile_off[r + 1] - w.tile_off[r];
    const int64_t local = c - w.cand_off[p];
    const int64_t m = local / (tiles * a.K);
    const int64_t rem = local - m * tiles * a.K;
    const int t = (int)(rem / a.K);
    const int k = (int)(rem - (int64_t)t * a.K);
    const int64_t g = w.motion_off[r] + m;
    const int64_t tile = w.tile_off[r] + t;
    keep = item_may_hit(w.tile_sph[tile], w.wave_sph + 4 * tile, w.spheres + ((size_t)g * a.K + k) * w.nb_max,
                        w.gspheres + ((size_t)g * a.K + k) * w.ng_max,
                        cull_block_count(a.reqs[r].motions.T, a.reqs[r].motions.kind, a.div_lin, a.div_spl),
                        key_dist(w.keys[g]));
    g32 = (int)g;
    tk = (t << 4) | k;
  }
  const unsigned long long ballot = __ballot(keep);
  if (!ballot) return;
  // kept items go to their request's segment of the list, in any order within it;
  // one atomic per wave when the wave's kept items share a request
  const int first = __ffsll((long long)ballot) - 1;
  const int r0 = __shfl(r, first, 64);
  int slot;
  if (__ballot(keep && r != r0) == 0) {
    int base = 0;
    if ((threadIdx.x & 63) == 0) base = atomicAdd(w.fill + r0, __popcll(ballot));
    base = __shfl(base, 0, 64);
    slot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0));
  } else {
    slot = keep ? atomicAdd(w.fill + r, 1) : 0;
  }
  if (keep) {
    const int at = w.req[r].list_off + slot;
    w.list_g[at] = g32;
    w.list_tk[at] = tk;
  }
}

__global__ __launch_bounds__(256) void k_batch_cull_list(BatchArgs a) {
  const int64_t total = a.w.plan->total_cands;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x)
    cull_list_step(a, base + threadIdx.x, total);   // whole waves: the step appends per wave
}

// One block per request: its listed items become its remaining count; a request with
// no listed item (no motion or no point) is finalized here.
__global__ __launch_bounds__(256) void k_batch_counts(BatchArgs a) {
  __shared__ int s_band;
  const int r = blockIdx.x;
  if (r >= a.n_req || (a.w.plan->status & (SV_BATCH_BAD_REQUEST | SV_BATCH_OVER_CAPACITY))) return;   // nothing runs
  const int items = a.w.fill[r];
  if (threadIdx.x == 0) {
    s_band = 0;
    a.w.remaining[r] = items;
  }
  __syncthreads();
  if (items == 0) finalize_request<256>(a, r, &s_band);
}

// One thread: requests are dealt to the gangs in work order (smallest estimated work
// first), each to the gang with the fewest items so far.
__global__ void k_batch_gangs(BatchArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const BatchWs& w = a.w;
  const int G = a.gangs;
  int load[kMaxGangs], cnt[kMaxGangs];
  for (int g = 0; g < G; ++g) {
    load[g] = 0;
    cnt[g] = 0;
    w.gang_head[g] = 0;
  }
  const bool run = (w.plan->status & (SV_BATCH_BAD_REQUEST | SV_BATCH_OVER_CAPACITY)) == 0;
  const int R = a.max_requests;
  for (int p = 0; run && p < a.n_req; ++p) {
    const int r = w.order[p];
    const int items = w.fill[r];
    if (items == 0) continue;
    int best = 0;
    for (int g = 1; g < G; ++g) best = load[g] < load[best] ? g : best;
    w.gang_req[best * R + cnt[best]] = r;
    w.gang_off[best * (R + 1) + cnt[best]] = load[best];
    load[best] += items;
    ++cnt[best];
  }
  for (int g = 0; g < G; ++g) {
    w.gang_off[g * (R + 1) + cnt[g]] = load[g];
    w.gang_n[g] = cnt[g];
    w.gang_total[g] = load[g];
  }
}

// Thread 0: the next item for a block of gang *gang (moving to the next gang when its
// queue is empty): *r its request (-1: none left), *slot its list slot.
__device__ void claim_item(const BatchArgs& a, int* gang, int g0, int* r, int* slot) {
  const BatchWs& w = a.w;
  for (;;) {
    const int g = *gang;
    const unsigned idx = atomicAdd(w.gang_head + g, 1u);
    if ((int)idx < w.gang_total[g]) {
      const int* off = w.gang_off + g * (a.max_requests + 1);
      int lo = 0, hi = w.gang_n[g];   // last j with off[j] <= idx
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= (int)idx) lo = mid; else hi = mid;
      }
      *r = w.gang_req[g * a.max_requests + lo];
      *slot = w.req[*r].list_off + ((int)idx - off[lo]);
      return;
    }
    *gang = (g + 1) % a.gangs;
    if (*gang == g0) {
      *r = -1;
      return;
    }
  }
}

// Persistent blocks take listed items from their gang's queue (the next item is
// claimed while the current one runs).  A gang works through its requests in order, so
// a block touches only a few requests; it counts the items it retires per request and
// publishes the count (one release fence) when it moves to another request or runs
// out of items.
template <int P, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_cull(BatchArgs a) {
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ unsigned long long wexec[NT / 64];
  __shared__ int s_last, s_band, s_r, s_slot;
  const BatchWs& w = a.w;
  const int g0 = blockIdx.x % a.gangs;
  int gang = g0;   // thread 0's current queue
  unsigned long long executed = 0;
  int cur = -1, pending = 0;   // request of the current run, items retired in it (block-uniform)
  if (threadIdx.x == 0) claim_item(a, &gang, g0, &s_r, &s_slot);
  __syncthreads();
  for (;;) {
    const int r = s_r, slot = s_slot;
    if (r < 0) break;
    int nr = -1, nslot = 0;
    if (threadIdx.x == 0) claim_item(a, &gang, g0, &nr, &nslot);
    if (r != cur) {
      if (pending) retire_run<NT>(a, cur, pending, &s_last, &s_band);
      cur = r;
      pending = 0;
    }
    const int su = __builtin_amdgcn_readfirstlane(slot);   // scalar loads of the item's header
    const int g = w.list_g[su];
    const int tk = w.list_tk[su];
    const int t = tk >> 4, k = tk & 15;
    const BatchReq q = w.req[r];
    const int64_t m = g - q.motion_off;
    const int64_t po = q.point_off;
    const float G = key_dist(__hip_atomic_load(w.keys + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long k2 = cull_item<P, NT>(
        (ConstF4Ptr)w.table, (size_t)(q.sample_off + m * q.T) * a.K + (size_t)k * q.T, q.T,
        w.spheres + ((size_t)g * a.K + k) * w.nb_max, q.nb, q.blen,
        (ConstF4Ptr)(w.wave_sph + 4 * ((size_t)q.tile_off + t)), w.sx + po, w.sy + po, w.sz + po, w.sidx + po,
        q.n_points, t, G, wmin, executed);
    if (threadIdx.x == 0) {
      if (k2 < __hip_atomic_load(w.keys + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(w.keys + g, k2);
      s_r = nr;
      s_slot = nslot;
    }
    ++pending;
    __syncthreads();   // s_r, s_slot written; wmin reused by the next item
  }
  if (pending) retire_run<NT>(a, cur, pending, &s_last, &s_band);
  // executed tests: one add per block, spread over kWorkSlots counters
  if ((threadIdx.x & 63) == 0) wexec[threadIdx.x >> 6] = executed;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long ex = 0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) ex += wexec[q];
    if (ex) atomicAdd(w.work + blockIdx.x % kWorkSlots, ex);
  }
}

// FP64 recheck: entries of band slot s at table64[(s K + k) max_T + t].
__global__ __launch_bounds__(256) void k_batch_fk64(Robot64 rb, BatchArgs a) {
  const BatchWs& w = a.w;
  const int nb = min(w.plan->band_count, a.max_band);
  const int64_t work = (int64_t)nb * a.max_T;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < work; g += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(g / a.max_T);
    const int t = (int)(g - (int64_t)s * a.max_T);
    const int64_t gm = w.band_list[s];
    const int r = find_seg(w.motion_off, a.n_req, gm);
    const sv_motions mo = a.reqs[r].motions;
    if (t >= mo.T) continue;
    const int64_t m = gm - w.motion_off[r];
    write_entries64(rb, mo.kind, mo.q0 + m * rb.dof, mo.q1 + m * rb.dof, mo.via ? mo.via + m * 2 * rb.dof : nullptr,
                    t, mo.T, w.table64 + (size_t)s * rb.n_caps * a.max_T + t, a.max_T);
  }
}

// Grid-stride over (band slot, tile of 256 points of its request's cloud).
__global__ __launch_bounds__(256) void k_batch_exact64(BatchArgs a, int tiles_max) {
  const BatchWs& w = a.w;
  __shared__ unsigned long long wmin[4];
  const int nb = min(w.plan->band_count, a.max_band);
  const int64_t work = (int64_t)nb * tiles_max;
  for (int64_t it = blockIdx.x; it < work; it += gridDim.x) {
    const int s = (int)(it / tiles_max);
    const int tile = (int)(it - (int64_t)s * tiles_max);
    const int r = find_seg(w.motion_off, a.n_req, w.band_list[s]);
    const sv_cloud cl = a.reqs[r].cloud;
    if ((int64_t)tile * 256 >= cl.n) continue;   // uniform across the block
    const int T = a.reqs[r].motions.T;
    const int i = tile * 256 + threadIdx.x;
    double best = INFINITY;
    if (i < cl.n) best = swept_min64(w.table64 + (size_t)s * a.K * a.max_T, T, a.max_T, a.K, cl.x[i], cl.y[i], cl.z[i]);
    unsigned long long key = i < cl.n ? ord_f64(best) : kKeyEmpty;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(key, off, 64);
      key = o < key ? o : key;
    }
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long k2 = wmin[0];
      for (int q = 1; q < 4; ++q) k2 = wmin[q] < k2 ? wmin[q] : k2;
      if (k2 != kKeyEmpty) atomicMin(w.keys64 + s, k2);
    }
    __syncthreads();
  }
}

// FP64 distances and verdicts of the band motions, their requests' stamps, and the
// status word.  One block: the band list is short.
__global__ __launch_bounds__(256) void k_batch_finalize64(BatchArgs a) {
  const BatchWs& w = a.w;
  const int nb = min(w.plan->band_count, a.max_band);
  for (int s = threadIdx.x; s < nb; s += blockDim.x) {
    const int64_t gm = w.band_list[s];
    const int r = find_seg(w.motion_off, a.n_req, gm);
    const sv_results out = a.reqs[r].out;
    const int64_t m = gm - w.motion_off[r];
    const double d = unord_f64(w.keys64[s]);
    if (out.min_dist) out.min_dist[m] = (float)d;
    if (out.verdict) out.verdict[m] = (uint8_t)(d <= (double)a.eps);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nb; s += blockDim.x) {
    const int r = find_seg(w.motion_off, a.n_req, w.band_list[s]);
    if (a.done_ticks) a.done_ticks[r] = wall_clock64();
  }
  if (threadIdx.x == 0 && a.status_out) *a.status_out = w.plan->status;
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

int device_cus() {
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

// Blocks of kernel f (threads per block nt) that the device holds at once: the grid of
// a persistent kernel (more would wait for a slot and run as a tail).
template <auto F>
unsigned resident_blocks(int nt) {
  static int per_cu[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (per_cu[dev] == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, F, nt, 0) != hipSuccess || b < 1) b = 1;
    per_cu[dev] = b;
  }
  return (unsigned)(device_cus() * per_cu[dev]);
}

template <int P, int NT>
hipError_t launch_exact_batch(const BatchArgs& a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_batch_exact<P, NT>), dim3(blocks), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace

sv_tile default_batch_tile() {
  sv_tile t{};
  t.ppl = 2;
  t.threads = 256;
  t.blocks_per_cu = 8;
  t.tiles_per_item = 4;
  t.cull = 1;
  t.cull_blocks_per_cu = 0;
  t.cull_gangs = 8;
  t.cull_div_linear = kCullDivLinear;
  t.cull_div_spline = kCullDivSpline;
  return t;
}

bool batch_tile_supported(const sv_tile& t) {
  const bool ppl = t.ppl == 1 || t.ppl == 2 || t.ppl == 4;
  const bool thr = t.threads == 64 || t.threads == 128 || t.threads == 256;
  const bool unculled = ppl && thr && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32 && t.tiles_per_item >= 1 &&
                        t.tiles_per_item <= 64;
  bool dl = false, ds = false;
  for (int d : kCullDivsLinear) dl = dl || t.cull_div_linear == d;
  for (int d : kCullDivsSpline) ds = ds || t.cull_div_spline == d;
  const bool gangs = t.cull_gangs == 1 || t.cull_gangs == 2 || t.cull_gangs == 4 || t.cull_gangs == 8 ||
                     t.cull_gangs == 16;
  const bool culled = t.cull_blocks_per_cu >= 0 && t.cull_blocks_per_cu <= 8 && gangs && dl && ds;
  return (t.cull == 0 || t.cull == 1) && unculled && culled;
}

BatchWs carve_batch(void* ws, const sv_robot& rb, const sv_batch_caps& caps, size_t* bytes) {
  Carver cv(ws);
  BatchWs w{};
  const size_t R = (size_t)caps.max_requests;
  w.work = cv.take<unsigned long long>(kWorkSlots);   // first: callers read it at offset 0
  w.plan = cv.take<BatchPlan>(1);
  w.motion_off = cv.take<int64_t>(R + 1);
  w.sample_off = cv.take<int64_t>(R + 1);
  w.item_off = cv.take<int64_t>(R + 1);
  w.n_motions = cv.take<int64_t>(R);
  w.n_samples = cv.take<int64_t>(R);
  w.n_items = cv.take<int64_t>(R);
  w.order = cv.take<int>(R);
  w.tiles = cv.take<int>(R);
  w.chunks = cv.take<int>(R);
  w.remaining = cv.take<int>(R);
  w.keys = cv.take<unsigned long long>((size_t)caps.max_motions);
  w.table = cv.take<CapEntry>((size_t)caps.max_samples * rb.n_caps);
  w.band_list = cv.take<int>((size_t)caps.max_band);
  w.keys64 = cv.take<unsigned long long>((size_t)caps.max_band);
  w.table64 = cv.take<CapEntry64>((size_t)caps.max_band * rb.n_caps * caps.max_T);
  // culled pass
  w.point_cap = caps.max_total_points > 0 ? caps.max_total_points : (int64_t)caps.max_requests * caps.max_points;
  w.tile_cap = w.point_cap / kCullTilePts + caps.max_requests;
  w.nb_max = cull_block_count_max(caps.max_T);
  w.ng_max = cull_group_count(w.nb_max);
  w.cand_cap = caps.max_motions * ((caps.max_points + kCullTilePts - 1) / kCullTilePts) * rb.n_caps;
  w.n_points = cv.take<int64_t>(R);
  w.point_off = cv.take<int64_t>(R + 1);
  w.tile_off = cv.take<int64_t>(R + 1);
  w.n_cands = cv.take<int64_t>(R);
  w.cand_off = cv.take<int64_t>(R + 1);
  w.bounds = cv.take<unsigned>(R * 6);
  w.level = cv.take<int>(R);
  w.bin_off = cv.take<int64_t>(R + 1);
  w.bin_cap = w.point_cap * kBinCellsPerPoint + caps.max_requests;
  const size_t P = (size_t)w.point_cap, B = (size_t)w.bin_cap;
  w.pbin = cv.take<int>(P);
  w.pslot = cv.take<int>(P);
  w.bin_count = cv.take<int>(B);
  w.bin_start = cv.take<int>(B);
  const size_t G = (size_t)bin_scan_groups(w.bin_cap);
  w.group_sum = cv.take<int>(G);
  w.group_off = cv.take<int64_t>(G + 1);
  w.sx = cv.take<float>(P);
  w.sy = cv.take<float>(P);
  w.sz = cv.take<float>(P);
  w.sidx = cv.take<int>(P);
  w.tile_sph = cv.take<float4>((size_t)w.tile_cap);
  w.wave_sph = cv.take<float4>((size_t)w.tile_cap * 4);
  w.spheres = cv.take<float4>((size_t)caps.max_motions * rb.n_caps * w.nb_max);
  w.gspheres = cv.take<float4>((size_t)caps.max_motions * rb.n_caps * w.ng_max);
  w.list_g = cv.take<int>((size_t)w.cand_cap);
  w.list_tk = cv.take<int>((size_t)w.cand_cap);
  w.req = cv.take<BatchReq>(R);
  w.fill = cv.take<int>(R);
  w.gang_n = cv.take<int>(kMaxGangs);
  w.gang_total = cv.take<int>(kMaxGangs);
  w.gang_head = cv.take<unsigned>(kMaxGangs);
  w.gang_req = cv.take<int>(kMaxGangs * R);
  w.gang_off = cv.take<int>(kMaxGangs * (R + 1));
  *bytes = cv.off;
  return w;
}

hipError_t launch_batch(const sv_robot& rb, const sv_request* reqs, int n_req, const sv_batch_caps& caps, float eps,
                        float band, const sv_tile& tile, unsigned long long* done_ticks, int* status,
                        const BatchWs& w, hipStream_t st) {
  BatchArgs a{};
  a.reqs = reqs;
  a.n_req = n_req;
  a.max_requests = caps.max_requests;
  a.K = rb.n_caps;
  a.max_T = caps.max_T;
  a.max_band = caps.max_band;
  a.max_motions = caps.max_motions;
  a.max_samples = caps.max_samples;
  a.max_points = caps.max_points;
  a.eps = eps;
  a.band = band;
  a.tile_pts = tile.ppl * tile.threads;
  a.tpi = tile.tiles_per_item;
  a.culled = tile.cull;
  a.gangs = tile.cull_gangs;
  a.div_lin = tile.cull_div_linear;
  a.div_spl = tile.cull_div_spline;
  a.w = w;
  a.done_ticks = done_ticks;
  a.status_out = status;
  hipError_t e;
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned tgrid = (unsigned)std::min<int64_t>(std::max<int64_t>(grid_for(caps.max_samples, 256), 1), 8192);
  hipLaunchKernelGGL(k_batch_tables, dim3(tgrid), dim3(256), 0, st, robot_to_dev<float>(rb), a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int blocks = device_cus() * tile.blocks_per_cu;
  if (a.culled) {
    const int64_t P = w.point_cap;
    const unsigned pg = std::min<unsigned>(grid_for(std::max<int64_t>(P, 1), 256), 8192);
    hipLaunchKernelGGL(k_batch_bounds, dim3(std::min<unsigned>(pg, 2048)), dim3(256), 0, st, a);
    auto capped = [](int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>(n, 1), 16384); };
    hipLaunchKernelGGL(k_batch_clear_bins, dim3(capped(grid_for(w.bin_cap, 256))), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_bin, dim3(pg), dim3(256), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_bin_scan(w.bin_count, 0, &w.plan->total_bins, w.bin_cap, w.group_sum, w.group_off, w.bin_start,
                             st)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_batch_scatter, dim3(pg), dim3(256), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_tile_spheres, dim3(capped(w.tile_cap)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_block_spheres, dim3(capped(grid_for(caps.max_motions * rb.n_caps * w.nb_max, 256))),
                       dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_group_spheres, dim3(capped(grid_for(caps.max_motions * rb.n_caps * w.ng_max, 256))),
                       dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_seed, dim3(capped(caps.max_motions * rb.n_caps)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_cull_list, dim3(capped(grid_for(w.cand_cap, 256))), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_counts, dim3(std::max(n_req, 1)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_gangs, dim3(1), dim3(64), 0, st, a);
    const unsigned resident = resident_blocks<k_batch_cull<kCullP, kCullNT>>(kCullNT);
    const unsigned cgrid = tile.cull_blocks_per_cu > 0
                               ? std::min<unsigned>(resident, (unsigned)(device_cus() * tile.cull_blocks_per_cu))
                               : resident;
    hipLaunchKernelGGL((k_batch_cull<kCullP, kCullNT>), dim3(cgrid), dim3(kCullNT), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
#define SV_BATCH_CASE(P, NT) \
  else if (tile.ppl == P && tile.threads == NT) e = launch_exact_batch<P, NT>(a, blocks, st);
    if (false) {
    }
    SV_BATCH_CASE(1, 64) SV_BATCH_CASE(1, 128) SV_BATCH_CASE(1, 256)
    SV_BATCH_CASE(2, 64) SV_BATCH_CASE(2, 128) SV_BATCH_CASE(2, 256)
    SV_BATCH_CASE(4, 64) SV_BATCH_CASE(4, 128) SV_BATCH_CASE(4, 256)
    else e = hipErrorInvalidValue;
#undef SV_BATCH_CASE
    if (e != hipSuccess) return e;
  }
  const unsigned fgrid = (unsigned)std::min<int64_t>(
      std::max<int64_t>(grid_for((int64_t)caps.max_band * caps.max_T, 256), 1), 1024);
  hipLaunchKernelGGL(k_batch_fk64, dim3(fgrid), dim3(256), 0, st, robot_to_dev<double>(rb), a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int tiles_max = (int)std::max<int64_t>((caps.max_points + 255) / 256, 1);
  const unsigned egrid = (unsigned)std::min<int64_t>((int64_t)caps.max_band * tiles_max, 2048);
  hipLaunchKernelGGL(k_batch_exact64, dim3(egrid), dim3(256), 0, st, a, tiles_max);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_finalize64, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace sv
