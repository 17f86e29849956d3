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
#include "sv_geom_common.h"

namespace sv {
namespace {

constexpr int kPlanThreads = 1024;

struct BatchArgs {
  const sv_request* reqs;
  int n_req;
  int K;
  int max_T;
  int max_band;
  int64_t max_motions, max_samples, max_points;
  float eps, band;
  int tile_pts;  // points per tile (threads * ppl)
  int tpi;       // tiles per work item
  BatchWs w;
  unsigned long long* done_ticks;
  int* status_out;
};

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
    w.remaining[r] = (int)items;
    cost[r] = M * N * T;
    if (a.done_ticks) a.done_ticks[r] = 0;
  }
  for (int s = tid; s < a.max_band; s += kPlanThreads) w.keys64[s] = kKeyEmpty;
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
  if (tid == 0) {
    int st = s_status;
    if (tm > a.max_motions || ts > a.max_samples || tm > 0x7fffffffLL) st |= SV_BATCH_OVER_CAPACITY;
    const bool run = (st & (SV_BATCH_BAD_REQUEST | SV_BATCH_OVER_CAPACITY)) == 0;
    w.plan->status = st;
    w.plan->band_count = 0;
    w.plan->total_items = run ? ti : 0;
    w.plan->total_samples = run ? ts : 0;
    w.plan->next_item = 0;
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

template <int P, int NT>
__global__ __launch_bounds__(NT) void k_batch_exact(BatchArgs a) {
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ int64_t s_item;
  __shared__ int s_last, s_band;
  const BatchWs& w = a.w;
  const int tid = threadIdx.x;
  const int64_t total = w.plan->total_items;
  const ConstF4Ptr tab = (ConstF4Ptr)w.table;
  for (;;) {
    if (tid == 0) {
      s_item = (int64_t)atomicAdd(&w.plan->next_item, 1ull);
      s_band = 0;
    }
    __syncthreads();
    const int64_t item = s_item;
    if (item >= total) break;
    const int pos = find_seg(w.item_off, a.n_req, item);
    const int r = w.order[pos];
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
    if (tid == 0) {
      __threadfence();
      s_last = atomicSub(w.remaining + r, 1) == 1;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      finalize_request<NT>(a, r, &s_band);
    }
    __syncthreads();
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

template <int P, int NT>
hipError_t launch_exact_batch(const BatchArgs& a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_batch_exact<P, NT>), dim3(blocks), dim3(NT), 0, st, a);
  return hipGetLastError();
}

}  // namespace

bool batch_tile_supported(const sv_tile& t) {
  const bool ppl = t.ppl == 1 || t.ppl == 2 || t.ppl == 4;
  const bool thr = t.threads == 64 || t.threads == 128 || t.threads == 256;
  return ppl && thr && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32 && t.tiles_per_item >= 1 &&
         t.tiles_per_item <= 64;
}

BatchWs carve_batch(void* ws, const sv_robot& rb, const sv_batch_caps& caps, size_t* bytes) {
  Carver cv(ws);
  BatchWs w{};
  const size_t R = (size_t)caps.max_requests;
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
  *bytes = cv.off;
  return w;
}

hipError_t launch_batch(const sv_robot& rb, const sv_request* reqs, int n_req, const sv_batch_caps& caps, float eps,
                        float band, const sv_tile& tile, unsigned long long* done_ticks, int* status,
                        const BatchWs& w, hipStream_t st) {
  BatchArgs a{};
  a.reqs = reqs;
  a.n_req = n_req;
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
