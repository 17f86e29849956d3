// First collision-free motion of a set (paper Alg. 1) on one GPU.
//
// Alg. 1 walks the motions one at a time: a first loop visits them in the given order
// and runs the exact check only where the network's proxy d_hat(X, m) exceeds the
// margin; a second loop visits the rest by d_hat descending.  The answer is the first
// motion, in that visiting order, whose exact distance exceeds the margin.  Here the
// visiting order is built in one block (k_search_order), and the exact checks of all
// motions run in one persistent launch over that order (k_search_exact): blocks take
// (position, chunk of point tiles) items from a queue in visiting order, and skip items
// whose position lies after an answer already found.  Every position before the final
// answer is therefore checked completely, so the answer is the sequential one; motions
// past it may be checked too (in parallel), which only costs work.  Motions within the
// certified band of eps are recomputed in FP64 (the per-call recheck) and only then may
// count as free (k_search_resolve).
#include "sv_geom_common.h"

namespace sv {
namespace {

constexpr int kOrderThreads = 1024;
constexpr int kSearchP = 2, kSearchNT = 256;   // exact-check tile of the search

struct SearchArgs {
  int M, K, T;
  float eps, band;
  const float* d_hat;        // NULL: the given order
  CloudArgs c;
  int tiles, tpi, chunks;    // point tiles per motion, tiles per item, items per motion
  SearchWs w;
  sv_search_result* result;
  int* order_out;
};

// Visiting order (Alg. 1): positions of the first-loop motions (d_hat > eps) in index
// order, then the others by d_hat descending, equal values by index; NaN counts as -inf.
__global__ __launch_bounds__(kOrderThreads) void k_search_order(SearchArgs a) {
  __shared__ float key[kMaxSearchMotions];
  __shared__ int s_first;
  const int M = a.M, tid = threadIdx.x;
  const SearchWs& w = a.w;
  if (tid == 0) s_first = 0;
  for (int m = tid; m < M; m += kOrderThreads) {
    const float v = a.d_hat ? a.d_hat[m] : 0.f;
    key[m] = isnan(v) ? -INFINITY : v;
    w.keys[m] = kKeyEmpty;
    w.remaining[m] = a.chunks;
  }
  __syncthreads();
  for (int m = tid; m < M; m += kOrderThreads) {
    int pos = m;
    if (a.d_hat) {
      const float v = key[m];
      pos = 0;
      if (v > a.eps) {
        for (int j = 0; j < m; ++j) pos += key[j] > a.eps;
        atomicAdd(&s_first, 1);
      } else {
        for (int j = 0; j < M; ++j) {
          const float u = key[j];
          pos += (u > a.eps) || (u > v) || (u == v && j < m);
        }
      }
    }
    w.order[pos] = m;
  }
  __syncthreads();
  if (a.order_out)
    for (int p = tid; p < M; p += kOrderThreads) a.order_out[p] = w.order[p];
  if (tid == 0) {
    w.hdr->answer = M;
    w.hdr->n_run = 0;
    w.hdr->band_count = 0;
    w.hdr->n_first = a.d_hat ? s_first : 0;
    w.hdr->next_item = 0;
  }
}

template <int P, int NT>
__global__ __launch_bounds__(NT) void k_search_exact(SearchArgs a) {
  __shared__ unsigned long long wmin[NT / 64];
  __shared__ long long s_item;
  __shared__ int s_answer, s_last;
  const SearchWs& w = a.w;
  const int tid = threadIdx.x;
  const long long total = (long long)a.M * a.chunks;
  const ConstF4Ptr tab = (ConstF4Ptr)w.table;
  for (;;) {
    if (tid == 0) {
      s_item = (long long)atomicAdd(&w.hdr->next_item, 1ull);
      s_answer = __hip_atomic_load(&w.hdr->answer, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const long long item = s_item;
    if (item >= total) break;
    const int p = (int)(item / a.chunks);
    const int c = (int)(item - (long long)p * a.chunks);
    if (p < s_answer) {   // later positions cannot change the answer
      const int m = w.order[p];
      if (a.tiles > 0) {
        unsigned long long key = kKeyEmpty;
        const int t1 = min((c + 1) * a.tpi, a.tiles);
        for (int tile = c * a.tpi; tile < t1; ++tile) {
          const int base = tile * (NT * P) + tid;
          float x[P], y[P], z[P], best[P];
          int idx[P];
#pragma unroll
          for (int q = 0; q < P; ++q) {
            const int j = base + q * NT;
            const bool ok = j < a.c.n;
            idx[q] = ok ? j : -1;
            x[q] = ok ? a.c.x[j] : 0.f;
            y[q] = ok ? a.c.y[j] : 0.f;
            z[q] = ok ? a.c.z[j] : 0.f;
          }
          swept_min<P>(tab, (size_t)m * a.K * a.T, a.T, a.K, x, y, z, best);
          const unsigned long long kk = lane_min_key<P>(best, idx);
          key = kk < key ? kk : key;
        }
        const unsigned long long k2 = block_min_key<NT>(key, wmin);
        if (tid == 0 && k2 != kKeyEmpty) atomicMin(w.keys + m, k2);
      }
      if (tid == 0) {
        // release this item's key; only the block that completes the motion acquires
        // (an acquire fence invalidates the compute unit's L2)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        s_last = __hip_atomic_fetch_add(w.remaining + p, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1;
        if (s_last) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          float d;
          int arg;
          decode_key(__hip_atomic_load(w.keys + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), &d, &arg);
          w.dist_pos[p] = d;
          atomicAdd(&w.hdr->n_run, 1);
          if (fabsf(d - a.eps) <= a.band) {
            const int s = atomicAdd(&w.hdr->band_count, 1);   // at most M entries
            w.band_list[s] = m;
            w.band_pos[s] = p;
          } else if (d > a.eps) {
            atomicMin(&w.hdr->answer, p);
          }
        }
      }
    }
    __syncthreads();
  }
}

// The answer: the first position that is free by its FP32 distance outside the band
// (k_search_exact) or by its FP64 verdict inside it.
__global__ void k_search_resolve(SearchArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const SearchWs& w = a.w;
  const SearchHdr* h = w.hdr;
  const int M = a.M;
  int fin = h->answer;
  bool from_band = false;
  for (int s = 0; s < h->band_count; ++s) {
    const int p = w.band_pos[s];
    if (w.v64[w.band_list[s]] == 0 && p < fin) {
      fin = p;
      from_band = true;
    }
  }
  sv_search_result r;
  r.position = fin;
  r.motion = fin < M ? w.order[fin] : -1;
  r.dist = fin < M ? (from_band ? w.d64[w.order[fin]] : w.dist_pos[fin]) : INFINITY;
  r.n_exact = fin < M ? fin + 1 : M;
  r.n_exact_run = h->n_run;
  r.n_first = h->n_first;
  r.n_nn = a.d_hat ? (fin < h->n_first ? w.order[fin] + 1 : M) : 0;
  r.status = 0;
  *a.result = r;
}

__global__ void k_decode_min(const unsigned* __restrict__ keys, int64_t M, float* __restrict__ d_hat) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) d_hat[m] = keys[m] == 0xffffffffu ? INFINITY : unord_f32(keys[m]);
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }
int device_cus_search() {
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

}  // namespace

SearchWs carve_search(void* ws, const sv_robot& rb, int64_t M, int T, size_t* bytes) {
  Carver cv(ws);
  SearchWs w{};
  const size_t K = (size_t)rb.n_caps;
  w.hdr = cv.take<SearchHdr>(1);
  w.order = cv.take<int>((size_t)M);
  w.remaining = cv.take<int>((size_t)M);
  w.keys = cv.take<unsigned long long>((size_t)M);
  w.dist_pos = cv.take<float>((size_t)M);
  w.table = cv.take<CapEntry>((size_t)M * K * T);
  w.band_list = cv.take<int>((size_t)M);
  w.band_pos = cv.take<int>((size_t)M);
  w.keys64 = cv.take<unsigned long long>((size_t)M);
  w.d64 = cv.take<float>((size_t)M);
  w.v64 = cv.take<uint8_t>((size_t)M);
  *bytes = cv.off;
  return w;
}

hipError_t launch_search(const sv_robot& rb, const MotionArgs& mo, const CloudArgs& c, float eps, float band,
                         const float* d_hat, sv_search_result* result, int* order_out, const SearchWs& w,
                         hipStream_t st) {
  SearchArgs a{};
  a.M = (int)mo.n;
  a.K = rb.n_caps;
  a.T = mo.T;
  a.eps = eps;
  a.band = band;
  a.d_hat = d_hat;
  a.c = c;
  a.tiles = (c.n + kSearchNT * kSearchP - 1) / (kSearchNT * kSearchP);
  a.tpi = 1;
  a.chunks = a.tiles > 0 ? (a.tiles + a.tpi - 1) / a.tpi : 1;
  a.w = w;
  a.result = result;
  a.order_out = order_out;
  hipError_t e;
  hipLaunchKernelGGL(k_search_order, dim3(1), dim3(kOrderThreads), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.M > 0) {
    if ((e = launch_motion_table(rb, mo, w.table, st)) != hipSuccess) return e;
    const int blocks = device_cus_search() * 8;
    hipLaunchKernelGGL((k_search_exact<kSearchP, kSearchNT>), dim3(blocks), dim3(kSearchNT), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const sv_results r64{w.d64, nullptr, w.v64, nullptr};
    if ((e = launch_recheck64(rb, mo, c, w.band_list, &w.hdr->band_count, w.keys64, eps, r64, st)) !=
        hipSuccess)
      return e;
  }
  hipLaunchKernelGGL(k_search_resolve, dim3(1), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_decode_min(const unsigned* keys, int64_t M, float* d_hat, hipStream_t st) {
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode_min, dim3(grid_for(M, 256)), dim3(256), 0, st, keys, M, d_hat);
  return hipGetLastError();
}

}  // namespace sv
