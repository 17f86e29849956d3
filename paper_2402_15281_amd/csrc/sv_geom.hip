// Geometric kernels of the exact swept-volume check (gfx950).
//
// Paper: Sec. III (eq. (1)-(4): f_d(x, m) = signed distance of x to the swept volume
// V_S(m) = union over s of V_R(c(m, s))) and Sec. IV-B (d(X, m) = min over the cloud,
// free iff d > eps_S).  The continuous union over s is sampled at T configurations
// s_t = t / (T - 1); V_R(q) is a union of capsules placed by forward kinematics.
//
// Kernels:
//   k_fk_configs   forward kinematics of independent configurations (sv_fk)
//   k_motion_table per (motion, t): motion sample + FK -> one capsule entry per link
//   k_exact        per (motion, point tile): min over capsules and samples, FP32 VALU;
//                  optional per-point output and per-motion (distance, index) min keys
//   k_finalize     keys -> min distance, argmin, verdict; certified-band list
//   k_exact64 / k_finalize64: FP64 recheck of the band list (FK in LDS, no table)
#include "sv_geom_common.h"

namespace sv {
namespace {

// ---------------------------------------------------------------- sv_fk
template <typename R>
__global__ __launch_bounds__(256) void k_fk_configs(RobotT<R> rb, const float* __restrict__ q, int64_t n,
                                                    float* __restrict__ caps) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  R qq[SV_MAX_DOF];
#pragma unroll
  for (int j = 0; j < SV_MAX_DOF; ++j) qq[j] = j < rb.dof ? (R)q[c * rb.dof + j] : (R)0;
  R A[SV_MAX_CAPS][3], B[SV_MAX_CAPS][3];
  fk_capsules<R>(rb, qq, A, B);
  float* o = caps + c * rb.n_caps * 8;
#pragma unroll
  for (int k = 0; k < SV_MAX_CAPS; ++k)
    if (k < rb.n_caps) {
      float4 lo = make_float4((float)A[k][0], (float)A[k][1], (float)A[k][2], (float)B[k][0]);
      float4 hi = make_float4((float)B[k][1], (float)B[k][2], (float)rb.r[k], 0.f);
      reinterpret_cast<float4*>(o + 8 * k)[0] = lo;
      reinterpret_cast<float4*>(o + 8 * k)[1] = hi;
    }
}

// ------------------------------------------------------- motion tables
// One thread per (motion, t); writes the entry of every capsule at [m][k][t].
__global__ __launch_bounds__(256) void k_motion_table(Robot32 rb, MotionArgs mo, CapEntry* __restrict__ table) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= mo.n * mo.T) return;
  const int64_t m = g / mo.T;
  const int t = (int)(g - m * mo.T);
  write_entries(rb, mo.kind, mo.q0 + m * rb.dof, mo.q1 + m * rb.dof, mo.via ? mo.via + m * 2 * rb.dof : nullptr, t,
                mo.T, table + (size_t)m * rb.n_caps * mo.T + t, mo.T);
}

// ------------------------------------------------------------ exact check
// grid: one block per (motion slot, tile of NT*P points), tile fastest.
// Lanes own points base + p*NT + tid.  For every capsule k: running min over t of
// the squared distance, then sqrt - r; the point's distance is the min over k.
// With a point list, lane slot j of motion m stands for point plist[m * N + j],
// j < pcount[m], and tiles beyond the list exit at once.  With seg > 0 motion m owns
// the points m * seg .. m * seg + seg - 1 (and sdf is indexed by point).
template <int P, int NT>
__global__ __launch_bounds__(NT) void k_exact(const CapEntry* __restrict__ table, int T, int K,
                                              const float* __restrict__ px, const float* __restrict__ py,
                                              const float* __restrict__ pz, int N, int tiles,
                                              const int* __restrict__ mlist, const int* __restrict__ mcount,
                                              const int* __restrict__ plist, const int* __restrict__ pcount, int seg,
                                              float* __restrict__ sdf, unsigned long long* __restrict__ keys) {
  const int slot = blockIdx.x / tiles;
  const int tile = blockIdx.x - slot * tiles;
  if (mcount && slot >= *mcount) return;
  const int m = mlist ? mlist[slot] : slot;
  const int n_here = pcount ? pcount[m] : (seg ? seg : N);
  if (tile * (NT * P) >= n_here) return;
  const int base = tile * (NT * P) + threadIdx.x;

  float x[P], y[P], z[P], best[P];
  int idx[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = base + p * NT;
    const bool ok = j < n_here;
    const int i = ok ? (plist ? plist[(size_t)m * N + j] : (seg ? m * seg + j : j)) : -1;
    idx[p] = i;
    x[p] = ok ? px[i] : 0.f;
    y[p] = ok ? py[i] : 0.f;
    z[p] = ok ? pz[i] : 0.f;
  }
  swept_min<P>((ConstF4Ptr)table, (size_t)m * K * T, T, K, x, y, z, best);

  if (sdf) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int i = idx[p];
      if (i >= 0) sdf[seg ? (size_t)i : (size_t)m * N + i] = best[p];
    }
  }
  if (keys) {
    __shared__ unsigned long long wmin[NT / 64];
    const unsigned long long k2 = block_min_key<NT>(lane_min_key<P>(best, idx), wmin);
    if (threadIdx.x == 0 && k2 != kKeyEmpty) atomicMin(keys + m, k2);
  }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int* __restrict__ p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Start values of a motion check, in one launch: per-motion keys empty, the band count
// and the executed-test counters zero.
__global__ void k_check_init(unsigned long long* __restrict__ keys, int64_t M, int* __restrict__ band_count,
                             unsigned long long* __restrict__ work, int n_work) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) keys[i] = kKeyEmpty;
  if (i < n_work) work[i] = 0ull;
  if (i == 0) *band_count = 0;
}

// Grid-stride over the motions of (mlist, mcount), or all M.
__global__ void k_finalize(const unsigned long long* __restrict__ keys, int64_t M, const int* __restrict__ mlist,
                           const int* __restrict__ mcount, float eps, float band, sv_results out,
                           int* __restrict__ list, int* __restrict__ count) {
  const int64_t n = mcount ? (int64_t)*mcount : M;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = mlist ? mlist[s] : s;
    float d;
    int arg;
    decode_key(keys[m], &d, &arg);
    write_result(out, m, d, arg, eps);
    if (list && fabsf(d - eps) <= band) list[atomicAdd(count, 1)] = (int)m;
  }
}

__global__ void k_screen_decide(unsigned long long* __restrict__ keys, int64_t M, const int* __restrict__ pcount,
                                float eps, float band, int certified, sv_results out, int* __restrict__ full,
                                int* __restrict__ full_count) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  if (out.n_fallback) out.n_fallback[m] = pcount[m];
  if (!certified) return;   // trust mode: the keys of the sent points are final
  float d;
  int arg;
  decode_key(keys[m], &d, &arg);
  if (d <= eps - band) {
    write_result(out, m, d, arg, eps);
  } else {
    keys[m] = kKeyEmpty;
    full[atomicAdd(full_count, 1)] = (int)m;
  }
}

// --------------------------------------------------------- FP64 recheck
constexpr int kFk64Chunk = 32;   // samples placed in LDS per stage

// Grid-stride over (slot, tile of 256 points) of the motions listed by k_finalize: per
// slot the min over the tile of the FP64 swept distance.  The block places the listed
// motion's capsules in FP64 for kFk64Chunk samples at a time in LDS (one thread per
// sample) and every thread folds them into its point's per-capsule minimum of squared
// distances (kept in LDS, so that the FK's registers are free); the minimum is exact in
// any order, so the result is that of a full FP64 table, without one in memory.
__global__ __launch_bounds__(256) void k_exact64(Robot64 rb, MotionArgs mo, const int* __restrict__ list,
                                                 const int* __restrict__ count, CloudArgs c, int tiles,
                                                 unsigned long long* __restrict__ keys64) {
  __shared__ CapEntry64 ent[SV_MAX_CAPS * kFk64Chunk];   // [k][t - t0]
  __shared__ double m2[SV_MAX_CAPS][256];                // [k][thread]
  __shared__ unsigned long long wmin[4];
  const int K = rb.n_caps, T = mo.T, dof = rb.dof;
  const int64_t work = (int64_t)(*count) * tiles;
  for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
    const int64_t slot = w / tiles;
    const int tile = (int)(w - slot * tiles);
    const int64_t m = list[slot];
    const int i = tile * 256 + threadIdx.x;
    const bool valid = i < c.n;
    const double x = valid ? (double)c.x[i] : 0.0, y = valid ? (double)c.y[i] : 0.0,
                 z = valid ? (double)c.z[i] : 0.0;
    for (int k = 0; k < K; ++k) m2[k][threadIdx.x] = INFINITY;
    for (int t0 = 0; t0 < T; t0 += kFk64Chunk) {
      const int nt = min(kFk64Chunk, T - t0);
      __syncthreads();   // the previous stage (or item) is consumed
      if ((int)threadIdx.x < nt)
        write_entries64(rb, mo.kind, mo.q0 + m * dof, mo.q1 + m * dof, mo.via ? mo.via + m * 2 * dof : nullptr,
                        t0 + (int)threadIdx.x, T, ent + threadIdx.x, kFk64Chunk);
      __syncthreads();
      for (int k = 0; k < K; ++k) {
        double v = m2[k][threadIdx.x];
        for (int t = 0; t < nt; ++t) v = fmin(v, seg_d2_64(ent[k * kFk64Chunk + t], x, y, z));
        m2[k][threadIdx.x] = v;
      }
    }
    double best = INFINITY;
    for (int k = 0; k < K; ++k) best = fmin(best, sqrt(m2[k][threadIdx.x]) - ent[k * kFk64Chunk].r);
    unsigned long long key = valid ? ord_f64(best) : kKeyEmpty;
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
      if (k2 != kKeyEmpty) atomicMin(keys64 + slot, k2);
    }
  }
}

__global__ void k_finalize64(const int* __restrict__ list, const int* __restrict__ count,
                             const unsigned long long* __restrict__ keys64, float eps, sv_results out) {
  const int n = *count;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const int m = list[s];
    const double d = unord_f64(keys64[s]);
    if (out.min_dist) out.min_dist[m] = (float)d;
    if (out.verdict) out.verdict[m] = (uint8_t)(d <= (double)eps);
  }
}

inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// ---- continuous certification -------------------------------------------------------
// The exact check samples the path at s_t = t / (T - 1) (eq. (2), (3)); every s lies
// within h = 1 / (2 (T - 1)) of a sample (h = 1 for T = 1).  If every point of capsule k
// moves at most L_k per unit of s, a point's distance to the capsule changes at most
// L_k per unit of s, so d_cont >= d_T - max_k L_k h.  Speed bound (standard DH, joint j
// turns about the z axis of frame j-1 through O_{j-1}): a point fixed in frame f >= j
// moves under joint j at |dq_j/ds| times its distance from that axis, at most
// sum_{i=j..f} l_i + |p| (l_i = sqrt(a_i^2 + d_i^2), p its coordinates in frame f);
// segment points are convex combinations of the two endpoints.

// max over s of |dq_j/ds| for one joint: linear |y3 - y0|; spline (knots at 0, 1/3,
// 2/3, 1 with the slopes of motion_config): per Hermite segment the derivative is a
// quadratic a u^2 + b u + c in u in [0, 1], largest in magnitude at an end or the vertex.
__device__ double joint_speed_max(int kind, double y0, double y1, double y2, double y3) {
  if (kind == SV_LINEAR) return fabs(y3 - y0);
  const double hm1 = (4.0 * (y2 - y0) - (y3 - y1)) / 5.0, hm2 = (4.0 * (y3 - y1) - (y2 - y0)) / 5.0;
  const double y[4] = {y0, y1, y2, y3}, hm[4] = {0.0, hm1, hm2, 0.0};
  double best = 0.0;
  for (int seg = 0; seg < 3; ++seg) {
    const double ya = y[seg], yb = y[seg + 1], ma = hm[seg], mb = hm[seg + 1];
    const double a = 6.0 * (ya - yb) + 3.0 * (ma + mb), b = 6.0 * (yb - ya) - 4.0 * ma - 2.0 * mb, c = ma;
    double v = fmax(fabs(c), fabs(a + b + c));
    if (a != 0.0) {
      const double u = -b / (2.0 * a);
      if (u > 0.0 && u < 1.0) v = fmax(v, fabs((a * u + b) * u + c));
    }
    best = fmax(best, 3.0 * v);   // ds = du / 3
  }
  return best;
}

// One thread per motion: gap[m] (rounded up to FP32) and, with min_dist, verdict[m] = 0
// iff min_dist[m] - gap[m] > eps + band (certified free along the continuous motion).
__global__ __launch_bounds__(256) void k_motion_gap(Robot64 rb, MotionArgs mo, const float* __restrict__ min_dist,
                                                    float eps, float band, float* __restrict__ gap,
                                                    uint8_t* __restrict__ verdict) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= mo.n) return;
  const int dof = rb.dof;
  double omega[SV_MAX_DOF], tail[SV_MAX_DOF + 1];   // tail[j] = sum_{i=j..dof-1} l_i (0-based links)
  for (int j = 0; j < dof; ++j) {
    const float* q0 = mo.q0 + m * dof;
    const float* q1 = mo.q1 + m * dof;
    const float* v = mo.via ? mo.via + m * 2 * dof : nullptr;
    omega[j] = joint_speed_max(mo.kind, q0[j], v ? v[j] : 0.0, v ? v[dof + j] : 0.0, q1[j]);
  }
  tail[dof] = 0.0;
  for (int i = dof - 1; i >= 0; --i) tail[i] = tail[i + 1] + sqrt(rb.dh[i][0] * rb.dh[i][0] + rb.dh[i][2] * rb.dh[i][2]);
  double L = 0.0;
  for (int k = 0; k < rb.n_caps; ++k)
    for (int e = 0; e < 2; ++e) {
      const int f = e ? rb.fb[k] : rb.fa[k];
      const double* p = e ? rb.pb[k] : rb.pa[k];
      const double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      double v = 0.0;
      for (int j = 0; j < f; ++j) v += omega[j] * (tail[j] - tail[f] + pn);   // links j..f-1 (0-based)
      L = fmax(L, v);
    }
  const double g = L * (mo.T > 1 ? 0.5 / (double)(mo.T - 1) : 1.0);
  float gf = (float)g;
  if ((double)gf < g) gf = nextafterf(gf, INFINITY);
  gap[m] = gf;
  if (verdict) verdict[m] = (min_dist[m] - gf > eps + band) ? 0 : 1;
}


template <int P, int NT>
hipError_t launch_exact_t(const CapEntry* table, const MotionArgs& m, const CloudArgs& c, int K, const int* mlist,
                          const int* mcount, int64_t n_slots, const int* plist, const int* pcount, int seg,
                          float* sdf, unsigned long long* keys, hipStream_t st) {
  const int per_motion = seg ? seg : c.n;
  const int tiles = (per_motion + NT * P - 1) / (NT * P);
  const int64_t blocks = n_slots * tiles;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_exact<P, NT>), dim3((unsigned)blocks), dim3(NT), 0, st, table, m.T, K, c.x, c.y, c.z, c.n,
                     tiles, mlist, mcount, plist, pcount, seg, sdf, keys);
  return hipGetLastError();
}

hipError_t launch_exact_any(const sv_robot& rb, const CapEntry* table, const MotionArgs& m, const CloudArgs& c,
                            const int* mlist, const int* mcount, int64_t n_slots, const int* plist, const int* pcount,
                            int seg, float* sdf, unsigned long long* keys, ExactShape s, hipStream_t st) {
  const int K = rb.n_caps;
#define SV_EXACT_CASE(P, NT)            \
  if (s.ppl == P && s.threads == NT)    \
    return launch_exact_t<P, NT>(table, m, c, K, mlist, mcount, n_slots, plist, pcount, seg, sdf, keys, st);
  SV_EXACT_CASE(1, 64) SV_EXACT_CASE(1, 128) SV_EXACT_CASE(1, 256)
  SV_EXACT_CASE(2, 64) SV_EXACT_CASE(2, 128) SV_EXACT_CASE(2, 256)
  SV_EXACT_CASE(4, 64) SV_EXACT_CASE(4, 128) SV_EXACT_CASE(4, 256)
#undef SV_EXACT_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------------ training data
// rnd per motion: [3 n_uniform] then [6 n_cand] numbers in [0, 1).
__global__ void k_uniform_points(int64_t M, int nu, int stride, const float* __restrict__ rnd, float half,
                                 float* __restrict__ x, float* __restrict__ y, float* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M * nu) return;
  const int64_t m = g / nu;
  const int u = (int)(g - m * nu);
  const float* r = rnd + m * stride + 3 * u;
  x[g] = half * (2.f * r[0] - 1.f);
  y[g] = half * (2.f * r[1] - 1.f);
  z[g] = half * (2.f * r[2] - 1.f);
}

// Candidate c of motion m: sample t, capsule k, axis point A + u AB, unit direction d
// (uniform on the sphere), position at radius r_k + o from the axis point, o in
// [-band, band].
__global__ void k_near_candidates(const CapEntry* __restrict__ table, int64_t M, int T, int K, int nu, int nc,
                                  int stride, const float* __restrict__ rnd, float band, float* __restrict__ x,
                                  float* __restrict__ y, float* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M * nc) return;
  const int64_t m = g / nc;
  const int c = (int)(g - m * nc);
  const float* r = rnd + m * stride + 3 * nu + 6 * c;
  const int t = min((int)(r[0] * T), T - 1);
  const int k = min((int)(r[1] * K), K - 1);
  const CapEntry e = table[(m * K + k) * T + t];
  const float cz = 2.f * r[3] - 1.f;
  const float sz = sqrtf(fmaxf(0.f, 1.f - cz * cz));
  float sphi, cphi;
  sincosf(6.28318530717958648f * r[4], &sphi, &cphi);
  const float rad = e.r + band * (2.f * r[5] - 1.f);
  x[g] = e.ax + r[2] * e.bx + rad * sz * cphi;
  y[g] = e.ay + r[2] * e.by + rad * sz * sphi;
  z[g] = e.az + r[2] * e.bz + rad * cz;
}

__device__ __forceinline__ void write_row(float* __restrict__ row, int dof, const float* q0, const float* q1, float x,
                                          float y, float z, float d) {
  row[0] = x;
  row[1] = y;
  row[2] = z;
  for (int j = 0; j < dof; ++j) {
    row[3 + j] = q0[j];
    row[3 + dof + j] = q1[j];
  }
  row[3 + 2 * dof] = d;
}

// One wave per motion: uniform rows, then the first n_near in-band candidates in
// candidate order (then, if short, the first out-of-band ones).
__global__ __launch_bounds__(256) void k_assemble_samples(int64_t M, int dof, int nu, int nn, int nc, float band,
                                                          const float* __restrict__ q0, const float* __restrict__ q1,
                                                          const float* __restrict__ ux, const float* __restrict__ uy,
                                                          const float* __restrict__ uz, const float* __restrict__ ud,
                                                          const float* __restrict__ cx, const float* __restrict__ cy,
                                                          const float* __restrict__ cz, const float* __restrict__ cd,
                                                          float* __restrict__ out, int* __restrict__ n_short) {
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= M) return;
  const int width = 3 + 2 * dof + 1;
  const float* mq0 = q0 + m * dof;
  const float* mq1 = q1 + m * dof;
  float* rows = out + (size_t)m * (nu + nn) * width;
  for (int u = lane; u < nu; u += 64) {
    const int64_t g = m * nu + u;
    write_row(rows + (size_t)u * width, dof, mq0, mq1, ux[g], uy[g], uz[g], ud[g]);
  }
  float* near = rows + (size_t)nu * width;
  int taken = 0;
  for (int pass = 0; pass < 2 && taken < nn; ++pass) {
    for (int c0 = 0; c0 < nc && taken < nn; c0 += 64) {
      const int c = c0 + lane;
      const int64_t g = m * nc + c;
      bool ok = false;
      if (c < nc) {
        const bool in_band = fabsf(cd[g]) <= band;
        ok = pass == 0 ? in_band : !in_band;
      }
      const unsigned long long mask = __ballot(ok);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
      if (ok && taken + rank < nn)
        write_row(near + (size_t)(taken + rank) * width, dof, mq0, mq1, cx[g], cy[g], cz[g], cd[g]);
      taken += __popcll(mask);
    }
    if (pass == 0 && taken < nn && lane == 0 && n_short) atomicAdd(n_short, nn - taken);
  }
}

// ------------------------------------------------------ paper-style training data
// Per motion (Sec. IV-C): uniform box points; swept-surface points; for each surface
// point two Gaussian points around it and one point on the chord to another surface
// point.  rnd per motion: [3 n_uniform] then [5 n_cand] then [8 n_surface] numbers in
// [0, 1).  The swept surface is sampled through candidates uniform over the total area
// of the capsule instances (capsule k by area, sample t uniformly, a point uniform on
// the capsule's surface); a candidate is on the swept surface iff no other instance
// contains it, i.e. iff its swept distance is 0, and every piece of the surface belongs
// to exactly one instance's surface, so accepted candidates are uniform on it.
constexpr float kSurfAccept = -1e-6f;   // m: FP32 swept distance of an accepted candidate, at least

__global__ void k_surface_candidates(const CapEntry* __restrict__ table, int64_t M, int T, int K, int nu, int nc,
                                     int stride, const float* __restrict__ rnd, float* __restrict__ x,
                                     float* __restrict__ y, float* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M * nc) return;
  const int64_t m = g / nc;
  const int c = (int)(g - m * nc);
  const float* r = rnd + m * stride + 3 * nu + 5 * c;
  const CapEntry* base = table + m * K * T;   // [k][t]
  // capsule k with probability proportional to its area 2 pi r L + 4 pi r^2 (rigid: from t = 0)
  float cum[SV_MAX_CAPS];
  float tot = 0.f;
  for (int k = 0; k < K; ++k) {
    const CapEntry e = base[(size_t)k * T];
    const float L = sqrtf(e.bx * e.bx + e.by * e.by + e.bz * e.bz);
    tot += 6.28318530717958648f * e.r * L + 12.5663706143591730f * e.r * e.r;
    cum[k] = tot;
  }
  const float pick = r[0] * tot;
  int k = K - 1;
  for (int kk = K - 1; kk >= 0; --kk)
    if (cum[kk] > pick) k = kk;   // the first capsule whose cumulative area exceeds pick
  const int t = min((int)(r[1] * T), T - 1);
  const CapEntry e = base[(size_t)k * T + t];
  const float L = sqrtf(e.bx * e.bx + e.by * e.by + e.bz * e.bz);
  const float pc = L + 2.f * e.r > 0.f ? L / (L + 2.f * e.r) : 0.f;
  float px, py, pz;
  if (r[2] < pc) {   // the cylinder: axial position and angle
    const float ax = e.bx / L, ay = e.by / L, az = e.bz / L;
    const bool useX = fabsf(ax) < 0.9f;   // helper axis not parallel to the segment
    const float hx = useX ? 1.f : 0.f, hy = useX ? 0.f : 1.f;
    float e1x = ay * 0.f - az * hy, e1y = az * hx - ax * 0.f, e1z = ax * hy - ay * hx;   // a x h
    const float n1 = 1.f / sqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x *= n1; e1y *= n1; e1z *= n1;
    const float e2x = ay * e1z - az * e1y, e2y = az * e1x - ax * e1z, e2z = ax * e1y - ay * e1x;   // a x e1
    float sp, cp;
    sincosf(6.28318530717958648f * r[4], &sp, &cp);
    px = e.ax + r[3] * e.bx + e.r * (cp * e1x + sp * e2x);
    py = e.ay + r[3] * e.by + e.r * (cp * e1y + sp * e2y);
    pz = e.az + r[3] * e.bz + e.r * (cp * e1z + sp * e2z);
  } else {           // the caps: a direction uniform on the sphere, around the end it points away at
    const float cz = 2.f * r[3] - 1.f;
    const float sz = sqrtf(fmaxf(0.f, 1.f - cz * cz));
    float sp, cp;
    sincosf(6.28318530717958648f * r[4], &sp, &cp);
    const float dx = sz * cp, dy = sz * sp, dz = cz;
    const bool atB = L > 0.f && (dx * e.bx + dy * e.by + dz * e.bz) > 0.f;
    px = e.ax + (atB ? e.bx : 0.f) + e.r * dx;
    py = e.ay + (atB ? e.by : 0.f) + e.r * dy;
    pz = e.az + (atB ? e.bz : 0.f) + e.r * dz;
  }
  x[g] = px;
  y[g] = py;
  z[g] = pz;
}

// One wave per motion: the first n_surface accepted candidates in candidate order (then,
// if short, the first rejected ones); n_acc[m] = accepted candidates of the motion.
__global__ __launch_bounds__(256) void k_pick_surface(int64_t M, int nc, int ns, const float* __restrict__ cx,
                                                      const float* __restrict__ cy, const float* __restrict__ cz,
                                                      const float* __restrict__ cd, float* __restrict__ sx,
                                                      float* __restrict__ sy, float* __restrict__ sz,
                                                      float* __restrict__ sd, int* __restrict__ n_acc,
                                                      int* __restrict__ n_short) {
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= M) return;
  int taken = 0, accepted = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int c0 = 0; c0 < nc && (pass == 0 || taken < ns); c0 += 64) {
      const int c = c0 + lane;
      const int64_t g = m * nc + c;
      bool ok = false;
      if (c < nc) {
        const bool acc = cd[g] >= kSurfAccept;
        ok = pass == 0 ? acc : !acc;
      }
      const unsigned long long mask = __ballot(ok);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
      if (ok && taken + rank < ns) {
        const int64_t o = m * ns + taken + rank;
        sx[o] = cx[g];
        sy[o] = cy[g];
        sz[o] = cz[g];
        sd[o] = cd[g];
      }
      taken += __popcll(mask);
      if (pass == 0) accepted += __popcll(mask);
    }
    if (pass == 0) {
      if (lane == 0 && n_acc) n_acc[m] = accepted;
      if (taken >= ns) break;
      if (lane == 0 && n_short) atomicAdd(n_short, ns - taken);
    }
  }
}

// Two standard normals from two uniforms in [0, 1) (Box-Muller; 1 - u1 keeps the log finite).
__device__ __forceinline__ void box_muller(float u1, float u2, float* n0, float* n1) {
  const float rad = sqrtf(-2.f * logf(1.f - u1));
  float s, c;
  sincosf(6.28318530717958648f * u2, &s, &c);
  *n0 = rad * c;
  *n1 = rad * s;
}

// One thread per (motion, surface point): its two Gaussian points and its chord point,
// at kid[(m ns + s) 3 + 0..2].
__global__ void k_surface_children(int64_t M, int nu, int nc, int ns, int stride, const float* __restrict__ rnd,
                                   float sigma, const float* __restrict__ sx, const float* __restrict__ sy,
                                   const float* __restrict__ sz, float* __restrict__ kx, float* __restrict__ ky,
                                   float* __restrict__ kz) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M * ns) return;
  const int64_t m = g / ns;
  const int s = (int)(g - m * ns);
  const float* r = rnd + m * stride + 3 * nu + 5 * nc + 8 * s;
  float n[6];
  box_muller(r[0], r[1], &n[0], &n[1]);
  box_muller(r[2], r[3], &n[2], &n[3]);
  box_muller(r[4], r[5], &n[4], &n[5]);
  const float x = sx[g], y = sy[g], z = sz[g];
  const int64_t o = g * 3;
  kx[o] = x + sigma * n[0];
  ky[o] = y + sigma * n[1];
  kz[o] = z + sigma * n[2];
  kx[o + 1] = x + sigma * n[3];
  ky[o + 1] = y + sigma * n[4];
  kz[o + 1] = z + sigma * n[5];
  const int64_t p = m * ns + min((int)(r[6] * ns), ns - 1);
  const float lam = r[7];
  kx[o + 2] = x + lam * (sx[p] - x);
  ky[o + 2] = y + lam * (sy[p] - y);
  kz[o + 2] = z + lam * (sz[p] - z);
}

// One wave per motion: rows [uniform | surface | per surface point: two Gaussian, chord].
__global__ __launch_bounds__(256) void k_assemble_paper(int64_t M, int dof, int nu, int ns,
                                                        const float* __restrict__ q0, const float* __restrict__ q1,
                                                        const float* __restrict__ ux, const float* __restrict__ uy,
                                                        const float* __restrict__ uz, const float* __restrict__ ud,
                                                        const float* __restrict__ sx, const float* __restrict__ sy,
                                                        const float* __restrict__ sz, const float* __restrict__ sd,
                                                        const float* __restrict__ kx, const float* __restrict__ ky,
                                                        const float* __restrict__ kz, const float* __restrict__ kd,
                                                        float* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= M) return;
  const int width = 3 + 2 * dof + 1;
  const float* mq0 = q0 + m * dof;
  const float* mq1 = q1 + m * dof;
  float* rows = out + (size_t)m * (nu + 4 * ns) * width;
  for (int u = lane; u < nu; u += 64) {
    const int64_t g = m * nu + u;
    write_row(rows + (size_t)u * width, dof, mq0, mq1, ux[g], uy[g], uz[g], ud[g]);
  }
  for (int s = lane; s < ns; s += 64) {
    const int64_t g = m * ns + s;
    write_row(rows + (size_t)(nu + s) * width, dof, mq0, mq1, sx[g], sy[g], sz[g], sd[g]);
  }
  for (int i = lane; i < 3 * ns; i += 64) {
    const int64_t g = m * 3 * ns + i;
    write_row(rows + (size_t)(nu + ns + i) * width, dof, mq0, mq1, kx[g], ky[g], kz[g], kd[g]);
  }
}

}  // namespace

ExactShape default_exact_shape() { return ExactShape{2, 256}; }

hipError_t launch_fk_configs(const sv_robot& rb, const float* q, int64_t n, float* caps, int fp64,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(k_fk_configs<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, robot_to_dev<double>(rb), q, n,
                       caps);
  else
    hipLaunchKernelGGL(k_fk_configs<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, robot_to_dev<float>(rb), q, n,
                       caps);
  return hipGetLastError();
}

hipError_t launch_motion_table(const sv_robot& rb, const MotionArgs& m, CapEntry* table, hipStream_t st) {
  const int64_t n = m.n * m.T;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_motion_table, dim3(grid_for(n, 256)), dim3(256), 0, st, robot_to_dev<float>(rb), m, table);
  return hipGetLastError();
}

hipError_t launch_exact(const sv_robot& rb, const CapEntry* table, const MotionArgs& m, const CloudArgs& c,
                        const int* mlist, const int* mcount, int64_t n_slots, const int* plist, const int* pcount,
                        float* sdf, unsigned long long* keys, ExactShape s, hipStream_t st) {
  return launch_exact_any(rb, table, m, c, mlist, mcount, n_slots, plist, pcount, 0, sdf, keys, s, st);
}

hipError_t launch_make_samples(const sv_robot& rb, const MotionArgs& m, const CapEntry* table, float half, int nu,
                               int nn, int nc, float band, const float* rnd, float* ux, float* uy, float* uz,
                               float* ud, float* cx, float* cy, float* cz, float* cd, float* out, int* n_short,
                               hipStream_t st) {
  const int stride = 3 * nu + 6 * nc;
  const ExactShape shape = default_exact_shape();
  hipError_t e;
  if (nu > 0) {
    hipLaunchKernelGGL(k_uniform_points, dim3(grid_for(m.n * nu, 256)), dim3(256), 0, st, m.n, nu, stride, rnd, half,
                       ux, uy, uz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const CloudArgs cu{(int)(m.n * nu), ux, uy, uz};
    if ((e = launch_exact_any(rb, table, m, cu, nullptr, nullptr, m.n, nullptr, nullptr, nu, ud, nullptr, shape,
                              st)) != hipSuccess)
      return e;
  }
  if (nc > 0) {
    hipLaunchKernelGGL(k_near_candidates, dim3(grid_for(m.n * nc, 256)), dim3(256), 0, st, table, m.n, m.T, rb.n_caps,
                       nu, nc, stride, rnd, band, cx, cy, cz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const CloudArgs cc{(int)(m.n * nc), cx, cy, cz};
    if ((e = launch_exact_any(rb, table, m, cc, nullptr, nullptr, m.n, nullptr, nullptr, nc, cd, nullptr, shape,
                              st)) != hipSuccess)
      return e;
  }
  hipLaunchKernelGGL(k_assemble_samples, dim3(grid_for(m.n, 4)), dim3(256), 0, st, m.n, rb.dof, nu, nn, nc, band, m.q0,
                     m.q1, ux, uy, uz, ud, cx, cy, cz, cd, out, n_short);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_check_init(unsigned long long* keys, int64_t M, int* band_count, unsigned long long* work,
                             int n_work, hipStream_t st) {
  hipLaunchKernelGGL(k_check_init, dim3(grid_for(std::max<int64_t>(std::max<int64_t>(M, n_work), 1), 256)), dim3(256), 0,
                     st, keys, M, band_count, work, n_work);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_finalize(const unsigned long long* keys, int64_t M, const int* mlist, const int* mcount, float eps,
                           float band, sv_results out, int* list, int* count, hipStream_t st) {
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)std::min<int64_t>(grid_for(M, 256), 1024)), dim3(256), 0, st, keys, M,
                     mlist, mcount, eps, band, out, list, count);
  return hipGetLastError();
}

hipError_t launch_screen_decide(unsigned long long* keys, int64_t M, const int* pcount, float eps, float band,
                                int certified, sv_results out, int* full, int* full_count, hipStream_t st) {
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_screen_decide, dim3(grid_for(M, 256)), dim3(256), 0, st, keys, M, pcount, eps, band, certified,
                     out, full, full_count);
  return hipGetLastError();
}

hipError_t launch_recheck64(const sv_robot& rb, const MotionArgs& m, const CloudArgs& c, const int* list,
                            const int* count, unsigned long long* keys64, float eps, sv_results out,
                            hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  hipError_t e = launch_fill_u64(keys64, m.n, kKeyEmpty, st);
  if (e != hipSuccess) return e;
  const int tiles = (c.n + 255) / 256;
  if (tiles > 0) {
    hipLaunchKernelGGL(k_exact64, dim3((unsigned)std::min<int64_t>(m.n * tiles, 2048)), dim3(256), 0, st,
                       robot_to_dev<double>(rb), m, list, count, c, tiles, keys64);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_finalize64, dim3(4), dim3(256), 0, st, list, count, keys64, eps, out);
  return hipGetLastError();
}

hipError_t launch_motion_gap(const sv_robot& rb, const MotionArgs& m, const float* min_dist, float eps, float band,
                             float* gap, uint8_t* verdict, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_motion_gap, dim3(grid_for(m.n, 256)), dim3(256), 0, st, robot_to_dev<double>(rb), m, min_dist,
                     eps, band, gap, verdict);
  return hipGetLastError();
}

hipError_t launch_make_samples_paper(const sv_robot& rb, const MotionArgs& m, const CapEntry* table, float half,
                                     int nu, int ns, int nc, float sigma, const float* rnd, const PaperSamplesWs& w,
                                     float* out, int* n_acc, int* n_short, hipStream_t st) {
  const int stride = 3 * nu + 5 * nc + 8 * ns;
  const ExactShape shape = default_exact_shape();
  hipError_t e;
  if (nu > 0) {
    hipLaunchKernelGGL(k_uniform_points, dim3(grid_for(m.n * nu, 256)), dim3(256), 0, st, m.n, nu, stride, rnd, half,
                       w.ux, w.uy, w.uz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const CloudArgs cu{(int)(m.n * nu), w.ux, w.uy, w.uz};
    if ((e = launch_exact_any(rb, table, m, cu, nullptr, nullptr, m.n, nullptr, nullptr, nu, w.ud, nullptr, shape,
                              st)) != hipSuccess)
      return e;
  }
  if (ns > 0) {
    hipLaunchKernelGGL(k_surface_candidates, dim3(grid_for(m.n * nc, 256)), dim3(256), 0, st, table, m.n, m.T,
                       rb.n_caps, nu, nc, stride, rnd, w.cx, w.cy, w.cz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const CloudArgs cc{(int)(m.n * nc), w.cx, w.cy, w.cz};
    if ((e = launch_exact_any(rb, table, m, cc, nullptr, nullptr, m.n, nullptr, nullptr, nc, w.cd, nullptr, shape,
                              st)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_pick_surface, dim3(grid_for(m.n, 4)), dim3(256), 0, st, m.n, nc, ns, w.cx, w.cy, w.cz, w.cd,
                       w.sx, w.sy, w.sz, w.sd, n_acc, n_short);
    hipLaunchKernelGGL(k_surface_children, dim3(grid_for(m.n * ns, 256)), dim3(256), 0, st, m.n, nu, nc, ns, stride,
                       rnd, sigma, w.sx, w.sy, w.sz, w.kx, w.ky, w.kz);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const CloudArgs ck{(int)(m.n * 3 * ns), w.kx, w.ky, w.kz};
    if ((e = launch_exact_any(rb, table, m, ck, nullptr, nullptr, m.n, nullptr, nullptr, 3 * ns, w.kd, nullptr,
                              shape, st)) != hipSuccess)
      return e;
  }
  hipLaunchKernelGGL(k_assemble_paper, dim3(grid_for(m.n, 4)), dim3(256), 0, st, m.n, rb.dof, nu, ns, m.q0, m.q1, w.ux,
                     w.uy, w.uz, w.ud, w.sx, w.sy, w.sz, w.sd, w.kx, w.ky, w.kz, w.kd, out);
  return hipGetLastError();
}

}  // namespace sv
