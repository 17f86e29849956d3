// Device building blocks of the exact swept-volume check, shared by the per-call
// kernels (sv_geom.hip) and the batched kernels (sv_batch.hip), so that both compute
// every distance with the same instructions and agree bit for bit.
//
// Paper: Sec. III, eq. (1)-(4) (signed distance to the swept volume, a union over the
// path of the robot's occupancy) and Sec. IV-B (cloud distance, verdict).
#pragma once

#include <math.h>

#include "sv_internal.h"

namespace sv {
namespace {

constexpr unsigned long long kKeyEmpty = ~0ull;

// Monotone map of a float onto uint32 so that unsigned order equals float order.
__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}
__device__ __forceinline__ unsigned long long ord_f64(double f) {
  unsigned long long u = (unsigned long long)__double_as_longlong(f);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double unord_f64(unsigned long long o) {
  unsigned long long u = (o >> 63) ? (o & ~(1ull << 63)) : ~o;
  return __longlong_as_double((long long)u);
}

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// Path parameter of sample t of T.
template <typename R>
__device__ __forceinline__ R sample_s(int t, int T) {
  return T > 1 ? (R)t / (R)(T - 1) : (R)0;
}

// Joint configuration q_s of one motion (eq. (2)).
// Linear: q0 + s (q1 - q0).  Spline: per joint, the C2 cubic through (0, q0),
// (1/3, v1), (2/3, v2), (1, q1) with zero end slopes.  With knot spacing 1/3 the
// two interior slopes, already multiplied by the spacing, are
//   h m1 = (4 (v2 - q0) - (q1 - v1)) / 5,   h m2 = (4 (q1 - v1) - (v2 - q0)) / 5,
// and each segment is a cubic Hermite in u = 3 s - segment.
template <typename R>
__device__ __forceinline__ void motion_config(int kind, int dof, const float* q0, const float* q1,
                                              const float* via, R s, R* q) {
  if (kind == SV_LINEAR) {
#pragma unroll
    for (int j = 0; j < SV_MAX_DOF; ++j)
      if (j < dof) {
        R a = (R)q0[j], b = (R)q1[j];
        q[j] = a + s * (b - a);
      }
    return;
  }
  R s3 = s * (R)3;
  int seg = (int)s3;
  seg = seg > 2 ? 2 : (seg < 0 ? 0 : seg);
  R u = s3 - (R)seg;
  R u2 = u * u, u3 = u2 * u;
  R h00 = (R)2 * u3 - (R)3 * u2 + (R)1;
  R h10 = u3 - (R)2 * u2 + u;
  R h01 = (R)3 * u2 - (R)2 * u3;
  R h11 = u3 - u2;
#pragma unroll
  for (int j = 0; j < SV_MAX_DOF; ++j)
    if (j < dof) {
      R y0 = (R)q0[j], y1 = (R)via[j], y2 = (R)via[dof + j], y3 = (R)q1[j];
      R hm1 = ((R)4 * (y2 - y0) - (y3 - y1)) / (R)5;
      R hm2 = ((R)4 * (y3 - y1) - (y2 - y0)) / (R)5;
      R ya = seg == 0 ? y0 : (seg == 1 ? y1 : y2);
      R yb = seg == 0 ? y1 : (seg == 1 ? y2 : y3);
      R ma = seg == 0 ? (R)0 : (seg == 1 ? hm1 : hm2);
      R mb = seg == 0 ? hm1 : (seg == 1 ? hm2 : (R)0);
      q[j] = h00 * ya + h10 * ma + h01 * yb + h11 * mb;
    }
}

// World endpoints of every capsule at configuration q (standard DH chain).
// F holds the running frame [R | p] (3x4, row-major); after joint i it is frame i.
template <typename R>
__device__ __forceinline__ void fk_capsules(const RobotT<R>& rb, const R* q, R (&A)[SV_MAX_CAPS][3],
                                            R (&B)[SV_MAX_CAPS][3]) {
  R F[12] = {(R)1, (R)0, (R)0, (R)0, (R)0, (R)1, (R)0, (R)0, (R)0, (R)0, (R)1, (R)0};
  for (int f = 0; f <= rb.dof; ++f) {
    if (f > 0) {
      const int i = f - 1;
      R st, ct, sa, ca;
      sincos_r(q[i] + rb.dh[i][3], &st, &ct);
      sincos_r(rb.dh[i][1], &sa, &ca);
      const R a = rb.dh[i][0], d = rb.dh[i][2];
      // F <- F * [[ct, -st ca, st sa, a ct], [st, ct ca, -ct sa, a st], [0, sa, ca, d]]
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const R f0 = F[4 * r], f1 = F[4 * r + 1], f2 = F[4 * r + 2], f3 = F[4 * r + 3];
        const R c0 = f0 * ct + f1 * st;
        const R s0 = f1 * ct - f0 * st;   // row . (-st, ct, 0)
        F[4 * r + 0] = c0;
        F[4 * r + 1] = s0 * ca + f2 * sa;
        F[4 * r + 2] = f2 * ca - s0 * sa;
        F[4 * r + 3] = a * c0 + d * f2 + f3;
      }
    }
#pragma unroll
    for (int k = 0; k < SV_MAX_CAPS; ++k) {
      if (k < rb.n_caps) {
        if (rb.fa[k] == f)
#pragma unroll
          for (int r = 0; r < 3; ++r)
            A[k][r] = F[4 * r] * rb.pa[k][0] + F[4 * r + 1] * rb.pa[k][1] + F[4 * r + 2] * rb.pa[k][2] + F[4 * r + 3];
        if (rb.fb[k] == f)
#pragma unroll
          for (int r = 0; r < 3; ++r)
            B[k][r] = F[4 * r] * rb.pb[k][0] + F[4 * r + 1] * rb.pb[k][1] + F[4 * r + 2] * rb.pb[k][2] + F[4 * r + 3];
      }
    }
  }
}

// Capsule entries are uniform across a wave: read them through the constant
// address space so that they arrive in scalar registers (s_load).
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const vf4* ConstF4Ptr;

__device__ __forceinline__ CapEntry load_entry(ConstF4Ptr p, size_t idx) {
  const vf4 lo = p[3 * idx], mid = p[3 * idx + 1], hi = p[3 * idx + 2];
  CapEntry e;
  e.ax = lo.x; e.ay = lo.y; e.az = lo.z; e.r = lo.w;
  e.bx = mid.x; e.by = mid.y; e.bz = mid.z; e.inv_l2 = mid.w;
  e.hx = hi.x; e.hy = hi.y; e.hz = hi.z; e.pad = hi.w;
  return e;
}

// Squared distance from (x, y, z) to the segment of entry e.  The closest-point
// parameter (p - A) . H, H = AB / |AB|^2, is clamped to [0, 1]; the residual is formed
// explicitly (never as |ap|^2 - dot^2 / |ab|^2, which cancels near the segment's axis).
__device__ __forceinline__ float seg_d2(const CapEntry& e, float x, float y, float z) {
  const float px = x - e.ax, py = y - e.ay, pz = z - e.az;
  const float u = __builtin_amdgcn_fmed3f(px * e.hx + py * e.hy + pz * e.hz, 0.0f, 1.0f);
  const float ex = px - u * e.bx, ey = py - u * e.by, ez = pz - u * e.bz;
  return ex * ex + ey * ey + ez * ez;
}

__device__ __forceinline__ void decode_key(unsigned long long key, float* d, int* arg) {
  if (key == kKeyEmpty) {
    *d = INFINITY;
    *arg = -1;
  } else {
    *d = unord_f32((uint32_t)(key >> 32));
    *arg = (int)(uint32_t)(key & 0xffffffffu);
  }
}

__device__ __forceinline__ void write_result(const sv_results& out, int64_t m, float d, int arg, float eps) {
  if (out.min_dist) out.min_dist[m] = d;
  if (out.argmin) out.argmin[m] = arg;
  if (out.verdict) out.verdict[m] = (uint8_t)(d <= eps);
}

__device__ __forceinline__ double seg_d2_64(const CapEntry64& e, double x, double y, double z) {
  const double px = x - e.ax, py = y - e.ay, pz = z - e.az;
  double u = 0.0;
  if (e.l2 > 0.0) {
    u = (px * e.bx + py * e.by + pz * e.bz) / e.l2;
    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
  }
  const double ex = px - u * e.bx, ey = py - u * e.by, ez = pz - u * e.bz;
  return ex * ex + ey * ey + ez * ez;
}

// Capsule entries of sample t of T of one motion (q0, q1 and, for splines, via: the
// motion's rows) written to dst[k * stride], k < n_caps.
__device__ __forceinline__ void write_entries(const Robot32& rb, int kind, const float* q0, const float* q1,
                                              const float* via, int t, int T, CapEntry* __restrict__ dst,
                                              int64_t stride) {
  float q[SV_MAX_DOF];
  motion_config<float>(kind, rb.dof, q0, q1, via, sample_s<float>(t, T), q);
  float A[SV_MAX_CAPS][3], B[SV_MAX_CAPS][3];
  fk_capsules<float>(rb, q, A, B);
#pragma unroll
  for (int k = 0; k < SV_MAX_CAPS; ++k)
    if (k < rb.n_caps) {
      const float bx = B[k][0] - A[k][0], by = B[k][1] - A[k][1], bz = B[k][2] - A[k][2];
      const float l2 = bx * bx + by * by + bz * bz;
      CapEntry e;
      e.ax = A[k][0]; e.ay = A[k][1]; e.az = A[k][2];
      e.inv_l2 = l2 > 0.f ? 1.0f / l2 : 0.f;
      e.bx = bx; e.by = by; e.bz = bz; e.r = rb.r[k];
      e.hx = bx * e.inv_l2; e.hy = by * e.inv_l2; e.hz = bz * e.inv_l2; e.pad = 0.f;
      dst[(size_t)k * stride] = e;
    }
}

// The same in FP64 (motion sample, FK and entries), for the certified-band recheck.
__device__ __forceinline__ void write_entries64(const Robot64& rb, int kind, const float* q0, const float* q1,
                                                const float* via, int t, int T, CapEntry64* __restrict__ dst,
                                                int64_t stride) {
  double q[SV_MAX_DOF];
  motion_config<double>(kind, rb.dof, q0, q1, via, sample_s<double>(t, T), q);
  double A[SV_MAX_CAPS][3], B[SV_MAX_CAPS][3];
  fk_capsules<double>(rb, q, A, B);
#pragma unroll
  for (int k = 0; k < SV_MAX_CAPS; ++k)
    if (k < rb.n_caps) {
      CapEntry64 e;
      e.ax = A[k][0]; e.ay = A[k][1]; e.az = A[k][2];
      e.bx = B[k][0] - A[k][0]; e.by = B[k][1] - A[k][1]; e.bz = B[k][2] - A[k][2];
      e.l2 = e.bx * e.bx + e.by * e.by + e.bz * e.bz;
      e.r = rb.r[k];
      dst[(size_t)k * stride] = e;
    }
}

// FP64 swept distance of one point: entries e0[k * stride + t], t < T, k < K.
__device__ __forceinline__ double swept_min64(const CapEntry64* __restrict__ e0, int T, int64_t stride, int K,
                                              double x, double y, double z) {
  double best = INFINITY;
  for (int k = 0; k < K; ++k) {
    double m2 = INFINITY;
    for (int t = 0; t < T; ++t) m2 = fmin(m2, seg_d2_64(e0[(size_t)k * stride + t], x, y, z));
    best = fmin(best, sqrt(m2) - e0[(size_t)k * stride].r);
  }
  return best;
}

// Per lane: m2[p] <- min(m2[p], squared distance from point p to the segments of entries
// e + t, t0 <= t < t1).  Samples are taken two at a time (the compiler merges the pair
// into one three-way min); the minimum is exact, so how a range is split does not
// change the result.
template <int P>
__device__ __forceinline__ void swept_range(ConstF4Ptr tab, size_t e, int t0, int t1, const float (&x)[P],
                                            const float (&y)[P], const float (&z)[P], float (&m2)[P]) {
  int t = t0;
  for (; t + 1 < t1; t += 2) {
    const CapEntry a = load_entry(tab, e + t);
    const CapEntry b = load_entry(tab, e + t + 1);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const float da = seg_d2(a, x[p], y[p], z[p]);
      const float db = seg_d2(b, x[p], y[p], z[p]);
      m2[p] = fminf(m2[p], fminf(da, db));
    }
  }
  if (t < t1) {
    const CapEntry a = load_entry(tab, e + t);
#pragma unroll
    for (int p = 0; p < P; ++p) m2[p] = fminf(m2[p], seg_d2(a, x[p], y[p], z[p]));
  }
}

// swept_range for the culled passes' sample blocks (2 to 16 samples, one block per
// call): the entries of four samples are loaded before any of their tests, so that one
// latency of the scalar loads covers four tests per point (with the sparser bound
// updates of the culled passes: 0.562 -> 0.528 ms per culled pass at T = 256 and 1.40 ->
// 1.17 ms at T = 1,024 on bin20k; eight samples at a time measured slower).
// The same squared distances as swept_range, so the minima are bit-identical.
template <int P>
__device__ __forceinline__ void swept_block(ConstF4Ptr tab, size_t e, int t0, int t1, const float (&x)[P],
                                            const float (&y)[P], const float (&z)[P], float (&m2)[P]) {
  int t = t0;
  for (; t + 3 < t1; t += 4) {
    CapEntry q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = load_entry(tab, e + t + i);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      float d[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = seg_d2(q[i], x[p], y[p], z[p]);
      m2[p] = fminf(m2[p], fminf(fminf(d[0], d[1]), fminf(d[2], d[3])));
    }
  }
  for (; t < t1; ++t) {
    const CapEntry a = load_entry(tab, e + t);
#pragma unroll
    for (int p = 0; p < P; ++p) m2[p] = fminf(m2[p], seg_d2(a, x[p], y[p], z[p]));
  }
}

// Per lane: best[p] = min over capsules k of (sqrt(min over samples t of the squared
// distance from point p to segment k at t) - r_k), for the motion whose table entries
// start at entry e0 and run [K][T].
template <int P>
__device__ __forceinline__ void swept_min(ConstF4Ptr tab, size_t e0, int T, int K, const float (&x)[P],
                                          const float (&y)[P], const float (&z)[P], float (&best)[P]) {
#pragma unroll
  for (int p = 0; p < P; ++p) best[p] = INFINITY;
  for (int k = 0; k < K; ++k) {
    const size_t e = e0 + (size_t)k * T;
    float m2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) m2[p] = INFINITY;
    swept_range<P>(tab, e, 0, T, x, y, z, m2);
    const float r = load_entry(tab, e).r;
#pragma unroll
    for (int p = 0; p < P; ++p) best[p] = fminf(best[p], sqrtf(m2[p]) - r);
  }
}

// Smallest (distance, index) key of a lane's points (idx < 0: no point).
template <int P>
__device__ __forceinline__ unsigned long long lane_min_key(const float (&best)[P], const int (&idx)[P]) {
  unsigned long long key = kKeyEmpty;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (idx[p] >= 0) {
      const unsigned long long kk = ((unsigned long long)ord_f32(best[p]) << 32) | (uint32_t)idx[p];
      key = kk < key ? kk : key;
    }
  }
  return key;
}

// Minimum of one key per thread over a block of NT threads; the result is valid in
// thread 0.  wmin: NT / 64 words of LDS.  Contains one barrier; a second call on the
// same wmin must be separated from this one by another barrier.
template <int NT>
__device__ __forceinline__ unsigned long long block_min_key(unsigned long long key, unsigned long long* wmin) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(key, off, 64);
    key = o < key ? o : key;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wmin[wid] = key;
  __syncthreads();
  unsigned long long k2 = kKeyEmpty;
  if (threadIdx.x == 0) {
    k2 = wmin[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) k2 = wmin[w] < k2 ? wmin[w] : k2;
  }
  return k2;
}

}  // namespace
}  // namespace sv
