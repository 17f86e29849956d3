/*
 * sv_oracle.c -- plain FP64 CPU oracle for the exact swept-volume check.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * library: it is written from the paper's definitions and nothing else.
 *
 * What it computes (paper, Sec. III and IV-B):
 *   - the robot occupancy V_R(q) as a union of capsules carried by the links of a
 *     serial arm (standard Denavit-Hartenberg kinematics; the paper asks for "the
 *     sequence of poses of each link", Sec. IV-C);
 *   - the joint path c(m, s) of a motion m = (q0, q1), eq. (2): linear joint
 *     interpolation, or a clamped cubic spline through q0, two vias and q1;
 *   - the swept volume V_S(m) = union over s of V_R(q_s), eq. (3)-(4), with s
 *     discretised at T samples s_t = t / (T - 1) including both ends (the paper
 *     discretises its linear motions into 200 steps, Sec. IV-C);
 *   - the signed distance f_d(x, m) of eq. (1) for a union of capsules: the
 *     minimum over samples and capsules of |x - segment| - radius;
 *   - the cloud distance d(X, m) = min over x in X (Sec. IV-B) and the verdict
 *     "free iff d(X, m) > eps_S" (Alg. 1 and Sec. III).
 *
 * Every routine below is the definition written out in straightforward loops, in
 * double precision, without blocking, fusion or reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_DOF 16

/* ---------------------------------------------------------------- kinematics */

/* One standard DH transform A = Rz(theta) Tz(d) Tx(a) Rx(alpha), as a 3x4 matrix
 * [R | p] in row-major order. */
static void dh_matrix(double a, double alpha, double d, double theta, double A[12]) {
  double ct = cos(theta), st = sin(theta), ca = cos(alpha), sa = sin(alpha);
  A[0] = ct;  A[1] = -st * ca; A[2] = st * sa;   A[3] = a * ct;
  A[4] = st;  A[5] = ct * ca;  A[6] = -ct * sa;  A[7] = a * st;
  A[8] = 0.0; A[9] = sa;       A[10] = ca;       A[11] = d;
}

/* C = A * B for 3x4 rigid transforms (implicit last row 0 0 0 1). */
static void compose(const double A[12], const double B[12], double C[12]) {
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      C[4 * r + c] = A[4 * r + 0] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c];
    C[4 * r + 3] = A[4 * r + 0] * B[3] + A[4 * r + 1] * B[7] + A[4 * r + 2] * B[11] + A[4 * r + 3];
  }
}

/* Frames T_0 .. T_dof of the arm at configuration q: T_0 = identity and
 * T_i = T_{i-1} A_i(q_i), theta_i = q_i + theta_offset_i.
 * dh: [dof][4] rows (a, alpha, d, theta_offset).  frames: [(dof+1)][12]. */
void orc_frames(int dof, const double* dh, const double* q, double* frames) {
  static const double I[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  memcpy(frames, I, sizeof I);
  for (int i = 0; i < dof; ++i) {
    double A[12];
    dh_matrix(dh[4 * i + 0], dh[4 * i + 1], dh[4 * i + 2], q[i] + dh[4 * i + 3], A);
    compose(frames + 12 * i, A, frames + 12 * (i + 1));
  }
}

/* World endpoints of every capsule at configuration q.
 * cap_frame: [K][2] frame of each endpoint; cap_p: [K][2][3] endpoint in that frame.
 * out: [K][6] = (A.xyz, B.xyz). */
void orc_capsules(int dof, const double* dh, int n_caps, const int* cap_frame,
                  const double* cap_p, const double* q, double* out) {
  double frames[(ORC_MAX_DOF + 1) * 12];
  orc_frames(dof, dh, q, frames);
  for (int k = 0; k < n_caps; ++k)
    for (int e = 0; e < 2; ++e) {
      const double* F = frames + 12 * cap_frame[2 * k + e];
      const double* p = cap_p + 6 * k + 3 * e;
      for (int r = 0; r < 3; ++r)
        out[6 * k + 3 * e + r] = F[4 * r] * p[0] + F[4 * r + 1] * p[1] + F[4 * r + 2] * p[2] + F[4 * r + 3];
    }
}

/* ------------------------------------------------------------------- motions */

/* Path parameter of sample t out of T (both ends included); T = 1 gives s = 0. */
double orc_sample_s(int t, int T) { return T > 1 ? (double)t / (double)(T - 1) : 0.0; }

/* Configuration q_s = c(m, s).  kind 0: linear joint interpolation q0 + s (q1 - q0).
 * kind 1: per joint, the cubic spline through (0, q0), (1/3, v1), (2/3, v2), (1, q1)
 * with zero slope at both ends and continuous second derivative at the two vias.
 * via: [2][dof] (kind 1 only). */
void orc_motion_q(int kind, int dof, const double* q0, const double* q1, const double* via,
                  double s, double* q) {
  if (kind == 0) {
    for (int j = 0; j < dof; ++j) q[j] = q0[j] + s * (q1[j] - q0[j]);
    return;
  }
  const double h = 1.0 / 3.0;
  for (int j = 0; j < dof; ++j) {
    double y[4] = {q0[j], via[j], via[dof + j], q1[j]};
    /* Slopes m0 = m3 = 0.  C2 continuity at the interior knots of a uniform grid:
     *   m_{i-1} + 4 m_i + m_{i+1} = 3 (y_{i+1} - y_{i-1}) / h,  i = 1, 2.
     * Solve the 2x2 system by Cramer's rule. */
    double r1 = 3.0 * (y[2] - y[0]) / h, r2 = 3.0 * (y[3] - y[1]) / h;
    double m[4];
    m[0] = 0.0;
    m[3] = 0.0;
    m[1] = (4.0 * r1 - r2) / 15.0;
    m[2] = (4.0 * r2 - r1) / 15.0;
    int i = (int)floor(s / h);
    if (i > 2) i = 2;
    if (i < 0) i = 0;
    double u = (s - i * h) / h;
    double h00 = 2 * u * u * u - 3 * u * u + 1, h10 = u * u * u - 2 * u * u + u;
    double h01 = -2 * u * u * u + 3 * u * u, h11 = u * u * u - u * u;
    q[j] = h00 * y[i] + h10 * h * m[i] + h01 * y[i + 1] + h11 * h * m[i + 1];
  }
}

/* ------------------------------------------------------------------ distances */

/* Signed distance of x to a capsule (segment A-B, radius r): |x - closest| - r,
 * closest = A + u (B - A), u = clamp(((x - A).(B - A)) / |B - A|^2, 0, 1). */
double orc_capsule_dist(const double* x, const double* A, const double* B, double r) {
  double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double ap[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
  double L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
  double u = 0.0;
  if (L2 > 0.0) {
    u = (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / L2;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
  }
  double e[3] = {ap[0] - u * ab[0], ap[1] - u * ab[1], ap[2] - u * ab[2]};
  return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) - r;
}

typedef struct {
  int dof, n_caps;
  const double* dh;
  const int* cap_frame;
  const double* cap_p;
  const double* cap_r;
} robot_t;

/* Capsule endpoints of one motion at all T samples: table [T][K][6]. */
static void motion_table(const robot_t* R, int kind, const double* q0, const double* q1,
                         const double* via, int T, double* table) {
  double q[ORC_MAX_DOF];
  for (int t = 0; t < T; ++t) {
    orc_motion_q(kind, R->dof, q0, q1, via, orc_sample_s(t, T), q);
    orc_capsules(R->dof, R->dh, R->n_caps, R->cap_frame, R->cap_p, q, table + (size_t)t * R->n_caps * 6);
  }
}

/* f_d(x, m) over the discretised swept volume: min over t and k. */
static double swept_dist(const robot_t* R, const double* table, int T, const double* x) {
  double best = INFINITY;
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < R->n_caps; ++k) {
      const double* c = table + ((size_t)t * R->n_caps + k) * 6;
      double d = orc_capsule_dist(x, c, c + 3, R->cap_r[k]);
      if (d < best) best = d;
    }
  return best;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Per-point swept SDF for every (motion, point): out [M][N].
 * q0, q1: [M][dof]; via: [M][2][dof] or NULL; pts: [N][3]. */
int orc_exact_sdf(int dof, const double* dh, int n_caps, const int* cap_frame, const double* cap_p,
                  const double* cap_r, int kind, int T, int64_t M, const double* q0, const double* q1,
                  const double* via, int64_t N, const double* pts, double* out, int nthreads) {
  if (dof > ORC_MAX_DOF || T < 1) return -1;
  robot_t R = {dof, n_caps, dh, cap_frame, cap_p, cap_r};
  set_threads(nthreads);
#pragma omp parallel
  {
    double* table = (double*)malloc(sizeof(double) * (size_t)T * n_caps * 6);
#pragma omp for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
      motion_table(&R, kind, q0 + m * dof, q1 + m * dof, via ? via + m * 2 * dof : NULL, T, table);
      for (int64_t i = 0; i < N; ++i) out[m * N + i] = swept_dist(&R, table, T, pts + 3 * i);
    }
    free(table);
  }
  return 0;
}

/* Cloud distance d(X, m) = min over points, the lowest point index among equal
 * minima, and the verdict (1 = collision iff d <= eps, 0 = free).  N = 0 gives
 * d = +inf, argmin = -1, verdict free. */
int orc_check_motions(int dof, const double* dh, int n_caps, const int* cap_frame, const double* cap_p,
                      const double* cap_r, int kind, int T, int64_t M, const double* q0, const double* q1,
                      const double* via, int64_t N, const double* pts, double eps, double* min_dist,
                      int64_t* argmin, uint8_t* verdict, int nthreads) {
  if (dof > ORC_MAX_DOF || T < 1) return -1;
  robot_t R = {dof, n_caps, dh, cap_frame, cap_p, cap_r};
  set_threads(nthreads);
#pragma omp parallel
  {
    double* table = (double*)malloc(sizeof(double) * (size_t)T * n_caps * 6);
#pragma omp for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
      motion_table(&R, kind, q0 + m * dof, q1 + m * dof, via ? via + m * 2 * dof : NULL, T, table);
      double best = INFINITY;
      int64_t arg = -1;
      for (int64_t i = 0; i < N; ++i) {
        double d = swept_dist(&R, table, T, pts + 3 * i);
        if (d < best) { best = d; arg = i; }
      }
      min_dist[m] = best;
      argmin[m] = arg;
      verdict[m] = (uint8_t)(best <= eps);
    }
    free(table);
  }
  return 0;
}

/* Swept SDF of independent (point, linear motion) samples, as used for training
 * labels: out[b] = f_d(x_b, (q0_b, q1_b)) at T samples.  x: [B][3]; q0, q1: [B][dof]. */
int orc_sample_sdf(int dof, const double* dh, int n_caps, const int* cap_frame, const double* cap_p,
                   const double* cap_r, int T, int64_t B, const double* x, const double* q0,
                   const double* q1, double* out, int nthreads) {
  if (dof > ORC_MAX_DOF || T < 1) return -1;
  robot_t R = {dof, n_caps, dh, cap_frame, cap_p, cap_r};
  set_threads(nthreads);
#pragma omp parallel
  {
    double* table = (double*)malloc(sizeof(double) * (size_t)T * n_caps * 6);
#pragma omp for schedule(dynamic, 16)
    for (int64_t b = 0; b < B; ++b) {
      motion_table(&R, 0, q0 + b * dof, q1 + b * dof, NULL, T, table);
      out[b] = swept_dist(&R, table, T, x + 3 * b);
    }
    free(table);
  }
  return 0;
}
