/*
 * sv.h -- C ABI of libsv, the MI355X (gfx950) swept-volume collision checker.
 *
 * Method: Joho, Schwinn, Safronov, "Neural Implicit Swept Volume Models for Fast
 * Collision Detection" (ICRA 2024).  The library evaluates, on one GPU,
 *   - the signed distance f_d(x, m) of a point x to the swept volume V_S(m) of a
 *     motion m (Sec. III, eq. (1)-(4)), exactly, by sampling the motion at T
 *     configurations, placing the robot's capsules with forward kinematics and
 *     taking the minimum point-to-capsule distance;
 *   - the cloud distance d(X, m) = min over x in X and the verdict "free iff
 *     d(X, m) > eps_S" (Sec. IV-B, Alg. 1);
 *   - the learned model f_theta(x, q0, q1) (Sec. IV-A) as a softplus MLP, and
 *     per-point screening with that model in front of the exact check.
 *
 * Conventions shared by every entry point:
 *   - Units are metres and radians.  Distances are signed: negative inside.
 *   - "dev" pointers are device (HBM) pointers the caller owns; "host" pointers
 *     are read during the call only.  The library never allocates or frees
 *     memory and never synchronises: scratch memory comes in through
 *     (ws, ws_bytes), sized with sv_workspace_size(), and every call is
 *     asynchronous on `stream` (a hipStream_t; NULL is the default stream).
 *   - Arguments are validated on the host before anything is launched.  On a
 *     validation failure the call returns a negative sv_status, launches
 *     nothing, and sv_last_error() describes the problem.  A HIP launch error
 *     is returned as SV_ERR_HIP.  Input values must be finite; they are not
 *     checked.
 *   - Verdicts: 1 = collision (d <= eps), 0 = free (d > eps).
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SV_OK = 0,
  SV_ERR_ARG = -1,          /* null pointer or value out of range */
  SV_ERR_SHAPE = -2,        /* inconsistent sizes */
  SV_ERR_WORKSPACE = -3,    /* workspace missing or too small */
  SV_ERR_UNSUPPORTED = -4,  /* valid request the library does not implement */
  SV_ERR_HIP = -5           /* a HIP runtime call failed */
} sv_status;

#define SV_MAX_DOF 8
#define SV_MAX_CAPS 16

/* Robot model (host struct, read during the call).
 * Kinematics: standard Denavit-Hartenberg, frame i = frame i-1 * Rz(q_i + theta_off_i)
 * Tz(d_i) Tx(a_i) Rx(alpha_i), frame 0 = world.  The paper needs "the sequence of
 * poses of each link" along a motion (Sec. IV-C); the robot's volume V_R(q)
 * (Sec. III) is a union of capsules.  Capsule k is the segment between point
 * cap_p[k][0] fixed in frame cap_frame[k][0] and point cap_p[k][1] fixed in frame
 * cap_frame[k][1], inflated by radius cap_r[k] >= 0.  Frame indices run 0..dof. */
typedef struct {
  int32_t dof;                          /* 1..SV_MAX_DOF */
  int32_t n_caps;                       /* 1..SV_MAX_CAPS */
  double dh[SV_MAX_DOF][4];             /* rows (a, alpha, d, theta_off) */
  int32_t cap_frame[SV_MAX_CAPS][2];
  double cap_p[SV_MAX_CAPS][2][3];
  double cap_r[SV_MAX_CAPS];
} sv_robot;

/* Motion types.  The path c(m, s), s in [0, 1] (Sec. III, eq. (2)) is sampled at
 * s_t = t / (T - 1), t = 0..T-1 (T = 1: s = 0).
 *   SV_LINEAR: q_s = q0 + s (q1 - q0) (the paper's linear joint-space motion, Sec. IV-C).
 *   SV_SPLINE: per joint, the cubic spline through q0, via[0], via[1], q1 at
 *              s = 0, 1/3, 2/3, 1 with zero end slopes and continuous second
 *              derivative (a joint-space stand-in for the paper's task-space spline). */
enum { SV_LINEAR = 0, SV_SPLINE = 1 };

typedef struct {
  int32_t kind;        /* SV_LINEAR or SV_SPLINE */
  int32_t T;           /* samples per motion, >= 1 */
  int64_t n;           /* number of motions M, >= 0 */
  const float* q0;     /* dev [M][dof] */
  const float* q1;     /* dev [M][dof] */
  const float* via;    /* dev [M][2][dof] for SV_SPLINE, else ignored */
} sv_motions;

/* Point cloud X (Sec. IV-B), structure of arrays. */
typedef struct {
  int64_t n;           /* number of points N, >= 0 (indices must fit in int32) */
  const float* x;      /* dev [N] */
  const float* y;      /* dev [N] */
  const float* z;      /* dev [N] */
} sv_cloud;

/* Per-motion results, all dev [M]; any pointer may be NULL to skip that output. */
typedef struct {
  float* min_dist;     /* d(X, m); +inf when N = 0 */
  int32_t* argmin;     /* index of a point attaining min_dist (the lowest among FP32
                          ties); -1 when N = 0 */
  uint8_t* verdict;    /* 1 = collision (d <= eps), 0 = free */
  int32_t* n_fallback; /* screening only: points sent to the exact check */
} sv_results;

/* Swept-volume network f_theta(x, q0, q1) -> delta_hat (Sec. IV-A), with input
 * x_in = [x; q0; q1] (in that order, the inputs of Fig. 1).  Two architectures:
 *
 * SV_NET_MLP: a plain MLP with softplus activations, h_1 = softplus(W_1 x_in + b_1),
 *   h_l = softplus(W_l h_{l-1} + b_l) for l = 2..L, delta_hat = w_out . h_L + b_out,
 *   softplus(z) = max(z, 0) + log(1 + exp(-|z|)).
 *   params: W_1 [W][in_dim], b_1 [W], then for l = 2..L: W_l [W][W], b_l [W]; then
 *   w_out [W], b_out [1].
 *
 * SV_NET_RESIDUAL: the paper's network (Sec. IV-A, Fig. 1): an initial linear layer
 *   h_0 = W_0 x_in + b_0 (no activation), then L blocks, each a linear layer on the
 *   block input with the network input concatenated (the jump connection), a ReLU, a
 *   BatchNorm (inference form, running statistics) and a skip connection:
 *     z_b = W_b [h_{b-1}; x_in] + c_b,
 *     h_b = h_{b-1} + gamma_b (relu(z_b) - mu_b) / sqrt(var_b + bn_eps) + beta_b,
 *   then delta_hat = w_out . h_L + b_out.
 *   params: W_0 [W][in_dim], b_0 [W], then per block b = 1..L: Wh_b [W][W] (the columns
 *   of W_b acting on h), Wx_b [W][in_dim] (the columns acting on x_in), c_b [W],
 *   gamma_b [W], beta_b [W], mu_b [W], var_b [W]; then w_out [W], b_out [1].
 *
 * Weights row-major [out][in], FP32.  The network applies to linear motions only:
 * (q0, q1) determines a linear motion but not a spline (Sec. IV-C). */
enum { SV_NET_MLP = 0, SV_NET_RESIDUAL = 1 };
typedef struct {
  int32_t in_dim;      /* 3 + 2 * dof; SV_NET_RESIDUAL in BF16: dof <= 6 */
  int32_t width;       /* hidden width W: FP32 path W % 64 == 0, W <= 1024; BF16 path 128, 256, 512
                          or 1024 (training: up to 512) */
  int32_t n_hidden;    /* L >= 1: softplus layers (SV_NET_MLP) or blocks (SV_NET_RESIDUAL) */
  const float* params; /* dev FP32, flat, in the order given above */
  int32_t kind;        /* SV_NET_MLP or SV_NET_RESIDUAL */
  float bn_eps;        /* SV_NET_RESIDUAL: the BatchNorm epsilon (> 0) */
} sv_mlp;

/* Arithmetic of the network evaluation. */
enum {
  SV_FP32 = 0,  /* FP32 throughout */
  SV_BF16 = 1   /* hidden layers: BF16 weights and activations (round to nearest even) on MFMA with
                   FP32 accumulation; first and output layers in FP32 */
};

/* Screening modes of sv_check_motions.  A point is sent to the exact check iff the
 * network predicts delta_hat < tau (the network is a proxy for the exact distance,
 * Sec. IV-B).  SV_SCREEN_TRUST: a motion collides iff a sent point has exact distance
 * <= eps; SV_SCREEN_CERTIFIED: as TRUST, and every motion without such a witness is
 * checked exactly over all its points, so that verdicts equal the exact check's (as
 * Alg. 1 confirms with the geometric checker every motion it reports free). */
enum { SV_SCREEN_NONE = 0, SV_SCREEN_TRUST = 1, SV_SCREEN_CERTIFIED = 2 };
/* May be OR'd into the screen argument of sv_check_motions: the exact passes over all
 * points of a motion run every test instead of skipping provably distant groups.  The
 * results are the same bit for bit; a measurement aid (per call, no global state). */
enum { SV_CHECK_UNCULLED = 0x100 };

/* Workspace sizes per operation. */
enum { SV_OP_EXACT_SDF = 0, SV_OP_CHECK = 1, SV_OP_NN_SDF = 2 };

/* Human-readable name of a status code. */
const char* sv_status_string(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* sv_last_error(void);

/* Bytes of workspace the operation `op` needs for these arguments (host, no launch).
 * SV_OP_EXACT_SDF: robot, motions, cloud.  SV_OP_CHECK: robot, motions, cloud and mlp
 * (NULL = exact only).  SV_OP_NN_SDF: mlp, motions, cloud and `precision` (robot may be
 * NULL).  Returns SV_OK and writes *bytes. */
int sv_workspace_size(int op, const sv_robot* robot, const sv_mlp* mlp, int precision,
                      const sv_motions* motions, const sv_cloud* cloud, size_t* bytes);

/* Forward kinematics (paper Sec. IV-C: the poses of every link along a motion).
 * q: dev [n_cfg][dof] joint configurations (FP32).
 * caps: dev [n_cfg][n_caps][8] output; entry = (Ax, Ay, Az, Bx, By, Bz, r, 0), the
 *       world endpoints and radius of every capsule.
 * fp64: 0 = FP32 arithmetic, 1 = FP64 arithmetic rounded to FP32 at the end.
 * No workspace.  n_cfg = 0 is a no-op. */
int sv_fk(const sv_robot* robot, const float* q, int64_t n_cfg, float* caps, int fp64, void* stream);

/* Exact swept signed distance of every point to every motion (Sec. III, eq. (1)-(4)):
 *   sdf[m][i] = min over t < T, k < n_caps of ( |x_i - segment_k(q_t)| - r_k ),
 * computed in FP32.  sdf: dev [M][N] row-major.  Workspace: SV_OP_EXACT_SDF. */
int sv_exact_sdf(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud, float* sdf,
                 void* ws, size_t ws_bytes, void* stream);

/* Network prediction delta_hat = f_theta(x_i, q0_m, q1_m) for every (motion, point):
 * sdf_hat dev [M][N] row-major.  Linear motions only (T is ignored).
 * precision: SV_FP32 or SV_BF16.  Workspace: SV_OP_NN_SDF (0 bytes for SV_FP32). */
int sv_nn_sdf(const sv_mlp* mlp, int precision, const sv_motions* motions, const sv_cloud* cloud, float* sdf_hat,
              void* ws, size_t ws_bytes, void* stream);

/* Collision check of M motions against one cloud (Sec. IV-B: d(X, m) and the
 * safety-margin test of Alg. 1).
 *   mlp == NULL, screen == SV_SCREEN_NONE: exact check of every (motion, point).
 *   mlp != NULL, screen TRUST or CERTIFIED: the BF16 network screens every (motion,
 *     point) first and only points with delta_hat < tau go to the exact check (linear
 *     motions; mlp->width 128, 256, 512 or 1024).  n_fallback[m] counts them.  min_dist of a
 *     motion decided by a witness is the minimum over the sent points; of any other
 *     motion it is the minimum over all points (CERTIFIED) or over the sent points,
 *     +inf if none (TRUST).
 * Exact distances are FP32; every motion whose FP32 distance lies within 1e-5 m of eps
 * is recomputed in FP64 over all its points so that its verdict is the FP64 one
 * (min_dist then holds the FP64 value rounded to FP32).
 * The exact passes over all points of a motion skip groups of (point, capsule, sample)
 * tests that bounding spheres prove to lie above the motion's minimum (the cloud is
 * put in Morton order internally; reported indices are the caller's).  Skipping never
 * changes min_dist, argmin or verdict: they equal the unskipped computation bit for
 * bit (screen | SV_CHECK_UNCULLED runs them unskipped).  Workspace: SV_OP_CHECK; after a
 * call its first 256 uint64 words sum to the number of segment tests the skipping
 * passes executed (a measurement aid). */
int sv_check_motions(const sv_robot* robot, const sv_mlp* mlp, int screen, float eps, float tau,
                     const sv_motions* motions, const sv_cloud* cloud, sv_results* out, void* ws,
                     size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): sv_check_motions without a workspace
 * argument.  Its scratch memory is a static device array of SV_STATIC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on, from the first call with that device
 * current until the process ends; the call itself allocates and frees nothing and
 * records no profiler events.  Arguments, results and arithmetic are those of
 * sv_check_motions (the same kernels).  A check whose workspace (sv_workspace_size,
 * SV_OP_CHECK) exceeds SV_STATIC_SCRATCH_BYTES returns SV_ERR_WORKSPACE and launches
 * nothing; the exact and the screened check of 512 motions at T = 256 against 20,000
 * points with a 15 -> 8 x 512 -> 1 network fit (46 and 88 MiB).  Every call on one GPU
 * uses that GPU's one array and leaves its contents behind (each call initialises what
 * it reads): calls that overlap in time on one GPU -- other streams, other threads --
 * race and give wrong results, so the caller must order them. */
#define SV_STATIC_SCRATCH_BYTES ((size_t)96 << 20)
int sv_check_motions_static(const sv_robot* robot, const sv_mlp* mlp, int screen, float eps, float tau,
                            const sv_motions* motions, const sv_cloud* cloud, sv_results* out, void* stream);

/* ---- continuous certification (Sec. III, eq. (3)) ---------------------------------
 * The swept volume is a union over the continuous path parameter s in [0, 1]; the
 * exact check evaluates it at the T samples s_t, so its distance is an upper bound of
 * the continuous one.  For every motion, gap[m] bounds the difference:
 *   d_cont(x, m) >= d_T(x, m) - gap[m]  for every point x,
 * with gap[m] = max_k L_k h, h = 1 / (2 (T - 1)) (1 for T = 1) the largest distance from
 * any s to a sample and L_k a bound of the speed (per unit s) of capsule k's points:
 * for an endpoint fixed in frame f at coordinates p, sum over joints j <= f of
 * max_s |dq_j/ds| (sum_{i=j..f} sqrt(a_i^2 + d_i^2) + |p|).  max_s |dq_j/ds| is
 * |q1_j - q0_j| for linear motions and the exact maximum of the spline's derivative
 * for splines.  Computed in FP64, rounded up to FP32.
 * With min_dist (dev [M], e.g. sv_results.min_dist of the same motions and cloud),
 * verdict[m] = 0 iff min_dist[m] - gap[m] > eps + 1e-5 (free along the whole
 * continuous motion, with the FP32 error band of min_dist), else 1.
 * gap: dev [M]; min_dist and verdict: both NULL or both dev [M]. */
int sv_continuous_gap(const sv_robot* robot, const sv_motions* motions, const float* min_dist, float eps, float* gap,
                      uint8_t* verdict, void* stream);

/* ---- batches of uneven requests (Sec. IV-B's check, many callers at once) --------
 * A request is one set of motions checked against one cloud: exactly the question of
 * sv_check_motions without a network, answered with the same per-point arithmetic, so
 * a request's results equal those of sv_check_motions on it bit for bit.
 * sv_check_requests answers a whole batch with a fixed sequence of kernels whose
 * launch shapes depend only on the capacities and the tile below, never on the
 * request contents:
 *   1. plan: validate every request, order them by estimated work (smallest first:
 *      small requests then finish early), lay out per-request offsets;
 *   2. capsule tables of every motion of every request;
 *   3. the exact check, skipping (as sv_check_motions does) the (motion, 512-point
 *      tile, capsule) items and the sample blocks that provably cannot lower a
 *      motion's minimum: all clouds are sorted together by (request, Morton code), a
 *      seed bound and bounding spheres are computed for every request, the surviving
 *      items are listed in work order, and one persistent kernel takes them in that
 *      order; the block that retires a request's last item writes the request's
 *      results and stamps done_ticks.  With tile->cull = 0 a persistent kernel of the
 *      given shape takes (request, motion, chunk of point tiles) items from a device
 *      work queue instead;
 *   4. FP64 recheck of the motions within 1e-5 m of eps (as sv_check_motions).
 * The call can therefore be captured in a HIP graph once and replayed after the
 * caller rewrites the request table (and the buffers it points to) within the same
 * capacities. */
typedef struct {
  sv_motions motions;  /* LINEAR or SPLINE, any T in [1, caps.max_T] */
  sv_cloud cloud;      /* cloud.n <= caps.max_points */
  sv_results out;      /* dev [motions.n] each; n_fallback is not written */
} sv_request;          /* the request table lives in device memory: dev [n_req] */

typedef struct {
  int32_t max_requests;  /* n_req <= max_requests <= 4096 */
  int32_t max_T;         /* every request's T <= max_T */
  int64_t max_motions;   /* sum of motions.n over the batch */
  int64_t max_samples;   /* sum of motions.n * T over the batch */
  int64_t max_points;    /* every request's cloud.n <= max_points < 2^31 */
  int32_t max_band;      /* motions that can be rechecked in FP64 per call, >= 1 */
  int64_t max_total_points; /* sum of cloud.n over the batch (< 2^30); 0: max_requests * max_points,
                               which must then be < 2^30 */
} sv_batch_caps;          /* also max_motions * ceil(max_points / 512) * 16 < 2^31 */

/* Launch shape of sv_check_requests (chosen by an autotuner, sv_tile_candidates).  Every
 * shape gives the same results bit for bit. */
typedef struct {
  /* the unculled persistent kernel (cull = 0) */
  int32_t ppl;            /* points per lane: 1, 2 or 4 */
  int32_t threads;        /* threads per block: 64, 128 or 256 */
  int32_t blocks_per_cu;  /* persistent blocks per compute unit: 1..32 */
  int32_t tiles_per_item; /* point tiles (threads * ppl points each) per work item: 1..64 */
  /* which pass runs */
  int32_t cull;           /* 1: the culled pass (the default), 0: the unculled kernel above */
  /* the culled pass (cull = 1; 512-point tiles of 256 threads x 2 points) */
  int32_t cull_blocks_per_cu; /* persistent blocks per compute unit, 1..8; 0: as many as fit */
  int32_t cull_gangs;     /* queues the persistent blocks are dealt to (block index mod gangs): 1, 2, 4,
                             8 or 16; requests are spread over the queues, an idle block helps the next */
  int32_t cull_div_linear; /* a linear motion of T samples is bounded by spheres over blocks of
                              min(16, max(2, ceil(T / div))) samples: 16, 32 or 64 */
  int32_t cull_div_spline; /* the same for splines: 32, 64 or 128 */
} sv_tile;

/* Bits of the device status word written by sv_check_requests. */
enum {
  SV_BATCH_BAD_REQUEST = 1,   /* a request is malformed (kind, T, sizes, NULL pointers): nothing computed */
  SV_BATCH_OVER_CAPACITY = 2, /* the batch exceeds caps: nothing computed */
  SV_BATCH_BAND_OVERFLOW = 4  /* more than max_band motions fell in the FP64 band: the excess keep
                                 their FP32 verdicts */
};

/* Workspace bytes for batches within caps. */
int sv_batch_workspace_size(const sv_robot* robot, const sv_batch_caps* caps, size_t* bytes);

/* Exact check of every request of the batch.
 * reqs: dev [n_req] request table (read by the kernels during the call).
 * done_ticks: dev [n_req + 1] (may be NULL): done_ticks[r] = device wall-clock tick at
 *   which request r's results became final (0 if nothing was computed);
 *   done_ticks[n_req] = tick at which the batch started.  Ticks run at
 *   sv_wall_clock_hz().
 * status: dev [1] (may be NULL): 0, or an OR of SV_BATCH_* bits.  With
 *   SV_BATCH_BAD_REQUEST or SV_BATCH_OVER_CAPACITY no result is written.
 * tile: launch shape (NULL: the library's default).
 * ws: after a call, its first 256 uint64 words sum to the number of segment tests the
 *   culled pass executed (a measurement aid; 0 with tile->cull = 0).
 * Host checks: robot, caps, tile, n_req <= caps->max_requests, workspace size.
 * Concurrent calls must not share a workspace. */
int sv_check_requests(const sv_robot* robot, const sv_request* reqs, int32_t n_req, const sv_batch_caps* caps,
                      float eps, const sv_tile* tile, uint64_t* done_ticks, int32_t* status, void* ws,
                      size_t ws_bytes, void* stream);

/* The launch shapes an autotuner may try (all accepted by sv_check_requests): the unculled
 * shapes (cull = 0, culled fields at their defaults), then the culled ones (cull = 1,
 * unculled fields at their defaults).  Writes up to `capacity` of them to tiles (may be
 * NULL) and their total count to *n. */
int sv_tile_candidates(sv_tile* tiles, int32_t capacity, int32_t* n);

/* The default launch shape: the culled pass with 8 gangs (one per XCD under the
 * round-robin dispatch of workgroups), as many blocks as fit and divisors 32 and 64. */
int sv_default_tile(sv_tile* tile);

/* Frequency of the device wall clock that stamps done_ticks (current device). */
int sv_wall_clock_hz(int64_t* hz);

/* ---- finding the first collision-free motion (Sec. IV-B, Alg. 1) ----------------- */

/* Network proxy of the cloud distance, d_hat(X, m) = min over x in X of f_theta(x, q0_m,
 * q1_m) (Sec. IV-B), for every motion: d_hat dev [M] (+inf when N = 0; NaN
 * predictions are skipped).  BF16 network (mlp->width 128, 256, 512 or 1024), linear motions.
 * Workspace: sv_nn_min_workspace_size. */
int sv_nn_min(const sv_mlp* mlp, const sv_motions* motions, const sv_cloud* cloud, float* d_hat, void* ws,
              size_t ws_bytes, void* stream);
int sv_nn_min_workspace_size(const sv_mlp* mlp, const sv_motions* motions, size_t* bytes);

/* Result of sv_first_free (written to device memory). */
typedef struct {
  int32_t motion;      /* index of the motion returned, -1 if no motion is free */
  int32_t position;    /* its position in the visiting order (M if none) */
  float dist;          /* its exact distance d(X, m) (+inf if none) */
  int32_t n_exact;     /* exact checks made when the search runs one motion at a time: the
                          visiting-order position of the answer + 1, or M */
  int32_t n_exact_run; /* motions whose exact check this call completed (checks run in
                          parallel, so motions past the answer may be checked too) */
  int32_t n_first;     /* motions visited in the first loop (d_hat > eps); 0 without d_hat */
  int32_t n_nn;        /* network evaluations of the one-at-a-time search: the original
                          index of the answer + 1 if the first loop found it, else M; 0
                          without d_hat */
  int32_t status;      /* 0 */
} sv_search_result;

/* First collision-free motion of a set (Alg. 1).  The visiting order is:
 *   d_hat == NULL: the given order (checking each motion in turn);
 *   d_hat != NULL (dev [M], e.g. from sv_nn_min): first the motions with d_hat > eps in
 *     the given order (the first loop), then the others by d_hat descending, equal
 *     values in the given order (the second loop; NaN counts as -inf).
 * The answer is the first motion in that order whose exact distance d(X, m) > eps,
 * which is the motion Alg. 1 returns.  Exact checks run as one persistent launch over
 * the visiting order; blocks stop taking motions that lie after an answer already
 * found.  Distances are FP32; motions within 1e-5 m of eps are recomputed in FP64
 * before they count as free.  1 <= M <= 4096 (M = 0 is a no-op that reports none).
 * order: dev [M] (may be NULL) receives the visiting order.  result: dev, one record.
 * Workspace: sv_first_free_workspace_size. */
int sv_first_free(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud, float eps,
                  const float* d_hat, sv_search_result* result, int32_t* order, void* ws, size_t ws_bytes,
                  void* stream);
int sv_first_free_workspace_size(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud,
                                 size_t* bytes);

/* ---- learning the network from the exact check (Sec. IV-C, Sec. V) ---------------- */

/* Training rows: samples[s] = (x[3], q0[dof], q1[dof], delta), i.e. in_dim + 1 floats per
 * row, the tuples (x, q0, q1, delta) of Sec. IV-C with delta in metres. */

/* Training data generated by the exact check (Sec. IV-C: uniform coverage of the task
 * space plus points close to the swept surface).  For every linear motion m of
 * `motions` it writes n_uniform + n_near rows to out (dev [M * (n_uniform + n_near)]
 * [in_dim + 1], motion-major, uniform rows first):
 *   - uniform rows: x = cube_half * (2 u - 1) per coordinate;
 *   - near rows: candidates are placed around the capsules of the motion's sampled
 *     configurations (sample t, capsule k, axis position, direction on the unit sphere
 *     and a radial offset in [-band, band] from the capsule surface, all from rnd);
 *     each motion keeps, in candidate order, the first n_near candidates whose exact
 *     distance satisfies |delta| <= band; if fewer qualify, the remaining slots take the
 *     first non-qualifying candidates and *n_short (dev int, accumulated, may be NULL)
 *     counts them.
 * delta is the exact FP32 swept distance at motions->T samples (as sv_exact_sdf).
 * rnd: dev [M][3 n_uniform + 6 n_cand] numbers in [0, 1) from the caller's generator.
 * Workspace: sv_make_samples_workspace_size. */
int sv_make_samples(const sv_robot* robot, const sv_motions* motions, float cube_half, int32_t n_uniform,
                    int32_t n_near, int32_t n_cand, float band, const float* rnd, float* out, int32_t* n_short,
                    void* ws, size_t ws_bytes, void* stream);
int sv_make_samples_workspace_size(const sv_robot* robot, const sv_motions* motions, int32_t n_uniform,
                                   int32_t n_cand, size_t* bytes);

/* Training samples in the paper's proportions (Sec. IV-C, dataset generation), for
 * linear motions.  Per motion, rows [x, y, z, q0, q1, delta] (in_dim + 1 floats):
 *   n_uniform points uniform in [-box_half, box_half]^3;
 *   n_surface points on the swept surface (delta ~ 0): candidates are drawn uniformly
 *     over the total area of the capsule instances (capsule k with probability
 *     proportional to its area, sample t uniformly, a point uniform on the capsule's
 *     surface: cylinder or caps by area) and a candidate is on the swept surface iff
 *     its swept distance is 0 (FP32 >= -1e-6 m): no other instance contains it.  Every
 *     piece of the swept surface belongs to one instance's surface, so accepted
 *     candidates are uniform on it.  The first n_surface accepted ones in candidate
 *     order are kept; if fewer are accepted, the first rejected ones fill the rest and
 *     *n_short counts them;
 *   then for each surface point: two points from a spherical Gaussian around it
 *     (standard deviation sigma, Box-Muller), and one point uniform on the segment to
 *     another of the motion's surface points (chosen at random).
 * Row order per motion: uniform, surface, then (Gaussian, Gaussian, chord) per surface
 * point: n_uniform + 4 n_surface rows.  Labels from the exact check (T samples).
 * rnd: dev [M][3 n_uniform + 5 n_cand + 8 n_surface] uniforms in [0, 1): 3 per uniform
 *   point, 5 per candidate, 8 per surface point (6 for the Gaussians, 2 for the chord).
 * n_accepted: dev [M] (may be NULL): accepted candidates per motion; the swept surface
 *   area is about n_accepted / n_cand times the total instance area.
 * n_short: dev [1] (may be NULL), advanced.  n_cand >= n_surface.
 * Workspace: sv_make_samples_paper_workspace_size. */
int sv_make_samples_paper(const sv_robot* robot, const sv_motions* motions, float box_half, int32_t n_uniform,
                          int32_t n_surface, int32_t n_cand, float sigma, const float* rnd, float* out,
                          int32_t* n_accepted, int32_t* n_short, void* ws, size_t ws_bytes, void* stream);
int sv_make_samples_paper_workspace_size(const sv_robot* robot, const sv_motions* motions, int32_t n_uniform,
                                         int32_t n_surface, int32_t n_cand, size_t* bytes);

/* Network prediction for arbitrary rows (x, q0, q1, ...): out[s] = f_theta(rows[s][0:in_dim]),
 * rows dev with row_stride floats per row (>= in_dim).  Workspace: SV_OP_NN_SDF sizes
 * (motions and cloud unused: pass any valid ones) -- 0 bytes for SV_FP32. */
int sv_nn_predict(const sv_mlp* mlp, int precision, const float* rows, int64_t row_stride, int64_t n, float* out,
                  void* ws, size_t ws_bytes, void* stream);

typedef struct {
  float lr;            /* Adam step size (PyTorch default 1e-3, as used in Sec. V) */
  float beta1, beta2;  /* Adam moment decays (0.9, 0.999) */
  float adam_eps;      /* 1e-8 */
  int64_t step;        /* 1-based index of this update, for Adam's bias correction */
  float clamp_sigma;   /* s > 0: the loss is an L1 on distances clamped to [-s, s] */
  int32_t clamp_pred;  /* 0: clamp the targets only, loss = mean |y - clamp(delta)| (the prediction
                          always has a gradient); 1: clamp both, loss = mean |clamp(y) - clamp(delta)|
                          (the form of DeepSDF, whose jump connections Sec. IV-A adopts; a prediction
                          with |y| >= s then has no gradient) */
} sv_train_hparams;

/* One training step of the BF16 network (mlp->width 128, 256 or 512): forward pass of
 * the batch rows samples[batch_idx[i]], i < batch, clamped-L1 loss, backward pass,
 * Adam update.
 * SV_NET_RESIDUAL (the paper's network, Sec. IV-A; target-only clamp, in_dim <= 16): its
 * BatchNorm layers normalise with the statistics of the batch (mean and biased variance
 * over the batch rows, as PyTorch's layers do in training), the gradient flows through
 * them, and after the step every block's running statistics move towards the batch's
 * with momentum 0.1 (mu <- 0.9 mu + 0.1 mean, var <- 0.9 var + 0.1 var_B B / (B - 1)).
 * Their entries of the gradient are zero and Adam leaves them alone.  mlp->params holds the FP32 master weights and is updated in place
 * (it must point to writable device memory); adam_m, adam_v: dev [n_params] FP32
 * Adam moments (zero before the first step).  Hidden layers run in BF16 on MFMA
 * with FP32 accumulation; gradient reductions are in fixed order, so a step is
 * bitwise reproducible.
 * loss_out: dev [1], the batch loss before the update (may be NULL).
 * grad_out: dev [n_params], the batch gradient (may be NULL).
 * Workspace: sv_train_workspace_size. */
int sv_train_step(const sv_mlp* mlp, float* adam_m, float* adam_v, const sv_train_hparams* hp,
                  const float* samples, int64_t n_samples, const int32_t* batch_idx, int64_t batch,
                  float* loss_out, float* grad_out, void* ws, size_t ws_bytes, void* stream);
int sv_train_workspace_size(const sv_mlp* mlp, int64_t batch, size_t* bytes);

/* ---- measurement support (not part of the method) --------------------------------
 * Per calling thread: when enabled, every later call made from this thread records a
 * HIP event pair on its stream around each of its kernel groups ("motion_table",
 * "exact", "exact_sdf", "finalize", "recheck64", ...).  sv_profile_read waits for the
 * events this thread recorded and returns the summed elapsed milliseconds and the
 * number of recorded launches of that group since this thread's last reset.  Calls
 * from other threads are not affected.  Do not enable while capturing a HIP graph. */
int sv_profile_enable(int on);
void sv_profile_reset(void);
int sv_profile_read(const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
