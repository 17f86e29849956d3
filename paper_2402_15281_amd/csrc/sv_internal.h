// Internal declarations shared by the libsv translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv.h"

namespace sv {

// Robot model in the precision of the kernel that reads it; passed by value as a
// kernel argument.  fa/fb: frame of each capsule endpoint; pa/pb: endpoint in it.
template <typename R>
struct RobotT {
  int dof, n_caps;
  R dh[SV_MAX_DOF][4];
  int fa[SV_MAX_CAPS], fb[SV_MAX_CAPS];
  R pa[SV_MAX_CAPS][3], pb[SV_MAX_CAPS][3];
  R r[SV_MAX_CAPS];
};
using Robot32 = RobotT<float>;
using Robot64 = RobotT<double>;

template <typename R>
RobotT<R> robot_to_dev(const sv_robot& in) {
  RobotT<R> o{};
  o.dof = in.dof;
  o.n_caps = in.n_caps;
  for (int i = 0; i < SV_MAX_DOF; ++i)
    for (int j = 0; j < 4; ++j) o.dh[i][j] = (R)in.dh[i][j];
  for (int k = 0; k < SV_MAX_CAPS; ++k) {
    o.fa[k] = in.cap_frame[k][0];
    o.fb[k] = in.cap_frame[k][1];
    for (int c = 0; c < 3; ++c) {
      o.pa[k][c] = (R)in.cap_p[k][0][c];
      o.pb[k][c] = (R)in.cap_p[k][1][c];
    }
    o.r[k] = (R)in.cap_r[k];
  }
  return o;
}

// Motion description for kernels (device pointers).
struct MotionArgs {
  int kind, T;
  int64_t n;
  const float* q0;
  const float* q1;
  const float* via;
};

// Network description for kernels: flat FP32 parameters (see sv_mlp in sv.h).
// BF16 residual network: the network input enters every block's MFMA loop as kResXCols
// extra columns of the activation tile, each input split into a BF16 high and low part
// (so in_dim <= kResMaxIn), the remaining columns zero.
constexpr int kResXCols = 32;
constexpr int kResMaxIn = kResXCols / 2;

struct MlpArgs {
  int in_dim, width, n_hidden, dof;
  const float* params;
  int kind;       // SV_NET_MLP or SV_NET_RESIDUAL
  float bn_eps;
};

struct CloudArgs {
  int n;
  const float* x;
  const float* y;
  const float* z;
};

// Capsule-sample table entry of the FP32 exact check: segment start A, radius, segment
// vector AB, 1/|AB|^2 (0 for a sphere), and H = AB / |AB|^2, so that the closest-point
// parameter of a point p is the clamped dot product (p - A) . H: one multiply per test
// fewer than (p - A) . AB / |AB|^2 (the dense kernel's 13.5 -> 12.5 VALU instructions
// per test, 5.31 -> 4.88 ms on bin20k; the culled passes read 48 instead of 32 bytes per
// sample and take the same time).  Layout [motion][capsule][t], 48 bytes each.
struct alignas(16) CapEntry {
  float ax, ay, az, r;
  float bx, by, bz, inv_l2;
  float hx, hy, hz, pad;
};
// FP64 entry for the certified-band recheck: A, |AB|^2, AB, radius.
struct alignas(64) CapEntry64 {
  double ax, ay, az, l2;
  double bx, by, bz, r;
};

// Tunable launch shape of the exact kernel: points per lane and threads per block.
struct ExactShape {
  int ppl;      // 1, 2, 4
  int threads;  // 64, 128, 256
};

// Sequential carving of the caller's workspace (256-byte aligned pieces); with a NULL
// base it only counts bytes.
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// ---- batched requests (sv_batch.hip) ----------------------------------------------
constexpr int kMaxBatchRequests = 4096;

// Device-side header of a batch call, written by the plan kernel.
struct BatchPlan {
  int status;                       // SV_BATCH_* bits
  int band_count;                   // motions queued for the FP64 recheck (may exceed capacity)
  int64_t total_items;              // work items of the batch (0 if nothing runs)
  int64_t total_samples;            // (motion, sample) pairs of the batch
  unsigned long long next_item;     // head of the work queue
  // culled pass
  int64_t total_motions, total_points, total_tiles, total_cands, total_bins;
};

// What the culled pass needs of request r per item, in one 32-byte record.
struct BatchReq {
  int64_t sample_off;              // first (motion, sample) pair
  int point_off, motion_off;       // first sorted point; first global motion
  int n_points, T, nb;             // cloud size; samples; sample blocks
  int list_off;                    // first slot of the request's listed items
  int tile_off;                    // first tile of the request's sorted points
  int blen;                        // samples per sample block
};

// The culled batched kernel's blocks form tile.cull_gangs gangs (block index mod gangs;
// 8, the default, puts one gang on each XCD under the round-robin dispatch of workgroups
// to XCDs).  Each gang has a queue over the requests assigned to it; an idle gang takes
// items from the others.  Arrays are sized for kMaxGangs.
constexpr int kMaxGangs = 16;
// Sample-block divisors of the culled passes (a block spans about 1/div of a motion):
// the defaults, and the sets a launch shape may choose (sv_tile.cull_div_linear,
// cull_div_spline).
constexpr int kCullDivLinear = 32, kCullDivSpline = 64;
constexpr int kCullDivsLinear[3] = {16, 32, 64}, kCullDivsSpline[3] = {32, 64, 128};

// Workspace of a batch call: per-request arrays [max_requests] (offsets [+1]), keys
// [max_motions], capsule table [max_samples * K], band arrays [max_band].
struct BatchWs {
  unsigned long long* work;                       // [kWorkSlots] segment tests of the culled pass
  BatchPlan* plan;
  int64_t *motion_off, *sample_off, *item_off;   // request order; item_off in work order
  int64_t *n_motions, *n_samples, *n_items;
  int *order, *tiles, *chunks, *remaining;        // order: work position -> request
  unsigned long long* keys;
  CapEntry* table;
  int* band_list;                                 // global motion index
  unsigned long long* keys64;
  CapEntry64* table64;                            // [max_band][K][max_T]
  // culled pass (all requests' clouds sorted together by (request, Morton code))
  int64_t *n_points, *point_off, *tile_off, *n_cands, *cand_off;   // cand_off in work order
  unsigned* bounds;                               // [max_requests][6] per-request cloud bounds
  int* level;                                     // [max_requests] Morton cells per axis 2^level
  int64_t* bin_off;                               // [max_requests + 1] first bin of each request
  int *pbin, *pslot;                              // [point_cap] bin of each point, slot within it
  int *bin_count, *bin_start;                     // [bin_cap]
  int* group_sum;                                 // [bin_cap / 2048] counts of groups of bins
  int64_t* group_off;                             // their exclusive scan
  float *sx, *sy, *sz;                            // [point_cap] sorted points
  int* sidx;                                      // [point_cap] their index in the request's cloud
  float4* tile_sph;                               // [tile_cap]
  float4* wave_sph;                               // [tile_cap][4] the culled kernel's wave groups
  float4* spheres;                                // [max_motions][K][nb_max]
  float4* gspheres;                               // [max_motions][K][ng_max] group spheres (item filter)
  int *list_g, *list_tk;                          // [cand_cap] motion, tile << 4 | capsule
  BatchReq* req;                                  // [max_requests]
  int* fill;                                      // [max_requests] listed items per request
  int* gang_n;                                    // [kMaxGangs] requests per gang
  int* gang_total;                                // [kMaxGangs] items per gang
  unsigned* gang_head;                            // [kMaxGangs] queue heads
  int* gang_req;                                  // [kMaxGangs][max_requests] requests in gang order
  int* gang_off;                                  // [kMaxGangs][max_requests + 1] their first gang item
  int64_t point_cap, tile_cap, cand_cap, bin_cap;
  int nb_max, ng_max;
};

bool batch_tile_supported(const sv_tile& t);
sv_tile default_batch_tile();

// Carves ws (NULL: only sizes); *bytes = total.
BatchWs carve_batch(void* ws, const sv_robot& rb, const sv_batch_caps& caps, size_t* bytes);
hipError_t launch_batch(const sv_robot& rb, const sv_request* reqs, int n_req, const sv_batch_caps& caps, float eps,
                        float band, const sv_tile& tile, unsigned long long* done_ticks, int* status,
                        const BatchWs& w, hipStream_t st);

// ---- first collision-free motion (sv_search.hip) ----------------------------------
constexpr int kMaxSearchMotions = 4096;

struct SearchHdr {
  int answer;                    // earliest position found free outside the band (M: none yet)
  int n_run;                     // motions whose exact check completed
  int band_count;                // motions queued for the FP64 recheck
  int n_first;                   // first-loop motions (d_hat > eps)
  unsigned long long next_item;  // head of the work queue
};

// Workspace of a search over M motions: per-position / per-motion arrays [M] and the
// capsule table [M][K][T].
struct SearchWs {
  SearchHdr* hdr;
  int *order, *remaining;
  unsigned long long* keys;
  float* dist_pos;
  CapEntry* table;
  int *band_list, *band_pos;
  unsigned long long* keys64;
  float* d64;
  uint8_t* v64;
};

SearchWs carve_search(void* ws, const sv_robot& rb, int64_t M, int T, size_t* bytes);
hipError_t launch_search(const sv_robot& rb, const MotionArgs& mo, const CloudArgs& c, float eps, float band,
                         const float* d_hat, sv_search_result* result, int* order_out, const SearchWs& w,
                         hipStream_t st);
// d_hat[m] <- the float of min key keys[m] (+inf for the empty key ~0u).
hipError_t launch_decode_min(const unsigned* keys, int64_t M, float* d_hat, hipStream_t st);

// ---- culled per-motion minimum (sv_cull.hip) ----------------------------------------
// Workspace of the culled exact pass: cloud bounds and Morton sort, the sorted cloud
// (SoA) with its permutation to the caller's indices, radix-sort scratch, and one
// bounding sphere per (motion, capsule, block of samples).
// Counting sort of a cloud by Morton cell (both culled passes): 2^L cells per axis,
// at most kBinCellsPerPoint cells per point and kBinMaxLevel levels.
constexpr int kBinCellsPerPoint = 2;
constexpr int kBinMaxLevel = 7;
__host__ __device__ inline int morton_level(int64_t n) {
  int L = 0;
  while (L < kBinMaxLevel && ((int64_t)1 << (3 * (L + 1))) <= n * kBinCellsPerPoint) ++L;
  return L;
}
// Exclusive scan of count[0..n) into start[0..n) (n = *n_dev if n_dev, else n_host);
// group_sum [bin_scan_groups(cap)], group_off [bin_scan_groups(cap) + 1] for n <= cap.
int64_t bin_scan_groups(int64_t cap);
hipError_t launch_bin_scan(const int* count, int64_t n_host, const int64_t* n_dev, int64_t cap, int* group_sum,
                           int64_t* group_off, int* start, hipStream_t st);

struct CullWs {
  unsigned* bounds;                 // [6]
  int level;                        // Morton cells per axis 2^level (morton_level(N))
  int *pbin, *pslot;                // [N] cell of each point, slot within it
  int *bin_count, *bin_start;       // [8^level]
  int* group_sum;                   // [bin_scan_groups(8^level)]
  int64_t* group_off;               // [bin_scan_groups(8^level) + 1]
  int* perm;                        // [N] caller's index of each sorted point
  float *sx, *sy, *sz;              // [N] sorted points
  float4* spheres;                  // [M][K][cull_blocks(T)]
  float4* group_spheres;            // [M][K][cull_group_count(cull_blocks(T))]
  float4* tile_spheres;             // [cull_tiles(N)]
  float4* wave_spheres;             // [cull_tiles(N)][4] the culled kernel's wave groups
  int* list;                        // [M * cull_tiles(N) * K] surviving (motion slot, tile) items
  int* list_caps;                  // [M * cull_tiles(N) * K] the capsule each item checks
  int* list_count;                  // [2] listed items, queue head
  unsigned long long* work;         // [kWorkSlots] executed segment tests, summed (may be NULL)
};
constexpr int kWorkSlots = 256;
int cull_blocks(int T, int kind);
// Sample blocks per group sphere of the culled passes' item filter (item_may_hit).
constexpr int kGroupBlocks = 8;
__host__ __device__ constexpr int cull_group_count(int nb) { return (nb + kGroupBlocks - 1) / kGroupBlocks; }
int cull_tiles(int64_t N);
// Per-motion (distance, index) keys of the motion slots (mlist/mcount as launch_exact)
// over all points, with groups of tests that provably exceed the minimum skipped.
// keys must hold kKeyEmpty or a valid upper bound on entry.
hipError_t launch_exact_culled(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                               const int* mlist, const int* mcount, int64_t n_slots, unsigned long long* keys,
                               const CullWs& w, hipStream_t st);
// The two halves of launch_exact_culled: the Morton sort of the cloud into w (sx, sy, sz,
// perm) and the sample-block spheres of every motion; then the pass itself (seed bound,
// tile spheres, item list, culled kernel) over the motion slots, which needs the sort
// (reset: clear the item queue first, when the sort did not run just before).
hipError_t launch_cull_sort(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                            const CullWs& w, hipStream_t st);
hipError_t launch_cull_pass(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, const CloudArgs& c,
                            const int* mlist, const int* mcount, int64_t n_slots, unsigned long long* keys,
                            const CullWs& w, bool reset, hipStream_t st);
// Per-motion keys over the points a screen sent, plist[m N ..] (indices into the sorted
// cloud of w, pcount[m] per motion), with sample blocks skipped that the sphere test
// proves to lie above min(g0, the current key); needs launch_cull_sort.  Exact (the
// minimum over the sent points and its lowest caller index) whenever that minimum is
// <= g0; g0 = +inf makes it exact always.
hipError_t launch_fallback_culled(const sv_robot& rb, const CapEntry* table, const MotionArgs& mo, int N,
                                  const int* plist, const int* pcount, float g0, unsigned long long* keys,
                                  const CullWs& w, hipStream_t st);

// ---- launchers (sv_geom.hip) ------------------------------------------------------
// Paper-style training samples (Sec. IV-C): workspace arrays [M][n_uniform] (u*),
// [M][n_cand] (c*), [M][n_surface] (s*), [M][3 n_surface] (k*).
struct PaperSamplesWs {
  float *ux, *uy, *uz, *ud, *cx, *cy, *cz, *cd, *sx, *sy, *sz, *sd, *kx, *ky, *kz, *kd;
};
hipError_t launch_make_samples_paper(const sv_robot& rb, const MotionArgs& m, const CapEntry* table, float half,
                                     int nu, int ns, int nc, float sigma, const float* rnd, const PaperSamplesWs& w,
                                     float* out, int* n_acc, int* n_short, hipStream_t st);

// Per-motion gap between the sampled and the continuous swept distance, and (with
// min_dist) the continuous verdict.
hipError_t launch_motion_gap(const sv_robot& rb, const MotionArgs& m, const float* min_dist, float eps, float band,
                             float* gap, uint8_t* verdict, hipStream_t st);
hipError_t launch_fk_configs(const sv_robot& rb, const float* q, int64_t n, float* caps, int fp64,
                             hipStream_t st);
hipError_t launch_motion_table(const sv_robot& rb, const MotionArgs& m, CapEntry* table, hipStream_t st);
// Exact kernel.  Motion slots: mlist/mcount (device) select motions, else slot = motion.
// Points: plist/pcount (device, per motion: plist[m * N + j], j < pcount[m]) select
// points, else all N points.
hipError_t launch_exact(const sv_robot& rb, const CapEntry* table, const MotionArgs& m, const CloudArgs& c,
                        const int* mlist, const int* mcount, int64_t n_slots, const int* plist, const int* pcount,
                        float* sdf, unsigned long long* keys, ExactShape shape, hipStream_t st);
// Training rows (x, q0, q1, delta) for every motion: uniform points and near-surface
// candidates (SoA scratch u*, c*), labelled by the exact kernel, assembled into out.
hipError_t launch_make_samples(const sv_robot& rb, const MotionArgs& m, const CapEntry* table, float half, int nu,
                               int nn, int nc, float band, const float* rnd, float* ux, float* uy, float* uz,
                               float* ud, float* cx, float* cy, float* cz, float* cd, float* out, int* n_short,
                               hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_check_init(unsigned long long* keys, int64_t M, int* band_count, unsigned long long* work,
                             int n_work, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
// Decode FP32 keys into results for the motions in (mlist, mcount) (all M if mlist is
// NULL); motions within `band` of eps are appended to (list, count) for the FP64 recheck.
hipError_t launch_finalize(const unsigned long long* keys, int64_t M, const int* mlist, const int* mcount, float eps,
                           float band, sv_results out, int* list, int* count, hipStream_t st);
// Screening decision after the fallback check of the listed points: motions with a
// witness below eps - band are final collisions; in certified mode every other motion
// is appended to (full, full_count) with its key reset, for a check over all points;
// in trust mode every motion is final.
hipError_t launch_screen_decide(unsigned long long* keys, int64_t M, const int* pcount, float eps, float band,
                                int certified, sv_results out, int* full, int* full_count, hipStream_t st);
hipError_t launch_recheck64(const sv_robot& rb, const MotionArgs& m, const CloudArgs& c, const int* list,
                            const int* count, unsigned long long* keys64, float eps,
                            sv_results out, hipStream_t st);

ExactShape default_exact_shape();

// ---- network (sv_mlp.hip) --------------------------------------------------------
bool mlp_bf16_supported(int width);
constexpr int kTrainMaxWidth = 512;   // the training kernels take W = 128, 256, 512
size_t mlp_packed_elems(const MlpArgs& net);
hipError_t launch_mlp_f32(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, float* out, hipStream_t st);
// Hidden-layer weights (layers 2..L) to BF16 in MFMA A-operand order; transpose = 1
// packs W_l^T (the backward pass's operand).
hipError_t launch_pack_bf16(const MlpArgs& net, int transpose, __bf16* packed, hipStream_t st);
// W_l and W_l^T of the softplus network in one launch (training).
hipError_t launch_pack_bf16_both(const MlpArgs& net, __bf16* packed, __bf16* packedT, hipStream_t st);
// Network on n independent rows rows[i][0:in_dim] (row_stride floats apart); bf16
// selects the BF16 kernel (packed weights required) over the FP32 one.
hipError_t launch_mlp_rows(const MlpArgs& net, int bf16, const __bf16* packed, const float* rows, int64_t row_stride,
                           int64_t n, float* out, hipStream_t st);

// ---- training (sv_train.hip) -----------------------------------------------------
int64_t train_rows_padded(int64_t B);
size_t train_part_w_elems(const MlpArgs& n);
size_t train_part_w1_elems(const MlpArgs& n, int64_t Bp);
// Forward, loss, backward and gradient of one batch (rows idx[0..B) of samples);
// writes the flat FP32 gradient to grad and the batch loss to loss_out (optional).
hipError_t launch_train_step(const MlpArgs& net, const float* samples, const int* idx, int B, int Bp, __bf16* aT,
                             __bf16* dzT, float* h0T, float* y, float* dy, const __bf16* packed,
                             const __bf16* packedT, float* grad, float* part_w, float* part_w1, float sigma,
                             int clamp_pred, float* loss_out, hipStream_t st);
// Training of the residual network (SV_NET_RESIDUAL) with batch-statistic BatchNorm:
// buffers of one step (Bp rows; slabs of W x Bp values in the tiled layout of aT).
struct ResTrainWs {
  __bf16 *packed, *packedT;   // forward operands (mlp_packed_elems), Wh_b^T [L][W][W]
  float* xT;                  // [in_dim][Bp]
  __bf16 *hT, *aT, *dzT;      // [L], [L] and [L + 1] slabs
  float *g, *part, *stats, *bsum, *y, *dy, *pout;   // [slab], [Bp/64][2][W], [L][3][W], [2][W], [Bp], [Bp], [Bp/64][W+2]
  float *part_w, *part_w1;    // dW splits
};
size_t train_res_part_w_elems(const MlpArgs& n);
size_t train_res_part_w1_elems(const MlpArgs& n, int64_t Bp);
// Forward, loss, backward and gradient of one batch; grad[n_params] (running-statistic
// entries zero), loss_out (optional).  Leaves the batch statistics in w.stats.
hipError_t launch_train_step_res(const MlpArgs& net, const float* samples, const int* idx, int B, int Bp,
                                 const ResTrainWs& w, float sigma, float* grad, float* loss_out, hipStream_t st);
// Moves every block's running statistics in params towards the batch statistics of
// the last launch_train_step_res (momentum 0.1, unbiased variance).
hipError_t launch_bn_running(const MlpArgs& net, const ResTrainWs& w, int B, float* params, hipStream_t st);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t st);

// Per-motion minimum of the BF16 prediction over the cloud, folded into min_keys[m]
// (order-preserving unsigned keys of the float; the caller fills them with ~0u first).
hipError_t launch_mlp_min(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const __bf16* packed,
                          unsigned* min_keys, hipStream_t st);

// out (optional): [M][N] predictions.  lists/counts (optional): per motion, the points
// with prediction < tau are appended to lists[m * N ...] and counted in counts[m].
hipError_t launch_mlp_bf16(const MlpArgs& net, const MotionArgs& mo, const CloudArgs& c, const __bf16* packed,
                           float* out, float tau, int* lists, int* counts, hipStream_t st);

}  // namespace sv
