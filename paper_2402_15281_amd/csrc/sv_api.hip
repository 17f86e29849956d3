// C ABI of libsv: argument validation, workspace carving and kernel dispatch.
// The entry points and their contracts are declared and documented in sv.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sv_internal.h"
#include "sv_mlp_common.h"

namespace sv {
namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(SV_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// ---- optional per-kernel timing with HIP events (sv_profile_*), per calling thread:
// a thread's switch, pending events and totals are its own, so no call from another
// thread sees them and no lock is needed.
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
thread_local bool t_prof_on = false;
thread_local bool t_prof_suspended = false;   // within a call that may not create events
thread_local std::vector<ProfRec> t_prof_pending;
thread_local std::map<std::string, std::pair<double, int64_t>> t_prof_acc;

// Records a HIP event pair around the launches in its scope, on the launch stream.
struct ProfScope {
  ProfRec rec{nullptr, nullptr, nullptr};
  hipStream_t st;
  ProfScope(const char* name, hipStream_t s) : st(s) {
    if (!t_prof_on || t_prof_suspended) return;
    if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess) return;
    rec.name = name;
    (void)hipEventRecord(rec.a, st);
  }
  ~ProfScope() {
    if (!rec.name) return;
    (void)hipEventRecord(rec.b, st);
    t_prof_pending.push_back(rec);
  }
};

void prof_resolve() {
  for (auto& r : t_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& acc = t_prof_acc[r.name];
      acc.first += ms;
      acc.second += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  t_prof_pending.clear();
}


int check_robot(const sv_robot* r) {
  if (!r) return fail(SV_ERR_ARG, "robot is NULL");
  if (r->dof < 1 || r->dof > SV_MAX_DOF) return fail(SV_ERR_ARG, "robot dof %d outside 1..%d", r->dof, SV_MAX_DOF);
  if (r->n_caps < 1 || r->n_caps > SV_MAX_CAPS)
    return fail(SV_ERR_ARG, "robot n_caps %d outside 1..%d", r->n_caps, SV_MAX_CAPS);
  for (int k = 0; k < r->n_caps; ++k) {
    for (int e = 0; e < 2; ++e)
      if (r->cap_frame[k][e] < 0 || r->cap_frame[k][e] > r->dof)
        return fail(SV_ERR_ARG, "capsule %d endpoint %d frame %d outside 0..%d", k, e, r->cap_frame[k][e], r->dof);
    if (!(r->cap_r[k] >= 0.0) || !isfinite(r->cap_r[k]))
      return fail(SV_ERR_ARG, "capsule %d radius must be finite and >= 0", k);
  }
  return SV_OK;
}

int check_motions(const sv_motions* m, int dof) {
  if (!m) return fail(SV_ERR_ARG, "motions is NULL");
  if (m->kind != SV_LINEAR && m->kind != SV_SPLINE) return fail(SV_ERR_ARG, "unknown motion kind %d", m->kind);
  if (m->T < 1) return fail(SV_ERR_ARG, "T = %d, need T >= 1", m->T);
  if (m->n < 0) return fail(SV_ERR_SHAPE, "negative motion count");
  if (m->n > 0 && (!m->q0 || !m->q1)) return fail(SV_ERR_ARG, "motion q0/q1 is NULL");
  if (m->n > 0 && m->kind == SV_SPLINE && !m->via) return fail(SV_ERR_ARG, "spline motions need via points");
  if (m->n > (int64_t)0x7fffffff / 2) return fail(SV_ERR_SHAPE, "too many motions");
  (void)dof;
  return SV_OK;
}

int check_cloud(const sv_cloud* c) {
  if (!c) return fail(SV_ERR_ARG, "cloud is NULL");
  if (c->n < 0 || c->n > 0x7fffffffLL) return fail(SV_ERR_SHAPE, "cloud size %lld outside 0..2^31-1", (long long)c->n);
  if (c->n > 0 && (!c->x || !c->y || !c->z)) return fail(SV_ERR_ARG, "cloud coordinate pointer is NULL");
  return SV_OK;
}

MotionArgs to_args(const sv_motions& m) {
  return MotionArgs{m.kind, m.T, m.n, m.q0, m.q1, m.kind == SV_SPLINE ? m.via : nullptr};
}
CloudArgs to_args(const sv_cloud& c) { return CloudArgs{(int)c.n, c.x, c.y, c.z}; }

int check_mlp(const sv_mlp* n, int precision, int dof) {
  if (!n) return fail(SV_ERR_ARG, "mlp is NULL");
  if (!n->params) return fail(SV_ERR_ARG, "mlp params is NULL");
  if (n->in_dim < 5 || (n->in_dim - 3) % 2 != 0 || (n->in_dim - 3) / 2 > SV_MAX_DOF)
    return fail(SV_ERR_ARG, "mlp in_dim %d is not 3 + 2*dof", n->in_dim);
  if (dof > 0 && n->in_dim != 3 + 2 * dof)
    return fail(SV_ERR_SHAPE, "mlp in_dim %d does not match robot dof %d", n->in_dim, dof);
  if (n->n_hidden < 1) return fail(SV_ERR_ARG, "mlp n_hidden %d < 1", n->n_hidden);
  if (n->kind != SV_NET_MLP && n->kind != SV_NET_RESIDUAL) return fail(SV_ERR_ARG, "unknown network kind %d", n->kind);
  if (n->kind == SV_NET_RESIDUAL && !(n->bn_eps > 0.f)) return fail(SV_ERR_ARG, "bn_eps must be > 0");
  if (n->kind == SV_NET_RESIDUAL && precision == SV_BF16 && n->in_dim > kResMaxIn)
    return fail(SV_ERR_UNSUPPORTED, "BF16 residual network: in_dim %d > %d", n->in_dim, kResMaxIn);
  if (precision == SV_FP32) {
    if (n->width < 64 || n->width > 1024 || n->width % 64)
      return fail(SV_ERR_UNSUPPORTED, "FP32 network width %d: need a multiple of 64 up to 1024", n->width);
  } else if (precision == SV_BF16) {
    if (!mlp_bf16_supported(n->width))
      return fail(SV_ERR_UNSUPPORTED, "BF16 network width %d: need 128, 256, 512 or 1024", n->width);
  } else {
    return fail(SV_ERR_ARG, "unknown precision %d", precision);
  }
  return SV_OK;
}

MlpArgs to_args(const sv_mlp& n) {
  return MlpArgs{n.in_dim, n.width, n.n_hidden, (n.in_dim - 3) / 2, n.params, n.kind, n.bn_eps};
}

// Workspace layout of sv_check_motions.  The screening arrays are empty without a network.
struct CheckWs {
  unsigned long long* work;   // first 8 bytes: segment tests of the culled exact pass
  CullWs cull;
  CapEntry* table;
  unsigned long long* keys;
  int* band;          // motions in the certified band (FP64 recheck)
  int* band_count;
  unsigned long long* keys64;
  __bf16* packed;     // BF16 hidden-layer weights
  int* plist;         // [M][N] points sent to the exact check
  int* pcount;        // [M]
  int* full;          // motions without a witness (certified mode)
  int* full_count;
  size_t bytes;
};

CheckWs carve_check(void* ws, const sv_robot& r, const sv_motions& m, const sv_cloud& c, const sv_mlp* mlp) {
  Carver cv(ws);
  CheckWs w{};
  const size_t entries = (size_t)m.n * r.n_caps * m.T;
  w.work = cv.take<unsigned long long>(kWorkSlots);
  const size_t N = (size_t)c.n;
  w.cull.bounds = cv.take<unsigned>(8);
  w.cull.level = morton_level(N);
  const size_t bins = (size_t)1 << (3 * w.cull.level);
  w.cull.pbin = cv.take<int>(N);
  w.cull.pslot = cv.take<int>(N);
  w.cull.bin_count = cv.take<int>(bins);
  w.cull.bin_start = cv.take<int>(bins);
  w.cull.group_sum = cv.take<int>((size_t)bin_scan_groups((int64_t)bins));
  w.cull.group_off = cv.take<int64_t>((size_t)bin_scan_groups((int64_t)bins) + 1);
  w.cull.perm = cv.take<int>(N);
  w.cull.sx = cv.take<float>(N);
  w.cull.sy = cv.take<float>(N);
  w.cull.sz = cv.take<float>(N);
  w.cull.spheres = cv.take<float4>((size_t)m.n * r.n_caps * cull_blocks(m.T, m.kind));
  w.cull.group_spheres = cv.take<float4>((size_t)m.n * r.n_caps * cull_group_count(cull_blocks(m.T, m.kind)));
  w.cull.tile_spheres = cv.take<float4>((size_t)cull_tiles(c.n));
  w.cull.wave_spheres = cv.take<float4>((size_t)cull_tiles(c.n) * 4);
  w.cull.list = cv.take<int>((size_t)m.n * cull_tiles(c.n) * r.n_caps);
  w.cull.list_caps = cv.take<int>((size_t)m.n * cull_tiles(c.n) * r.n_caps);
  w.cull.list_count = cv.take<int>(2);
  w.cull.work = w.work;
  w.table = cv.take<CapEntry>(entries);
  w.keys = cv.take<unsigned long long>(m.n);
  w.band = cv.take<int>(m.n);
  w.band_count = cv.take<int>(1);
  w.keys64 = cv.take<unsigned long long>(m.n);
  if (mlp) {
    w.packed = cv.take<__bf16>(mlp_packed_elems(to_args(*mlp)));
    w.plist = cv.take<int>((size_t)m.n * c.n);
    w.pcount = cv.take<int>(m.n);
    w.full = cv.take<int>(m.n);
    w.full_count = cv.take<int>(1);
  }
  w.bytes = cv.off;
  return w;
}

size_t exact_sdf_bytes(const sv_robot& r, const sv_motions& m) {
  Carver c(nullptr);
  c.take<CapEntry>((size_t)m.n * r.n_caps * m.T);
  return c.off;
}

size_t nn_sdf_bytes(const sv_mlp& n, int precision) {
  if (precision == SV_FP32) return 0;
  Carver c(nullptr);
  c.take<__bf16>(mlp_packed_elems(to_args(n)));
  return c.off;
}

// Motions whose FP32 cloud distance lies within this band of eps are recomputed in FP64.
constexpr float kCertBand = 1e-5f;

int check_caps(const sv_batch_caps* c) {
  if (!c) return fail(SV_ERR_ARG, "caps is NULL");
  if (c->max_requests < 1 || c->max_requests > kMaxBatchRequests)
    return fail(SV_ERR_ARG, "caps.max_requests %d outside 1..%d", c->max_requests, kMaxBatchRequests);
  if (c->max_T < 1) return fail(SV_ERR_ARG, "caps.max_T must be >= 1");
  if (c->max_motions < 1 || c->max_motions > 0x7fffffffLL)
    return fail(SV_ERR_ARG, "caps.max_motions outside 1..2^31-1");
  if (c->max_samples < 1) return fail(SV_ERR_ARG, "caps.max_samples must be >= 1");
  if (c->max_points < 0 || c->max_points > 0x7fffffffLL) return fail(SV_ERR_ARG, "caps.max_points outside 0..2^31-1");
  if (c->max_band < 1 || c->max_band > (1 << 20)) return fail(SV_ERR_ARG, "caps.max_band outside 1..2^20");
  if (c->max_total_points < 0) return fail(SV_ERR_ARG, "caps.max_total_points is negative");
  const int64_t pts = c->max_total_points > 0 ? c->max_total_points : (int64_t)c->max_requests * c->max_points;
  if (pts >= (1LL << 30))
    return fail(SV_ERR_ARG, "total points (caps.max_total_points, or max_requests * max_points when 0) must be "
                            "below 2^30");
  if (c->max_motions * ((c->max_points + 511) / 512) * SV_MAX_CAPS > 0x7fffffffLL)
    return fail(SV_ERR_ARG, "caps.max_motions * ceil(caps.max_points / 512) * 16 exceeds 2^31-1");
  return SV_OK;
}

// The launch shapes offered to an autotuner (all accepted by sv_check_requests): the
// unculled shapes, then the culled ones, each with the other pass's fields at their
// defaults.
std::vector<sv_tile> tile_candidates() {
  const sv_tile d = default_batch_tile();
  std::vector<sv_tile> v;
  for (int ppl : {1, 2, 4})
    for (int threads : {64, 128, 256})
      for (int bpc : {1, 2, 4, 8, 16, 32})
        for (int tpi : {1, 2, 4, 8, 16, 32}) {
          sv_tile t = d;
          t.ppl = ppl;
          t.threads = threads;
          t.blocks_per_cu = bpc;
          t.tiles_per_item = tpi;
          t.cull = 0;
          v.push_back(t);
        }
  for (int bpc : {1, 2, 4, 0})
    for (int gangs : {1, 2, 4, 8, 16})
      for (int dl : kCullDivsLinear)
        for (int ds : kCullDivsSpline) {
          sv_tile t = d;
          t.cull_blocks_per_cu = bpc;
          t.cull_gangs = gangs;
          t.cull_div_linear = dl;
          t.cull_div_spline = ds;
          v.push_back(t);
        }
  return v;
}

}  // namespace
}  // namespace sv

// Scratch memory of sv_check_motions_static: one copy on every GPU the library runs on,
// held until the process ends.  Host code never uses this name for the memory (on the
// host it is only a stand-in): it takes the device address that hipGetSymbolAddress
// returns for the current device, once per device (static_scratch).
static __device__ __align__(256) unsigned char scratch[SV_STATIC_SCRATCH_BYTES];

namespace sv {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, resolved on the first call
// with that device current and kept.
int static_scratch(void** p) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SV_ERR_UNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SV_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *p = g_scratch_ptr[dev];
  return SV_OK;
}

// Suspends the thread's profiler for the scope (it would create HIP events).
struct ProfSuspend {
  bool was;
  ProfSuspend() : was(t_prof_suspended) { t_prof_suspended = true; }
  ~ProfSuspend() { t_prof_suspended = was; }
};

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

const char* sv_status_string(int s) {
  switch (s) {
    case SV_OK: return "ok";
    case SV_ERR_ARG: return "invalid argument";
    case SV_ERR_SHAPE: return "inconsistent shape";
    case SV_ERR_WORKSPACE: return "workspace missing or too small";
    case SV_ERR_UNSUPPORTED: return "unsupported request";
    case SV_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* sv_last_error(void) { return g_last_error.c_str(); }

int sv_profile_enable(int on) {
  t_prof_on = on != 0;
  return SV_OK;
}

void sv_profile_reset(void) {
  prof_resolve();
  t_prof_acc.clear();
}

int sv_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return fail(SV_ERR_ARG, "NULL argument");
  prof_resolve();
  auto it = t_prof_acc.find(kernel);
  *total_ms = it == t_prof_acc.end() ? 0.0 : it->second.first;
  *launches = it == t_prof_acc.end() ? 0 : it->second.second;
  return SV_OK;
}

int sv_workspace_size(int op, const sv_robot* robot, const sv_mlp* mlp, int precision, const sv_motions* motions,
                      const sv_cloud* cloud, size_t* bytes) {
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  int s;
  if (op == SV_OP_NN_SDF) {
    if ((s = check_mlp(mlp, precision, 0)) || (s = check_motions(motions, 0)) || (s = check_cloud(cloud))) return s;
    *bytes = nn_sdf_bytes(*mlp, precision);
    return SV_OK;
  }
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) || (s = check_cloud(cloud))) return s;
  switch (op) {
    case SV_OP_EXACT_SDF: *bytes = exact_sdf_bytes(*robot, *motions); return SV_OK;
    case SV_OP_CHECK:
      if (mlp && (s = check_mlp(mlp, SV_BF16, robot->dof))) return s;
      *bytes = carve_check(nullptr, *robot, *motions, *cloud, mlp).bytes;
      return SV_OK;
    default: return fail(SV_ERR_ARG, "unknown workspace op %d", op);
  }
}

int sv_continuous_gap(const sv_robot* robot, const sv_motions* motions, const float* min_dist, float eps, float* gap,
                      uint8_t* verdict, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof))) return s;
  if (motions->n == 0) return SV_OK;
  if (!gap) return fail(SV_ERR_ARG, "gap is NULL");
  if (!verdict != !min_dist) return fail(SV_ERR_ARG, "verdict and min_dist go together");
  if (isnan(eps)) return fail(SV_ERR_ARG, "eps is NaN");
  hipStream_t st = (hipStream_t)stream;
  ProfScope ps("motion_gap", st);
  const hipError_t e = launch_motion_gap(*robot, to_args(*motions), min_dist, eps, kCertBand, gap, verdict, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "continuous gap");
}

int sv_fk(const sv_robot* robot, const float* q, int64_t n_cfg, float* caps, int fp64, void* stream) {
  int s;
  if ((s = check_robot(robot))) return s;
  if (n_cfg < 0) return fail(SV_ERR_SHAPE, "negative configuration count");
  if (n_cfg > 0 && (!q || !caps)) return fail(SV_ERR_ARG, "q or caps is NULL");
  hipError_t e = launch_fk_configs(*robot, q, n_cfg, caps, fp64 ? 1 : 0, (hipStream_t)stream);
  return e == hipSuccess ? SV_OK : hip_fail(e, "sv_fk");
}

int sv_exact_sdf(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud, float* sdf, void* ws,
                 size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) || (s = check_cloud(cloud))) return s;
  if (motions->n == 0 || cloud->n == 0) return SV_OK;
  if (!sdf) return fail(SV_ERR_ARG, "sdf is NULL");
  const size_t need = exact_sdf_bytes(*robot, *motions);
  if (!ws || ws_bytes < need) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  hipStream_t st = (hipStream_t)stream;
  CapEntry* table = static_cast<CapEntry*>(ws);
  const MotionArgs ma = to_args(*motions);
  hipError_t e;
  {
    ProfScope ps("motion_table", st);
    e = launch_motion_table(*robot, ma, table, st);
  }
  if (e != hipSuccess) return hip_fail(e, "motion table");
  ProfScope ps("exact_sdf", st);
  e = launch_exact(*robot, table, ma, to_args(*cloud), nullptr, nullptr, motions->n, nullptr, nullptr, sdf, nullptr,
                   default_exact_shape(), st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "exact kernel");
}

int sv_nn_sdf(const sv_mlp* mlp, int precision, const sv_motions* motions, const sv_cloud* cloud, float* sdf_hat,
              void* ws, size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_mlp(mlp, precision, 0)) || (s = check_motions(motions, 0)) || (s = check_cloud(cloud))) return s;
  if (motions->kind != SV_LINEAR) return fail(SV_ERR_UNSUPPORTED, "the network applies to linear motions only");
  if (motions->n == 0 || cloud->n == 0) return SV_OK;
  if (!sdf_hat) return fail(SV_ERR_ARG, "sdf_hat is NULL");
  const size_t need = nn_sdf_bytes(*mlp, precision);
  if (need && (!ws || ws_bytes < need))
    return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  hipStream_t st = (hipStream_t)stream;
  const MlpArgs na = to_args(*mlp);
  hipError_t e;
  if (precision == SV_FP32) {
    ProfScope ps("mlp_f32", st);
    e = launch_mlp_f32(na, to_args(*motions), to_args(*cloud), sdf_hat, st);
    return e == hipSuccess ? SV_OK : hip_fail(e, "FP32 network");
  }
  __bf16* packed = static_cast<__bf16*>(ws);
  {
    ProfScope ps("pack_bf16", st);
    e = launch_pack_bf16(na, 0, packed, st);
  }
  if (e != hipSuccess) return hip_fail(e, "pack weights");
  ProfScope ps("mlp_bf16", st);
  e = launch_mlp_bf16(na, to_args(*motions), to_args(*cloud), packed, sdf_hat, 0.f, nullptr, nullptr, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "BF16 network");
}

int sv_check_motions(const sv_robot* robot, const sv_mlp* mlp, int screen, float eps, float tau,
                     const sv_motions* motions, const sv_cloud* cloud, sv_results* out, void* ws, size_t ws_bytes,
                     void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) || (s = check_cloud(cloud))) return s;
  if (!out) return fail(SV_ERR_ARG, "results is NULL");
  if (!isfinite(eps)) return fail(SV_ERR_ARG, "eps must be finite");
  const bool cull = (screen & SV_CHECK_UNCULLED) == 0;
  screen &= ~SV_CHECK_UNCULLED;
  const bool screened = screen != SV_SCREEN_NONE;
  if (screen < SV_SCREEN_NONE || screen > SV_SCREEN_CERTIFIED) return fail(SV_ERR_ARG, "unknown screen mode %d", screen);
  if (screened != (mlp != nullptr)) return fail(SV_ERR_ARG, "a screen mode needs a network and a network a screen mode");
  if (screened) {
    if ((s = check_mlp(mlp, SV_BF16, robot->dof))) return s;
    if (motions->kind != SV_LINEAR) return fail(SV_ERR_UNSUPPORTED, "the network applies to linear motions only");
    if (isnan(tau)) return fail(SV_ERR_ARG, "tau is NaN");
  }
  if (motions->n == 0) return SV_OK;
  const CheckWs w0 = carve_check(nullptr, *robot, *motions, *cloud, mlp);
  if (!ws || ws_bytes < w0.bytes)
    return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w0.bytes, ws_bytes);
  const CheckWs w = carve_check(ws, *robot, *motions, *cloud, mlp);
  hipStream_t st = (hipStream_t)stream;
  const MotionArgs ma = to_args(*motions);
  const CloudArgs ca = to_args(*cloud);
  const int64_t M = motions->n;
  const ExactShape shape = default_exact_shape();
  hipError_t e;
#define SV_TRY(name, call)                    \
  do {                                        \
    {                                         \
      ProfScope ps_(name, st);                \
      e = (call);                             \
    }                                         \
    if (e != hipSuccess) return hip_fail(e, name); \
  } while (0)

  SV_TRY("init", launch_check_init(w.keys, M, w.band_count, w.work, kWorkSlots, st));
  const int* mlist = nullptr;
  const int* mcount = nullptr;
  if (cloud->n > 0) {
    SV_TRY("motion_table", launch_motion_table(*robot, ma, w.table, st));
    if (!screened) {
      if (cull) {
        SV_TRY("exact", launch_exact_culled(*robot, w.table, ma, ca, nullptr, nullptr, M, w.keys, w.cull, st));
      } else {
        SV_TRY("exact", launch_exact(*robot, w.table, ma, ca, nullptr, nullptr, M, nullptr, nullptr, nullptr, w.keys,
                                     shape, st));
      }
    } else {
      const MlpArgs na = to_args(*mlp);
      const bool certified = screen == SV_SCREEN_CERTIFIED;
      SV_TRY("init", launch_fill_i32(w.pcount, M, 0, st));
      SV_TRY("init", launch_fill_i32(w.full_count, 1, 0, st));
      SV_TRY("pack_bf16", launch_pack_bf16(na, 0, w.packed, st));
      if (cull) {
        // Screen the Morton-sorted cloud (a prediction does not depend on the order), so
        // that the points sent per motion come in sorted order and the culled check of
        // them bounds each wave's points by a small sphere.  Certified screening only
        // asks whether a sent point lies within eps - band: groups provably above that
        // are skipped from the start.
        SV_TRY("sort", launch_cull_sort(*robot, w.table, ma, ca, w.cull, st));
        CloudArgs sorted = ca;
        sorted.x = w.cull.sx;
        sorted.y = w.cull.sy;
        sorted.z = w.cull.sz;
        SV_TRY("screen", launch_mlp_bf16(na, ma, sorted, w.packed, nullptr, tau, w.plist, w.pcount, st));
        SV_TRY("fallback", launch_fallback_culled(*robot, w.table, ma, cloud->n, w.plist, w.pcount,
                                                  certified ? eps - kCertBand : INFINITY, w.keys, w.cull, st));
      } else {
        SV_TRY("screen", launch_mlp_bf16(na, ma, ca, w.packed, nullptr, tau, w.plist, w.pcount, st));
        SV_TRY("fallback", launch_exact(*robot, w.table, ma, ca, nullptr, nullptr, M, w.plist, w.pcount, nullptr,
                                        w.keys, shape, st));
      }
      SV_TRY("decide", launch_screen_decide(w.keys, M, w.pcount, eps, kCertBand, certified, *out, w.full,
                                            w.full_count, st));
      if (certified) {
        if (cull) {
          SV_TRY("confirm", launch_cull_pass(*robot, w.table, ma, ca, w.full, w.full_count, M, w.keys, w.cull, true,
                                             st));
        } else {
          SV_TRY("confirm", launch_exact(*robot, w.table, ma, ca, w.full, w.full_count, M, nullptr, nullptr, nullptr,
                                         w.keys, shape, st));
        }
        mlist = w.full;
        mcount = w.full_count;
      }
    }
  } else if (screened) {
    SV_TRY("init", launch_fill_i32(w.pcount, M, 0, st));
    SV_TRY("init", launch_fill_i32(w.full_count, 1, 0, st));
    SV_TRY("decide", launch_screen_decide(w.keys, M, w.pcount, eps, kCertBand, screen == SV_SCREEN_CERTIFIED, *out,
                                          w.full, w.full_count, st));
    if (screen == SV_SCREEN_CERTIFIED) {
      mlist = w.full;
      mcount = w.full_count;
    }
  }
  SV_TRY("finalize", launch_finalize(w.keys, M, mlist, mcount, eps, kCertBand, *out, w.band, w.band_count, st));
  SV_TRY("recheck64", launch_recheck64(*robot, ma, ca, w.band, w.band_count, w.keys64, eps, *out, st));
#undef SV_TRY
  return SV_OK;
}

int sv_check_motions_static(const sv_robot* robot, const sv_mlp* mlp, int screen, float eps, float tau,
                            const sv_motions* motions, const sv_cloud* cloud, sv_results* out, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) || (s = check_cloud(cloud))) return s;
  const bool screened = (screen & ~SV_CHECK_UNCULLED) != SV_SCREEN_NONE;
  if (screened && mlp && (s = check_mlp(mlp, SV_BF16, robot->dof))) return s;
  const size_t need = carve_check(nullptr, *robot, *motions, *cloud, screened ? mlp : nullptr).bytes;
  if (need > SV_STATIC_SCRATCH_BYTES)
    return fail(SV_ERR_WORKSPACE, "this check needs %zu bytes of scratch; the static scratch holds %zu", need,
                (size_t)SV_STATIC_SCRATCH_BYTES);
  void* ptr = nullptr;
  if ((s = static_scratch(&ptr))) return s;
  ProfSuspend no_events;
  return sv_check_motions(robot, mlp, screen, eps, tau, motions, cloud, out, ptr, SV_STATIC_SCRATCH_BYTES, stream);
}

// ---- training data, row prediction, training step --------------------------------

namespace {
struct SamplesWs {
  CapEntry* table;
  float *ux, *uy, *uz, *ud, *cx, *cy, *cz, *cd;
  size_t bytes;
};
SamplesWs carve_samples(void* ws, const sv_robot& r, const sv_motions& m, int nu, int nc) {
  Carver cv(ws);
  SamplesWs w{};
  w.table = cv.take<CapEntry>((size_t)m.n * r.n_caps * m.T);
  const size_t U = (size_t)m.n * nu, C = (size_t)m.n * nc;
  w.ux = cv.take<float>(U);
  w.uy = cv.take<float>(U);
  w.uz = cv.take<float>(U);
  w.ud = cv.take<float>(U);
  w.cx = cv.take<float>(C);
  w.cy = cv.take<float>(C);
  w.cz = cv.take<float>(C);
  w.cd = cv.take<float>(C);
  w.bytes = cv.off;
  return w;
}

struct TrainWs {
  __bf16 *packed, *packedT, *aT, *dzT;
  float *h0T, *y, *dy, *grad, *part_w, *part_w1;
  size_t bytes;
};
size_t n_params(const sv_mlp& n) {
  const size_t W = n.width;
  if (n.kind == SV_NET_RESIDUAL) return res_block_base(n.width, n.in_dim, n.n_hidden) + W + 1;
  return W * n.in_dim + W + (size_t)(n.n_hidden - 1) * (W * W + W) + W + 1;
}
struct TrainResWs {
  ResTrainWs r;
  float* grad;
  size_t bytes;
};
TrainResWs carve_train_res(void* ws, const sv_mlp& mlp, int64_t B) {
  const MlpArgs na = to_args(mlp);
  const int64_t Bp = train_rows_padded(B);
  const size_t W = mlp.width, L = mlp.n_hidden, slab = W * (size_t)Bp, tiles = (size_t)Bp / 64;
  Carver cv(ws);
  TrainResWs w{};
  w.r.packed = cv.take<__bf16>(mlp_packed_elems(na));
  w.r.packedT = cv.take<__bf16>(L * W * W);
  w.r.xT = cv.take<float>((size_t)mlp.in_dim * Bp);
  w.r.hT = cv.take<__bf16>(L * slab);
  w.r.aT = cv.take<__bf16>(L * slab);
  w.r.dzT = cv.take<__bf16>((L + 1) * slab);
  w.r.g = cv.take<float>(slab);
  w.r.part = cv.take<float>(tiles * 2 * W);
  w.r.stats = cv.take<float>(L * 3 * W);
  w.r.bsum = cv.take<float>(2 * W);
  w.r.y = cv.take<float>(Bp);
  w.r.dy = cv.take<float>(Bp);
  w.r.pout = cv.take<float>(tiles * (W + 2));
  w.r.part_w = cv.take<float>(train_res_part_w_elems(na));
  w.r.part_w1 = cv.take<float>(train_res_part_w1_elems(na, Bp));
  w.grad = cv.take<float>(n_params(mlp));
  w.bytes = cv.off;
  return w;
}
TrainWs carve_train(void* ws, const sv_mlp& mlp, int64_t B) {
  const MlpArgs na = to_args(mlp);
  const int64_t Bp = train_rows_padded(B);
  const size_t W = mlp.width, L = mlp.n_hidden;
  Carver cv(ws);
  TrainWs w{};
  w.packed = cv.take<__bf16>(mlp_packed_elems(na));
  w.packedT = cv.take<__bf16>(mlp_packed_elems(na));
  w.aT = cv.take<__bf16>(L * W * Bp);
  w.dzT = cv.take<__bf16>(L * W * Bp);
  w.h0T = cv.take<float>((size_t)mlp.in_dim * Bp);
  w.y = cv.take<float>(Bp);
  w.dy = cv.take<float>(Bp);
  w.grad = cv.take<float>(n_params(mlp));
  w.part_w = cv.take<float>(train_part_w_elems(na));
  w.part_w1 = cv.take<float>(train_part_w1_elems(na, Bp));
  w.bytes = cv.off;
  return w;
}
size_t train_bytes(const sv_mlp& mlp, int64_t B) {
  return mlp.kind == SV_NET_RESIDUAL ? carve_train_res(nullptr, mlp, B).bytes : carve_train(nullptr, mlp, B).bytes;
}
}  // namespace

int sv_make_samples_workspace_size(const sv_robot* robot, const sv_motions* motions, int32_t n_uniform,
                                   int32_t n_cand, size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof))) return s;
  if (n_uniform < 0 || n_cand < 0) return fail(SV_ERR_ARG, "negative sample counts");
  *bytes = carve_samples(nullptr, *robot, *motions, n_uniform, n_cand).bytes;
  return SV_OK;
}

int sv_make_samples(const sv_robot* robot, const sv_motions* motions, float cube_half, int32_t n_uniform,
                    int32_t n_near, int32_t n_cand, float band, const float* rnd, float* out, int32_t* n_short,
                    void* ws, size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof))) return s;
  if (motions->kind != SV_LINEAR) return fail(SV_ERR_UNSUPPORTED, "training samples are drawn for linear motions");
  if (n_uniform < 0 || n_near < 0 || n_cand < n_near)
    return fail(SV_ERR_ARG, "need n_uniform >= 0, n_near >= 0 and n_cand >= n_near");
  if (!(cube_half > 0.f) || !(band >= 0.f)) return fail(SV_ERR_ARG, "cube_half must be > 0 and band >= 0");
  if (motions->n * (int64_t)std::max(n_uniform, n_cand) > 0x7fffffffLL)
    return fail(SV_ERR_SHAPE, "too many points for one call; split the motions");
  if (motions->n == 0 || (n_uniform == 0 && n_near == 0)) return SV_OK;
  if (!rnd || !out) return fail(SV_ERR_ARG, "rnd or out is NULL");
  const SamplesWs w0 = carve_samples(nullptr, *robot, *motions, n_uniform, n_cand);
  if (!ws || ws_bytes < w0.bytes) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w0.bytes, ws_bytes);
  const SamplesWs w = carve_samples(ws, *robot, *motions, n_uniform, n_cand);
  hipStream_t st = (hipStream_t)stream;
  const MotionArgs ma = to_args(*motions);
  hipError_t e;
  {
    ProfScope ps("motion_table", st);
    e = launch_motion_table(*robot, ma, w.table, st);
  }
  if (e != hipSuccess) return hip_fail(e, "motion table");
  ProfScope ps("make_samples", st);
  e = launch_make_samples(*robot, ma, w.table, cube_half, n_uniform, n_near, n_cand, band, rnd, w.ux, w.uy, w.uz, w.ud,
                          w.cx, w.cy, w.cz, w.cd, out, n_short, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "make samples");
}

struct PaperWs {
  CapEntry* table;
  PaperSamplesWs a;
  size_t bytes;
};
PaperWs carve_paper(void* ws, const sv_robot& r, const sv_motions& m, int nu, int ns, int nc) {
  Carver cv(ws);
  PaperWs w{};
  w.table = cv.take<CapEntry>((size_t)m.n * r.n_caps * m.T);
  const size_t U = (size_t)m.n * nu, C = (size_t)m.n * nc, S = (size_t)m.n * ns;
  float** arrays[16] = {&w.a.ux, &w.a.uy, &w.a.uz, &w.a.ud, &w.a.cx, &w.a.cy, &w.a.cz, &w.a.cd,
                        &w.a.sx, &w.a.sy, &w.a.sz, &w.a.sd, &w.a.kx, &w.a.ky, &w.a.kz, &w.a.kd};
  const size_t sizes[4] = {U, C, S, 3 * S};
  for (int i = 0; i < 16; ++i) *arrays[i] = cv.take<float>(sizes[i / 4]);
  w.bytes = cv.off;
  return w;
}

int check_paper_counts(const sv_motions* m, int32_t nu, int32_t ns, int32_t nc) {
  if (nu < 0 || ns < 0 || nc < ns) return fail(SV_ERR_ARG, "need n_uniform >= 0, n_surface >= 0, n_cand >= n_surface");
  if (m->n * (int64_t)std::max(std::max(nu, nc), 3 * ns) > 0x7fffffffLL)
    return fail(SV_ERR_SHAPE, "too many points for one call; split the motions");
  return SV_OK;
}

int sv_make_samples_paper_workspace_size(const sv_robot* robot, const sv_motions* motions, int32_t n_uniform,
                                         int32_t n_surface, int32_t n_cand, size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) ||
      (s = check_paper_counts(motions, n_uniform, n_surface, n_cand)))
    return s;
  *bytes = carve_paper(nullptr, *robot, *motions, n_uniform, n_surface, n_cand).bytes;
  return SV_OK;
}

int sv_make_samples_paper(const sv_robot* robot, const sv_motions* motions, float box_half, int32_t n_uniform,
                          int32_t n_surface, int32_t n_cand, float sigma, const float* rnd, float* out,
                          int32_t* n_accepted, int32_t* n_short, void* ws, size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) ||
      (s = check_paper_counts(motions, n_uniform, n_surface, n_cand)))
    return s;
  if (motions->kind != SV_LINEAR) return fail(SV_ERR_UNSUPPORTED, "training samples are drawn for linear motions");
  if (!(box_half > 0.f) || !(sigma >= 0.f)) return fail(SV_ERR_ARG, "box_half must be > 0 and sigma >= 0");
  if (motions->n == 0 || (n_uniform == 0 && n_surface == 0)) return SV_OK;
  if (!rnd || !out) return fail(SV_ERR_ARG, "rnd or out is NULL");
  const PaperWs w0 = carve_paper(nullptr, *robot, *motions, n_uniform, n_surface, n_cand);
  if (!ws || ws_bytes < w0.bytes) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w0.bytes, ws_bytes);
  const PaperWs w = carve_paper(ws, *robot, *motions, n_uniform, n_surface, n_cand);
  hipStream_t st = (hipStream_t)stream;
  const MotionArgs ma = to_args(*motions);
  hipError_t e;
  {
    ProfScope ps("motion_table", st);
    e = launch_motion_table(*robot, ma, w.table, st);
  }
  if (e != hipSuccess) return hip_fail(e, "motion table");
  ProfScope ps("make_samples_paper", st);
  e = launch_make_samples_paper(*robot, ma, w.table, box_half, n_uniform, n_surface, n_cand, sigma, rnd, w.a, out,
                                n_accepted, n_short, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "make paper samples");
}

int sv_nn_predict(const sv_mlp* mlp, int precision, const float* rows, int64_t row_stride, int64_t n, float* out,
                  void* ws, size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_mlp(mlp, precision, 0))) return s;
  if (n < 0 || n > 0x7fffffffLL) return fail(SV_ERR_SHAPE, "row count %lld outside 0..2^31-1", (long long)n);
  if (row_stride < mlp->in_dim) return fail(SV_ERR_ARG, "row_stride %lld < in_dim", (long long)row_stride);
  if (n == 0) return SV_OK;
  if (!rows || !out) return fail(SV_ERR_ARG, "rows or out is NULL");
  const size_t need = nn_sdf_bytes(*mlp, precision);
  if (need && (!ws || ws_bytes < need))
    return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  hipStream_t st = (hipStream_t)stream;
  const MlpArgs na = to_args(*mlp);
  hipError_t e = hipSuccess;
  __bf16* packed = static_cast<__bf16*>(ws);
  if (precision == SV_BF16) {
    ProfScope ps("pack_bf16", st);
    e = launch_pack_bf16(na, 0, packed, st);
  }
  if (e != hipSuccess) return hip_fail(e, "pack weights");
  ProfScope ps("mlp_rows", st);
  e = launch_mlp_rows(na, precision == SV_BF16, packed, rows, row_stride, n, out, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "network rows");
}

int sv_train_workspace_size(const sv_mlp* mlp, int64_t batch, size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_mlp(mlp, SV_BF16, 0))) return s;
  if (mlp->width > kTrainMaxWidth) return fail(SV_ERR_UNSUPPORTED, "training width %d > %d", mlp->width, kTrainMaxWidth);
  if (batch < 1 || batch > (1 << 24)) return fail(SV_ERR_SHAPE, "batch %lld outside 1..2^24", (long long)batch);
  *bytes = train_bytes(*mlp, batch);
  return SV_OK;
}

int sv_train_step(const sv_mlp* mlp, float* adam_m, float* adam_v, const sv_train_hparams* hp, const float* samples,
                  int64_t n_samples, const int32_t* batch_idx, int64_t batch, float* loss_out, float* grad_out,
                  void* ws, size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_mlp(mlp, SV_BF16, 0))) return s;
  if (mlp->width > kTrainMaxWidth) return fail(SV_ERR_UNSUPPORTED, "training width %d > %d", mlp->width, kTrainMaxWidth);
  if (!hp) return fail(SV_ERR_ARG, "hparams is NULL");
  if (hp->step < 1) return fail(SV_ERR_ARG, "Adam step must be >= 1");
  if (!(hp->clamp_sigma > 0.f) || !(hp->lr >= 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) ||
      !(hp->beta2 >= 0.f && hp->beta2 < 1.f) || !(hp->adam_eps > 0.f) || (hp->clamp_pred != 0 && hp->clamp_pred != 1))
    return fail(SV_ERR_ARG, "hyper-parameter out of range");
  if (batch < 1 || batch > (1 << 24)) return fail(SV_ERR_SHAPE, "batch %lld outside 1..2^24", (long long)batch);
  if (n_samples < 1) return fail(SV_ERR_SHAPE, "no samples");
  if (!adam_m || !adam_v || !samples || !batch_idx) return fail(SV_ERR_ARG, "NULL device pointer");
  if (mlp->kind == SV_NET_RESIDUAL) {
    if (hp->clamp_pred) return fail(SV_ERR_UNSUPPORTED, "the residual network trains with the target-only clamp");
    const TrainResWs w0 = carve_train_res(nullptr, *mlp, batch);
    if (!ws || ws_bytes < w0.bytes)
      return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w0.bytes, ws_bytes);
    const TrainResWs w = carve_train_res(ws, *mlp, batch);
    hipStream_t st = (hipStream_t)stream;
    const MlpArgs na = to_args(*mlp);
    float* grad = grad_out ? grad_out : w.grad;
    hipError_t e;
    {
      ProfScope ps("train_grad", st);
      e = launch_train_step_res(na, samples, batch_idx, (int)batch, (int)train_rows_padded(batch), w.r,
                                hp->clamp_sigma, grad, loss_out, st);
    }
    if (e != hipSuccess) return hip_fail(e, "residual train step");
    ProfScope ps("adam", st);
    e = launch_bn_running(na, w.r, (int)batch, const_cast<float*>(mlp->params), st);
    if (e == hipSuccess)
      e = launch_adam(const_cast<float*>(mlp->params), adam_m, adam_v, grad, (int64_t)n_params(*mlp), hp->lr,
                      hp->beta1, hp->beta2, hp->adam_eps, hp->step, st);
    return e == hipSuccess ? SV_OK : hip_fail(e, "adam");
  }
  const TrainWs w0 = carve_train(nullptr, *mlp, batch);
  if (!ws || ws_bytes < w0.bytes) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", w0.bytes, ws_bytes);
  const TrainWs w = carve_train(ws, *mlp, batch);
  hipStream_t st = (hipStream_t)stream;
  const MlpArgs na = to_args(*mlp);
  float* grad = grad_out ? grad_out : w.grad;
  const int64_t Bp = train_rows_padded(batch);
  hipError_t e;
  {
    ProfScope ps("pack_bf16", st);
    e = launch_pack_bf16_both(na, w.packed, w.packedT, st);
  }
  if (e != hipSuccess) return hip_fail(e, "pack weights");
  {
    ProfScope ps("train_grad", st);
    e = launch_train_step(na, samples, batch_idx, (int)batch, (int)Bp, w.aT, w.dzT, w.h0T, w.y, w.dy, w.packed,
                          w.packedT, grad, w.part_w, w.part_w1, hp->clamp_sigma, hp->clamp_pred, loss_out, st);
  }
  if (e != hipSuccess) return hip_fail(e, "train step");
  ProfScope ps("adam", st);
  e = launch_adam(const_cast<float*>(mlp->params), adam_m, adam_v, grad, (int64_t)n_params(*mlp), hp->lr, hp->beta1,
                  hp->beta2, hp->adam_eps, hp->step, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "adam");
}

int sv_batch_workspace_size(const sv_robot* robot, const sv_batch_caps* caps, size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_robot(robot)) || (s = check_caps(caps))) return s;
  carve_batch(nullptr, *robot, *caps, bytes);
  return SV_OK;
}

int sv_check_requests(const sv_robot* robot, const sv_request* reqs, int32_t n_req, const sv_batch_caps* caps,
                      float eps, const sv_tile* tile, uint64_t* done_ticks, int32_t* status, void* ws,
                      size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_robot(robot)) || (s = check_caps(caps))) return s;
  if (n_req < 0 || n_req > caps->max_requests)
    return fail(SV_ERR_SHAPE, "n_req %d outside 0..caps.max_requests (%d)", n_req, caps->max_requests);
  if (n_req > 0 && !reqs) return fail(SV_ERR_ARG, "request table is NULL");
  if (isnan(eps)) return fail(SV_ERR_ARG, "eps is NaN");
  const sv_tile t = tile ? *tile : default_batch_tile();
  if (!batch_tile_supported(t))
    return fail(SV_ERR_ARG,
                "unsupported tile (ppl %d, threads %d, blocks/CU %d, tiles/item %d, cull %d, culled blocks/CU %d, "
                "gangs %d, divisors %d/%d)", t.ppl, t.threads, t.blocks_per_cu, t.tiles_per_item, t.cull,
                t.cull_blocks_per_cu, t.cull_gangs, t.cull_div_linear, t.cull_div_spline);
  size_t need = 0;
  carve_batch(nullptr, *robot, *caps, &need);
  if (!ws || ws_bytes < need) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  if (n_req == 0) return SV_OK;
  size_t unused = 0;
  const BatchWs w = carve_batch(ws, *robot, *caps, &unused);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps("batch", st);
    e = launch_batch(*robot, reqs, n_req, *caps, eps, kCertBand, t, reinterpret_cast<unsigned long long*>(done_ticks),
                     status, w, st);
  }
  return e == hipSuccess ? SV_OK : hip_fail(e, "batched check");
}

int sv_nn_min_workspace_size(const sv_mlp* mlp, const sv_motions* motions, size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_mlp(mlp, SV_BF16, 0)) || (s = check_motions(motions, 0))) return s;
  Carver cv(nullptr);
  cv.take<__bf16>(mlp_packed_elems(to_args(*mlp)));
  cv.take<unsigned>((size_t)motions->n);
  *bytes = cv.off;
  return SV_OK;
}

int sv_nn_min(const sv_mlp* mlp, const sv_motions* motions, const sv_cloud* cloud, float* d_hat, void* ws,
              size_t ws_bytes, void* stream) {
  int s;
  if ((s = check_mlp(mlp, SV_BF16, 0)) || (s = check_motions(motions, 0)) || (s = check_cloud(cloud))) return s;
  if (motions->kind != SV_LINEAR) return fail(SV_ERR_UNSUPPORTED, "the network applies to linear motions only");
  if (motions->n > 0 && !d_hat) return fail(SV_ERR_ARG, "d_hat is NULL");
  size_t need = 0;
  if ((s = sv_nn_min_workspace_size(mlp, motions, &need))) return s;
  if (motions->n == 0) return SV_OK;
  if (!ws || ws_bytes < need) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  Carver cv(ws);
  const MlpArgs na = to_args(*mlp);
  __bf16* packed = cv.take<__bf16>(mlp_packed_elems(na));
  unsigned* keys = cv.take<unsigned>((size_t)motions->n);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_fill_i32(reinterpret_cast<int*>(keys), motions->n, -1, st);
  if (e == hipSuccess && cloud->n > 0) {
    {
      ProfScope ps("pack_bf16", st);
      e = launch_pack_bf16(na, 0, packed, st);
    }
    if (e == hipSuccess) {
      ProfScope ps("nn_min", st);
      e = launch_mlp_min(na, to_args(*motions), to_args(*cloud), packed, keys, st);
    }
  }
  if (e == hipSuccess) e = launch_decode_min(keys, motions->n, d_hat, st);
  return e == hipSuccess ? SV_OK : hip_fail(e, "network minimum");
}

int sv_first_free_workspace_size(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud,
                                 size_t* bytes) {
  int s;
  if (!bytes) return fail(SV_ERR_ARG, "bytes is NULL");
  if ((s = check_robot(robot)) || (s = check_motions(motions, robot->dof)) || (s = check_cloud(cloud))) return s;
  if (motions->n > kMaxSearchMotions) return fail(SV_ERR_SHAPE, "more than %d motions", kMaxSearchMotions);
  carve_search(nullptr, *robot, motions->n, motions->T, bytes);
  return SV_OK;
}

int sv_first_free(const sv_robot* robot, const sv_motions* motions, const sv_cloud* cloud, float eps,
                  const float* d_hat, sv_search_result* result, int32_t* order, void* ws, size_t ws_bytes,
                  void* stream) {
  int s;
  size_t need = 0;
  if ((s = sv_first_free_workspace_size(robot, motions, cloud, &need))) return s;
  if (!result) return fail(SV_ERR_ARG, "result is NULL");
  if (isnan(eps)) return fail(SV_ERR_ARG, "eps is NaN");
  if (!ws || ws_bytes < need) return fail(SV_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  size_t unused = 0;
  const SearchWs w = carve_search(ws, *robot, motions->n, motions->T, &unused);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps("search", st);
    e = launch_search(*robot, to_args(*motions), to_args(*cloud), eps, kCertBand, d_hat, result, order, w, st);
  }
  return e == hipSuccess ? SV_OK : hip_fail(e, "first free motion");
}

int sv_tile_candidates(sv_tile* tiles, int32_t capacity, int32_t* n) {
  if (!n) return fail(SV_ERR_ARG, "n is NULL");
  const std::vector<sv_tile> v = tile_candidates();
  *n = (int32_t)v.size();
  if (tiles)
    for (int32_t i = 0; i < capacity && i < (int32_t)v.size(); ++i) tiles[i] = v[i];
  return SV_OK;
}

int sv_default_tile(sv_tile* tile) {
  if (!tile) return fail(SV_ERR_ARG, "tile is NULL");
  *tile = default_batch_tile();
  return SV_OK;
}

int sv_wall_clock_hz(int64_t* hz) {
  if (!hz) return fail(SV_ERR_ARG, "hz is NULL");
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "wall clock rate");
  *hz = (int64_t)khz * 1000;
  return SV_OK;
}

}  // extern "C"
