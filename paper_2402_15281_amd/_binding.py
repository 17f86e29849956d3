"""ctypes binding of libsv (argument marshalling only).

Every function here has the name of the C entry point it wraps and does nothing
but turn torch device tensors into the pointers and sizes of the C ABI (see
include/sv.h).  All arithmetic runs in the HIP kernels of libsv.so; if the
library is missing this module raises at import time rather than fall back to
anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_MAX_DOF = 8
SV_MAX_CAPS = 16
SV_LINEAR, SV_SPLINE = 0, 1
SV_OP_EXACT_SDF, SV_OP_CHECK, SV_OP_NN_SDF = 0, 1, 2
SV_FP32, SV_BF16 = 0, 1
SV_SCREEN_NONE, SV_SCREEN_TRUST, SV_SCREEN_CERTIFIED = 0, 1, 2
SV_CHECK_UNCULLED = 0x100

_STATUS = {0: "SV_OK", -1: "SV_ERR_ARG", -2: "SV_ERR_SHAPE", -3: "SV_ERR_WORKSPACE",
           -4: "SV_ERR_UNSUPPORTED", -5: "SV_ERR_HIP"}


class SvError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_STATUS.get(status, status)}: {detail}")
        self.status = status


class sv_robot(ctypes.Structure):
    _fields_ = [("dof", ctypes.c_int32), ("n_caps", ctypes.c_int32),
                ("dh", (ctypes.c_double * 4) * SV_MAX_DOF),
                ("cap_frame", (ctypes.c_int32 * 2) * SV_MAX_CAPS),
                ("cap_p", ((ctypes.c_double * 3) * 2) * SV_MAX_CAPS),
                ("cap_r", ctypes.c_double * SV_MAX_CAPS)]


class sv_motions(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("T", ctypes.c_int32), ("n", ctypes.c_int64),
                ("q0", ctypes.c_void_p), ("q1", ctypes.c_void_p), ("via", ctypes.c_void_p)]


class sv_cloud(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


SV_NET_MLP, SV_NET_RESIDUAL = 0, 1


class sv_mlp(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("width", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("kind", ctypes.c_int32), ("bn_eps", ctypes.c_float)]


class sv_train_hparams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("adam_eps", ctypes.c_float), ("step", ctypes.c_int64), ("clamp_sigma", ctypes.c_float),
                ("clamp_pred", ctypes.c_int32)]


class sv_results(ctypes.Structure):
    _fields_ = [("min_dist", ctypes.c_void_p), ("argmin", ctypes.c_void_p), ("verdict", ctypes.c_void_p),
                ("n_fallback", ctypes.c_void_p)]


class sv_request(ctypes.Structure):
    _fields_ = [("motions", sv_motions), ("cloud", sv_cloud), ("out", sv_results)]


class sv_batch_caps(ctypes.Structure):
    _fields_ = [("max_requests", ctypes.c_int32), ("max_T", ctypes.c_int32), ("max_motions", ctypes.c_int64),
                ("max_samples", ctypes.c_int64), ("max_points", ctypes.c_int64), ("max_band", ctypes.c_int32),
                ("max_total_points", ctypes.c_int64)]


class sv_tile(ctypes.Structure):
    _fields_ = [("ppl", ctypes.c_int32), ("threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tiles_per_item", ctypes.c_int32), ("cull", ctypes.c_int32), ("cull_blocks_per_cu", ctypes.c_int32),
                ("cull_gangs", ctypes.c_int32), ("cull_div_linear", ctypes.c_int32),
                ("cull_div_spline", ctypes.c_int32)]

    def as_tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "sv_tile(" + ", ".join(f"{k}={v}" for k, v in self.as_dict().items()) + ")"


SV_BATCH_BAD_REQUEST, SV_BATCH_OVER_CAPACITY, SV_BATCH_BAND_OVERFLOW = 1, 2, 4


class sv_search_result(ctypes.Structure):
    _fields_ = [("motion", ctypes.c_int32), ("position", ctypes.c_int32), ("dist", ctypes.c_float),
                ("n_exact", ctypes.c_int32), ("n_exact_run", ctypes.c_int32), ("n_first", ctypes.c_int32),
                ("n_nn", ctypes.c_int32), ("status", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsv.so not built at {LIB_PATH}; run `python -m paper_2402_15281_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.sv_status_string.restype = ctypes.c_char_p
    lib.sv_status_string.argtypes = [ctypes.c_int]
    lib.sv_last_error.restype = ctypes.c_char_p
    lib.sv_workspace_size.argtypes = [ctypes.c_int, ctypes.POINTER(sv_robot), ctypes.POINTER(sv_mlp), ctypes.c_int,
                                      ctypes.POINTER(sv_motions), ctypes.POINTER(sv_cloud),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.sv_nn_sdf.argtypes = [ctypes.POINTER(sv_mlp), ctypes.c_int, ctypes.POINTER(sv_motions),
                              ctypes.POINTER(sv_cloud), P, P, ctypes.c_size_t, P]
    lib.sv_fk.argtypes = [ctypes.POINTER(sv_robot), P, ctypes.c_int64, P, ctypes.c_int, P]
    lib.sv_exact_sdf.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), ctypes.POINTER(sv_cloud), P,
                                 P, ctypes.c_size_t, P]
    lib.sv_check_motions.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_mlp), ctypes.c_int, ctypes.c_float,
                                     ctypes.c_float,
                                     ctypes.POINTER(sv_motions), ctypes.POINTER(sv_cloud),
                                     ctypes.POINTER(sv_results), P, ctypes.c_size_t, P]
    lib.sv_check_motions_static.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_mlp), ctypes.c_int,
                                            ctypes.c_float, ctypes.c_float, ctypes.POINTER(sv_motions),
                                            ctypes.POINTER(sv_cloud), ctypes.POINTER(sv_results), P]
    lib.sv_profile_enable.argtypes = [ctypes.c_int]
    lib.sv_profile_reset.argtypes = []
    lib.sv_profile_reset.restype = None
    lib.sv_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    I32, I64, F32, SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.POINTER(ctypes.c_size_t)
    lib.sv_make_samples.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), F32, I32, I32, I32, F32, P,
                                    P, P, P, ctypes.c_size_t, P]
    lib.sv_make_samples_workspace_size.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), I32, I32,
                                                   SZ]
    lib.sv_nn_predict.argtypes = [ctypes.POINTER(sv_mlp), ctypes.c_int, P, I64, I64, P, P, ctypes.c_size_t, P]
    lib.sv_train_step.argtypes = [ctypes.POINTER(sv_mlp), P, P, ctypes.POINTER(sv_train_hparams), P, I64, P, I64, P,
                                  P, P, ctypes.c_size_t, P]
    lib.sv_train_workspace_size.argtypes = [ctypes.POINTER(sv_mlp), I64, SZ]
    lib.sv_batch_workspace_size.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_batch_caps), SZ]
    lib.sv_check_requests.argtypes = [ctypes.POINTER(sv_robot), P, I32, ctypes.POINTER(sv_batch_caps), F32,
                                      ctypes.POINTER(sv_tile), P, P, P, ctypes.c_size_t, P]
    lib.sv_tile_candidates.argtypes = [ctypes.POINTER(sv_tile), I32, ctypes.POINTER(I32)]
    lib.sv_default_tile.argtypes = [ctypes.POINTER(sv_tile)]
    lib.sv_wall_clock_hz.argtypes = [ctypes.POINTER(I64)]
    lib.sv_nn_min.argtypes = [ctypes.POINTER(sv_mlp), ctypes.POINTER(sv_motions), ctypes.POINTER(sv_cloud), P, P,
                              ctypes.c_size_t, P]
    lib.sv_nn_min_workspace_size.argtypes = [ctypes.POINTER(sv_mlp), ctypes.POINTER(sv_motions), SZ]
    lib.sv_first_free.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), ctypes.POINTER(sv_cloud),
                                  F32, P, P, P, P, ctypes.c_size_t, P]
    lib.sv_first_free_workspace_size.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions),
                                                 ctypes.POINTER(sv_cloud), SZ]
    lib.sv_continuous_gap.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), P, F32, P, P, P]
    lib.sv_make_samples_paper.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), F32, I32, I32, I32,
                                          F32, P, P, P, P, P, ctypes.c_size_t, P]
    lib.sv_make_samples_paper_workspace_size.argtypes = [ctypes.POINTER(sv_robot), ctypes.POINTER(sv_motions), I32,
                                                         I32, I32, SZ]
    for fn in ("sv_workspace_size", "sv_fk", "sv_exact_sdf", "sv_nn_sdf", "sv_check_motions", "sv_profile_enable",
               "sv_profile_read", "sv_make_samples", "sv_make_samples_workspace_size", "sv_nn_predict",
               "sv_train_step", "sv_train_workspace_size", "sv_batch_workspace_size", "sv_check_requests",
               "sv_tile_candidates", "sv_default_tile", "sv_wall_clock_hz", "sv_nn_min", "sv_nn_min_workspace_size",
               "sv_first_free", "sv_first_free_workspace_size", "sv_continuous_gap", "sv_check_motions_static",
               "sv_make_samples_paper", "sv_make_samples_paper_workspace_size"):
        getattr(lib, fn).restype = ctypes.c_int
    return lib


lib = _load()


def _check(status: int):
    if status != 0:
        raise SvError(status, lib.sv_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- host structs

def make_robot(arm) -> sv_robot:
    """sv_robot from an arm description (dh [dof][4], cap_frame [K][2], cap_p [K][2][3], cap_r [K])."""
    r = sv_robot()
    dh = np.asarray(arm.dh, np.float64)
    cf = np.asarray(arm.cap_frame, np.int32)
    cp = np.asarray(arm.cap_p, np.float64)
    cr = np.asarray(arm.cap_r, np.float64)
    r.dof, r.n_caps = dh.shape[0], cr.shape[0]
    for i in range(dh.shape[0]):
        for j in range(4):
            r.dh[i][j] = float(dh[i, j])
    for k in range(cr.shape[0]):
        r.cap_frame[k][0], r.cap_frame[k][1] = int(cf[k, 0]), int(cf[k, 1])
        for e in range(2):
            for c in range(3):
                r.cap_p[k][e][c] = float(cp[k, e, c])
        r.cap_r[k] = float(cr[k])
    return r


class DeviceMotions:
    """Motions resident in device memory (FP32) plus their sv_motions descriptor."""

    def __init__(self, motions, device="cuda"):
        self.kind = SV_SPLINE if motions.kind == "spline" else SV_LINEAR
        self.T = int(motions.T)
        self.q0 = torch.as_tensor(np.asarray(motions.q0, np.float32), device=device).contiguous()
        self.q1 = torch.as_tensor(np.asarray(motions.q1, np.float32), device=device).contiguous()
        self.via = None
        if motions.via is not None:
            self.via = torch.as_tensor(np.asarray(motions.via, np.float32), device=device).contiguous()
        self.n = int(self.q0.shape[0])

    def desc(self) -> sv_motions:
        return sv_motions(self.kind, self.T, self.n, self.q0.data_ptr() if self.n else None,
                          self.q1.data_ptr() if self.n else None,
                          self.via.data_ptr() if self.via is not None and self.n else None)


class DeviceCloud:
    """Point cloud in device memory as structure of arrays (FP32)."""

    def __init__(self, pts, device="cuda"):
        p = torch.as_tensor(np.asarray(pts, np.float32).reshape(-1, 3).T.copy(), device=device).contiguous()
        self.xyz = p                      # [3][N]
        self.n = int(p.shape[1])

    def desc(self) -> sv_cloud:
        if self.n == 0:
            return sv_cloud(0, None, None, None)
        base = self.xyz.data_ptr()
        return sv_cloud(self.n, base, base + 4 * self.n, base + 8 * self.n)


class DeviceMLP:
    """Flat FP32 network parameters in device memory plus their sv_mlp descriptor."""

    def __init__(self, params, in_dim: int, width: int, n_hidden: int, device="cuda", kind: int = 0,
                 bn_eps: float = 1e-5):
        if isinstance(params, torch.Tensor):
            self.params = params.to(device=device, dtype=torch.float32).contiguous()
        else:
            self.params = torch.as_tensor(np.asarray(params, np.float32), device=device).contiguous()
        self.in_dim, self.width, self.n_hidden = int(in_dim), int(width), int(n_hidden)
        self.kind, self.bn_eps = int(kind), float(bn_eps)

    def desc(self) -> sv_mlp:
        return sv_mlp(self.in_dim, self.width, self.n_hidden, self.params.data_ptr(), self.kind, self.bn_eps)


class DeviceResults:
    def __init__(self, M, device="cuda"):
        self.min_dist = torch.empty(M, dtype=torch.float32, device=device)
        self.argmin = torch.empty(M, dtype=torch.int32, device=device)
        self.verdict = torch.empty(M, dtype=torch.uint8, device=device)
        self.n_fallback = torch.zeros(M, dtype=torch.int32, device=device)

    def desc(self) -> sv_results:
        return sv_results(self.min_dist.data_ptr(), self.argmin.data_ptr(), self.verdict.data_ptr(),
                          self.n_fallback.data_ptr())


# ------------------------------------------------------------------ entry points

def _mlp_ref(mlp):
    if mlp is None:
        return None, None
    d = mlp.desc()
    return d, ctypes.byref(d)


def sv_workspace_size(op: int, robot, motions: DeviceMotions, cloud: DeviceCloud, mlp=None,
                      precision: int = SV_BF16) -> int:
    n = ctypes.c_size_t(0)
    md, cd = motions.desc(), cloud.desc()
    keep, mref = _mlp_ref(mlp)
    rref = ctypes.byref(robot) if robot is not None else None
    _check(lib.sv_workspace_size(op, rref, mref, int(precision), ctypes.byref(md), ctypes.byref(cd), ctypes.byref(n)))
    return int(n.value)


def workspace(nbytes: int, device="cuda"):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def sv_make_samples_paper(robot: sv_robot, motions: DeviceMotions, box_half: float, n_uniform: int, n_surface: int,
                          n_cand: int, sigma: float, rnd: torch.Tensor, out: torch.Tensor,
                          n_accepted: torch.Tensor = None, n_short: torch.Tensor = None, ws=None, stream=None):
    """out[M][n_uniform + 4 n_surface][in_dim + 1] <- paper-style training rows (Sec. IV-C)."""
    md = motions.desc()
    if ws is None:
        n = ctypes.c_size_t(0)
        _check(lib.sv_make_samples_paper_workspace_size(ctypes.byref(robot), ctypes.byref(md), int(n_uniform),
                                                        int(n_surface), int(n_cand), ctypes.byref(n)))
        ws = workspace(n.value)
    _check(lib.sv_make_samples_paper(ctypes.byref(robot), ctypes.byref(md), float(box_half), int(n_uniform),
                                     int(n_surface), int(n_cand), float(sigma), _ptr(rnd), _ptr(out),
                                     _ptr(n_accepted), _ptr(n_short), _ptr(ws), ws.numel(), _stream(stream)))


def sv_continuous_gap(robot: sv_robot, motions: DeviceMotions, gap: torch.Tensor, min_dist: torch.Tensor = None,
                      eps: float = 0.0, verdict: torch.Tensor = None, stream=None):
    """gap[m] <- bound of (sampled - continuous) swept distance; with min_dist, verdict[m]."""
    md = motions.desc()
    _check(lib.sv_continuous_gap(ctypes.byref(robot), ctypes.byref(md), _ptr(min_dist), float(eps), _ptr(gap),
                                 _ptr(verdict), _stream(stream)))


def sv_fk(robot: sv_robot, q: torch.Tensor, caps: torch.Tensor, fp64: bool = False, stream=None):
    """caps[n][n_caps][8] <- FK of q[n][dof] (device tensors, FP32)."""
    n = int(q.shape[0])
    _check(lib.sv_fk(ctypes.byref(robot), _ptr(q), n, _ptr(caps), int(bool(fp64)), _stream(stream)))


def sv_exact_sdf(robot: sv_robot, motions: DeviceMotions, cloud: DeviceCloud, sdf: torch.Tensor, ws=None,
                 stream=None):
    """sdf[M][N] <- exact swept SDF (device FP32)."""
    md, cd = motions.desc(), cloud.desc()
    if ws is None:
        ws = workspace(sv_workspace_size(SV_OP_EXACT_SDF, robot, motions, cloud))
    _check(lib.sv_exact_sdf(ctypes.byref(robot), ctypes.byref(md), ctypes.byref(cd), _ptr(sdf), _ptr(ws),
                            ws.numel(), _stream(stream)))
    return ws


def sv_nn_sdf(mlp: DeviceMLP, precision: int, motions: DeviceMotions, cloud: DeviceCloud, sdf_hat: torch.Tensor,
              ws=None, stream=None):
    """sdf_hat[M][N] <- network prediction for every (motion, point) (device FP32)."""
    md, cd = motions.desc(), cloud.desc()
    keep, mref = _mlp_ref(mlp)
    if ws is None:
        ws = workspace(sv_workspace_size(SV_OP_NN_SDF, None, motions, cloud, mlp, precision))
    _check(lib.sv_nn_sdf(mref, int(precision), ctypes.byref(md), ctypes.byref(cd), _ptr(sdf_hat), _ptr(ws),
                         ws.numel(), _stream(stream)))
    return ws


def sv_check_motions(robot: sv_robot, motions: DeviceMotions, cloud: DeviceCloud, out: DeviceResults, eps: float,
                     mlp: DeviceMLP = None, screen: int = SV_SCREEN_NONE, tau: float = 0.0, ws=None, stream=None,
                     unculled: bool = False):
    """Per-motion min distance, argmin, verdict (and fallback counts when screening);
    unculled: run every exact test (screen | SV_CHECK_UNCULLED; same results)."""
    md, cd, rd = motions.desc(), cloud.desc(), out.desc()
    keep, mref = _mlp_ref(mlp)
    if ws is None:
        ws = workspace(sv_workspace_size(SV_OP_CHECK, robot, motions, cloud, mlp))
    mode = int(screen) | (SV_CHECK_UNCULLED if unculled else 0)
    _check(lib.sv_check_motions(ctypes.byref(robot), mref, mode, float(eps), float(tau), ctypes.byref(md),
                                ctypes.byref(cd), ctypes.byref(rd), _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def sv_check_motions_static(robot: sv_robot, motions: DeviceMotions, cloud: DeviceCloud, out: DeviceResults,
                            eps: float, mlp: DeviceMLP = None, screen: int = SV_SCREEN_NONE, tau: float = 0.0,
                            stream=None, unculled: bool = False):
    """sv_check_motions on the library's static scratch memory (no workspace, no allocation)."""
    md, cd, rd = motions.desc(), cloud.desc(), out.desc()
    keep, mref = _mlp_ref(mlp)
    mode = int(screen) | (SV_CHECK_UNCULLED if unculled else 0)
    _check(lib.sv_check_motions_static(ctypes.byref(robot), mref, mode, float(eps), float(tau), ctypes.byref(md),
                                       ctypes.byref(cd), ctypes.byref(rd), _stream(stream)))


def executed_tests(ws: torch.Tensor) -> int:
    """Segment tests the culled exact passes of the last sv_check_motions or
    sv_check_requests call on ws ran."""
    return int(ws[:8 * 256].cpu().numpy().view(np.uint64).sum())


def sv_profile_enable(on: bool = True):
    _check(lib.sv_profile_enable(int(bool(on))))


def sv_profile_reset():
    lib.sv_profile_reset()


def sv_profile_read(kernel: str):
    """(total milliseconds, launches) recorded for a kernel group since the last reset."""
    ms, n = ctypes.c_double(0), ctypes.c_int64(0)
    _check(lib.sv_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def sv_make_samples(robot: sv_robot, motions: DeviceMotions, cube_half: float, n_uniform: int, n_near: int,
                    n_cand: int, band: float, rnd: torch.Tensor, out: torch.Tensor, n_short: torch.Tensor = None,
                    ws=None, stream=None):
    """out[M*(n_uniform+n_near)][in_dim+1] <- training rows (x, q0, q1, delta) labelled by the exact check."""
    md = motions.desc()
    if ws is None:
        n = ctypes.c_size_t(0)
        _check(lib.sv_make_samples_workspace_size(ctypes.byref(robot), ctypes.byref(md), int(n_uniform), int(n_cand),
                                                  ctypes.byref(n)))
        ws = workspace(n.value)
    _check(lib.sv_make_samples(ctypes.byref(robot), ctypes.byref(md), float(cube_half), int(n_uniform), int(n_near),
                               int(n_cand), float(band), _ptr(rnd), _ptr(out), _ptr(n_short), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return ws


def sv_nn_predict(mlp: DeviceMLP, precision: int, rows: torch.Tensor, out: torch.Tensor, ws=None, stream=None):
    """out[n] <- network prediction for rows[n][stride] (first in_dim columns)."""
    d = mlp.desc()
    n, stride = int(rows.shape[0]), int(rows.shape[1])
    if ws is None:   # the network's workspace does not depend on the rows
        n_ws = ctypes.c_size_t(0)
        none_m, none_c = sv_motions(SV_LINEAR, 1, 0, None, None, None), sv_cloud(0, None, None, None)
        _check(lib.sv_workspace_size(SV_OP_NN_SDF, None, ctypes.byref(d), int(precision), ctypes.byref(none_m),
                                     ctypes.byref(none_c), ctypes.byref(n_ws)))
        ws = workspace(n_ws.value)
    _check(lib.sv_nn_predict(ctypes.byref(d), int(precision), _ptr(rows), stride, n, _ptr(out), _ptr(ws), ws.numel(),
                             _stream(stream)))
    return ws


def sv_train_workspace_size(mlp: DeviceMLP, batch: int) -> int:
    d = mlp.desc()
    n = ctypes.c_size_t(0)
    _check(lib.sv_train_workspace_size(ctypes.byref(d), int(batch), ctypes.byref(n)))
    return int(n.value)


def sv_train_step(mlp: DeviceMLP, adam_m: torch.Tensor, adam_v: torch.Tensor, step: int, samples: torch.Tensor,
                  batch_idx: torch.Tensor, lr: float = 1e-3, betas=(0.9, 0.999), adam_eps: float = 1e-8,
                  clamp_sigma: float = 0.1, loss_out: torch.Tensor = None, grad_out: torch.Tensor = None, ws=None,
                  stream=None, clamp_pred: bool = False):
    """One Adam step of the BF16 network on samples[batch_idx]; mlp.params is updated in place."""
    d = mlp.desc()
    hp = sv_train_hparams(float(lr), float(betas[0]), float(betas[1]), float(adam_eps), int(step), float(clamp_sigma),
                          int(bool(clamp_pred)))
    B = int(batch_idx.shape[0])
    if ws is None:
        ws = workspace(sv_train_workspace_size(mlp, B))
    _check(lib.sv_train_step(ctypes.byref(d), _ptr(adam_m), _ptr(adam_v), ctypes.byref(hp), _ptr(samples),
                             int(samples.shape[0]), _ptr(batch_idx), B, _ptr(loss_out), _ptr(grad_out), _ptr(ws),
                             ws.numel(), _stream(stream)))
    return ws


# ------------------------------------------------------------- batched requests

class DeviceRequests:
    """A batch of requests (motions, cloud, results) and its request table in device memory.

    requests: list of (DeviceMotions, DeviceCloud, DeviceResults).  The table is one
    device tensor of sv_request records; rewrite() refreshes it in place (same
    storage), so a captured graph that reads it sees the new contents.
    """

    def __init__(self, requests, device="cuda"):
        self.requests = list(requests)
        n = max(len(self.requests), 1)
        self.table = torch.zeros(n * ctypes.sizeof(sv_request), dtype=torch.uint8, device=device)
        self.rewrite()

    @property
    def n(self) -> int:
        return len(self.requests)

    def rewrite(self, requests=None):
        if requests is not None:
            if len(requests) > self.table.numel() // ctypes.sizeof(sv_request):
                raise ValueError("more requests than the table holds")
            self.requests = list(requests)
        arr = (sv_request * max(self.n, 1))()
        for i, (m, c, o) in enumerate(self.requests):
            arr[i] = sv_request(m.desc(), c.desc(), o.desc())
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        self.table[:host.numel()].copy_(host)

    def caps(self, max_band: int = 64, slack: float = 1.0) -> sv_batch_caps:
        """Capacities that hold this batch (times slack)."""
        ms = [m for m, _, _ in self.requests]
        tot_m = sum(m.n for m in ms)
        tot_s = sum(m.n * m.T for m in ms)
        tot_p = sum(c.n for _, c, _ in self.requests)
        return sv_batch_caps(max(self.n, 1), max([m.T for m in ms] + [1]), max(int(tot_m * slack), 1),
                             max(int(tot_s * slack), 1), max([c.n for _, c, _ in self.requests] + [0]), int(max_band),
                             max(int(tot_p * slack), 1))


def sv_batch_workspace_size(robot: sv_robot, caps: sv_batch_caps) -> int:
    n = ctypes.c_size_t(0)
    _check(lib.sv_batch_workspace_size(ctypes.byref(robot), ctypes.byref(caps), ctypes.byref(n)))
    return int(n.value)


def sv_check_requests(robot: sv_robot, reqs: DeviceRequests, caps: sv_batch_caps, eps: float, tile: sv_tile = None,
                      done_ticks: torch.Tensor = None, status: torch.Tensor = None, ws=None, n_req: int = None,
                      stream=None):
    """Exact check of every request of the batch (results into each request's DeviceResults)."""
    if ws is None:
        ws = workspace(sv_batch_workspace_size(robot, caps))
    n = reqs.n if n_req is None else int(n_req)
    _check(lib.sv_check_requests(ctypes.byref(robot), _ptr(reqs.table), n, ctypes.byref(caps), float(eps),
                                 ctypes.byref(tile) if tile is not None else None, _ptr(done_ticks), _ptr(status),
                                 _ptr(ws), ws.numel(), _stream(stream)))
    return ws


def sv_tile_candidates():
    n = ctypes.c_int32(0)
    _check(lib.sv_tile_candidates(None, 0, ctypes.byref(n)))
    arr = (sv_tile * n.value)()
    _check(lib.sv_tile_candidates(arr, n.value, ctypes.byref(n)))
    return [sv_tile(*t.as_tuple()) for t in arr]


def sv_default_tile() -> sv_tile:
    t = sv_tile()
    _check(lib.sv_default_tile(ctypes.byref(t)))
    return t


def sv_wall_clock_hz() -> int:
    hz = ctypes.c_int64(0)
    _check(lib.sv_wall_clock_hz(ctypes.byref(hz)))
    return int(hz.value)


# ------------------------------------------------------------- first free motion

def sv_nn_min(mlp: DeviceMLP, motions: DeviceMotions, cloud: DeviceCloud, d_hat: torch.Tensor, ws=None,
              stream=None):
    """d_hat[m] <- min over the cloud of the BF16 network's prediction for motion m."""
    md, cd, nd = motions.desc(), cloud.desc(), mlp.desc()
    if ws is None:
        n = ctypes.c_size_t(0)
        _check(lib.sv_nn_min_workspace_size(ctypes.byref(nd), ctypes.byref(md), ctypes.byref(n)))
        ws = workspace(n.value)
    _check(lib.sv_nn_min(ctypes.byref(nd), ctypes.byref(md), ctypes.byref(cd), _ptr(d_hat), _ptr(ws), ws.numel(),
                         _stream(stream)))
    return ws


def search_result_tensor(device="cuda"):
    """Device buffer for one sv_search_result record."""
    return torch.zeros(ctypes.sizeof(sv_search_result) // 4, dtype=torch.int32, device=device)


def read_search_result(t: torch.Tensor) -> dict:
    r = sv_search_result.from_buffer_copy(t.cpu().numpy().tobytes())
    return {f: getattr(r, f) for f, _ in sv_search_result._fields_}


def sv_first_free(robot: sv_robot, motions: DeviceMotions, cloud: DeviceCloud, eps: float, result: torch.Tensor,
                  d_hat: torch.Tensor = None, order: torch.Tensor = None, ws=None, stream=None):
    """First collision-free motion (Alg. 1); result is a search_result_tensor()."""
    md, cd = motions.desc(), cloud.desc()
    if ws is None:
        n = ctypes.c_size_t(0)
        _check(lib.sv_first_free_workspace_size(ctypes.byref(robot), ctypes.byref(md), ctypes.byref(cd),
                                                ctypes.byref(n)))
        ws = workspace(n.value)
    _check(lib.sv_first_free(ctypes.byref(robot), ctypes.byref(md), ctypes.byref(cd), float(eps), _ptr(d_hat),
                             _ptr(result), _ptr(order), _ptr(ws), ws.numel(), _stream(stream)))
    return ws
