"""FP64 CPU oracle for the swept-volume collision check (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library; the only thing both sides share is the seeded input
generator (``svgen``), which holds none of the method's arithmetic.

The geometric part is plain C (``sv_oracle.c``, compiled with gcc -O2, no
fast-math, OpenMP over motions); the network part is numpy (``mlp.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libsv_oracle.so")
_lib = None


def build(out=_LIB, extra_flags=()) -> str:
    """Compile the C oracle with gcc (-O2, IEEE semantics, OpenMP)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
           "-std=c11", *extra_flags, _SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path=_LIB):
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(path)
    lib = ctypes.CDLL(path)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(ctypes.c_int)
    i64 = ctypes.c_int64
    lib.orc_frames.argtypes = [ctypes.c_int, D, D, D]
    lib.orc_capsules.argtypes = [ctypes.c_int, D, ctypes.c_int, I, D, D, D]
    lib.orc_motion_q.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, ctypes.c_double, D]
    lib.orc_sample_s.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.orc_sample_s.restype = ctypes.c_double
    lib.orc_capsule_dist.argtypes = [D, D, D, ctypes.c_double]
    lib.orc_capsule_dist.restype = ctypes.c_double
    robot = [ctypes.c_int, D, ctypes.c_int, I, D, D]
    lib.orc_exact_sdf.argtypes = robot + [ctypes.c_int, ctypes.c_int, i64, D, D, D, i64, D, D, ctypes.c_int]
    lib.orc_check_motions.argtypes = robot + [ctypes.c_int, ctypes.c_int, i64, D, D, D, i64, D,
                                              ctypes.c_double, D, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
    lib.orc_sample_sdf.argtypes = robot + [ctypes.c_int, i64, D, D, D, D, ctypes.c_int]
    lib.orc_max_threads.restype = ctypes.c_int
    if path == _LIB:
        _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _robot_args(arm):
    dh, pdh = _d(arm.dh)
    cf = np.ascontiguousarray(arm.cap_frame, dtype=np.int32)
    cp, pcp = _d(arm.cap_p)
    cr, pcr = _d(arm.cap_r)
    keep = (dh, cf, cp, cr)
    args = [arm.dof, pdh, arm.n_caps, cf.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pcp, pcr]
    return keep, args


_KIND = {"linear": 0, "spline": 1}


def frames(arm, q, lib=None):
    """[(dof+1)][3][4] frames T_0..T_dof at configuration q."""
    lib = lib or load()
    dh, pdh = _d(arm.dh)
    qq, pq = _d(q)
    out = np.zeros(((arm.dof + 1) * 12,))
    lib.orc_frames(arm.dof, pdh, pq, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out.reshape(arm.dof + 1, 3, 4)


def capsules(arm, q, lib=None):
    """[K][2][3] world capsule endpoints at configuration q."""
    lib = lib or load()
    keep, args = _robot_args(arm)
    qq, pq = _d(q)
    out = np.zeros((arm.n_caps * 6,))
    lib.orc_capsules(*args[:5], pq, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out.reshape(arm.n_caps, 2, 3)


def motion_q(kind, q0, q1, via, s, lib=None):
    lib = lib or load()
    dof = len(q0)
    a, pa = _d(q0)
    b, pb = _d(q1)
    v, pv = _d(via if via is not None else np.zeros((2, dof)))
    out = np.zeros(dof)
    lib.orc_motion_q(_KIND[kind], dof, pa, pb, pv, float(s), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def sample_s(t, T, lib=None):
    return (lib or load()).orc_sample_s(t, T)


def capsule_dist(x, A, B, r, lib=None):
    lib = lib or load()
    x, px = _d(x)
    A, pA = _d(A)
    B, pB = _d(B)
    return lib.orc_capsule_dist(px, pA, pB, float(r))


def _motion_args(motions):
    q0, p0 = _d(motions.q0)
    q1, p1 = _d(motions.q1)
    if motions.via is not None:
        via, pv = _d(motions.via)
    else:
        via, pv = None, ctypes.POINTER(ctypes.c_double)()
    return (q0, q1, via), [_KIND[motions.kind], motions.T, motions.n, p0, p1, pv]


def exact_sdf(arm, motions, pts, nthreads=0, lib=None):
    """[M][N] float64 swept SDF of every point for every motion."""
    lib = lib or load()
    k1, ra = _robot_args(arm)
    k2, ma = _motion_args(motions)
    pts, pp = _d(np.reshape(pts, (-1, 3)))
    out = np.zeros((motions.n, pts.shape[0]))
    rc = lib.orc_exact_sdf(*ra, *ma, pts.shape[0], pp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           int(nthreads))
    if rc:
        raise ValueError("orc_exact_sdf rejected its arguments")
    return out


def check_motions(arm, motions, pts, eps, nthreads=0, lib=None):
    """(min_dist [M] f64, argmin [M] i64, verdict [M] u8) per motion."""
    lib = lib or load()
    k1, ra = _robot_args(arm)
    k2, ma = _motion_args(motions)
    pts, pp = _d(np.reshape(pts, (-1, 3)))
    M = motions.n
    md = np.zeros(M)
    am = np.zeros(M, np.int64)
    vd = np.zeros(M, np.uint8)
    rc = lib.orc_check_motions(*ra, *ma, pts.shape[0], pp, float(eps),
                               md.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               am.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               vd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(nthreads))
    if rc:
        raise ValueError("orc_check_motions rejected its arguments")
    return md, am, vd


def sample_sdf(arm, x, q0, q1, T, nthreads=0, lib=None):
    """[B] swept SDF of independent (x_b, linear motion q0_b -> q1_b) samples."""
    lib = lib or load()
    k1, ra = _robot_args(arm)
    x, px = _d(np.reshape(x, (-1, 3)))
    a, pa = _d(q0)
    b, pb = _d(q1)
    out = np.zeros(x.shape[0])
    rc = lib.orc_sample_sdf(*ra, int(T), x.shape[0], px, pa, pb,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(nthreads))
    if rc:
        raise ValueError("orc_sample_sdf rejected its arguments")
    return out


def max_threads(lib=None) -> int:
    return int((lib or load()).orc_max_threads())
