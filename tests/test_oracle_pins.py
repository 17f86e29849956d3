"""Pins for the FP64 oracle against things other than itself.

Each check ties the oracle to the paper's definitions through an independent
route: hand-derived closed forms (tests/golden), a different formulation of the
same quantity (product of exponentials for the kinematics, cross products for
point-segment distance, point-to-arc geometry), library routines (scipy's
clamped cubic spline), brute force at a much finer time grid within the
Lipschitz discretisation bound, and invariants the swept volume must obey.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.spatial.transform import Rotation

import svgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")


def arm_from(dh, cap_frame, cap_p, cap_r, qlim=None):
    dh = np.asarray(dh, float)
    if qlim is None:
        qlim = np.tile([-math.pi, math.pi], (dh.shape[0], 1))
    return svgen.Arm(dh=dh, qlim=np.asarray(qlim, float), cap_frame=np.asarray(cap_frame, np.int32),
                     cap_p=np.asarray(cap_p, float), cap_r=np.asarray(cap_r, float))


def motions_from(q0, q1, T, kind="linear", via=None):
    return svgen.Motions(q0=np.atleast_2d(np.asarray(q0, float)), q1=np.atleast_2d(np.asarray(q1, float)),
                         T=T, kind=kind, via=None if via is None else np.asarray(via, float)[None])


# ----------------------------------------------------------------- distances

def seg_dist_crossproduct(x, A, B):
    """Point-segment distance via endpoint distances and |ap x ab| / |ab| (independent form)."""
    x, A, B = map(np.asarray, (x, A, B))
    ab, ap, bp = B - A, x - A, x - B
    if np.dot(ab, ab) == 0:
        return np.linalg.norm(ap)
    if np.dot(ap, ab) <= 0:
        return np.linalg.norm(ap)
    if np.dot(bp, ab) >= 0:
        return np.linalg.norm(bp)
    return np.linalg.norm(np.cross(ap, ab)) / np.linalg.norm(ab)


def test_capsule_distance_closed_forms(orc):
    rng = np.random.default_rng(0)
    c = np.array([0.1, -0.2, 0.3])
    for _ in range(200):
        x = rng.uniform(-1, 1, 3)
        # sphere: A == B
        assert orc.capsule_dist(x, c, c, 0.07) == pytest.approx(np.linalg.norm(x - c) - 0.07, abs=1e-15)
        A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        r = rng.uniform(0.01, 0.1)
        assert orc.capsule_dist(x, A, B, r) == pytest.approx(seg_dist_crossproduct(x, A, B) - r, abs=1e-12)
    A, B = np.array([0., 0, 0]), np.array([0., 0, 1])
    assert orc.capsule_dist([0, 0, 0.3], A, B, 0.05) == pytest.approx(-0.05, abs=1e-15)   # on the axis
    assert orc.capsule_dist([0.05, 0, 0.3], A, B, 0.05) == pytest.approx(0.0, abs=1e-15)  # on the surface
    assert orc.capsule_dist([0, 0, 1.5], A, B, 0.05) == pytest.approx(0.45, abs=1e-15)    # beyond the cap


# ---------------------------------------------------------------- kinematics

def test_golden_planar_2r(orc):
    g = json.load(open(GOLD))["planar_2r"]
    arm = arm_from(g["dh"], g["cap_frame"], g["cap_p"], g["cap_r"])
    F = orc.frames(arm, g["q"])
    np.testing.assert_allclose(F[:, :, 3], g["origins"], atol=g["tol"])
    m = motions_from(g["q"], g["q"], 1)
    sdf = orc.exact_sdf(arm, m, np.array(g["points"]))[0]
    np.testing.assert_allclose(sdf, g["sdf"], atol=g["tol"])


def _elem(axis, v):
    T = np.eye(4)
    if axis in "xyz":
        T[:3, :3] = Rotation.from_euler(axis, v).as_matrix()
    else:
        T[:3, 3] = {"X": [v, 0, 0], "Z": [0, 0, v]}[axis]
    return T


def _screw_exp(w, p, theta):
    """exp of a unit rotation screw about axis w through point p, as a 4x4."""
    T = np.eye(4)
    R = Rotation.from_rotvec(np.asarray(w) * theta).as_matrix()
    T[:3, :3] = R
    T[:3, 3] = (np.eye(3) - R) @ p
    return T


def test_fk_matches_product_of_exponentials(orc):
    """Frames from the oracle's DH chain equal a product of exponentials built from
    the zero-configuration frames: T_i(q) = prod_{j<=i} exp([S_j] q_j) T_i(0),
    where joint j turns about the z axis of frame j-1 at q = 0."""
    arm = svgen.make_arm(3)
    rng = np.random.default_rng(1)
    # zero configuration frames from elementary transforms (scipy rotations)
    home = [np.eye(4)]
    for a, alpha, d, th in arm.dh:
        home.append(home[-1] @ _elem("z", th) @ _elem("Z", d) @ _elem("X", a) @ _elem("x", alpha))
    for _ in range(20):
        q = rng.uniform(-3, 3, arm.dof)
        F = orc.frames(arm, q)
        P = np.eye(4)
        for i in range(1, arm.dof + 1):
            w = home[i - 1][:3, 2]
            p = home[i - 1][:3, 3]
            P = P @ _screw_exp(w, p, q[i - 1])
            np.testing.assert_allclose(F[i], (P @ home[i])[:3], atol=1e-12)


def test_fk_z_rotation_equivariance(orc):
    arm = svgen.make_arm(1)
    rng = np.random.default_rng(2)
    for _ in range(10):
        q = rng.uniform(-2.5, 2.5, arm.dof)
        phi = rng.uniform(-0.5, 0.5)
        q2 = q.copy()
        q2[0] += phi
        R = Rotation.from_euler("z", phi).as_matrix()
        C1 = orc.capsules(arm, q)
        C2 = orc.capsules(arm, q2)
        np.testing.assert_allclose(C2, C1 @ R.T, atol=1e-12)


# -------------------------------------------------------------------- motions

def test_linear_motion_endpoints_and_grid(orc):
    q0, q1 = np.array([0.1, -0.2, 0.3]), np.array([-1.0, 2.0, 0.5])
    np.testing.assert_array_equal(orc.motion_q("linear", q0, q1, None, 0.0), q0)
    np.testing.assert_allclose(orc.motion_q("linear", q0, q1, None, 1.0), q1, atol=1e-15)
    np.testing.assert_allclose(orc.motion_q("linear", q0, q1, None, 0.25), q0 + 0.25 * (q1 - q0), atol=1e-15)
    assert orc.sample_s(0, 1) == 0.0
    for T in (2, 3, 64, 257):
        assert orc.sample_s(0, T) == 0.0 and orc.sample_s(T - 1, T) == 1.0
        for t in range(T):   # nested grids: sample t of T is sample 2t of 2T-1, bit for bit
            assert orc.sample_s(t, T) == orc.sample_s(2 * t, 2 * T - 1)


def test_spline_matches_scipy_clamped_cubic(orc):
    rng = np.random.default_rng(3)
    dof = 6
    for _ in range(5):
        q0, q1 = rng.uniform(-3, 3, dof), rng.uniform(-3, 3, dof)
        via = rng.uniform(-3, 3, (2, dof))
        knots = np.array([0, 1 / 3, 2 / 3, 1])
        ys = np.stack([q0, via[0], via[1], q1])
        cs = CubicSpline(knots, ys, bc_type="clamped", axis=0)
        for s in np.concatenate([np.linspace(0, 1, 37), knots]):
            np.testing.assert_allclose(orc.motion_q("spline", q0, q1, via, s), cs(s), atol=1e-12)


# ------------------------------------------------------------- swept distance

def test_golden_rotating_sphere(orc):
    g = json.load(open(GOLD))["rotating_sphere"]
    arm = arm_from(g["dh"], g["cap_frame"], g["cap_p"], g["cap_r"])
    sdf = orc.exact_sdf(arm, motions_from(g["q0"], g["q1"], g["T"]), np.array(g["points"]))[0]
    np.testing.assert_allclose(sdf, g["sdf"], atol=g["tol"])


def arc_distance(x, R, a0, a1):
    """Distance from x to the planar arc of radius R, angles a0..a1 (a0 < a1), z = 0."""
    rho = math.hypot(x[0], x[1])
    phi = math.atan2(x[1], x[0])
    ends = [np.array([R * math.cos(a), R * math.sin(a), 0.0]) for a in (a0, a1)]
    best = min(np.linalg.norm(np.asarray(x) - e) for e in ends)
    for k in (-1, 0, 1):   # angle of x within the arc (modulo 2 pi)
        if a0 <= phi + 2 * math.pi * k <= a1:
            best = min(best, math.hypot(rho - R, x[2]))
    return best


def test_rotating_sphere_between_continuous_and_bound(orc):
    """1-DOF arm sweeping a sphere along an arc: the continuous swept distance is the
    point-to-arc distance minus r; T samples overestimate it by at most the sagitta
    bound R * dq / (2 (T-1))."""
    R, r = 0.6, 0.05
    arm = arm_from([[R, 0, 0, 0]], [[1, 1]], [[[0, 0, 0], [0, 0, 0]]], [r])
    rng = np.random.default_rng(4)
    pts = rng.uniform(-1, 1, (300, 3))
    for a0, a1, T in [(-0.4, 1.3, 9), (0.2, 2.9, 33), (-2.0, 2.5, 64)]:
        sdf = orc.exact_sdf(arm, motions_from([a0], [a1], T), pts)[0]
        cont = np.array([arc_distance(p, R, a0, a1) - r for p in pts])
        bound = R * (a1 - a0) / (2 * (T - 1))
        assert np.all(sdf >= cont - 1e-12)
        assert np.all(sdf <= cont + bound + 1e-12)


def sector_distance(x, L, a0, a1):
    """Distance from x to the planar sector {rho <= L, a0 <= angle <= a1, z = 0}."""
    rho = math.hypot(x[0], x[1])
    phi = math.atan2(x[1], x[0])
    inside = any(a0 <= phi + 2 * math.pi * k <= a1 for k in (-1, 0, 1))
    if inside:
        return math.hypot(max(rho - L, 0.0), x[2])
    best = math.inf
    for a in (a0, a1):   # distance to the two bounding radial segments
        best = min(best, seg_dist_crossproduct(x, [0, 0, 0], [L * math.cos(a), L * math.sin(a), 0]))
    return best


def test_rotating_radial_capsule_sector(orc):
    L, r = 0.5, 0.04
    arm = arm_from([[L, 0, 0, 0]], [[0, 1]], [[[0, 0, 0], [0, 0, 0]]], [r])
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.8, 0.8, (300, 3))
    a0, a1, T = -0.7, 1.9, 41
    sdf = orc.exact_sdf(arm, motions_from([a0], [a1], T), pts)[0]
    cont = np.array([sector_distance(p, L, a0, a1) - r for p in pts])
    bound = L * (a1 - a0) / (2 * (T - 1))
    assert np.all(sdf >= cont - 1e-12)
    assert np.all(sdf <= cont + bound + 1e-12)


def _reach(arm):
    return float(np.sum(np.abs(arm.dh[:, 0]) + np.abs(arm.dh[:, 2])) + np.abs(arm.cap_p).max() * 2)


def test_dense_brute_force_within_lipschitz_bound(orc):
    """T = 65 samples versus 2^16 + 1: the coarse samples are a subset of the dense
    ones (bit-identical s), so d_dense <= d_T exactly, and d_T - d_dense is at most
    the motion's Lipschitz gap sum_j |dq_j| * reach / (2 (T - 1))."""
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 2, 65, 7)
    pts = svgen.uniform_cube(6, 8)
    coarse = orc.exact_sdf(arm, m, pts)
    dense = orc.exact_sdf(arm, svgen.Motions(m.q0, m.q1, 2**16 + 1), pts)
    assert np.all(dense <= coarse)
    for i in range(m.n):
        gap = np.sum(np.abs(m.q1[i] - m.q0[i])) * _reach(arm) / (2 * 64)
        assert np.all(coarse[i] - dense[i] <= gap)
    assert np.any(coarse > dense)    # the finer grid does find closer positions


def test_nested_grid_monotone_and_special_cases(orc):
    arm = svgen.make_arm(2)
    m = svgen.make_motions(arm, 3, 17, 9)
    pts = svgen.uniform_cube(500, 10)
    d17 = orc.exact_sdf(arm, m, pts)
    d33 = orc.exact_sdf(arm, svgen.Motions(m.q0, m.q1, 33), pts)
    assert np.all(d33 <= d17)
    # q0 == q1: the swept SDF is the static SDF, whatever T
    st = svgen.Motions(m.q0, m.q0, 1)
    s1 = orc.exact_sdf(arm, st, pts)
    for T in (2, 5, 64):
        np.testing.assert_array_equal(orc.exact_sdf(arm, svgen.Motions(m.q0, m.q0, T), pts), s1)
    # static SDF = min over capsules of the independent segment distance
    for i in range(m.n):
        caps = orc.capsules(arm, m.q0[i])
        ref = np.array([min(seg_dist_crossproduct(p, c[0], c[1]) - rk for c, rk in zip(caps, arm.cap_r))
                        for p in pts])
        np.testing.assert_allclose(s1[i], ref, atol=1e-12)
    # lower bound: never deeper than the largest radius
    assert d17.min() >= -arm.cap_r.max() - 1e-15


def test_reversal_rotation_and_lipschitz(orc):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 4, 48, 13)
    pts = svgen.uniform_cube(400, 14)
    d = orc.exact_sdf(arm, m, pts)
    rev = orc.exact_sdf(arm, svgen.Motions(m.q1, m.q0, m.T), pts)
    np.testing.assert_allclose(rev, d, atol=1e-12)
    phi = 0.37
    q0, q1 = m.q0.copy(), m.q1.copy()
    q0[:, 0] += phi
    q1[:, 0] += phi
    Rz = Rotation.from_euler("z", phi).as_matrix()
    rot = orc.exact_sdf(arm, svgen.Motions(q0, q1, m.T), pts @ Rz.T)
    np.testing.assert_allclose(rot, d, atol=1e-12)
    # 1-Lipschitz in x
    rng = np.random.default_rng(15)
    step = rng.normal(size=pts.shape) * 0.01
    d2 = orc.exact_sdf(arm, m, pts + step)
    assert np.all(np.abs(d2 - d) <= np.linalg.norm(step, axis=1) + 1e-12)


def test_check_motions_reduction_and_boundary(orc):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 6, 32, 16)
    pts = svgen.bin_cloud(700, 17)
    sdf = orc.exact_sdf(arm, m, pts)
    md, am, vd = orc.check_motions(arm, m, pts, 0.01)
    np.testing.assert_array_equal(md, sdf.min(axis=1))
    np.testing.assert_array_equal(am, sdf.argmin(axis=1))      # numpy: first index of the minimum
    np.testing.assert_array_equal(vd, (sdf.min(axis=1) <= 0.01).astype(np.uint8))
    # eps exactly at a motion's distance: d <= eps is a collision (free needs d > eps)
    _, _, v_tie = orc.check_motions(arm, svgen.Motions(m.q0[:1], m.q1[:1], m.T), pts, float(md[0]))
    assert v_tie[0] == 1
    _, _, v_up = orc.check_motions(arm, svgen.Motions(m.q0[:1], m.q1[:1], m.T), pts,
                                   float(np.nextafter(md[0], -np.inf)))
    assert v_up[0] == 0
    # duplicated point: the lower index wins
    dup = np.concatenate([pts, pts[am[:1]]])
    _, am2, _ = orc.check_motions(arm, m, dup, 0.01)
    assert am2[0] == am[0]
    # empty cloud: +inf, no argmin, free
    md0, am0, vd0 = orc.check_motions(arm, m, np.zeros((0, 3)), 0.01)
    assert np.all(np.isinf(md0)) and np.all(am0 == -1) and np.all(vd0 == 0)


def test_training_labels_match_cloud_sdf(orc):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 5, 40, 18)
    x = svgen.uniform_cube(5, 19)
    lab = orc.sample_sdf(arm, x, m.q0, m.q1, 40)
    full = orc.exact_sdf(arm, m, x)
    np.testing.assert_array_equal(lab, np.diag(full))
