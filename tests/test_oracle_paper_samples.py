"""Pins of the paper-style sample oracle (oracle/paper_samples.py), CPU only.

- one static capsule (q0 = q1, T = 1): every candidate is accepted and lies at exactly
  the radius from the segment; the share of points on the cylinder is its share of
  the area (binomial bound), axial positions and cap directions are uniform (means);
- surface points of a moving arm have swept distance ~0, rejected candidates lie inside
  another capsule instance (distance < -1e-6);
- Gaussian children: offsets with mean ~0 and standard deviation ~sigma per axis;
  chord points lie on the segment between two surface points of the motion;
- uniform points lie in the box; labels equal the exact oracle's distances.
"""
import math

import numpy as np

import oracle
import svgen
from oracle import paper_samples as ps


def static_capsule_arm(L=0.3, r=0.05):
    dh = np.array([[L, 0.0, 0.0, 0.0]])
    return svgen.Arm(dh=dh, qlim=np.array([[-3.0, 3.0]]), cap_frame=np.array([[0, 1]], np.int32),
                     cap_p=np.zeros((1, 2, 3)), cap_r=np.array([r]))


def seg_dist(p, A, B):
    ab = B - A
    u = np.clip(((p - A) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(p - (A + u[:, None] * ab), axis=1)


def test_static_capsule_surface_is_uniform():
    L, r = 0.3, 0.05
    arm = static_capsule_arm(L, r)
    mo = svgen.Motions(np.array([[0.4]]), np.array([[0.4]]), 1, "linear")
    nc = 4000
    rnd = svgen.uniforms(11, 1, 5 * nc + 8 * nc).ravel()
    rows, n_acc, short = ps.make_samples(arm, mo, 1.0, 0, nc, nc, 0.003, rnd)
    assert n_acc[0] == nc and short == 0
    S = rows[0, :nc, :3]
    A, B = oracle.capsules(arm, np.array([0.4]))[0]
    np.testing.assert_allclose(seg_dist(S, A, B), r, atol=1e-12)
    ab = B - A
    u = ((S - A) @ ab) / (ab @ ab)
    on_cyl = (u > 1e-9) & (u < 1 - 1e-9)
    p = L / (L + 2 * r)
    assert abs(on_cyl.mean() - p) <= 4 * math.sqrt(p * (1 - p) / nc)
    assert abs(u[on_cyl].mean() - 0.5) <= 4 * math.sqrt(1 / 12 / on_cyl.sum())
    caps = S[~on_cyl]
    d = np.where(((caps - A) @ ab < 0)[:, None], caps - A, caps - B) / r
    assert np.all(np.abs(d.mean(axis=0)[[1, 2]]) <= 4 * math.sqrt(1 / 3 / len(d)))   # symmetric about the axis (x)


def test_moving_arm_accepts_only_surface():
    arm = svgen.make_arm(1)
    mo = svgen.make_motions(arm, 2, 12, 5)
    nu, ns, nc, sig = 30, 40, 600, 0.003
    rnd = svgen.uniforms(12, mo.n, 3 * nu + 5 * nc + 8 * ns)
    rows, n_acc, short = ps.make_samples(arm, mo, 0.6, nu, ns, nc, sig, rnd)
    assert short == 0 and np.all(n_acc >= ns) and np.all(n_acc < nc)
    for m in range(mo.n):
        one = svgen.Motions(mo.q0[m:m + 1], mo.q1[m:m + 1], mo.T, "linear")
        R = rows[m]
        U, S, kids = R[:nu], R[nu:nu + ns], R[nu + ns:].reshape(ns, 3, -1)
        assert np.all(np.abs(U[:, :3]) <= 0.6)
        np.testing.assert_allclose(oracle.exact_sdf(arm, one, R[:, :3])[0], R[:, -1], atol=1e-12)
        assert np.all(np.abs(S[:, -1]) <= 1e-6)
        # rejected candidates are inside another instance
        C = rnd[m, 3 * nu:3 * nu + 5 * nc].reshape(nc, 5)
        inst = ps.capsule_instances(arm, mo, m)
        area = np.array([2 * math.pi * rk * np.linalg.norm(Bk - Ak) + 4 * math.pi * rk * rk for Ak, Bk, rk in inst[0]])
        cum = np.cumsum(area)
        P = []
        for c in range(nc):
            k = min(int(np.searchsorted(cum, C[c, 0] * cum[-1], side="right")), arm.n_caps - 1)
            t = min(int(C[c, 1] * mo.T), mo.T - 1)
            P.append(ps.surface_point(*inst[t][k], C[c, 2:5]))
        dC = oracle.exact_sdf(arm, one, np.array(P))[0]
        assert np.all(dC <= 1e-9)                 # every candidate is on or inside the swept volume
        assert np.all(dC[dC.astype(np.float32) < ps.ACCEPT] < -1e-6)
        # chords lie on the segment to another surface point
        for s in range(ns):
            c = kids[s, 2, :3]
            x = S[s, :3]
            others = S[:, :3]
            dev = [np.linalg.norm(np.cross(c - x, o - x)) / max(np.linalg.norm(o - x), 1e-30) if np.linalg.norm(o - x) > 0
                   else np.linalg.norm(c - x) for o in others]
            assert min(dev) <= 1e-12


def test_gaussian_children_statistics():
    L, r, sig = 0.3, 0.05, 0.003
    arm = static_capsule_arm(L, r)
    mo = svgen.Motions(np.array([[0.1]]), np.array([[0.1]]), 1, "linear")
    ns = 3000
    rnd = svgen.uniforms(13, 1, 5 * ns + 8 * ns).ravel()
    rows, _, _ = ps.make_samples(arm, mo, 1.0, 0, ns, ns, sig, rnd)
    S = rows[0, :ns, :3]
    kids = rows[0, ns:, :3].reshape(ns, 3, 3)
    off = np.concatenate([kids[:, 0] - S, kids[:, 1] - S])
    assert np.all(np.abs(off.mean(axis=0)) <= 4 * sig / math.sqrt(len(off)))
    assert np.all(np.abs(off.std(axis=0) / sig - 1) <= 0.05)


def test_box_muller_closed_form():
    n0, n1 = ps.box_muller(1 - math.exp(-0.5), 0.0)       # radius 1, angle 0
    assert abs(n0 - 1.0) < 1e-12 and abs(n1) < 1e-12
    n0, n1 = ps.box_muller(1 - math.exp(-2.0), 0.25)      # radius 2, angle pi/2
    assert abs(n0) < 1e-12 and abs(n1 - 2.0) < 1e-12
