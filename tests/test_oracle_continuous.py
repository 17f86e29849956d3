"""Pins of the continuous-certification oracle (oracle/continuous.py), CPU only.

- link lengths against the distances between consecutive frame origins of the FK
  oracle at random configurations;
- spline speed maxima against central differences of the oracle's own spline
  evaluation (which is pinned against scipy elsewhere), and the interior slopes;
- the bound itself: on random linear and spline motions the sampled distance never
  exceeds the distance at 16x finer sampling by more than the gap;
- a closed form: one link of length l turning by dq, radius 0, a point on the tip's
  circle half-way between two samples: sampled distance l sin(dq / (2 (T-1))), gap
  l dq / (2 (T-1)), continuous distance 0.
"""
import numpy as np
import pytest

import oracle
import svgen
from oracle import continuous as oc


def test_link_lengths_match_fk():
    arm = svgen.make_arm(1)
    g = np.random.default_rng(1)
    l = oc.link_lengths(arm)
    for _ in range(5):
        q = g.uniform(arm.qlim[:, 0], arm.qlim[:, 1])
        F = oracle.frames(arm, q)
        d = np.linalg.norm(F[1:, :, 3] - F[:-1, :, 3], axis=1)
        np.testing.assert_allclose(d, l, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_spline_speed_against_differences(seed):
    arm = svgen.make_arm(1)
    mo = svgen.make_motions(arm, 1, 8, seed, "spline")
    q0, q1, via = mo.q0[0], mo.q1[0], mo.via[0]
    s = np.linspace(0.0, 1.0, 30001)
    Q = np.array([oracle.motion_q("spline", q0, q1, via, si) for si in s])
    dq = np.diff(Q, axis=0) / np.diff(s)[:, None]
    fd_max = np.abs(dq).max(axis=0)
    bound = oc.joint_speed_max("spline", q0, q1, via)
    assert np.all(fd_max <= bound * (1 + 1e-9) + 1e-9)          # never above the maximum
    assert np.all(fd_max >= bound * (1 - 1e-3) - 1e-6)          # and attained up to the grid
    # interior slopes equal the spline's derivative at the knots
    for j in range(arm.dof):
        m = oc.spline_slopes(np.array([q0[j], via[0, j], via[1, j], q1[j]]))
        for knot, mk in zip((1 / 3, 2 / 3), m[1:3]):
            e = 1e-6
            d = (oracle.motion_q("spline", q0, q1, via, knot + e)[j] - oracle.motion_q("spline", q0, q1, via, knot - e)[j]) / (2 * e)
            assert abs(d - mk) <= 1e-5 * (1 + abs(mk))


@pytest.mark.parametrize("kind", ["linear", "spline"])
def test_gap_bounds_finer_sampling(kind):
    arm = svgen.make_arm(1)
    T = 9
    mo = svgen.make_motions(arm, 6, T, 40, kind)
    fine = svgen.Motions(mo.q0, mo.q1, 16 * (T - 1) + 1, kind, mo.via)
    pts = svgen.bin_cloud(400, 41)
    dT = oracle.exact_sdf(arm, mo, pts)
    dF = oracle.exact_sdf(arm, fine, pts)
    gap = oc.gaps(arm, mo)
    excess = (dT - dF).max(axis=1)
    assert np.all(excess >= -1e-12)          # the fine grid contains the coarse samples
    assert np.all(excess <= gap)
    print(f"{kind}: excess / gap = {np.round(excess / gap, 3)}")


def test_rotating_link_closed_form():
    l, dq, T = 0.4, 0.6, 5
    arm = svgen.Arm(dh=np.array([[l, 0.0, 0.0, 0.0]]), qlim=np.array([[-3.0, 3.0]]),
                    cap_frame=np.array([[0, 1]], np.int32), cap_p=np.zeros((1, 2, 3)), cap_r=np.zeros(1))
    mo = svgen.Motions(np.array([[0.0]]), np.array([[dq]]), T, "linear")
    step = dq / (T - 1)
    phi = step / 2.0                               # half-way between samples 0 and 1
    x = np.array([[l * np.cos(phi), l * np.sin(phi), 0.0]])
    d = oracle.exact_sdf(arm, mo, x)[0, 0]
    assert abs(d - l * np.sin(phi)) <= 1e-12
    gap = oc.gaps(arm, mo)[0]
    assert abs(gap - l * dq / (2 * (T - 1))) <= 1e-15
    assert d - gap <= 0.0 <= d                     # the continuous distance (0) lies in [d - gap, d]
