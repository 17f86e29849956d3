"""FP64 oracle of the gap between the sampled and the continuous swept-volume distance.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The swept volume is a union over the continuous path parameter s in [0, 1] (Sec. III,
eq. (3)); the exact check evaluates it at T samples s_t = t / (T - 1).  Every s lies
within h = 1 / (2 (T - 1)) of a sample (h = 1 for T = 1).  If every point of capsule k
moves at most L_k per unit of s, the distance of any point x to capsule k changes at
most L_k per unit of s, so the continuous distance is at least the sampled one minus
L_k h.  With L = max_k L_k:

    d_cont(x, m) >= d_T(x, m) - gap(m),    gap(m) = L h.

Speed bound (standard DH, joint j turns about the z axis of frame j-1 through its
origin O_{j-1}): a point fixed in frame f >= j moves under joint j at speed |dq_j/ds|
times its distance from that axis, which is at most its distance from O_{j-1}, at most
sum_{i=j..f} l_i + |p| (l_i = |O_i - O_{i-1}| = sqrt(a_i^2 + d_i^2), p the point's
coordinates in frame f).  A capsule's segment points are convex combinations of its
two endpoints, so its speed is at most the larger endpoint speed.

max_s |dq_j/ds|: |q1_j - q0_j| for a linear motion; for the spline, the derivative
of each cubic segment is a quadratic in the segment parameter, whose largest magnitude
on the segment is at an end or at its vertex.
"""
from __future__ import annotations

import numpy as np


def link_lengths(arm) -> np.ndarray:
    """l_i = |O_i - O_{i-1}| for i = 1..dof (constant for a DH chain)."""
    return np.hypot(arm.dh[:, 0], arm.dh[:, 2])


def spline_slopes(y):
    """Interior slopes (in s) of the clamped C2 cubic through y[0..3] at s = 0, 1/3,
    2/3, 1: continuity of the second derivative at the two interior knots gives a 2x2
    linear system (end slopes are zero)."""
    h = 1.0 / 3.0
    A = np.array([[4.0, 1.0], [1.0, 4.0]])
    rhs = np.array([3.0 * (y[2] - y[0]) / h, 3.0 * (y[3] - y[1]) / h])
    m1, m2 = np.linalg.solve(A, rhs)
    return np.array([0.0, m1, m2, 0.0])


def joint_speed_max(kind, q0, q1, via=None) -> np.ndarray:
    """max over s of |dq_j/ds| per joint."""
    q0, q1 = np.asarray(q0, np.float64), np.asarray(q1, np.float64)
    if kind == "linear":
        return np.abs(q1 - q0)
    via = np.asarray(via, np.float64)
    h = 1.0 / 3.0
    out = np.zeros(len(q0))
    for j in range(len(q0)):
        y = np.array([q0[j], via[0, j], via[1, j], q1[j]])
        m = spline_slopes(y)
        best = 0.0
        for seg in range(3):
            # Hermite segment in u in [0, 1], s = (seg + u) h:
            # q(u) = h00 y_a + h10 h m_a + h01 y_b + h11 h m_b; dq/ds = (dq/du) / h
            ya, yb, ma, mb = y[seg], y[seg + 1], h * m[seg], h * m[seg + 1]
            a = 6.0 * (ya - yb) + 3.0 * (ma + mb)
            b = 6.0 * (yb - ya) - 4.0 * ma - 2.0 * mb
            c = ma
            cands = [c, a + b + c]
            if a != 0.0 and 0.0 < -b / (2.0 * a) < 1.0:
                u = -b / (2.0 * a)
                cands.append(a * u * u + b * u + c)
            best = max(best, max(abs(v) for v in cands) / h)
        out[j] = best
    return out


def capsule_speeds(arm, omega) -> np.ndarray:
    """L_k for every capsule, given omega_j = max |dq_j/ds|."""
    l = link_lengths(arm)
    L = np.zeros(arm.n_caps)
    for k in range(arm.n_caps):
        best = 0.0
        for e in range(2):
            f = int(arm.cap_frame[k][e])
            p = float(np.linalg.norm(arm.cap_p[k][e]))
            v = sum(omega[j - 1] * (l[j - 1:f].sum() + p) for j in range(1, f + 1))
            best = max(best, v)
        L[k] = best
    return L


def half_spacing(T: int) -> float:
    return 1.0 / (2.0 * (T - 1)) if T > 1 else 1.0


def gaps(arm, motions) -> np.ndarray:
    """gap(m) for every motion of an svgen.Motions set."""
    out = np.zeros(motions.n)
    for m in range(motions.n):
        via = None if motions.via is None else motions.via[m]
        omega = joint_speed_max(motions.kind, motions.q0[m], motions.q1[m], via)
        out[m] = capsule_speeds(arm, omega).max() * half_spacing(motions.T)
    return out
