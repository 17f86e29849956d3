"""FP64 oracle of the paper-style training samples (Sec. IV-C, dataset generation).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The paper labels points against a swept-volume mesh; here the swept volume is the
union of the robot's capsules at the T samples of the motion, whose signed distance the
exact check gives.  Per motion:

1. n_uniform points uniform in the box [-h, h]^3 (the paper: a fixed box covering any
   motion, 0.25 points per dm^3);
2. points on the swept surface (the paper: 0.2 per cm^2).  Candidates are drawn
   uniformly over the total area of all capsule instances (capsule k with probability
   proportional to its area, sample t uniformly, then a point uniform on that capsule's
   surface: the cylinder or the two hemispherical caps, in proportion to their areas).
   A candidate lies on the swept surface iff no other instance contains it, i.e. iff
   its swept distance is 0 (accepted: FP32 distance >= -1e-6 m).  Every piece of the
   surface belongs to exactly one instance's surface, so the accepted candidates are
   uniform on the swept surface.  The first n_surface accepted candidates in candidate
   order are kept (if fewer are accepted, the first rejected ones fill the rest and
   are counted as short);
3. for each surface point two points from a spherical Gaussian around it (sigma; the
   paper: 3 mm), from Box-Muller on the supplied uniforms;
4. for each surface point another of the motion's surface points at random and a point
   uniform on the segment between them (the paper's cover of the interior).

Every random number comes from `rnd` (per motion: 3 per uniform point, 5 per candidate,
8 per surface point, in that order), so the GPU and this oracle draw the same samples.
Rows: [x, y, z, q0, q1, delta]; per motion uniform rows, then the surface rows, then
for each surface point its two Gaussian rows and its chord row.
"""
from __future__ import annotations

import math

import numpy as np

from . import capsules as _capsules
from . import exact_sdf as _exact_sdf
from . import motion_q as _motion_q
from . import sample_s as _sample_s

ACCEPT = np.float32(-1e-6)


def _one_motion(motions, m):
    import svgen
    via = None if motions.via is None else motions.via[m:m + 1]
    return svgen.Motions(motions.q0[m:m + 1], motions.q1[m:m + 1], motions.T, motions.kind, via)


def capsule_instances(arm, motions, m):
    """[T][K] (A, B, r) world capsules of motion m at its samples."""
    via = None if motions.via is None else motions.via[m]
    out = []
    for t in range(motions.T):
        q = _motion_q(motions.kind, motions.q0[m], motions.q1[m], via, _sample_s(t, motions.T))
        caps = _capsules(arm, q)
        out.append([(caps[k, 0], caps[k, 1], float(arm.cap_r[k])) for k in range(arm.n_caps)])
    return out


def surface_point(A, B, r, u):
    """A point of the capsule (A, B, r) surface from 4 uniforms: u[0] chooses the cylinder
    (probability L / (L + 2r), its share of the area) or the caps; then either the axial
    position u[1] and the angle 2 pi u[2] on the cylinder, or a direction uniform on the
    sphere (cos theta = 2 u[1] - 1, phi = 2 pi u[2]) around A or B (the end it points
    away from the segment at)."""
    u = np.asarray(u, np.float64)   # FP64 arithmetic whatever the uniforms' type
    A, B, r = np.asarray(A, np.float64), np.asarray(B, np.float64), float(r)
    ab = B - A
    L = float(np.linalg.norm(ab))
    pc = L / (L + 2.0 * r) if L + 2.0 * r > 0 else 0.0
    if u[0] < pc:
        a = ab / L
        h = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(a, h)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(a, e1)
        phi = 2.0 * math.pi * u[2]
        return A + u[1] * ab + r * (math.cos(phi) * e1 + math.sin(phi) * e2)
    cz = 2.0 * u[1] - 1.0
    sz = math.sqrt(max(0.0, 1.0 - cz * cz))
    phi = 2.0 * math.pi * u[2]
    d = np.array([sz * math.cos(phi), sz * math.sin(phi), cz])
    centre = B if (L > 0 and float(d @ ab) > 0) else A
    return centre + r * d


def box_muller(u1, u2):
    """Two standard normals from two uniforms in [0, 1) (1 - u1 keeps the log finite)."""
    u1, u2 = float(u1), float(u2)
    rad = math.sqrt(-2.0 * math.log(1.0 - u1))
    return rad * math.cos(2.0 * math.pi * u2), rad * math.sin(2.0 * math.pi * u2)


def make_samples(arm, motions, box_half, n_uniform, n_surface, n_cand, sigma, rnd):
    """(rows [M][n_uniform + 4 n_surface][in_dim + 1], n_accepted [M], n_short)."""
    M, T, K = motions.n, motions.T, arm.n_caps
    rnd = np.asarray(rnd, np.float64).reshape(M, 3 * n_uniform + 5 * n_cand + 8 * n_surface)
    dof = arm.dof
    rows = np.zeros((M, n_uniform + 4 * n_surface, 3 + 2 * dof + 1))
    n_acc = np.zeros(M, np.int64)
    n_short = 0
    for m in range(M):
        r = rnd[m]
        one = _one_motion(motions, m)
        inst = capsule_instances(arm, motions, m)
        # 1. uniform points
        U = box_half * (2.0 * r[:3 * n_uniform].reshape(n_uniform, 3) - 1.0)
        # 2. candidates over the capsule instances, by area
        area = np.array([2 * math.pi * rk * np.linalg.norm(B - A) + 4 * math.pi * rk * rk for A, B, rk in inst[0]])
        cum = np.cumsum(area)
        C = r[3 * n_uniform:3 * n_uniform + 5 * n_cand].reshape(n_cand, 5)
        P = np.zeros((n_cand, 3))
        for c in range(n_cand):
            k = min(int(np.searchsorted(cum, C[c, 0] * cum[-1], side="right")), K - 1)
            t = min(int(C[c, 1] * T), T - 1)
            A, B, rk = inst[t][k]
            P[c] = surface_point(A, B, rk, C[c, 2:5])
        dC = _exact_sdf(arm, one, P)[0] if n_cand else np.zeros(0)
        ok = dC.astype(np.float32) >= ACCEPT
        n_acc[m] = int(ok.sum())
        chosen = list(np.flatnonzero(ok)[:n_surface])
        if len(chosen) < n_surface:
            n_short += n_surface - len(chosen)
            chosen += list(np.flatnonzero(~ok)[:n_surface - len(chosen)])
        S, dS = P[chosen], dC[chosen]
        # 3, 4. Gaussian and chord points
        R = r[3 * n_uniform + 5 * n_cand:].reshape(n_surface, 8)
        kids = np.zeros((n_surface, 3, 3))
        for s in range(n_surface):
            n0, n1 = box_muller(R[s, 0], R[s, 1])
            n2, n3 = box_muller(R[s, 2], R[s, 3])
            n4, n5 = box_muller(R[s, 4], R[s, 5])
            kids[s, 0] = S[s] + sigma * np.array([n0, n1, n2])
            kids[s, 1] = S[s] + sigma * np.array([n3, n4, n5])
            p = min(int(R[s, 6] * n_surface), n_surface - 1)
            kids[s, 2] = S[s] + R[s, 7] * (S[p] - S[s])
        pts = np.concatenate([U, S, kids.reshape(-1, 3)])
        d = np.concatenate([_exact_sdf(arm, one, U)[0] if n_uniform else np.zeros(0), dS,
                            _exact_sdf(arm, one, kids.reshape(-1, 3))[0] if n_surface else np.zeros(0)])
        rows[m, :, 0:3] = pts
        rows[m, :, 3:3 + dof] = motions.q0[m]
        rows[m, :, 3 + dof:3 + 2 * dof] = motions.q1[m]
        rows[m, :, -1] = d
    return rows, n_acc, n_short
