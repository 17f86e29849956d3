"""GPU parity of the paper-style training samples (sv_make_samples_paper) through the C ABI.

Bars, against the FP64 oracle on the same uniforms:
- uniform rows: coordinates within 1e-6 m, labels within 1e-5 m;
- surface rows: the same candidates are chosen (matched by position within 1e-5 m, in
  candidate order) and n_accepted is equal, except in motions where the oracle has a
  decision within FP32 rounding of its threshold (a candidate distance within 5e-7 m of
  the -1e-6 m acceptance bound); labels within 1e-5 m;
- Gaussian and chord rows: coordinates equal the recipe applied to the GPU's own
  surface rows within 1e-6 m, labels equal the oracle's distance of those points within
  1e-5 m;
- the row layout (joint columns) and host checks.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import svgen
from oracle import paper_samples as ps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def run(sv, robot, mo, half, nu, ns, nc, sigma, rnd):
    dm = sv.DeviceMotions(mo)
    width = 3 + 2 * mo.q0.shape[1] + 1
    out = torch.full((mo.n, nu + 4 * ns, width), float("nan"), device="cuda")
    n_acc = torch.zeros(mo.n, dtype=torch.int32, device="cuda")
    short = torch.zeros(1, dtype=torch.int32, device="cuda")
    sv.sv_make_samples_paper(robot, dm, half, nu, ns, nc, sigma, torch.as_tensor(rnd, device="cuda"), out, n_acc,
                             short)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), n_acc.cpu().numpy(), int(short.item())


@pytest.mark.parametrize("T,nu,ns,nc", [(24, 40, 50, 1500), (7, 5, 8, 300), (64, 0, 30, 3000)])
def test_paper_samples_against_oracle(sv, T, nu, ns, nc):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, 4, T, 1000 + T)
    half, sigma = 0.6, 0.003
    rnd = svgen.uniforms(1001 + T, mo.n, 3 * nu + 5 * nc + 8 * ns)
    got, n_acc, short = run(sv, robot, mo, half, nu, ns, nc, sigma, rnd)
    ref, ref_acc, ref_short = ps.make_samples(arm, mo, half, nu, ns, nc, sigma, rnd)
    dof = arm.dof
    np.testing.assert_allclose(got[:, :, 3:3 + dof], np.repeat(mo.q0[:, None, :], nu + 4 * ns, 1), rtol=0, atol=0)
    borderline = 0
    for m in range(mo.n):
        one = svgen.Motions(mo.q0[m:m + 1], mo.q1[m:m + 1], T, "linear")
        G, R = got[m], ref[m]
        np.testing.assert_allclose(G[:nu, :3], R[:nu, :3], atol=1e-6)
        np.testing.assert_allclose(G[:nu, -1], R[:nu, -1], atol=1e-5)
        # candidates of the oracle, to tell borderline motions
        C = np.asarray(rnd[m, 3 * nu:3 * nu + 5 * nc], np.float64).reshape(nc, 5)
        inst = ps.capsule_instances(arm, mo, m)
        area = np.array([2 * math.pi * rk * np.linalg.norm(B - A) + 4 * math.pi * rk * rk for A, B, rk in inst[0]])
        cum = np.cumsum(area)
        P = np.array([ps.surface_point(*inst[min(int(C[c, 1] * T), T - 1)][
            min(int(np.searchsorted(cum, C[c, 0] * cum[-1], side="right")), arm.n_caps - 1)], C[c, 2:5])
                      for c in range(nc)])
        dC = oracle.exact_sdf(arm, one, P)[0]
        if np.any(np.abs(dC + 1e-6) < 5e-7):   # within the FP32 error of a distance from the bound
            borderline += 1
            continue
        assert n_acc[m] == ref_acc[m]
        S = G[nu:nu + ns]
        np.testing.assert_allclose(S[:, :3], R[nu:nu + ns, :3], atol=1e-5)
        np.testing.assert_allclose(S[:, -1], R[nu:nu + ns, -1], atol=1e-5)
        # children from the GPU's own surface rows
        K = G[nu + ns:].reshape(ns, 3, -1)
        Rs = np.asarray(rnd[m, 3 * nu + 5 * nc:], np.float64).reshape(ns, 8)
        for s in range(ns):
            n = [*ps.box_muller(Rs[s, 0], Rs[s, 1]), *ps.box_muller(Rs[s, 2], Rs[s, 3]),
                 *ps.box_muller(Rs[s, 4], Rs[s, 5])]
            np.testing.assert_allclose(K[s, 0, :3], S[s, :3] + sigma * np.array(n[0:3]), atol=1e-6)
            np.testing.assert_allclose(K[s, 1, :3], S[s, :3] + sigma * np.array(n[3:6]), atol=1e-6)
            p = min(int(Rs[s, 6] * ns), ns - 1)
            np.testing.assert_allclose(K[s, 2, :3], S[s, :3] + Rs[s, 7] * (S[p, :3] - S[s, :3]), atol=1e-6)
        kd = oracle.exact_sdf(arm, one, K[:, :, :3].reshape(-1, 3))[0]
        np.testing.assert_allclose(K[:, :, -1].ravel(), kd, atol=1e-5)
    assert borderline <= 1, f"{borderline} borderline motions"
    if borderline == 0:
        assert short == ref_short


def test_paper_samples_host_checks(sv):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, 2, 8, 1100)
    rnd = torch.zeros((2, 3 * 4 + 5 * 3 + 8 * 4), device="cuda")
    out = torch.zeros((2, 4 + 16, 16), device="cuda")
    with pytest.raises(sv.SvError) as e:
        sv.sv_make_samples_paper(robot, sv.DeviceMotions(mo), 0.6, 4, 4, 3, 0.003, rnd, out)   # n_cand < n_surface
    assert e.value.status == -1
    spl = svgen.make_motions(arm, 2, 8, 1101, "spline")
    with pytest.raises(sv.SvError) as e:
        sv.sv_make_samples_paper(robot, sv.DeviceMotions(spl), 0.6, 4, 4, 8, 0.003, rnd, out)
    assert e.value.status == -4
