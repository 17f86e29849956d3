"""The culled exact passes of sv_check_motions against the unculled kernels.

Skipped test groups are proven to exceed the motion's minimum, so min_dist, argmin
and verdict must be bit-identical with culling on and off: on the bin-picking
workload (linear and spline motions), with duplicated points (exact ties), tiny and
ragged clouds, and in screening (the check of the sent points and certified
screening's confirmation pass are culled).  The
sample blocks follow T and the motion kind (2 to 16 samples: about T / 32 for linear
motions, T / 64 for splines), so the cases span every block length regime, including
the largest block count below T = 1024 (a spline at T = 256: 64 blocks of 4).  The
oracle checks a sample of the culled results directly.
"""
import numpy as np
import pytest
import torch

import svgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def check(sv, arm, motions, pts, eps, cull, mlp=None, screen=0, tau=0.0):
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    out = sv.DeviceResults(dm.n)
    ws = sv.sv_check_motions(sv.make_robot(arm), dm, dc, out, eps, mlp=mlp, screen=screen, tau=tau,
                             unculled=not cull)
    torch.cuda.synchronize()
    return (out.min_dist.cpu().numpy(), out.argmin.cpu().numpy(), out.verdict.cpu().numpy(),
            sv.executed_tests(ws))


def assert_same(a, b):
    np.testing.assert_array_equal(a[0].view(np.int32), b[0].view(np.int32))
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("kind,T,M,N", [("linear", 256, 64, 20000), ("spline", 100, 24, 7000),
                                        ("linear", 33, 16, 513), ("spline", 2, 9, 130), ("linear", 1, 5, 3),
                                        ("linear", 47, 12, 2000), ("linear", 64, 20, 3000),
                                        ("spline", 200, 8, 1500), ("linear", 300, 6, 1100),
                                        ("spline", 256, 6, 1200)])
def test_culled_equals_unculled(sv, orc, kind, T, M, N):
    arm = svgen.make_arm(1)
    motions = svgen.make_motions(arm, M, T, 400 + T, kind)
    pts = svgen.bin_cloud(N, 401 + T)
    on = check(sv, arm, motions, pts, 0.01, True)
    off = check(sv, arm, motions, pts, 0.01, False)
    assert_same(on, off)
    full = M * ((N + 511) // 512) * 512 * T * arm.n_caps
    print(f"{kind} T={T} M={M} N={N}: executed {on[3] / full:.3f} of the tests")
    idx = np.arange(0, M, max(1, M // 4))
    sub = svgen.Motions(motions.q0[idx], motions.q1[idx], T, kind, None if motions.via is None else motions.via[idx])
    ref, _, rv = orc.check_motions(arm, sub, pts, 0.01)
    assert np.abs(on[0][idx] - ref).max() <= 1e-5
    np.testing.assert_array_equal(on[2][idx], rv)


def test_culled_ties_and_full_workload(sv):
    arm = svgen.make_arm(1)
    w = svgen.WORKLOADS["bin20k"]
    motions = svgen.make_motions(arm, w["n_motions"], w["T"], w["motion_seed"])
    pts = svgen.bin_cloud(w["n_points"], w["cloud_seed"])
    on = check(sv, arm, motions, pts, w["eps"], True)
    off = check(sv, arm, motions, pts, w["eps"], False)
    assert_same(on, off)
    print(f"bin20k: executed {on[3] / (512 * 20480 * 256 * 7):.4f} of the tests")
    dup = np.concatenate([pts[:3000], pts[:3000]])          # every point twice: lowest index wins
    a = check(sv, arm, svgen.Motions(motions.q0[:32], motions.q1[:32], 64), dup, 0.01, True)
    b = check(sv, arm, svgen.Motions(motions.q0[:32], motions.q1[:32], 64), dup, 0.01, False)
    assert_same(a, b)
    assert np.all(a[1] < 3000)


def test_culled_confirmation_in_certified_screening(sv):
    arm = svgen.make_arm(1)
    motions = svgen.make_motions(arm, 48, 64, 420)
    pts = svgen.bin_cloud(5000, 421)
    spec = svgen.MLPSpec(15, 128, 3)
    mlp = sv.DeviceMLP(svgen.mlp_init(spec, 422), 15, 128, 3)
    on = check(sv, arm, motions, pts, 0.01, True, mlp=mlp, screen=sv.SV_SCREEN_CERTIFIED, tau=0.03)
    off = check(sv, arm, motions, pts, 0.01, False, mlp=mlp, screen=sv.SV_SCREEN_CERTIFIED, tau=0.03)
    assert_same(on, off)
    ex = check(sv, arm, motions, pts, 0.01, False)
    np.testing.assert_array_equal(on[2], ex[2])


@pytest.mark.parametrize("T,M,N,q", [(64, 40, 4000, 0.3), (33, 24, 2100, 0.6), (256, 8, 1500, 0.1)])
def test_culled_fallback_of_screening(sv, T, M, N, q):
    """The exact check of the points a screen sends runs culled over the Morton-sorted
    cloud (from min(eps - band, current minimum) in certified mode, from the current
    minimum in trust mode).  Both modes must give the unculled kernels' results bit for
    bit: minima over the sent points and their lowest caller indices (every sent point
    duplicated once: exact ties), verdicts and fallback counts.  tau is the q quantile of
    the predictions, so that a share of the points is sent and some motions have a
    witness and some do not."""
    arm = svgen.make_arm(1)
    motions = svgen.make_motions(arm, M, T, 430 + T)
    base = svgen.bin_cloud(N // 2, 431 + T)
    pts = np.concatenate([base, base[: N - N // 2]])
    mlp = sv.DeviceMLP(svgen.mlp_init(svgen.MLPSpec(15, 128, 3), 432), 15, 128, 3)
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    pred = torch.empty(M, pts.shape[0], device="cuda")
    sv.sv_nn_sdf(mlp, sv.SV_BF16, dm, dc, pred)
    tau = float(torch.quantile(pred.flatten()[:1 << 20], q).item())
    robot = sv.make_robot(arm)
    for mode in (sv.SV_SCREEN_TRUST, sv.SV_SCREEN_CERTIFIED):
        res = []
        for unculled in (False, True):
            out = sv.DeviceResults(dm.n)
            sv.sv_check_motions(robot, dm, dc, out, 0.01, mlp=mlp, screen=mode, tau=tau, unculled=unculled)
            torch.cuda.synchronize()
            res.append((out.min_dist.cpu().numpy(), out.argmin.cpu().numpy(), out.verdict.cpu().numpy(),
                        out.n_fallback.cpu().numpy()))
        on, off = res
        assert_same(on, off)
        np.testing.assert_array_equal(on[3], off[3])
        sent = on[3] > 0
        print(f"T={T} M={M} N={N} mode {mode}: {sent.sum()} motions with sent points, "
              f"{int((on[2] == 1).sum())} colliding, fallback fraction {on[3].sum() / (M * pts.shape[0]):.3f}")
        assert sent.any()
    ex = check(sv, arm, motions, pts, 0.01, False)
    np.testing.assert_array_equal(on[2], ex[2])   # certified verdicts are the exact check's
