"""GPU parity of the swept-volume network (sv_nn_sdf) and of screened checking
(sv_check_motions with a network) against the oracle, through the C ABI.

Bars:
  FP32 path: |y - y_ref| <= 1e-4 |y_ref| + 1e-4 rms(y_ref) per element (FP64 oracle).
  BF16 path: against the FP64 network, |y - y64| <= bar per output, the a-priori bar of
    oracle/bf16_error.py (first-order sum over every BF16 and FP32 rounding site with
    Hoeffding's inequality at lam = 7, from the BF16 unit roundoff 2^-8); against the
    oracle's emulation of the same rounding points, |y - y_bf| <= bar per output and the
    median |y - y_bf| / bar <= 0.005 (each misplaced rounding point moves it above 0.01).
  Screening: certified verdicts equal the exact oracle's bit for bit; tau = +inf
    reproduces the exact check bit for bit.
"""
import numpy as np
import pytest
import torch

import svgen
from oracle import bf16_error as be
from oracle import mlp as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def net_inputs(motions, pts):
    """[M*N][15] oracle input rows in (motion, point) order."""
    M, N = motions.n, pts.shape[0]
    x = np.tile(pts, (M, 1))
    q0 = np.repeat(motions.q0, N, axis=0)
    q1 = np.repeat(motions.q1, N, axis=0)
    return om.features(x, q0, q1)


def run_nn(sv, flat, shape, motions, pts, precision):
    dmlp = sv.DeviceMLP(flat, *shape)
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    out = torch.full((dm.n, dc.n), float("nan"), device="cuda")
    sv.sv_nn_sdf(dmlp, precision, dm, dc, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def rel_ok(y, ref, rtol=1e-4):
    rms = np.sqrt(np.mean(ref ** 2))
    return np.all(np.abs(y - ref) <= rtol * np.abs(ref) + rtol * rms)


def test_nn_fp32_tiny_workload(sv):
    """15 -> 4 x 256 softplus -> 1, seeded random init, 4096 cube points, one motion."""
    w = svgen.WORKLOADS["tiny"]
    arm = svgen.make_arm(w["arm_seed"])
    m = svgen.make_motions(arm, w["n_motions"], w["T"], w["motion_seed"])
    pts = svgen.uniform_cube(w["n_points"], w["cloud_seed"])
    shape = w["mlp"]
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), w["mlp_seed"])
    y = run_nn(sv, flat, shape, m, pts, sv.SV_FP32)
    ref, _ = om.forward(flat, *shape, net_inputs(m, pts))
    err = np.abs(y.ravel() - ref)
    print(f"fp32 tiny: max abs err {err.max():.2e}, max rel {np.max(err / np.abs(ref)):.2e}")
    assert rel_ok(y.ravel(), ref)


@pytest.mark.parametrize("shape,M,N", [((15, 64, 1), 3, 100), ((15, 512, 8), 2, 777), ((15, 128, 3), 5, 17),
                                       ((15, 1024, 2), 1, 40)])
def test_nn_fp32_shapes(sv, shape, M, N):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, M, 8, 100 + N)
    pts = svgen.bin_cloud(N, 101 + N)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 102)
    y = run_nn(sv, flat, shape, m, pts, sv.SV_FP32)
    ref, _ = om.forward(flat, *shape, net_inputs(m, pts))
    assert rel_ok(y.ravel(), ref)


@pytest.mark.parametrize("shape,M,N", [((15, 512, 8), 3, 3000), ((15, 256, 4), 4, 129), ((15, 128, 1), 2, 64),
                                       ((15, 512, 2), 1, 1), ((15, 1024, 3), 2, 200), ((15, 1024, 1), 1, 65)])
def test_nn_bf16_matches_rounding_oracle(sv, shape, M, N):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, M, 8, 200 + N)
    pts = svgen.bin_cloud(N, 201 + N)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 202)
    y = run_nn(sv, flat, shape, m, pts, sv.SV_BF16).ravel()
    X = net_inputs(m, pts)
    ref_bf = om.forward_bf16(flat, *shape, X)
    ref64, bar = be.mlp_bar(flat, *shape, X)
    ok, rep = be.compare(y, ref_bf, ref64, bar)
    print(f"bf16 {shape}: {rep}")
    assert ok, rep


def _screen_case(seed, M=24, N=2500, T=48):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, M, T, seed)
    pts = svgen.bin_cloud(N, seed + 1)
    shape = (15, 512, 8)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), seed + 2)
    return arm, m, pts, shape, flat


def run_screen(sv, arm, m, pts, shape, flat, mode, eps, tau):
    dm, dc = sv.DeviceMotions(m), sv.DeviceCloud(pts)
    out = sv.DeviceResults(dm.n)
    mlp = sv.DeviceMLP(flat, *shape) if mode else None
    sv.sv_check_motions(sv.make_robot(arm), dm, dc, out, eps, mlp=mlp, screen=mode, tau=tau)
    torch.cuda.synchronize()
    return (out.min_dist.cpu().numpy(), out.argmin.cpu().numpy(), out.verdict.cpu().numpy(),
            out.n_fallback.cpu().numpy())


def test_screen_tau_inf_reproduces_exact(sv):
    arm, m, pts, shape, flat = _screen_case(300)
    ex = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_NONE, 0.01, 0.0)
    for mode in (sv.SV_SCREEN_TRUST, sv.SV_SCREEN_CERTIFIED):
        sc = run_screen(sv, arm, m, pts, shape, flat, mode, 0.01, float("inf"))
        for a, b in zip(ex[:3], sc[:3]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(sc[3], pts.shape[0])


def test_screen_certified_verdicts_equal_oracle(sv, orc):
    """Random-init network (its predictions are poor): certified screening must still
    give the exact verdicts; trust mode's agreement is reported."""
    arm, m, pts, shape, flat = _screen_case(310)
    eps, tau = 0.01, 0.03
    ref_md, _, ref_vd = orc.check_motions(arm, m, pts, eps)
    md, am, vd, nf = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_CERTIFIED, eps, tau)
    np.testing.assert_array_equal(vd, ref_vd)
    free = ref_vd == 0
    assert np.abs(md[free] - ref_md[free]).max() <= 1e-5        # free motions: exact over all points
    assert np.all(md[~free] <= eps)                              # colliding motions: a witness
    tmd, _, tvd, tnf = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_TRUST, eps, tau)
    np.testing.assert_array_equal(tnf, nf)
    print(f"trust-mode verdict agreement {np.mean(tvd == ref_vd):.3f}; mean fallback fraction "
          f"{nf.mean() / pts.shape[0]:.3f}")


def test_screen_fallback_sets_follow_predictions(sv):
    """The points sent to the exact check are those with delta_hat < tau: counts match
    the BF16-rounding oracle except for points within their error bar of tau, where the
    GPU's FP32 arithmetic may decide either way."""
    arm, m, pts, shape, flat = _screen_case(320, M=6, N=1500)
    X = net_inputs(m, pts)
    yb = om.forward_bf16(flat, *shape, X).reshape(m.n, -1)
    bar = be.mlp_bar(flat, *shape, X)[1].reshape(m.n, -1)
    tau = float(np.median(yb))
    _, _, _, nf = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_TRUST, 0.01, tau)
    lo = np.sum(yb < tau - bar, axis=1)
    hi = np.sum(yb < tau + bar, axis=1)
    assert np.all((lo <= nf) & (nf <= hi)), (lo, nf, hi)


def test_screen_tau_minus_inf(sv, orc):
    arm, m, pts, shape, flat = _screen_case(330, M=8, N=800)
    md, am, vd, nf = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_TRUST, 0.01, float("-inf"))
    assert np.all(nf == 0) and np.all(vd == 0) and np.all(np.isinf(md)) and np.all(am == -1)
    md, am, vd, nf = run_screen(sv, arm, m, pts, shape, flat, sv.SV_SCREEN_CERTIFIED, 0.01, float("-inf"))
    _, _, ref_vd = orc.check_motions(arm, m, pts, 0.01)
    np.testing.assert_array_equal(vd, ref_vd)


def test_screen_empty_cloud(sv):
    arm, m, _, shape, flat = _screen_case(340, M=4, N=10)
    for mode in (sv.SV_SCREEN_TRUST, sv.SV_SCREEN_CERTIFIED):
        md, am, vd, nf = run_screen(sv, arm, m, np.zeros((0, 3)), shape, flat, mode, 0.01, 0.03)
        assert np.all(np.isinf(md)) and np.all(am == -1) and np.all(vd == 0) and np.all(nf == 0)
