"""GPU tests of the continuous certification (sv_continuous_gap) through the C ABI.

Bars:
- gap[m] against the FP64 oracle: never below it, and at most one FP32 rounding above
  it (the kernel computes in FP64 and rounds up);
- the verdict is the FP32 decision min_dist - gap > eps + 1e-5 (taken here in
  float32 on the same values), and agrees with the oracle's FP64 distances and gaps
  wherever those are more than 1e-5 m from the decision boundary;
- the bound holds for the GPU's own distances: the sampled minimum minus the gap never
  exceeds the minimum at 8x finer sampling;
- host checks: verdict without min_dist is rejected; M = 0 is a no-op.
"""
import numpy as np
import pytest
import torch

import svgen
from oracle import continuous as oc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def gpu_gap(sv, robot, mo, min_dist=None, eps=0.0):
    dm = sv.DeviceMotions(mo)
    gap = torch.full((mo.n,), float("nan"), device="cuda")
    verdict = None if min_dist is None else torch.full((mo.n,), 7, dtype=torch.uint8, device="cuda")
    sv.sv_continuous_gap(robot, dm, gap, min_dist=min_dist, eps=eps, verdict=verdict)
    torch.cuda.synchronize()
    return gap.cpu().numpy(), None if verdict is None else verdict.cpu().numpy()


@pytest.mark.parametrize("kind,T", [("linear", 64), ("linear", 2), ("linear", 1), ("spline", 128), ("spline", 5)])
def test_gap_against_oracle(sv, kind, T):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, 300, T, 700 + T, kind)
    g, _ = gpu_gap(sv, robot, mo)
    ref = oc.gaps(arm, mo)
    assert np.all(g.astype(np.float64) >= ref * (1 - 1e-12))
    assert np.all(g.astype(np.float64) <= ref * (1 + 2.0 ** -22))


@pytest.mark.parametrize("kind", ["linear", "spline"])
def test_verdict_and_bound(sv, orc, kind):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    T, eps = 512, 0.01   # at this T some motions are certified along the whole path, others not
    mo = svgen.make_motions(arm, 64, T, 800, kind)
    pts = svgen.bin_cloud(3000, 801)
    dm, dc = sv.DeviceMotions(mo), sv.DeviceCloud(pts)
    out = sv.DeviceResults(mo.n)
    sv.sv_check_motions(robot, dm, dc, out, eps)
    g, v = gpu_gap(sv, robot, mo, out.min_dist, eps)
    md = out.min_dist.cpu().numpy()
    v32 = np.where(np.float32(md) - np.float32(g) > np.float32(eps) + np.float32(1e-5), 0, 1).astype(np.uint8)
    np.testing.assert_array_equal(v, v32)
    # the oracle's FP64 decision, away from the boundary
    ref_md, _, _ = orc.check_motions(arm, mo, pts, eps)
    ref_g = oc.gaps(arm, mo)
    margin = ref_md - ref_g - eps - 1e-5
    clear = np.abs(margin) > 1e-5
    np.testing.assert_array_equal(v[clear], np.where(margin[clear] > 0, 0, 1))
    print(f"{kind}: {int((v == 0).sum())} of {mo.n} motions certified free along the continuous path; "
          f"{int((out.verdict.cpu().numpy() == 0).sum())} free at the samples")
    # the bound on the GPU's own distances: 8x finer sampling
    fine = svgen.Motions(mo.q0, mo.q1, 8 * (T - 1) + 1, kind, mo.via)
    out_f = sv.DeviceResults(mo.n)
    sv.sv_check_motions(robot, sv.DeviceMotions(fine), dc, out_f, eps)
    torch.cuda.synchronize()
    assert np.all(md.astype(np.float64) - g <= out_f.min_dist.cpu().numpy().astype(np.float64) + 1e-6)


def test_host_checks(sv):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, 4, 8, 900)
    dm = sv.DeviceMotions(mo)
    gap = torch.empty(4, device="cuda")
    with pytest.raises(sv.SvError) as e:
        sv.sv_continuous_gap(robot, dm, gap, verdict=torch.empty(4, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -1
    empty = svgen.Motions(np.zeros((0, arm.dof)), np.zeros((0, arm.dof)), 8, "linear")
    sv.sv_continuous_gap(robot, sv.DeviceMotions(empty), gap)
