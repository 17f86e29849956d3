"""GPU parity of the exact swept-volume path (sv_fk, sv_exact_sdf, sv_check_motions)
against the FP64 oracle, through the C ABI.

Bars: distances within 1e-5 m of the oracle; verdicts bit-exact; argmin valid
(the oracle's distance at the returned point equals the oracle's minimum within
1e-5 m, since several points can tie within FP32 rounding).
"""
import numpy as np
import pytest
import torch

import svgen

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def run_sdf(sv, arm, motions, pts):
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    sdf = torch.full((dm.n, dc.n), float("nan"), device="cuda")
    sv.sv_exact_sdf(sv.make_robot(arm), dm, dc, sdf)
    torch.cuda.synchronize()
    return sdf.cpu().numpy().astype(np.float64)


def run_check(sv, arm, motions, pts, eps):
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    out = sv.DeviceResults(dm.n)
    sv.sv_check_motions(sv.make_robot(arm), dm, dc, out, eps)
    torch.cuda.synchronize()
    return out.min_dist.cpu().numpy(), out.argmin.cpu().numpy(), out.verdict.cpu().numpy()


def test_fk_matches_oracle(sv, orc):
    arm = svgen.make_arm(1)
    rng = np.random.default_rng(0)
    q = svgen._f32(rng.uniform(arm.qlim[:, 0], arm.qlim[:, 1], (333, arm.dof)))
    ref = np.stack([orc.capsules(arm, qi) for qi in q])                    # [n][K][2][3]
    qd = torch.tensor(q, dtype=torch.float32, device="cuda")
    for fp64, tol in ((False, 2e-6), (True, 1.2e-7)):
        caps = torch.zeros(q.shape[0], arm.n_caps, 8, device="cuda")
        sv.sv_fk(sv.make_robot(arm), qd, caps, fp64=fp64)
        c = caps.cpu().numpy().astype(np.float64)
        got = np.stack([c[:, :, 0:3], c[:, :, 3:6]], axis=2)
        err = np.abs(got - ref).max()
        print(f"fk fp64={fp64}: max endpoint error {err:.3e} m")
        assert err <= tol
        np.testing.assert_array_equal(c[:, :, 6], np.broadcast_to(arm.cap_r.astype(np.float32), c[:, :, 6].shape))


def test_exact_sdf_tiny_workload(sv, orc):
    """1 linear motion, T = 64, 4096 points uniform in the 1.2 m cube."""
    w = svgen.WORKLOADS["tiny"]
    arm = svgen.make_arm(w["arm_seed"])
    m = svgen.make_motions(arm, w["n_motions"], w["T"], w["motion_seed"])
    pts = svgen.uniform_cube(w["n_points"], w["cloud_seed"])
    got = run_sdf(sv, arm, m, pts)
    ref = orc.exact_sdf(arm, m, pts)
    err = np.abs(got - ref).max()
    print(f"tiny: max |gpu - oracle| = {err:.3e} m")
    assert err <= TOL


@pytest.mark.parametrize("kind,M,T,N", [
    ("linear", 3, 1, 700),      # T = 1: static robot
    ("linear", 5, 2, 513),      # ragged tail
    ("linear", 4, 3, 1),
    ("linear", 7, 37, 1531),    # odd T: unpaired last sample
    ("spline", 6, 64, 2000),
    ("spline", 2, 129, 257),
])
def test_exact_sdf_shapes(sv, orc, kind, M, T, N):
    arm = svgen.make_arm(2)
    m = svgen.make_motions(arm, M, T, 40 + T, kind=kind)
    pts = svgen.uniform_cube(N, 50 + N)
    got = run_sdf(sv, arm, m, pts)
    ref = orc.exact_sdf(arm, m, pts)
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= TOL


def test_exact_sdf_static_motion_and_robot_variants(sv, orc):
    """q0 = q1 gives the static SDF; a robot with fewer capsules and a sphere capsule."""
    arm = svgen.make_arm(3)
    arm.cap_p[2, 1] = arm.cap_p[2, 0]
    arm.cap_frame[2, 1] = arm.cap_frame[2, 0]          # capsule 2 becomes a sphere
    m = svgen.make_motions(arm, 4, 16, 60)
    m.q1 = m.q0.copy()
    pts = svgen.uniform_cube(1000, 61)
    assert np.abs(run_sdf(sv, arm, m, pts) - orc.exact_sdf(arm, m, pts)).max() <= TOL
    small = svgen.Arm(dh=arm.dh[:3], qlim=arm.qlim[:3], cap_frame=arm.cap_frame[:3], cap_p=arm.cap_p[:3],
                      cap_r=arm.cap_r[:3])
    ms = svgen.Motions(m.q0[:, :3], svgen.make_motions(arm, 4, 16, 62).q1[:, :3], 16)
    assert np.abs(run_sdf(sv, small, ms, pts) - orc.exact_sdf(small, ms, pts)).max() <= TOL


def _check_against_oracle(orc, arm, m, pts, eps, md, am, vd, ref_md, ref_vd):
    np.testing.assert_array_equal(vd, ref_vd)
    assert np.abs(md.astype(np.float64) - ref_md).max() <= TOL
    for i in range(m.n):   # the returned point attains the minimum (within tolerance)
        one = svgen.Motions(m.q0[i:i + 1], m.q1[i:i + 1], m.T, m.kind, None if m.via is None else m.via[i:i + 1])
        d_at = orc.exact_sdf(arm, one, pts[am[i]:am[i] + 1])[0, 0]
        assert abs(d_at - ref_md[i]) <= TOL


def test_check_motions_bin_subsample(sv, orc):
    """64 of the bin-picking motions x the full 20,000-point bin cloud at T = 256."""
    w = svgen.WORKLOADS["bin20k"]
    arm = svgen.make_arm(w["arm_seed"])
    full = svgen.make_motions(arm, w["n_motions"], w["T"], w["motion_seed"])
    m = svgen.Motions(full.q0[::8], full.q1[::8], full.T)
    pts = svgen.bin_cloud(w["n_points"], w["cloud_seed"])
    md, am, vd = run_check(sv, arm, m, pts, w["eps"])
    ref_md, ref_am, ref_vd = orc.check_motions(arm, m, pts, w["eps"])
    assert np.min(np.abs(ref_md - w["eps"])) > 1e-9          # no exact tie at eps in this set
    print(f"collision fraction {ref_vd.mean():.3f}; max |d - d_ref| {np.abs(md - ref_md).max():.2e}")
    assert 0.05 <= ref_vd.mean() <= 0.95
    _check_against_oracle(orc, arm, m, pts, w["eps"], md, am, vd, ref_md, ref_vd)


def test_check_motions_full_size_sampled(sv, orc):
    """Full bin-picking workload (512 motions x 20,000 points, T = 256) in the
    launch configuration the benchmark times; 24 sampled motions are recomputed
    by the oracle."""
    w = svgen.WORKLOADS["bin20k"]
    arm = svgen.make_arm(w["arm_seed"])
    m = svgen.make_motions(arm, w["n_motions"], w["T"], w["motion_seed"])
    pts = svgen.bin_cloud(w["n_points"], w["cloud_seed"])
    md, am, vd = run_check(sv, arm, m, pts, w["eps"])
    idx = np.random.default_rng(7).choice(m.n, 24, replace=False)
    sub = svgen.Motions(m.q0[idx], m.q1[idx], m.T)
    ref_md, _, ref_vd = orc.check_motions(arm, sub, pts, w["eps"])
    _check_against_oracle(orc, arm, sub, pts, w["eps"], md[idx], am[idx], vd[idx], ref_md, ref_vd)
    assert np.isfinite(md).all() and set(np.unique(vd)) <= {0, 1}


def test_certified_band_recheck(sv, orc):
    """eps placed within a few micrometres of motions' oracle distances: the FP32
    distance alone could fall on either side; the FP64 recheck must give the
    oracle's verdict, and min_dist is then the FP64 value."""
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 8, 48, 70)
    pts = svgen.bin_cloud(3000, 71)
    ref_md, _, _ = orc.check_motions(arm, m, pts, 0.0)
    for i in range(4):
        for off in (-3e-6, -2e-7, 2e-7, 3e-6):
            eps = float(np.float32(ref_md[i] + off))
            if abs(eps - ref_md[i]) < 1e-9:
                continue
            md, am, vd = run_check(sv, arm, m, pts, eps)
            _, _, rv = orc.check_motions(arm, m, pts, eps)
            np.testing.assert_array_equal(vd, rv)
            assert abs(float(md[i]) - ref_md[i]) <= 1e-7


def test_check_motions_edge_cases(sv, orc):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 5, 8, 80)
    md, am, vd = run_check(sv, arm, m, np.zeros((0, 3)), 0.01)           # empty cloud
    assert np.all(np.isinf(md)) and np.all(am == -1) and np.all(vd == 0)
    empty = svgen.Motions(np.zeros((0, 6)), np.zeros((0, 6)), 8)
    md, am, vd = run_check(sv, arm, empty, svgen.uniform_cube(10, 1), 0.01)   # no motions: no-op
    assert md.size == 0
    pts = svgen.uniform_cube(1, 81)                                       # single point
    md, am, vd = run_check(sv, arm, m, pts, 0.01)
    ref_md, ref_am, ref_vd = orc.check_motions(arm, m, pts, 0.01)
    np.testing.assert_array_equal(am, 0)
    np.testing.assert_array_equal(vd, ref_vd)
    # duplicated points tie exactly in FP32: the lower index is reported
    pts = svgen.bin_cloud(500, 82)
    md1, am1, _ = run_check(sv, arm, m, pts, 0.01)
    dup = np.concatenate([pts, pts])
    md2, am2, _ = run_check(sv, arm, m, dup, 0.01)
    np.testing.assert_array_equal(md1, md2)
    np.testing.assert_array_equal(am1, am2)


def test_repeat_runs_bitwise_identical(sv):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, 32, 64, 90)
    pts = svgen.bin_cloud(5000, 91)
    a = run_check(sv, arm, m, pts, 0.01)
    b = run_check(sv, arm, m, pts, 0.01)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_invalid_arguments_rejected(sv):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    m = sv.DeviceMotions(svgen.make_motions(arm, 2, 8, 1))
    c = sv.DeviceCloud(svgen.uniform_cube(10, 1))
    out = sv.DeviceResults(2)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_motions(robot, m, c, out, 0.01, ws=small)
    assert e.value.status == -3
    bad = sv.make_robot(arm)
    bad.cap_frame[0][1] = 9
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_motions(bad, m, c, out, 0.01)
    assert e.value.status == -1
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_motions(robot, m, c, out, float("nan"))
    assert e.value.status == -1
