"""GPU parity of the paper's residual network (SV_NET_RESIDUAL) through the C ABI.

Bars (as for the softplus network):
  FP32 path: |y - y_ref| <= 1e-4 |y_ref| + 1e-4 rms(y_ref) per element (FP64 oracle).
  BF16 path: against the FP64 network, |y - y64| <= bar per output, the a-priori bar of
    oracle/bf16_error.py (first-order sum over every BF16 and FP32 rounding site with
    Hoeffding's inequality at lam = 7, from the BF16 unit roundoff 2^-8); against the
    oracle's emulation of the same rounding points, |y - y_bf| <= bar per output and the
    median |y - y_bf| / bar <= 0.005 (each misplaced rounding point moves it above 0.01).
  W = 1024 (one block of 8 waves per CU): the same bars, the kMin and screening modes.
  Modes of one kernel: the per-motion minimum (sv_nn_min) equals the minimum of the
    dense predictions bit for bit, and trust screening sends exactly the points whose
    dense prediction is below tau; certified verdicts equal the exact oracle's.
  Host checks: training rejects the architecture and width 1024; bn_eps must be positive.
"""
import numpy as np
import pytest
import torch

import svgen
from oracle import bf16_error as be
from oracle import mlp as om
from oracle import residual as ores

pytestmark = pytest.mark.gpu

IN = 15
EPS_BN = 1e-5


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def inputs(motions, pts):
    M, N = motions.n, pts.shape[0]
    return om.features(np.tile(pts, (M, 1)), np.repeat(motions.q0, N, axis=0), np.repeat(motions.q1, N, axis=0))


def device_net(sv, width, n_blocks, seed):
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), seed)
    return flat, sv.DeviceMLP(flat, IN, width, n_blocks, kind=sv.SV_NET_RESIDUAL, bn_eps=EPS_BN)


def dense(sv, dnet, motions, pts, precision):
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    out = torch.full((dm.n, dc.n), float("nan"), device="cuda")
    sv.sv_nn_sdf(dnet, precision, dm, dc, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def rel_ok(y, ref, rtol=1e-4):
    rms = np.sqrt(np.mean(ref ** 2))
    return np.all(np.abs(y - ref) <= rtol * np.abs(ref) + rtol * rms)


@pytest.mark.parametrize("width,n_blocks,M,N", [(64, 1, 3, 100), (128, 5, 2, 333), (512, 2, 1, 70), (1024, 1, 1, 20)])
def test_residual_fp32(sv, width, n_blocks, M, N):
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, M, 8, 200 + N)
    pts = svgen.bin_cloud(N, 201 + N)
    flat, dnet = device_net(sv, width, n_blocks, 202)
    y = dense(sv, dnet, m, pts, sv.SV_FP32).ravel()
    ref = ores.forward(flat, IN, width, n_blocks, inputs(m, pts), EPS_BN)
    print(f"fp32 residual {width}x{n_blocks}: max abs err {np.abs(y - ref).max():.2e}")
    assert rel_ok(y, ref)


@pytest.mark.parametrize("width,n_blocks,M,N", [(512, 5, 3, 1000), (512, 11, 1, 129), (256, 3, 4, 257),
                                                (128, 1, 2, 64), (128, 2, 1, 1), (1024, 3, 2, 150),
                                                (1024, 11, 1, 70)])
def test_residual_bf16(sv, width, n_blocks, M, N):
    """Several tiles of 64 rows with a ragged last tile; the paper's 5 x 512, 11 x 512 and
    11 x 1024 (one block of 8 waves per CU)."""
    arm = svgen.make_arm(1)
    m = svgen.make_motions(arm, M, 8, 300 + N)
    pts = svgen.bin_cloud(N, 301 + N)
    flat, dnet = device_net(sv, width, n_blocks, 302 + n_blocks)
    y = dense(sv, dnet, m, pts, sv.SV_BF16).ravel()
    X = inputs(m, pts)
    ref_bf = ores.forward_bf16(flat, IN, width, n_blocks, X, EPS_BN)
    ref, bar = be.residual_bar(flat, IN, width, n_blocks, X, EPS_BN)
    ok, rep = be.compare(y, ref_bf, ref, bar)
    print(f"bf16 residual {width}x{n_blocks}: {rep}")
    assert ok, rep


def test_residual_rows_mode(sv):
    """sv_nn_predict (explicit rows, layer 0 unsplit) in both precisions."""
    width, n_blocks, n = 256, 4, 500
    flat, dnet = device_net(sv, width, n_blocks, 400)
    g = np.random.default_rng(401)
    X = np.concatenate([g.uniform(-0.6, 0.6, (n, 3)), g.uniform(-3, 3, (n, IN - 3))], 1).astype(np.float32)
    rows = torch.as_tensor(np.concatenate([X, np.zeros((n, 1), np.float32)], 1), device="cuda").contiguous()
    for prec in (sv.SV_FP32, sv.SV_BF16):
        out = torch.full((n,), float("nan"), device="cuda")
        sv.sv_nn_predict(dnet, prec, rows, out)
        torch.cuda.synchronize()
        y = out.cpu().numpy().astype(np.float64)
        if prec == sv.SV_FP32:
            assert rel_ok(y, ores.forward(flat, IN, width, n_blocks, X, EPS_BN))
        else:
            ref_bf = ores.forward_bf16(flat, IN, width, n_blocks, X, EPS_BN)
            ref, bar = be.residual_bar(flat, IN, width, n_blocks, X, EPS_BN)
            ok, rep = be.compare(y, ref_bf, ref, bar)
            assert ok, rep


def test_residual_min_and_screening_modes(sv, orc):
    """kMin equals the dense minimum bit for bit; trust screening sends exactly the
    dense predictions below tau; certified verdicts equal the exact oracle."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    m = svgen.make_motions(arm, 6, 32, 500)
    pts = svgen.bin_cloud(900, 501)
    flat, dnet = device_net(sv, 512, 5, 502)
    y = dense(sv, dnet, m, pts, sv.SV_BF16).astype(np.float32)
    dm, dc = sv.DeviceMotions(m), sv.DeviceCloud(pts)
    d_hat = torch.empty(m.n, device="cuda")
    sv.sv_nn_min(dnet, dm, dc, d_hat)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_hat.cpu().numpy().view(np.int32), y.min(axis=1).view(np.int32))
    tau = float(np.median(y))
    out = sv.DeviceResults(m.n)
    sv.sv_check_motions(robot, dm, dc, out, 0.01, mlp=dnet, screen=sv.SV_SCREEN_TRUST, tau=tau)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.n_fallback.cpu().numpy(), (y < np.float32(tau)).sum(axis=1))
    outc = sv.DeviceResults(m.n)
    sv.sv_check_motions(robot, dm, dc, outc, 0.01, mlp=dnet, screen=sv.SV_SCREEN_CERTIFIED, tau=tau)
    torch.cuda.synchronize()
    _, _, ref_v = orc.check_motions(arm, m, pts, 0.01)
    np.testing.assert_array_equal(outc.verdict.cpu().numpy(), ref_v)


def test_residual_host_checks(sv):
    flat, dnet = device_net(sv, 128, 2, 600)
    assert sv.sv_train_workspace_size(dnet, 256) > 0        # the residual network trains (test_gpu_train_residual)
    n = flat.size
    rows = torch.zeros(256, IN + 1, device="cuda")
    with pytest.raises(sv.SvError) as e:                    # ... with the target-only clamp
        sv.sv_train_step(dnet, torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"), 1, rows,
                         torch.arange(256, dtype=torch.int32, device="cuda"), clamp_pred=True)
    assert e.value.status == -4
    bad = sv.DeviceMLP(flat, IN, 128, 2, kind=sv.SV_NET_RESIDUAL, bn_eps=0.0)
    m = svgen.make_motions(svgen.make_arm(1), 1, 8, 601)
    with pytest.raises(sv.SvError) as e:
        dense(sv, bad, m, svgen.bin_cloud(10, 602), sv.SV_BF16)
    assert e.value.status == -1
    wrong = sv.DeviceMLP(flat, IN, 128, 2, kind=7)
    with pytest.raises(sv.SvError) as e:
        dense(sv, wrong, m, svgen.bin_cloud(10, 602), sv.SV_FP32)
    assert e.value.status == -1


def test_residual_1024_min_and_screening(sv):
    """W = 1024: kMin equals the dense minimum bit for bit, and trust screening sends
    exactly the dense predictions below tau to the fallback."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    m = svgen.make_motions(arm, 3, 16, 510)
    pts = svgen.bin_cloud(300, 511)
    flat, dnet = device_net(sv, 1024, 2, 512)
    y = dense(sv, dnet, m, pts, sv.SV_BF16).astype(np.float32)
    dm, dc = sv.DeviceMotions(m), sv.DeviceCloud(pts)
    d_hat = torch.empty(m.n, device="cuda")
    sv.sv_nn_min(dnet, dm, dc, d_hat)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_hat.cpu().numpy().view(np.int32), y.min(axis=1).view(np.int32))
    tau = float(np.median(y))
    out = sv.DeviceResults(m.n)
    sv.sv_check_motions(robot, dm, dc, out, 0.01, mlp=dnet, screen=sv.SV_SCREEN_TRUST, tau=tau)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.n_fallback.cpu().numpy(), (y < np.float32(tau)).sum(axis=1))


def test_training_rejects_width_1024(sv):
    spec = svgen.MLPSpec(IN, 1024, 2)
    dnet = sv.DeviceMLP(svgen.mlp_init(spec, 5), IN, 1024, 2)
    with pytest.raises(sv.SvError) as e:
        sv.sv_train_workspace_size(dnet, 1024)
    assert e.value.status == -4
