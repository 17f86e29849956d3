"""GPU tests of the batched exact check (sv_check_requests) through the C ABI.

Bars:
- every request's results equal sv_check_motions on that request bit for bit
  (the same per-point arithmetic, only scheduled differently), for every launch
  shape of the unculled kernel;
- the culled pass (branch and bound over sorted clouds) equals the unculled one
  bit for bit: skipped tests provably exceed the final minimum;
- against the FP64 oracle: distances within 1e-5 m, verdicts exact, argmin valid;
- a captured HIP graph replays to the eager results, also after the request
  contents change;
- malformed or oversized batches are reported in the status word with nothing
  written.
Latency itself is measured by the benchmark only (parity unpinned).
"""
import numpy as np
import pytest
import torch

import svgen

pytestmark = pytest.mark.gpu

TOL = 1e-5
EPS = 0.01


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def tile(sv, **fields):
    """The default launch shape with some fields replaced (cull=0: the unculled kernel)."""
    t = sv.sv_default_tile()
    for k, v in fields.items():
        setattr(t, k, v)
    return t


def make_batch(sv, arm, specs, seed):
    """specs: (motions, points, T, kind) per request -> (host data, device requests)."""
    host, dev = [], []
    for i, (M, N, T, kind) in enumerate(specs):
        mo = svgen.make_motions(arm, M, T, seed + 2 * i, kind)
        pts = svgen.bin_cloud(N, seed + 2 * i + 1) if N > 0 else np.zeros((0, 3))
        host.append((mo, pts))
        dev.append((sv.DeviceMotions(mo), sv.DeviceCloud(pts), sv.DeviceResults(M)))
    return host, sv.DeviceRequests(dev)


def poison(reqs):
    for _, _, o in reqs.requests:
        o.min_dist.fill_(-7.0)
        o.argmin.fill_(-7)
        o.verdict.fill_(7)


def results(reqs):
    torch.cuda.synchronize()
    return [(o.min_dist.cpu().numpy().copy(), o.argmin.cpu().numpy().copy(), o.verdict.cpu().numpy().copy())
            for _, _, o in reqs.requests]


def per_request(sv, robot, reqs, eps=EPS, unculled=False):
    out = []
    for m, c, _ in reqs.requests:
        o = sv.DeviceResults(m.n)
        sv.sv_check_motions(robot, m, c, o, eps, unculled=unculled)
        out.append(o)
    torch.cuda.synchronize()
    return [(o.min_dist.cpu().numpy(), o.argmin.cpu().numpy(), o.verdict.cpu().numpy()) for o in out]


def assert_bitwise(got, ref):
    assert len(got) == len(ref)
    for r, ((a0, a1, a2), (b0, b1, b2)) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(a0.view(np.int32), b0.view(np.int32), err_msg=f"min_dist of request {r}")
        np.testing.assert_array_equal(a1, b1, err_msg=f"argmin of request {r}")
        np.testing.assert_array_equal(a2, b2, err_msg=f"verdict of request {r}")


MIXED = [(3, 1000, 64, "spline"), (0, 500, 64, "spline"), (5, 0, 64, "linear"), (1, 1, 1, "linear"),
         (7, 777, 2, "spline"), (2, 513, 3, "linear"), (16, 2500, 100, "spline"), (1, 4097, 64, "linear"),
         (9, 64, 64, "spline"), (4, 1500, 33, "linear"), (1, 2000, 128, "spline"), (12, 300, 64, "linear"),
         (0, 0, 64, "linear"), (6, 1025, 17, "spline")]


def test_batch_equals_per_request_calls(sv):
    """Mixed kinds, T, sizes (empty requests, empty clouds, single points, ragged tiles)."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    _, reqs = make_batch(sv, arm, MIXED, 500)
    caps = reqs.caps(max_band=8)
    ticks = torch.zeros(reqs.n + 1, dtype=torch.int64, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    poison(reqs)
    sv.sv_check_requests(robot, reqs, caps, EPS, done_ticks=ticks, status=status)
    got = results(reqs)
    assert int(status.item()) == 0
    assert_bitwise(got, per_request(sv, robot, reqs))
    t = ticks.cpu().numpy()
    assert t[-1] > 0 and np.all(t[:-1] >= t[-1]), t


def test_batch_against_oracle(sv, orc):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    specs = [(4, 600, 40, "spline"), (3, 900, 25, "linear"), (2, 300, 64, "spline")]
    host, reqs = make_batch(sv, arm, specs, 600)
    sv.sv_check_requests(robot, reqs, reqs.caps(), EPS)
    got = results(reqs)
    for (mo, pts), (md, am, vd) in zip(host, got):
        ref_md, _, ref_vd = orc.check_motions(arm, mo, pts, EPS)
        assert np.abs(md - ref_md).max() <= TOL
        np.testing.assert_array_equal(vd, ref_vd)
        for i in range(mo.n):
            one = svgen.Motions(mo.q0[i:i + 1], mo.q1[i:i + 1], mo.T, mo.kind,
                                None if mo.via is None else mo.via[i:i + 1])
            d_at = orc.exact_sdf(arm, one, pts[am[i]:am[i] + 1])[0, 0]
            assert abs(d_at - ref_md[i]) <= TOL


@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_every_launch_shape_bitwise(sv, ppl):
    """The unculled persistent kernel under every tile shape."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    _, reqs = make_batch(sv, arm, MIXED, 700)
    caps = reqs.caps(max_band=8)
    ref = per_request(sv, robot, reqs)
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    for threads in (64, 128, 256):
        for bpc, tpi in ((1, 1), (3, 2), (8, 64), (32, 5)):
            poison(reqs)
            sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws,
                                 tile=tile(sv, cull=0, ppl=ppl, threads=threads, blocks_per_cu=bpc, tiles_per_item=tpi))
            assert_bitwise(results(reqs), ref)


CULL_MIX = [(40, 20000, 64, "spline"), (3, 9000, 17, "linear"), (0, 3000, 64, "spline"), (25, 0, 48, "linear"),
            (1, 1, 1, "linear"), (60, 5000, 100, "spline"), (8, 513, 16, "linear"), (12, 40000, 33, "spline"),
            (2, 511, 2, "linear"), (30, 12345, 64, "linear")]


@pytest.mark.parametrize("specs", [MIXED, CULL_MIX], ids=["mixed", "multi_tile"])
def test_culled_batch_equals_unculled(sv, specs):
    """Culled and unculled batched passes bit for bit, and both equal per-request calls
    with and without culling (ragged tiles and sample blocks, empty requests and clouds,
    single points, T = 1)."""
    arm = svgen.make_arm(2)
    robot = sv.make_robot(arm)
    _, reqs = make_batch(sv, arm, specs, 1300)
    caps = reqs.caps(max_band=16)
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    poison(reqs)
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status, tile=tile(sv, cull=0))
    dense = results(reqs)
    assert int(status.item()) == 0
    assert_bitwise(dense, per_request(sv, robot, reqs, unculled=True))
    shapes = [None, None, tile(sv, cull_div_linear=16, cull_div_spline=32, cull_gangs=2),
              tile(sv, cull_div_linear=64, cull_div_spline=128, cull_gangs=16, cull_blocks_per_cu=1)]
    for shape in shapes:   # the default twice (workspace reuse), then extreme sample blocks and gangs
        poison(reqs)
        sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status, tile=shape)
        assert_bitwise(results(reqs), dense)
        assert int(status.item()) == 0
    assert_bitwise(per_request(sv, robot, reqs), dense)


def test_total_points_capacity(sv):
    """caps.max_total_points bounds the sum of cloud sizes: a batch over it is flagged,
    nothing written; the host rejects capacities the pass cannot index."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    _, reqs = make_batch(sv, arm, [(3, 900, 32, "linear"), (2, 700, 40, "spline")], 1400)
    caps = reqs.caps()
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    tight = sv.sv_batch_caps(caps.max_requests, caps.max_T, caps.max_motions, caps.max_samples, caps.max_points,
                             caps.max_band, 1599)
    poison(reqs)
    sv.sv_check_requests(robot, reqs, tight, EPS, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == sv.SV_BATCH_OVER_CAPACITY
    assert all((o.verdict.cpu() == 7).all() for _, _, o in reqs.requests)
    exact = sv.sv_batch_caps(caps.max_requests, caps.max_T, caps.max_motions, caps.max_samples, caps.max_points,
                             caps.max_band, 1600)
    sv.sv_check_requests(robot, reqs, exact, EPS, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    huge = sv.sv_batch_caps(4096, 64, 1000, 64000, 1 << 30, 8, 0)
    with pytest.raises(sv.SvError) as e:
        sv.sv_batch_workspace_size(robot, huge)
    assert e.value.status == -1


@pytest.mark.parametrize("culled", [True, False], ids=["culled", "unculled"])
def test_graph_capture_and_replay_with_new_contents(sv, culled):
    graph_replay_case(sv, tile(sv, cull=int(culled)))


def graph_replay_case(sv, shape):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    specs = [(5, 800, 48, "spline"), (1, 3000, 48, "linear"), (9, 150, 48, "spline")]
    host, reqs = make_batch(sv, arm, specs, 800)
    caps = reqs.caps(max_band=8)
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    ticks = torch.zeros(reqs.n + 1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, done_ticks=ticks, status=status, tile=shape)   # eager
    eager = results(reqs)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, done_ticks=ticks, status=status, stream=s,
                                 tile=shape)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        poison(reqs)
        ticks.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_bitwise(results(reqs), eager)
        assert int(status.item()) == 0 and int(ticks[:-1].min().item()) > 0
        _ = torch.randn(1000, device="cuda").sum().item()      # unrelated eager work between replays
    # new contents in the same buffers: other motions and points, same sizes
    for i, ((m, c, o), (mo, pts)) in enumerate(zip(reqs.requests, host)):
        mo2 = svgen.make_motions(arm, mo.n, mo.T, 900 + i, mo.kind)
        m.q0.copy_(torch.as_tensor(mo2.q0, dtype=torch.float32))
        m.q1.copy_(torch.as_tensor(mo2.q1, dtype=torch.float32))
        if m.via is not None:
            m.via.copy_(torch.as_tensor(mo2.via, dtype=torch.float32))
        c.xyz.copy_(sv.DeviceCloud(svgen.bin_cloud(c.n, 950 + i)).xyz)
    poison(reqs)
    g.replay()
    got = results(reqs)
    assert_bitwise(got, per_request(sv, robot, reqs))
    assert any(not np.array_equal(a[0], b[0]) for a, b in zip(got, eager))


def test_status_word_and_host_checks(sv):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    specs = [(3, 400, 32, "linear"), (2, 300, 40, "spline")]
    _, reqs = make_batch(sv, arm, specs, 1000)
    caps = reqs.caps()
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    ticks = torch.full((reqs.n + 1,), 5, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    # a request beyond the capacities: flagged on the device, nothing written
    small = sv.sv_batch_caps(caps.max_requests, 32, caps.max_motions, caps.max_samples, caps.max_points, 4,
                             caps.max_total_points)
    poison(reqs)
    sv.sv_check_requests(robot, reqs, small, EPS, ws=ws, done_ticks=ticks, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & sv.SV_BATCH_OVER_CAPACITY
    assert all((o.verdict.cpu() == 7).all() for _, _, o in reqs.requests)
    assert int(ticks[:-1].abs().max().item()) == 0
    # a malformed request (unknown motion kind)
    m0 = reqs.requests[0][0]
    m0.kind = 7
    reqs.rewrite()
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & sv.SV_BATCH_BAD_REQUEST
    assert all((o.verdict.cpu() == 7).all() for _, _, o in reqs.requests)
    m0.kind = sv.SV_LINEAR
    reqs.rewrite()
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    # host-side checks
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, n_req=caps.max_requests + 1)
    assert e.value.status == -2
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, tile=tile(sv, ppl=3))
    assert e.value.status == -1
    for bad in (dict(cull=2), dict(cull_gangs=3), dict(cull_gangs=32), dict(cull_div_linear=48),
                dict(cull_div_spline=16), dict(cull_blocks_per_cu=9), dict(cull_blocks_per_cu=-1)):
        with pytest.raises(sv.SvError) as e:
            sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, tile=tile(sv, **bad))
        assert e.value.status == -1, bad
    with pytest.raises(sv.SvError) as e:
        sv.sv_check_requests(robot, reqs, caps, EPS, ws=torch.empty(64, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -3


def test_band_recheck_in_batch(sv, orc):
    """eps within micrometres of motions' distances: FP64 recheck inside the batch,
    as in sv_check_motions; a band list too short for them says so."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    specs = [(6, 2000, 48, "linear"), (4, 1500, 48, "spline")]
    host, _ = make_batch(sv, arm, specs, 1100)
    mo = host[0][0]
    mo.q0[4], mo.q1[4] = mo.q0[2], mo.q1[2]           # motions 2 and 4 of request 0 coincide
    reqs = sv.DeviceRequests([(sv.DeviceMotions(m), sv.DeviceCloud(p), sv.DeviceResults(m.n)) for m, p in host])
    ref_md = [orc.check_motions(arm, m, p, 0.0)[0] for m, p in host]
    eps = float(np.float32(ref_md[0][2] + 2e-7))
    caps = reqs.caps(max_band=8)
    ticks = torch.zeros(reqs.n + 1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    sv.sv_check_requests(robot, reqs, caps, eps, done_ticks=ticks, status=status)
    got = results(reqs)
    assert int(status.item()) == 0
    assert_bitwise(got, per_request(sv, robot, reqs, eps))
    for (m, p), (md, am, vd) in zip(host, got):
        _, _, ref_vd = orc.check_motions(arm, m, p, eps)
        np.testing.assert_array_equal(vd, ref_vd)
    assert abs(float(got[0][0][2]) - ref_md[0][2]) <= 1e-7       # the FP64 value
    assert int(ticks[:-1].min().item()) > 0
    one = sv.sv_batch_caps(caps.max_requests, caps.max_T, caps.max_motions, caps.max_samples, caps.max_points, 1)
    sv.sv_check_requests(robot, reqs, one, eps, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == sv.SV_BATCH_BAND_OVERFLOW


def test_requests_workload_full_size(sv, orc):
    """64 uneven SPLINE requests, T = 512 (1-2048 motions x 2k-200k points, log-uniform):
    culled batch bitwise equal to per-request calls and to the unculled batch; sampled
    motions of small requests against the oracle."""
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    rq = svgen.make_requests(arm, 64, 4242)
    reqs = sv.DeviceRequests([(sv.DeviceMotions(r.motions), sv.DeviceCloud(r.cloud), sv.DeviceResults(r.motions.n))
                              for r in rq])
    caps = reqs.caps(max_band=64)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    print(f"{sum(r.motions.n for r in rq)} motions, {sum(r.motions.n * r.cloud.shape[0] for r in rq) / 1e6:.1f}M pairs")
    ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status)
    got = results(reqs)
    assert int(status.item()) == 0
    assert_bitwise(got, per_request(sv, robot, reqs))
    poison(reqs)
    sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status, tile=tile(sv, cull=0))
    assert_bitwise(results(reqs), got)
    # the culled pass under other launch shapes (gangs, blocks, sample-block divisors)
    for fields in (dict(cull_gangs=1, cull_blocks_per_cu=1), dict(cull_gangs=16, cull_div_linear=16,
                                                                   cull_div_spline=128),
                   dict(cull_gangs=4, cull_blocks_per_cu=2, cull_div_linear=64, cull_div_spline=32)):
        poison(reqs)
        sv.sv_check_requests(robot, reqs, caps, EPS, ws=ws, status=status, tile=tile(sv, **fields))
        assert int(status.item()) == 0
        assert_bitwise(results(reqs), got)
    order = np.argsort([r.motions.n * r.cloud.shape[0] for r in rq])
    for ri in order[:3]:
        r = rq[ri]
        one = svgen.Motions(r.motions.q0[:1], r.motions.q1[:1], r.motions.T, r.motions.kind, r.motions.via[:1])
        ref_md, _, ref_vd = orc.check_motions(arm, one, r.cloud, EPS)
        assert abs(got[ri][0][0] - ref_md[0]) <= TOL
        assert got[ri][2][0] == ref_vd[0]
