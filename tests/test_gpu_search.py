"""GPU tests of the first-collision-free-motion search (Alg. 1: sv_first_free) and of
the network proxy d_hat (sv_nn_min), through the C ABI.

Bars:
- with a proxy drawn by the seeded generator, or without one: motion, position,
  exact-check count, network count, first-loop size and the visiting order equal
  the oracle's (verdicts are exact: FP32 distances with the FP64 recheck of the band);
- the returned distance is within 1e-5 m of the oracle's;
- sv_nn_min is within the BF16 network bar of the oracle's BF16 emulation;
- network + search: the answer is free, every motion visited before it collides,
  and the order is a valid Alg. 1 order for the proxy values the GPU produced.
"""
import numpy as np
import pytest
import torch

import svgen
from oracle import bf16_error as obf
from oracle import mlp as omlp
from oracle import search as osearch

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def run_search(sv, arm, motions, pts, eps, d_hat=None):
    robot = sv.make_robot(arm)
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    res = sv.search_result_tensor()
    order = torch.full((max(dm.n, 1),), -7, dtype=torch.int32, device="cuda")
    dh = None if d_hat is None else torch.as_tensor(np.asarray(d_hat, np.float32), device="cuda")
    sv.sv_first_free(robot, dm, dc, eps, res, d_hat=dh, order=order)
    torch.cuda.synchronize()
    return sv.read_search_result(res), order.cpu().numpy()[:dm.n]


def seeded_proxy(seed, M, eps):
    """Proxy values around eps on a coarse grid (many ties), a few NaN."""
    u = svgen.uniforms(seed, 1, M)[0]
    v = np.round((u - 0.5) * 0.08 / 0.004) * 0.004 + eps
    v[(u * 997) % 1 < 0.03] = np.nan
    return v.astype(np.float32)


@pytest.mark.parametrize("scene", [0, 1, 2, 3])
def test_search_matches_oracle(sv, orc, scene):
    arm = svgen.make_arm(1)
    w = svgen.WORKLOADS["boxworld"]
    motions, pts = svgen.box_world_scene(arm, scene)
    eps = float(np.float32(w["eps"]))
    d, _, _ = orc.check_motions(arm, motions, pts, eps)
    assert np.min(np.abs(d - eps)) > 1e-9
    for proxy in (None, seeded_proxy(scene + 40, motions.n, eps)):
        got, order = run_search(sv, arm, motions, pts, eps, proxy)
        ref = osearch.first_free(list(d), eps, None if proxy is None else [float(v) for v in proxy])
        print(scene, "proxy" if proxy is not None else "plain", got, ref)
        assert (got["motion"], got["n_exact"], got["n_nn"], got["n_first"]) == ref
        assert got["position"] == (ref[1] - 1 if ref[0] >= 0 else motions.n)
        assert got["n_exact_run"] >= min(got["n_exact"], motions.n)
        if ref[0] >= 0:
            assert abs(got["dist"] - d[ref[0]]) <= TOL
        if proxy is None:
            np.testing.assert_array_equal(order, np.arange(motions.n))
        else:
            np.testing.assert_array_equal(order, osearch.visiting_order([float(v) for v in proxy], eps))


def test_search_edge_cases(sv, orc):
    arm = svgen.make_arm(1)
    motions, pts = svgen.box_world_scene(arm, 5)
    got, _ = run_search(sv, arm, motions, pts, 10.0)                       # nothing is free
    assert got["motion"] == -1 and got["n_exact"] == motions.n and got["n_exact_run"] == motions.n
    assert np.isinf(got["dist"])
    got, _ = run_search(sv, arm, motions, np.zeros((0, 3)), 0.005)        # empty cloud: all free
    assert got["motion"] == 0 and got["n_exact"] == 1 and np.isinf(got["dist"])
    empty = svgen.Motions(np.zeros((0, 6), np.float32), np.zeros((0, 6), np.float32), 200)
    got, _ = run_search(sv, arm, empty, pts, 0.005)                        # no motions
    assert got["motion"] == -1 and got["n_exact"] == 0
    one = svgen.Motions(motions.q0[:1], motions.q1[:1], 1)                 # T = 1, single motion
    d, _, _ = orc.check_motions(arm, one, pts, 0.0)
    got, _ = run_search(sv, arm, one, pts, float(np.float32(d[0] - 0.01)))
    assert got["motion"] == 0 and abs(got["dist"] - d[0]) <= TOL


def test_search_band_uses_fp64(sv, orc):
    """eps within micrometres of motions' distances: only the FP64 recheck decides."""
    arm = svgen.make_arm(1)
    motions, pts = svgen.box_world_scene(arm, 6)
    d, _, _ = orc.check_motions(arm, motions, pts, 0.0)
    order = np.argsort(d)
    for i in order[-3:]:
        for off in (-2e-7, 2e-7):
            eps = float(np.float32(d[i] + off))
            if abs(eps - d[i]) < 1e-9:
                continue
            got, _ = run_search(sv, arm, motions, pts, eps)
            ref = osearch.first_free(list(d), eps)
            assert (got["motion"], got["n_exact"]) == ref[:2]


def test_nn_min_matches_bf16_oracle(sv):
    arm = svgen.make_arm(1)
    spec = svgen.MLPSpec(15, 128, 3)
    params = svgen.mlp_init(spec, 77)
    motions = svgen.make_motions(arm, 6, 64, 78)
    pts = svgen.uniform_cube(700, 79)
    mlp = sv.DeviceMLP(params, 15, 128, 3)
    d_hat = torch.full((6,), float("nan"), device="cuda")
    sv.sv_nn_min(mlp, sv.DeviceMotions(motions), sv.DeviceCloud(pts), d_hat)
    torch.cuda.synchronize()
    got = d_hat.cpu().numpy()
    for m in range(6):
        rows = np.concatenate([pts, np.repeat(motions.q0[m:m + 1], len(pts), 0),
                               np.repeat(motions.q1[m:m + 1], len(pts), 0)], axis=1)
        ref = omlp.forward_bf16(params, 15, 128, 3, rows).min()
        ref64, bar = obf.mlp_bar(params, 15, 128, 3, rows)
        # a minimum moves by at most the largest change of its terms
        assert abs(got[m] - ref) <= bar.max(), (m, got[m], ref)
        assert abs(got[m] - ref64.min()) <= bar.max(), (m, got[m], ref64.min())
    empty = torch.zeros(6, device="cuda")
    sv.sv_nn_min(mlp, sv.DeviceMotions(motions), sv.DeviceCloud(np.zeros((0, 3))), empty)
    assert torch.isinf(empty).all()


def test_network_search_composition(sv, orc):
    """Proxy from the (untrained) network: the GPU's own order must be an Alg. 1 order
    for the values it produced, and the answer the first free motion of that order."""
    arm = svgen.make_arm(1)
    w = svgen.WORKLOADS["boxworld"]
    motions, pts = svgen.box_world_scene(arm, 7)
    eps = float(np.float32(w["eps"]))
    spec = svgen.MLPSpec(*w["mlp"])
    mlp = sv.DeviceMLP(svgen.mlp_init(spec, 5), *w["mlp"])
    dm, dc = sv.DeviceMotions(motions), sv.DeviceCloud(pts)
    d_hat = torch.empty(dm.n, device="cuda")
    sv.sv_nn_min(mlp, dm, dc, d_hat)
    res = sv.search_result_tensor()
    order = torch.empty(dm.n, dtype=torch.int32, device="cuda")
    sv.sv_first_free(sv.make_robot(arm), dm, dc, eps, res, d_hat=d_hat, order=order)
    torch.cuda.synchronize()
    got = sv.read_search_result(res)
    dh = d_hat.cpu().numpy()
    o = order.cpu().numpy()
    nf = got["n_first"]
    assert sorted(o.tolist()) == list(range(dm.n))
    assert np.all(dh[o[:nf]] > eps) and np.all(np.diff(o[:nf]) > 0)
    assert np.all(~(dh[o[nf:]] > eps))
    key = np.where(np.isnan(dh[o[nf:]]), -np.inf, dh[o[nf:]])
    assert np.all(np.diff(key) <= 0)
    d, _, vd = orc.check_motions(arm, motions, pts, eps)
    if got["motion"] >= 0:
        p = got["position"]
        assert o[p] == got["motion"] and d[got["motion"]] > eps
        assert np.all(d[o[:p]] <= eps)
        assert got["n_exact"] == p + 1
    else:
        assert np.all(d <= eps)
