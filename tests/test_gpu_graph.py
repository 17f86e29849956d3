"""sv_check_motions captured in a HIP graph (through torch.cuda.CUDAGraph) and replayed.

The per-call path allocates nothing and clears its counters with fill kernels, so the
whole call (capsule table, culled or dense exact pass, screening network, fallback,
certified confirmation, FP64 band recheck) can be captured once and replayed.  Bars:
- every replay equals the eager call bit for bit (min_dist, argmin, verdict,
  n_fallback), with the outputs poisoned before each replay and unrelated eager work
  and synchronisations between replays (n_fallback is compared where the call writes
  it, in screening);
- after new motions and points are copied into the captured buffers, a replay equals
  an eager call on the new contents bit for bit.
"""

import numpy as np
import pytest
import torch

import svgen

pytestmark = pytest.mark.gpu

EPS, TAU = 0.01, 0.03


@pytest.fixture(scope="module")
def sv():
    from paper_2402_15281_amd import _binding
    assert torch.cuda.is_available()
    return _binding


def results(out):
    return (out.min_dist.cpu().numpy().view(np.int32).copy(), out.argmin.cpu().numpy().copy(),
            out.verdict.cpu().numpy().copy(), out.n_fallback.cpu().numpy().copy())


def poison(out, screening):
    out.min_dist.fill_(float("nan"))
    out.argmin.fill_(-7)
    out.verdict.fill_(9)
    if screening:   # written only when screening
        out.n_fallback.fill_(-3)


def assert_same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("mode", ["culled", "dense", "certified"])
def test_check_motions_graph_replay(sv, mode):
    arm = svgen.make_arm(1)
    robot = sv.make_robot(arm)
    mo = svgen.make_motions(arm, 24, 64, 1300)
    pts = svgen.bin_cloud(2500, 1301)
    dm, dc = sv.DeviceMotions(mo), sv.DeviceCloud(pts)
    out = sv.DeviceResults(dm.n)
    mlp, screen = None, sv.SV_SCREEN_NONE
    if mode == "certified":
        spec = svgen.MLPSpec(15, 256, 4)
        mlp, screen = sv.DeviceMLP(svgen.mlp_init(spec, 1302), 15, 256, 4), sv.SV_SCREEN_CERTIFIED
    ws = sv.workspace(sv.sv_workspace_size(sv.SV_OP_CHECK, robot, dm, dc, mlp))

    def call(stream=None):
        sv.sv_check_motions(robot, dm, dc, out, EPS, mlp=mlp, screen=screen, tau=TAU, ws=ws, stream=stream,
                            unculled=mode == "dense")

    call()   # eager warm-up and reference
    torch.cuda.synchronize()
    eager = results(out)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for _ in range(3):
        poison(out, mlp is not None)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert_same(results(out), eager)
        _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
    # new contents in the captured buffers
    mo2 = svgen.make_motions(arm, 24, 64, 1310)
    dm.q0.copy_(torch.as_tensor(mo2.q0, dtype=torch.float32))
    dm.q1.copy_(torch.as_tensor(mo2.q1, dtype=torch.float32))
    dc.xyz.copy_(sv.DeviceCloud(svgen.bin_cloud(2500, 1311)).xyz)
    poison(out, mlp is not None)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    replayed = results(out)
    poison(out, mlp is not None)
    call()
    torch.cuda.synchronize()
    fresh = results(out)
    assert_same(replayed, fresh)
    assert not np.array_equal(replayed[0], eager[0])
    print(f"{mode}: {int(fresh[2].sum())} of {dm.n} motions colliding after the new contents")
