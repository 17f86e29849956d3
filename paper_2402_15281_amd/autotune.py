"""Autotuner for the launch shape of the batched exact check (sv_tile).

The unculled persistent kernel of sv_check_requests (the one that runs when exact-check
culling is switched off with sv_set_exact_culling(0); the culled pass has a fixed
shape) has four shape parameters:
- points per lane;
- threads per block;
- resident blocks per compute unit;
- point tiles per work item.

The best choice depends on the request mix: small clouds favour small tiles, and
many motions favour fewer, larger items.  The tuner times candidate shapes on the
caller's own batch through the C entry point (HIP events on the calling stream,
median of `reps` runs after one warm-up).  It searches in three stages:

1. every (points per lane, threads) pair, at full occupancy and a middle item size;
2. blocks per compute unit, for the best pair;
3. tiles per item.

The winner is cached in a JSON file, keyed by device and workload signature, so a
serving process tunes once per kind of batch.  Every candidate produces the same
results bit for bit; the tuner checks that too.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import _binding as sv


def _full_occupancy_bpc(threads: int) -> int:
    # 8 waves per SIMD, 4 SIMDs per compute unit
    return max(1, min(32, 32 * 64 // threads))


def signature(robot, reqs: "sv.DeviceRequests") -> str:
    """Device and coarse workload shape: the key of the tuning cache."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    ms = [m for m, _, _ in reqs.requests]
    cs = [c for _, c, _ in reqs.requests]
    tot_pairs = sum(m.n * c.n * m.T for m, c in zip(ms, cs))
    kinds = sorted({m.kind for m in ms})
    Ts = sorted({m.T for m in ms})
    bucket = lambda v: int(round(float(v) ** 0.25 * 4))   # coarse: 19% steps
    return (f"{props.name}|{getattr(props, 'gcnArchName', '')}|dof{robot.dof}|caps{robot.n_caps}|kinds{kinds}|"
            f"T{Ts if len(Ts) <= 4 else [Ts[0], Ts[-1]]}|req{reqs.n}|work{bucket(tot_pairs)}")


def _results(reqs):
    return [(o.min_dist.clone(), o.argmin.clone(), o.verdict.clone()) for _, _, o in reqs.requests]


def time_tile(robot, reqs, caps, eps, tile, ws, reps=3) -> float:
    """Median milliseconds of one sv_check_requests call with this launch shape."""
    sv.sv_check_requests(robot, reqs, caps, eps, tile=tile, ws=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        sv.sv_check_requests(robot, reqs, caps, eps, tile=tile, ws=ws)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(robot, reqs, caps, eps, ws=None, reps=3, cache_path=None, log=None):
    """Fastest launch shape for this batch: (sv_tile, {shape tuple: ms}, from_cache)."""
    key = signature(robot, reqs)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return sv.sv_tile(*cache[key]["tile"]), {}, True
    if ws is None:
        ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    allowed = {t.as_tuple() for t in sv.sv_tile_candidates()}
    timings = {}
    ref = None

    def run(t):
        nonlocal ref
        if t in timings or t not in allowed:
            return
        timings[t] = time_tile(robot, reqs, caps, eps, sv.sv_tile(*t), ws, reps)
        res = _results(reqs)
        if ref is None:
            ref = res
        else:
            for (a0, a1, a2), (b0, b1, b2) in zip(ref, res):
                if not (torch.equal(a0.view(torch.int32), b0.view(torch.int32)) and torch.equal(a1, b1)
                        and torch.equal(a2, b2)):
                    raise RuntimeError(f"launch shape {t} changed the results")
        if log:
            log(f"tile {t}: {timings[t]:.3f} ms")

    for ppl in (1, 2, 4):
        for threads in (64, 128, 256):
            run((ppl, threads, _full_occupancy_bpc(threads), 4))
    best = min(timings, key=timings.get)
    full = _full_occupancy_bpc(best[1])
    for bpc in sorted({max(1, full // 4), max(1, full // 2), full}):
        run((best[0], best[1], bpc, best[3]))
    best = min(timings, key=timings.get)
    for tpi in (1, 2, 4, 8, 16, 32):
        run((best[0], best[1], best[2], tpi))
    best = min(timings, key=timings.get)
    if cache_path:
        cache[key] = {"tile": list(best), "ms": timings[best]}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return sv.sv_tile(*best), timings, False
