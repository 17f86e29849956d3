"""Autotuner for the launch shape of the batched exact check (sv_tile).

sv_check_requests runs one of two passes, each with its own shape parameters:
- the culled pass (the default, tile.cull = 1): persistent blocks per compute unit,
  the number of gangs (queues) the blocks are dealt to, and the divisors that set
  the length of the sample blocks bounded by one sphere (linear motions, splines);
- the unculled persistent kernel (tile.cull = 0): points per lane, threads per
  block, resident blocks per compute unit and point tiles per work item.

The best choice depends on the request mix: long motions favour longer sample
blocks, a few large requests favour fewer gangs, small clouds favour small tiles.
The tuner times candidate shapes on the caller's own batch through the C entry point
(HIP events on the calling stream, median of `reps` runs after one warm-up) and
searches each pass in stages, one parameter group at a time from the library's
default shape:

culled:   1. the two sample-block divisors (all pairs);
          2. gangs, for the best pair;
          3. blocks per compute unit;
unculled: 1. every (points per lane, threads) pair, at full occupancy and a middle item size;
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


def signature(robot, reqs: "sv.DeviceRequests", passes=("culled",)) -> str:
    """Device, passes searched and coarse workload shape: the key of the tuning cache."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    ms = [m for m, _, _ in reqs.requests]
    cs = [c for _, c, _ in reqs.requests]
    tot_pairs = sum(m.n * c.n * m.T for m, c in zip(ms, cs))
    kinds = sorted({m.kind for m in ms})
    Ts = sorted({m.T for m in ms})
    bucket = lambda v: int(round(float(v) ** 0.25 * 4))   # coarse: 19% steps
    return (f"{props.name}|{getattr(props, 'gcnArchName', '')}|dof{robot.dof}|caps{robot.n_caps}|kinds{kinds}|"
            f"T{Ts if len(Ts) <= 4 else [Ts[0], Ts[-1]]}|req{reqs.n}|work{bucket(tot_pairs)}|"
            f"passes{sorted(passes)}")


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


def _with(base: tuple, **fields) -> tuple:
    t = sv.sv_tile(*base)
    for k, v in fields.items():
        setattr(t, k, v)
    return t.as_tuple()


def tune(robot, reqs, caps, eps, ws=None, reps=3, cache_path=None, log=None, passes=("culled",)):
    """Fastest launch shape for this batch among the passes named: (sv_tile, {shape tuple:
    ms}, from_cache)."""
    if not passes or any(p not in ("culled", "unculled") for p in passes):
        raise ValueError(f"passes must name 'culled' and/or 'unculled', got {passes!r}")
    key = signature(robot, reqs, passes)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return sv.sv_tile(*cache[key]["tile"]), {}, True
    if ws is None:
        ws = sv.workspace(sv.sv_batch_workspace_size(robot, caps))
    allowed = {t.as_tuple() for t in sv.sv_tile_candidates()}
    default = sv.sv_default_tile().as_tuple()
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
            log(f"tile {sv.sv_tile(*t)}: {timings[t]:.3f} ms")

    def best_of(pred):
        cands = [t for t in timings if pred(sv.sv_tile(*t))]
        return min(cands, key=timings.get)

    if "culled" in passes:
        is_culled = lambda t: t.cull == 1
        for dl in (16, 32, 64):
            for ds in (32, 64, 128):
                run(_with(default, cull=1, cull_div_linear=dl, cull_div_spline=ds))
        best = best_of(is_culled)
        for gangs in (1, 2, 4, 8, 16):
            run(_with(best, cull_gangs=gangs))
        best = best_of(is_culled)
        for bpc in (1, 2, 4, 0):
            run(_with(best, cull_blocks_per_cu=bpc))
    if "unculled" in passes:
        is_unculled = lambda t: t.cull == 0
        for ppl in (1, 2, 4):
            for threads in (64, 128, 256):
                run(_with(default, cull=0, ppl=ppl, threads=threads, blocks_per_cu=_full_occupancy_bpc(threads),
                          tiles_per_item=4))
        best = best_of(is_unculled)
        full = _full_occupancy_bpc(sv.sv_tile(*best).threads)
        for bpc in sorted({max(1, full // 4), max(1, full // 2), full}):
            run(_with(best, blocks_per_cu=bpc))
        best = best_of(is_unculled)
        for tpi in (1, 2, 4, 8, 16, 32):
            run(_with(best, tiles_per_item=tpi))
    best = min(timings, key=timings.get)
    if cache_path:
        cache[key] = {"tile": list(best), "ms": timings[best]}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return sv.sv_tile(*best), timings, False
