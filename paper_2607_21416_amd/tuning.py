"""Autotuner of the work decomposition: the binning tile edge and the compositing
schedule (long-tile threshold, workgroup widths, persistent grid sizes).  None of these
change a result beyond the FP32 rounding order of the compositing sums, only the time,
so the tuner times candidates on the caller's own workload and keeps the fastest.

Search, by coordinate descent on the measured time:
  1. tile edge in {8, 16, 32}: the whole step (decode .. backward), since the edge moves
     work between the bin sort (more pairs for smaller tiles) and the compositing
     (each 8x8 quadrant walks its whole tile's range, so larger tiles cull more);
  2. forward and backward grids (waves per workgroup, which is also how many waves
     share a long tile's quadrant, and workgroups per CU), each on its own kernel;
  3. long-tile threshold 2^k: the two compositing kernels (the bin sort re-run once per
     candidate to rebuild the work order);
  4. the grids again, under the chosen threshold.
Choices are cached per workload signature (scene kind, views and their resolutions,
Gaussian and anchor counts, loss); set GLAM_TUNE_CACHE to a file path to keep them
across processes.  Choices measured earlier ship in tune_choices.json beside this file
and are used when neither cache holds the workload; use_cache=False measures afresh.
The returned choice names where it came from under "source" ("measured", "cache",
"stored").
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from .pipeline import TILE, Pipeline

TILES = (8, 16, 32)
LONG_LOG2 = (8, 9, 10, 11, 12)
# (waves per workgroup, workgroups per CU) of the two compositing grids
FWD_GRIDS = ((4, 3), (4, 4), (4, 5), (8, 1), (8, 2), (16, 1))
BWD_GRIDS = ((4, 4), (4, 5), (4, 6), (8, 1), (8, 2), (16, 1))
DEFAULT = {"tile": TILE, "long_log2": 10, "fwd_blocks_per_cu": 5, "bwd_blocks_per_cu": 6, "fwd_group_waves": 4,
           "bwd_group_waves": 4}
SCHEDULE = ("long_log2", "fwd_blocks_per_cu", "bwd_blocks_per_cu", "fwd_group_waves", "bwd_group_waves")

_cache: dict = {}
STORED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_choices.json")


def workload_key(scene: dict) -> str:
    cams = scene["cams"]
    res = sorted({(int(c["W"]), int(c["H"])) for c in cams})
    if scene["kind"] == "plain":
        size = int(scene["mean"].shape[1])
    else:
        size = int(scene["feat"].shape[0]) * int(scene["K"])
    # Gaussian counts to two significant digits: nearby sizes share a choice
    size = int(float(f"{size:.2g}"))
    return json.dumps([scene["kind"], len(cams), res, size, float(scene.get("ssim_weight", 0.0))])


def _load_disk() -> dict:
    path = os.environ.get("GLAM_TUNE_CACHE")
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _load_stored() -> dict:
    if os.path.exists(STORED):
        with open(STORED) as f:
            return {k: v for k, v in json.load(f).items() if not k.startswith("_")}
    return {}


def _save_disk(d: dict) -> None:
    path = os.environ.get("GLAM_TUNE_CACHE")
    if path:
        with open(path, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)


def _time(fn, iters: int) -> float:
    """Median milliseconds of fn() over iters eager calls (events on the current stream)."""
    out = []
    for _ in range(iters):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def autotune(scene: dict, device="cuda", iters: int = 5, log=None, use_cache: bool = True) -> dict:
    """Returns {tile, long_log2, fwd/bwd_blocks_per_cu, fwd/bwd_group_waves} for this
    workload, and the measured times in ms under key "ms"."""
    key = workload_key(scene)
    if use_cache:
        if key in _cache:
            return dict(_cache[key], source="cache")
        disk = _load_disk()
        if key in disk:
            _cache[key] = disk[key]
            return dict(disk[key], source="cache")
        stored = _load_stored()
        if key in stored:
            _cache[key] = stored[key]
            return dict(stored[key], source="stored")
    say = log or (lambda msg: None)
    ms: dict = {}
    best = dict(DEFAULT)
    # 1. tile edge, whole step
    step_ms = {}
    for t in TILES:
        pipe = Pipeline(scene, device=device, tile=t)
        pipe.fit_capacity()
        pipe.status.zero_()
        for _ in range(2):
            pipe.step()
        torch.cuda.synchronize()
        pipe.check_status()
        step_ms[t] = _time(pipe.step, iters)
        say(f"tune: tile {t}: step {step_ms[t]:.3f} ms")
        del pipe
        torch.cuda.empty_cache()
    best["tile"] = min(step_ms, key=step_ms.get)
    ms["step_by_tile"] = step_ms
    # 2-4. the schedule, on the chosen tile edge
    pipe = Pipeline(scene, device=device, tile=best["tile"])
    pipe.fit_capacity()
    pipe.status.zero_()
    for _ in range(2):
        pipe.step()
    torch.cuda.synchronize()

    def sched(**kw):
        return {k: best[k] for k in SCHEDULE} | kw

    def grids(tag):
        fwd_ms, bwd_ms = {}, {}
        for gw, b in FWD_GRIDS:
            pipe.set_tuning(sched(fwd_group_waves=gw, fwd_blocks_per_cu=b))
            fwd_ms[f"{gw}x{b}"] = _time(pipe.render, iters)
        for gw, b in BWD_GRIDS:
            pipe.set_tuning(sched(bwd_group_waves=gw, bwd_blocks_per_cu=b))
            bwd_ms[f"{gw}x{b}"] = _time(pipe.composite_bwd, iters)
        f = min(fwd_ms, key=fwd_ms.get)
        g = min(bwd_ms, key=bwd_ms.get)
        best["fwd_group_waves"], best["fwd_blocks_per_cu"] = (int(x) for x in f.split("x"))
        best["bwd_group_waves"], best["bwd_blocks_per_cu"] = (int(x) for x in g.split("x"))
        say(f"tune: grids ({tag}): forward {f} ({fwd_ms[f]:.3f} ms), backward {g} ({bwd_ms[g]:.3f} ms) "
            "(waves x workgroups per CU)")
        return fwd_ms, bwd_ms

    pipe.forward()
    pipe.backward()
    grids("default threshold")
    long_ms = {}
    for k in LONG_LOG2:
        pipe.set_tuning(sched(long_log2=k))
        pipe.forward()
        pipe.backward()
        torch.cuda.synchronize()
        long_ms[k] = _time(lambda: (pipe.render(), pipe.composite_bwd()), iters)
        say(f"tune: long tiles >= 2^{k}: compositing {long_ms[k]:.3f} ms")
    best["long_log2"] = min(long_ms, key=long_ms.get)
    pipe.set_tuning(sched())
    pipe.bin_sort()
    fwd_ms, bwd_ms = grids(f"threshold 2^{best['long_log2']}")
    pipe.check_status()
    del pipe
    torch.cuda.empty_cache()
    ms.update(long=long_ms, fwd=fwd_ms, bwd=bwd_ms)
    best["ms"] = {k: {str(a): round(b, 4) for a, b in v.items()} for k, v in ms.items()}
    _cache[key] = best
    if use_cache and os.environ.get("GLAM_TUNE_CACHE"):
        disk = _load_disk()
        disk[key] = best
        _save_disk(disk)
    return dict(best, source="measured")


def schedule(choice: dict) -> dict:
    """The compositing-schedule part of a tuner choice (for Pipeline(tuning=...)); a
    choice without group widths takes the default four waves."""
    return {k: int(choice.get(k, DEFAULT[k])) for k in SCHEDULE}
