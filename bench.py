#!/usr/bin/env python
"""Mapping-iteration throughput of the anchor-decoded Gaussian-splatting render on one
MI355X: anchor-MLP decode -> projection -> tile bin + depth sort -> compositing ->
L1 + 0.2 (1 - SSIM) loss -> backward to anchor features, offsets, scales and MLP
weights (Sec. III-A and III-D of the paper).

Headline (M1): mapping iterations per second at the metric's configuration, 50k anchors
x 10 offsets = 500k Gaussians on the synthetic street corridor, 1226x370, one keyframe
view per iteration (the paper samples one keyframe per mapping iteration, Sec. IV-B):
the whole path for view 0 of config 3, replayed from a HIP graph; value = steps / s.

Also reported: M1' (config 3's four views in one batched step: steps/s and view
iterations/s), per-stage times and Gaussian-pixel evaluations/s, each kernel's
fraction of its roofline (the work per unit of the hot-path scope table: lane-op slots
for the compositing kernels, bytes for the HBM-bound stages, matrix-core FLOP for the
MLPs) against the published peaks and against ceilings measured on this GPU by
microbenchmarks, the batched-vs-plain speedup on 16 partitions x 4 views (one batched
graph replay against the 64 per-view launch sequences, eager and replayed from a graph
at the same tile edge and schedule), and the FP64 CPU oracle timed on this host.

Prints one JSON line on stdout; progress goes to stderr.  --headline-only runs the
headline workload alone (the profiler runs use it, so that every kernel's average is
the headline's).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit, after the hot-path scope table's roofline rows:
#   forward compositing: per Gaussian-pixel evaluation about 18 FP32 VALU operations and
#     one exp, the transcendental issuing at a quarter of the VALU rate: 22 lane-op slots
#   backward compositing: per evaluation about 45 VALU operations, one exp and one
#     reciprocal: 53 lane-op slots
# against the chip's FP32 VALU issue rate, 256 CU x 4 SIMD x 16 lanes x 2.4 GHz =
# 39.32 T lane-op slots/s (non-packed FP32; an FMA is one slot).  The same work in the
# FLOP convention of the kernels as built (an FMA counted as two, exp2 as one):
#   forward: offset 2, exponent form 7, exp2 1, opacity 1, clamp 1, threshold 1,
#            transmittance 2, stop test 1, weight 1, colour 6 -> 23 FLOP
#   backward: the forward's alpha 13, T_i recovery 2, colour gradient 4, alpha
#            gradient 9, behind-colour update 6, opacity/power 2, the five moments of
#            dL/dpower 5 -> 41 FLOP, against 78.6 TFLOP/s
SLOTS_FWD = 22
SLOTS_BWD = 53
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12  # T lane-op slots/s
FLOP_FWD = 23
FLOP_BWD = 41
PEAK_FP32_TFLOPS = 78.6   # 256 CU x 64 FP32 lanes x 2 (FMA) x 2.4 GHz, scalar (non-packed) FP32
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_FP32_TFLOPS = 157.3  # dense FP32 matrix cores

# The other stages, for their own fractions and the whole-step one (each stage's ideal
# time is the larger of its compute and HBM times at the peaks):
#   decode + projection: 13,952 FLOP per anchor-view (three MLPs 36 -> 32 -> {10, 30, 70},
#     FMA = 2, on the matrix cores); 264 B read per anchor (position 3, features 32,
#     log-scale 1, offsets 30 words) once per partition; 96 B written per view-Gaussian
#     (14 decoded words, 10 projected words)
#   bin + sort: 24 B per pair (key and value written once, ranges scanned) + 24 B per pair
#     and radix pass (key and value read and written)
#   loss: 36 B per pixel (image and target read, dL/dC written, 3 channels each)
#   projection adjoint: 132 B per view-Gaussian (23 words read, 10 written)
#   decode adjoint: 27,904 FLOP per anchor-view (the two products of each forward one),
#     264 B per anchor and 56 B of incoming gradients per view-Gaussian read
DECODE_FLOP, DECODE_READ_B, DECODE_WRITE_B = 13952, 264, 96
SORT_PAIR_B, SORT_PASS_B = 24, 24
LOSS_PIXEL_B = 36
PROJ_BWD_B = 132
DECODE_BWD_FLOP, DECODE_BWD_READ_B = 27904, 56


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def split_views(scene):
    """One single-view scene per view of an anchor scene (its partition's anchors,
    MLP set and target): the plain per-view form."""
    import numpy as np
    out = []
    K = scene["K"]
    for v, cam in enumerate(scene["cams"]):
        m = cam["partition"]
        a0, a1 = int(scene["part_begin"][m]), int(scene["part_begin"][m + 1])
        sub = dict(scene)
        sub.update(pos=np.ascontiguousarray(scene["pos"][:, a0:a1]), feat=scene["feat"][a0:a1],
                   log_scale=scene["log_scale"][a0:a1], offs=np.ascontiguousarray(scene["offs"][:, a0 * K:a1 * K]),
                   part_begin=np.array([0, a1 - a0], np.int32), mlp=scene["mlp"][m:m + 1],
                   cams=[dict(cam, partition=0)], targets=[scene["targets"][v]])
        out.append(sub)
    return out


def timed(torch, fn, iters, stream):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(iters):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / iters


def stage_times(torch, pipe, iters, use_graph=True, reps=5):
    """Average duration of each C-ABI call of the step, HIP events on the stream the
    kernels run on: `iters` replays of a HIP graph of `reps` consecutive calls (as the
    step runs them, without the host's launch gaps), or eager launches.  The calls run
    in the step's order, so each one's inputs are the previous one's outputs."""
    first = [("project", pipe.project)] if pipe.plain else [("decode_project", pipe.decode_project)]
    calls = first + [("bin_sort", pipe.bin_sort),
             ("render_fwd", pipe.render), ("loss", pipe.compute_loss),
             ("composite_bwd", pipe.composite_bwd), ("project_bwd", pipe.project_bwd),
             ("decode_bwd", pipe.decode_bwd)]
    cur = torch.cuda.current_stream()
    out = {}
    for k, f in calls:
        if use_graph:
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(cur)
            with torch.cuda.stream(s):
                f()  # warm, outside capture
            cur.wait_stream(s)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                for _ in range(reps):
                    f()
            g.replay()
            fn, n = g.replay, iters * reps
        else:
            fn, n, g = f, iters, None
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(cur)
        for _ in range(iters):
            fn()
        b.record(cur)
        torch.cuda.synchronize()
        out[k] = a.elapsed_time(b) / n
        del g
    return out


def make_graph(torch, fn, use_graph):
    if not use_graph:
        return fn, None
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm, outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g.replay, g


def make_step(torch, pipe, use_graph):
    return make_graph(torch, pipe.step, use_graph)


def profiled_traffic(kernel, launch, name):
    """HBM bytes per launch of `kernel` from the committed counter summary profiles/<name>,
    or None when the compositing source has changed since the counters were taken or they
    were taken at another launch configuration (tile edge and schedule)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256") or rec.get("launch") != launch:
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return int(round(k["fetch_bytes"] + k["write_bytes"]))


def stage_work(pipe, pairs, evals_fwd, evals_bwd):
    """Each stage's algorithmic work, counted from the pipeline's own sizes: matrix-core
    FLOP, HBM bytes and VALU lane-op slots (see the constants above)."""
    passes = int(pipe.status.cpu()[6].item())
    anchor_views = sum(int(pipe.vt.info[i].anchor_count) for i in range(pipe.vt.n))
    n_anchors = int(pipe.anchors.A) if getattr(pipe, "anchors", None) is not None else 0
    G, npix = int(pipe.vt.n_gauss), int(pipe.vt.n_pix)
    work = {
        "decode_project": {"mfma_flop": anchor_views * DECODE_FLOP,
                           "hbm_bytes": n_anchors * DECODE_READ_B + G * DECODE_WRITE_B},
        "bin_sort": {"hbm_bytes": pairs * (SORT_PAIR_B + passes * SORT_PASS_B)},
        "render_fwd": {"lane_ops": evals_fwd * SLOTS_FWD, "flop": evals_fwd * FLOP_FWD},
        "loss": {"hbm_bytes": npix * LOSS_PIXEL_B},
        "composite_bwd": {"lane_ops": evals_bwd * SLOTS_BWD, "flop": evals_bwd * FLOP_BWD},
        "project_bwd": {"hbm_bytes": G * PROJ_BWD_B},
        "decode_bwd": {"mfma_flop": anchor_views * DECODE_BWD_FLOP,
                       "hbm_bytes": n_anchors * DECODE_READ_B + G * DECODE_BWD_READ_B},
    }
    units = {"anchor_views": anchor_views, "anchors": n_anchors, "view_gaussians": G, "pairs": int(pairs),
             "radix_passes": passes, "pixels": npix, "evaluations_fwd": evals_fwd, "evaluations_bwd": evals_bwd}
    return work, units


def peaks(ceil=None):
    """Ceilings in units per second: the published ones, or those measured on this GPU."""
    if ceil is None:
        return {"hbm": PEAK_HBM_GBS * 1e9, "alu": PEAK_LANE_OPS * 1e12, "mfma": PEAK_MFMA_FP32_TFLOPS * 1e12}
    return {"hbm": ceil["hbm_copy_TBs"] * 1e12, "alu": ceil["fma_TFLOPs"] / 2 * 1e12,
            "mfma": ceil["mfma_fp32_TFLOPs"] * 1e12}


def ideal_times(work, pk):
    """Each stage's ideal time (s) and bound: the largest of its compute and HBM times."""
    out = {}
    for k, w in work.items():
        cands = []
        if "mfma_flop" in w:
            cands.append((w["mfma_flop"] / pk["mfma"], "mfma"))
        if "hbm_bytes" in w:
            cands.append((w["hbm_bytes"] / pk["hbm"], "hbm"))
        if "lane_ops" in w:
            cands.append((w["lane_ops"] / pk["alu"], "alu"))
        out[k] = max(cands)
    return out


def whole_step_roofline(pipe, ms, pairs, evals_fwd, evals_bwd, st=None, ceil=None):
    """Sum over the stages of the step of each stage's ideal time (the larger of its
    compute and HBM times at the peaks, for its algorithmic work counted from the
    pipeline's own sizes), against the measured step; per stage too when `st` holds the
    stages' measured times.  ceil: measured ceilings in place of the published ones."""
    work, units = stage_work(pipe, pairs, evals_fwd, evals_bwd)
    ideal = ideal_times(work, peaks(ceil))
    t_ideal = sum(t for t, _ in ideal.values())
    out = {"frac": round(t_ideal * 1e3 / ms, 4), "ideal_ms": round(t_ideal * 1e3, 4), "measured_ms": round(ms, 4)}
    if st is not None:
        out["stages"] = {k: {"bound": b, "ideal_ms": round(t * 1e3, 4), "frac": round(t * 1e3 / st[k], 4)}
                         for k, (t, b) in ideal.items()}
    else:
        out["stages_ideal_ms"] = {k: round(t * 1e3, 4) for k, (t, _) in ideal.items()}
    out["units"] = units
    return out


def measure_ceilings():
    """The chip's ceilings measured by the microbenchmarks of libglam_ceilings.so (run
    outside any timed region)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2607_21416_amd", "libglam_ceilings.so"))
    for f in ("glamc_fma_tflops", "glamc_exp_trate", "glamc_lds_read_tbs", "glamc_hbm_copy_tbs",
              "glamc_hbm_triad_tbs", "glamc_mfma_fp32_tflops", "glamc_atomic_grate"):
        getattr(lib, f).restype = C.c_double
    lib.glamc_hbm_copy_tbs.argtypes = [C.c_longlong]
    lib.glamc_hbm_triad_tbs.argtypes = [C.c_longlong]
    lib.glamc_atomic_grate.argtypes = [C.c_int]
    gib = 1 << 30
    out = {"fma_TFLOPs": lib.glamc_fma_tflops(), "exp_Tper_s": lib.glamc_exp_trate(),
           "lds_read_TBs": lib.glamc_lds_read_tbs(), "hbm_copy_TBs": lib.glamc_hbm_copy_tbs(gib),
           "hbm_triad_TBs": lib.glamc_hbm_triad_tbs(gib), "mfma_fp32_TFLOPs": lib.glamc_mfma_fp32_tflops(),
           "atomic_distinct_Gper_s": lib.glamc_atomic_grate(0), "atomic_one_word_Gper_s": lib.glamc_atomic_grate(1)}
    out = {k: round(v, 3) for k, v in out.items()}
    out["published"] = {"fma_TFLOPs": PEAK_FP32_TFLOPS, "exp_Tper_s": round(PEAK_LANE_OPS / 4, 3),
                        "hbm_TBs": PEAK_HBM_GBS / 1e3, "mfma_fp32_TFLOPs": PEAK_MFMA_FP32_TFLOPS,
                        "lds_read_TBs": round(256 * 128 * 2.4e9 / 1e12, 2)}
    return out


def kernel_rooflines(pipe, st, pairs, evals_fwd, evals_bwd, ceil):
    """Every stage's fraction of its roofline from its algorithmic work and its measured
    average duration, against the published peaks and against the measured ceilings."""
    work, _ = stage_work(pipe, pairs, evals_fwd, evals_bwd)
    pub, mea = ideal_times(work, peaks()), ideal_times(work, peaks(ceil))
    out = {}
    for k in work:
        t = st[k] * 1e-3
        b = pub[k][1]
        rate = {"hbm": work[k].get("hbm_bytes", 0) / t / 1e9, "alu": work[k].get("lane_ops", 0) / t / 1e12,
                "mfma": work[k].get("mfma_flop", 0) / t / 1e12}[b]
        out[k] = {"bound": b, "achieved": round(rate, 3),
                  "unit": {"hbm": "GB/s", "alu": "Tlane-op/s", "mfma": "TFLOP/s"}[b],
                  "frac": round(pub[k][0] / t, 4), "frac_measured_ceiling": round(mea[k][0] / t, 4),
                  "ms": round(st[k], 4)}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    """Threads of the oracle: the host CPUs this process may use, at most 16 (one GPU's
    share of a GPU node's cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def time_oracle(scene, views, threads, min_s=0.0):
    """Seconds per view iteration of the FP64 oracle (forward + loss + backward), over
    `views`, repeated until min_s has passed."""
    import oracle
    oracle.set_num_threads(threads)
    t0 = time.perf_counter()
    n = 0
    while True:
        fwd = oracle.forward(scene, views=views)
        oracle.backward(scene, fwd)
        n += len(views)
        if time.perf_counter() - t0 >= min_s:
            break
    return (time.perf_counter() - t0) / n, n


def cpu_baseline(scene, view, threads):
    """The oracle on the headline workload (one view of config 3) on this host."""
    per, n = time_oracle(scene, [view], threads, min_s=10.0)
    return dict(value=1.0 / per, unit="iterations/s", cores=threads, kind="oracle",
                sample=f"config-3 view {view}: one FP64 forward + loss + backward pass per iteration, "
                       f"{n} iterations in {n * per:.1f} s on {threads} threads ({cpu_model()}, "
                       f"os.cpu_count() {os.cpu_count()})")


def cpu_baselines(threads, evals4_per_view=None):
    """The oracle at the smaller configurations on 1 thread and on `threads`, and a
    sample of config 4 extrapolated by Gaussian-pixel evaluations."""
    import synth
    out = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads": threads}
    for name in ("C1", "C2"):
        sc = synth.config(name)
        one, _ = time_oracle(sc, [0], 1, min_s=0.5)
        allc, _ = time_oracle(sc, [0], threads, min_s=0.5)
        out[name] = {"iterations_per_s_1_thread": round(1.0 / one, 4),
                     f"iterations_per_s_{threads}_threads": round(1.0 / allc, 4)}
    if evals4_per_view is not None:
        s4 = synth.config("C4")
        sample = list(range(0, len(s4["cams"]), len(s4["cams"]) // 8))[:8]
        per, n = time_oracle(s4, sample, threads)
        ev_sample = sum(evals4_per_view[v] for v in sample)
        ev_all = sum(evals4_per_view)
        step_s = per * len(sample) * ev_all / max(ev_sample, 1)
        out["C4_extrapolated"] = {"views_timed": sample, "seconds_per_timed_view": round(per, 3),
                                  "step_s_extrapolated": round(step_s, 2),
                                  "view_iterations_per_s_extrapolated": round(len(evals4_per_view) / step_s, 4),
                                  "note": "extrapolated linearly by the step's Gaussian-pixel evaluations"}
    return out


def run_workload(torch, scene, choice, args, dev, label):
    """Builds the pipeline of one workload at the tuner's choice, times args.steps graph
    replays of its step (the timed region: HIP events on the stream, synchronised on
    both sides), then, outside that region, the spread of single replays, each stage's
    average duration and the Gaussian-pixel evaluations (over 16x16 tile ranges, the
    workload's definition of the work, whatever tile edge the tuner chose)."""
    import numpy as np
    from paper_2607_21416_amd import tuning
    from paper_2607_21416_amd.pipeline import Pipeline

    pipe = Pipeline(scene, device=dev, tile=choice["tile"], tuning=tuning.schedule(choice))
    need = pipe.fit_capacity()
    pipe.status.zero_()
    log(f"bench: {label}: {pipe.vt.n} view(s), {pipe.vt.n_gauss} view-Gaussians, {need} pairs, capacity "
        f"{pipe.capacity}")
    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()
    step, graph = make_step(torch, pipe, not args.no_graph)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    log(f"bench: {label}: timing {args.steps} steps ({'graph' if graph else 'eager'})")
    t0 = time.perf_counter()
    ms = timed(torch, step, args.steps, stream)
    wall = time.perf_counter() - t0
    pipe.check_status()
    log(f"bench: {label}: {ms:.3f} ms/step, {1000.0 / ms:.1f} steps/s (wall {wall:.2f} s)")
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
    for a, b in rev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    rt = np.array([a.elapsed_time(b) for a, b in rev])
    replay = {"n": len(rt), "median_ms": round(float(np.median(rt)), 4),
              "p10_ms": round(float(np.percentile(rt, 10)), 4), "p90_ms": round(float(np.percentile(rt, 90)), 4)}
    pipe.check_status()
    st = stage_times(torch, pipe, args.stage_iters, use_graph=not args.no_graph)
    pipe.check_status()
    ref = pipe if pipe.vt.tile == 16 else Pipeline(scene, device=dev)
    if ref is not pipe:
        ref.fit_capacity()
        ref.status.zero_()
        ref.forward()
    ref.count_evaluations()
    ref.render()
    torch.cuda.synchronize()
    evals_fwd = int(ref.n_eval.to(torch.int64).sum().item())
    evals_bwd = int(ref.n_contrib.to(torch.int64).sum().item())
    per_view = [int(t.to(torch.int64).sum().item()) for t in ref.per_pixel(ref.n_eval)]
    ref.count_evaluations(False)
    ref.check_status()
    del ref
    log(f"bench: {label}: stages " + ", ".join(f"{k} {v:.3f}" for k, v in st.items()))
    return dict(pipe=pipe, ms=ms, wall=wall, replay=replay, st=st, need=need, evals_fwd=evals_fwd,
                evals_bwd=evals_bwd, evals_per_view=per_view, graph=graph, step=step)


def dominant_roofline(w, choice, ceil, traffic_file):
    """The roofline object of the workload's dominant kernel (the slower compositing
    kernel), in the scope table's work units, with the FLOP convention and the measured
    ceiling beside it."""
    from paper_2607_21416_amd import tuning
    st = w["st"]
    dom = max(("render_fwd", "composite_bwd"), key=lambda k: st[k])
    evals = w["evals_fwd"] if dom == "render_fwd" else w["evals_bwd"]
    slots = SLOTS_FWD if dom == "render_fwd" else SLOTS_BWD
    flop = FLOP_FWD if dom == "render_fwd" else FLOP_BWD
    t = st[dom] * 1e-3
    achieved = evals * slots / t / 1e12
    achieved_flop = evals * flop / t / 1e12
    measured_peak = ceil["fma_TFLOPs"] / 2 if ceil else None
    return {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_LANE_OPS, 2),
            "unit": "Tlane-op/s", "frac": round(achieved / PEAK_LANE_OPS, 4),
            "traffic": profiled_traffic(dom, {"tile": choice["tile"], "schedule": tuning.schedule(choice)},
                                        traffic_file),
            "work": f"{evals} Gaussian-pixel evaluations x {slots} FP32 VALU lane-op slots per launch "
                    f"(exp and reciprocal at a quarter of the VALU rate); peak = 256 CU x 4 SIMD x 16 lanes "
                    f"x 2.4 GHz",
            "avg_ms": round(st[dom], 4),
            "avg_ms_is": "the C-ABI call, replayed from a graph of consecutive calls"
                         + (" (its clearing launch of the 2-D gradient buffer and the kernel)"
                            if dom == "composite_bwd" else ""),
            "measured_peak": round(measured_peak, 3) if measured_peak else None,
            "frac_measured_peak": round(achieved / measured_peak, 4) if measured_peak else None,
            "flop_convention": {"achieved": round(achieved_flop, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                "frac": round(achieved_flop / PEAK_FP32_TFLOPS, 4),
                                "work": f"{evals} evaluations x {flop} FLOP (FMA = 2, exp2 = 1)"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-graph", action="store_true", help="eager launches instead of a HIP graph replay")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-view batched-vs-plain comparison")
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline workload alone (no ceilings, four-view step, next rows, config 4, CPU)")
    ap.add_argument("--four-view-only", action="store_true",
                    help="config 3's four-view step alone (for profiling; prints its object, not the bench line)")
    ap.add_argument("--stage-iters", type=int, default=10)
    ap.add_argument("--no-config5", action="store_true",
                    help="skip config 5 (2 km path, 64 partitions x 8 views, mixed resolutions), which the "
                         "default run times from a graph after the other workloads")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (built-in tile edge and compositing schedule)")
    ap.add_argument("--retune", action="store_true",
                    help="measure the tuner's choice now instead of using a stored one")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this size (profiler byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); partitions shard across GPUs "
              "without communication, so there is no multi-GPU run to make here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2607_21416_amd import binding, tuning
    from paper_2607_21416_amd.pipeline import Pipeline

    binding.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ceil = None
    if not (args.headline_only or args.four_view_only):
        log("bench: ceilings of this GPU (microbenchmarks, outside any timed region)")
        ceil = measure_ceilings()
        log("bench: ceilings " + ", ".join(f"{k} {v}" for k, v in ceil.items() if k != "published"))

    def choose(sc):
        if args.no_tune:
            return dict(tuning.DEFAULT, source="built-in default")
        return tuning.autotune(sc, device=dev, log=log, use_cache=not args.retune)

    log("bench: generating config 3 (50k anchors, 4 views 1226x370)")
    scene = synth.config("C3")
    if args.four_view_only:
        choice = choose(scene)
        w4 = run_workload(torch, scene, choice, args, dev, "config 3, four views")
        m = {"workload": "config 3: the four keyframe views in one batched step", "ms_per_step": round(w4["ms"], 4),
             "tile": choice["tile"], "schedule": tuning.schedule(choice),
             "stages_ms": {k: round(v, 4) for k, v in w4["st"].items()},
             "roofline": dominant_roofline(w4, choice, None, "traffic_config3.json")}
        if args.copy_mib > 0:
            src = torch.ones(args.copy_mib * 262144, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"m1_prime": m}), flush=True)
        return
    scene1 = synth.one_view(scene, 0)
    choice1 = choose(scene1)
    sc1 = tuning.schedule(choice1)
    log("bench: headline (one view): tile %d, long tiles >= 2^%d, grids %dx%d / %dx%d (waves x workgroups per CU, "
        "forward / backward) (%s)" % (choice1["tile"], sc1["long_log2"], sc1["fwd_group_waves"],
                                      sc1["fwd_blocks_per_cu"], sc1["bwd_group_waves"], sc1["bwd_blocks_per_cu"],
                                      choice1["source"]))
    w1 = run_workload(torch, scene1, choice1, args, dev, "config 3, view 0")
    ms = w1["ms"]
    value = 1000.0 / ms
    roofline = dominant_roofline(w1, choice1, ceil, "traffic_view0_config3.json")
    step_roofline = whole_step_roofline(w1["pipe"], ms, w1["need"], w1["evals_fwd"], w1["evals_bwd"], w1["st"])
    log(f"bench: M1 {value:.1f} iterations/s; dominant kernel {roofline['kernel']} at {roofline['frac']:.3f} of "
        f"its roofline; whole step {step_roofline['frac']:.3f}")
    out = {
        "metric": "mapping iters/s fwd+bwd (500k Gaussians, 1226x370); batched vs plain speedup",
        "value": round(value, 2), "unit": "iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config 3 scale: 50k anchors x 10 offsets = 500k Gaussians, street corridor, "
                               "1226x370; one mapping iteration = one keyframe view (view 0) decoded, projected, "
                               "binned, composited, L1 + 0.2 (1 - SSIM), backward to anchors and MLPs",
                   "views_per_step": 1, "view_gaussians": int(w1["pipe"].vt.n_gauss), "pairs": int(w1["need"]),
                   "launch": "hip graph" if w1["graph"] else "eager",
                   "tile": choice1["tile"], "schedule": tuning.schedule(choice1), "tuning": choice1["source"]},
        "stages_ms": {k: round(v, 4) for k, v in w1["st"].items()},
        "evaluations_per_s": {"fwd": round(w1["evals_fwd"] / (w1["st"]["render_fwd"] * 1e-3), 1),
                              "bwd": round(w1["evals_bwd"] / (w1["st"]["composite_bwd"] * 1e-3), 1)},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "replays": w1["replay"],
    }
    if ceil is not None:
        out["ceilings"] = ceil
        out["kernel_rooflines"] = kernel_rooflines(w1["pipe"], w1["st"], w1["need"], w1["evals_fwd"],
                                                   w1["evals_bwd"], ceil)
        out["step_roofline"]["frac_measured_ceilings"] = whole_step_roofline(
            w1["pipe"], ms, w1["need"], w1["evals_fwd"], w1["evals_bwd"], ceil=ceil)["frac"]
    if "ms" in choice1:
        out["autotune_ms"] = choice1["ms"]
    del w1["graph"], w1["step"]
    if args.headline_only:
        if args.copy_mib > 0:
            src = torch.ones(args.copy_mib * 262144, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps(out), flush=True)
        return
    del w1

    # M1': config 3's four views in one batched step
    choice = choose(scene)
    w4 = run_workload(torch, scene, choice, args, dev, "config 3, four views")
    pipe = w4["pipe"]
    n_views = pipe.vt.n
    out["m1_prime"] = {"workload": "config 3: the four keyframe views in one batched step", "views": n_views,
                       "ms_per_step": round(w4["ms"], 4), "steps_per_s": round(1000.0 / w4["ms"], 2),
                       "view_iterations_per_s": round(n_views * 1000.0 / w4["ms"], 2),
                       "tile": choice["tile"], "schedule": tuning.schedule(choice), "tuning": choice["source"],
                       "stages_ms": {k: round(v, 4) for k, v in w4["st"].items()},
                       "roofline": dominant_roofline(w4, choice, ceil, "traffic_config3.json"),
                       "kernel_rooflines": kernel_rooflines(pipe, w4["st"], w4["need"], w4["evals_fwd"],
                                                            w4["evals_bwd"], ceil),
                       "step_roofline": whole_step_roofline(pipe, w4["ms"], w4["need"], w4["evals_fwd"],
                                                            w4["evals_bwd"], w4["st"]),
                       "replays": w4["replay"]}
    if "ms" in choice:
        out["m1_prime"]["autotune_ms"] = choice["ms"]
    del w4["graph"], w4["step"]
    stream = torch.cuda.current_stream()

    # the optimiser step that closes the mapping iteration (Adam over the anchors'
    # features, offsets, log-scales and the MLP sets); the headline rate excludes it.
    # Parameters are restored afterwards; a graph replay reuses the captured step number.
    saved = {k: v.clone() for k, v in pipe.params.items()}

    def restore():
        for k, v in saved.items():
            pipe.params[k].copy_(v)

    pipe.fit_capacity(slack=1.6)  # room for the pairs of parameters that move
    pipe.status.zero_()
    pipe.init_optimizer()
    # the Adam kernel alone, from a graph of ten steps (eager calls would time the host
    # launch of its group table instead)
    astep, ag = make_graph(torch, lambda: [pipe.adam_step(step=1) for _ in range(10)], True)
    t_adam = timed(torch, astep, max(1, args.stage_iters // 2), stream) / 10
    del ag
    restore()
    ostep, og = make_graph(torch, lambda: (pipe.step(), pipe.adam_step(step=1)), not args.no_graph)

    # every timed iteration starts from the same parameters (restored outside the timed
    # interval), so the iterations repeat the measured workload
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in ev:
        restore()
        a.record(stream)
        ostep()
        b.record(stream)
    torch.cuda.synchronize()
    t_opt = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    pipe.check_status()
    del og
    restore()
    n_opt = sum(int(pipe.opt_m[k].numel()) for k in pipe.opt_m)
    out["m1_prime"]["stages_ms"]["adam"] = round(t_adam, 4)
    log(f"bench: with the optimiser step {t_opt:.3f} ms/step ({n_views * 1000.0 / t_opt:.1f} view iterations/s), "
        f"Adam {t_adam:.3f} ms over {n_opt} parameters")

    # loop-closure deformation of config 3's anchors by 40 corrected keyframes (on
    # scratch copies of the anchor positions and offsets)
    fixes = synth.loop_fixes(77, 40, spacing=2.0)
    table = (binding.KeyframeFix * len(fixes))()
    for i, f in enumerate(fixes):
        c = table[i].before
        for k in range(9):
            c.R[k], table[i].R_new[k] = float(np.asarray(f["R_old"]).ravel()[k]), float(np.asarray(f["R_new"]).ravel()[k])
        for k in range(3):
            c.t[k], table[i].t_new[k] = float(f["t_old"][k]), float(f["t_new"][k])
        c.fx, c.fy, c.cx, c.cy, c.width, c.height = f["fx"], f["fy"], f["cx"], f["cy"], f["W"], f["H"]
    dtable = torch.from_numpy(np.frombuffer(bytes(table), np.uint8).copy()).to(dev)
    A3, K3 = pipe.anchors.A, pipe.anchors.K
    xpos, xoffs = pipe.params["pos"].clone(), pipe.params["offs"].clone()
    xown = torch.empty(A3, dtype=torch.int32, device=dev)
    dstep, dg_ = make_graph(torch, lambda: [binding.glam_deform_anchors(xpos, xoffs, A3, K3, dtable, len(fixes), 0.2,
                                                                        80.0, xown, torch.cuda.current_stream())
                                            for _ in range(10)], True)
    t_def = timed(torch, dstep, 3, stream) / 10
    moved = int((xown >= 0).sum().item())
    del dg_, xpos, xoffs
    log(f"bench: loop-closure deformation {t_def * 1e3:.1f} us for {A3} anchors x {len(fixes)} keyframes "
        f"({moved} anchors in a frustum)")

    # flow densification geometry: one flow field's correspondences between two
    # keyframes (a pair per pixel of a 1226x370 view), epipolar filter + triangulation
    from paper_2607_21416_amd.pipeline import camera_array
    npx = 1226 * 370
    fc1, fc2, fx1, fx2, _, _ = synth.flow_pairs(91, npx, baseline=1.0, noise_px=0.5, outlier_frac=0.2)
    fcams = camera_array([fc1, fc2])
    gx1, gx2 = torch.from_numpy(np.ascontiguousarray(fx1)).to(dev), torch.from_numpy(np.ascontiguousarray(fx2)).to(dev)
    fres = torch.empty(npx, device=dev)
    fkeep = torch.empty(npx, dtype=torch.int32, device=dev)
    fX = torch.empty((3, npx), device=dev)
    tau = 0.05  # unit-norm F: keeps ~95% of the inliers and drops most outliers here

    def epi():
        binding.glam_epipolar_triangulate(fcams[0], fcams[1], gx1, gx2, npx, tau, fres, fkeep, fX,
                                          torch.cuda.current_stream())

    estep, eg = make_graph(torch, lambda: [epi() for _ in range(10)], True)
    t_epi = timed(torch, estep, 3, stream) / 10
    kept = int(fkeep.sum().item())
    del eg
    log(f"bench: epipolar filter + triangulation {t_epi * 1e3:.1f} us for {npx} correspondences ({kept} kept)")

    # anchor growth (Eq. 4): the triangulated flow points above (NaN where rejected) and
    # 2,000 tracked points of the keyframe, snapped to 1 mm voxels and grown onto the key
    # set of config 3's anchors (built once by the same call with no existing keys)
    veps = 0.001
    tracked = torch.from_numpy(synth.fused_points(92, 2000, dup_frac=0.0)).to(dev)
    cloud = torch.cat([fX, tracked], dim=1).contiguous()
    nv = int(cloud.shape[1])
    vwsb = binding.glam_voxelize_workspace_bytes(max(nv, A3))
    vws = torch.empty(vwsb, dtype=torch.uint8, device=dev)
    akeys = torch.empty(A3, dtype=torch.int64, device=dev)
    acen = torch.empty((3, A3), device=dev)
    aset = torch.empty(A3, dtype=torch.int64, device=dev)
    acnt = torch.empty(2, dtype=torch.int64, device=dev)
    binding.glam_voxelize(pipe.params["pos"], A3, veps, None, 0, akeys, acen, A3, aset, acnt, vws, vwsb,
                          torch.cuda.current_stream())
    n_akeys = int(acnt[0].item())
    gkeys = torch.empty(nv, dtype=torch.int64, device=dev)
    gcen = torch.empty((3, nv), device=dev)
    gset = torch.empty(n_akeys + nv, dtype=torch.int64, device=dev)
    gcnt = torch.empty(2, dtype=torch.int64, device=dev)

    def grow():
        binding.glam_voxelize(cloud, nv, veps, aset, n_akeys, gkeys, gcen, nv, gset, gcnt, vws, vwsb,
                              torch.cuda.current_stream())

    vstep, vg = make_graph(torch, lambda: [grow() for _ in range(10)], True)
    t_vox = timed(torch, vstep, 3, stream) / 10
    n_new, n_drop = (int(x) for x in gcnt.cpu().tolist())
    del vg, vws
    log(f"bench: anchor growth {t_vox * 1e3:.1f} us for {nv} points onto {n_akeys} anchor voxels "
        f"({n_new} new voxels, {n_drop} points dropped)")
    # its bookkeeping: the new anchors inserted at the end of the last partition in the
    # four per-anchor arrays and the six Adam moments of config 3 (into scratch copies)
    F3 = pipe.anchors.F
    at3 = A3  # config 3 has one partition: its end is the end of the arrays
    lay = [(pipe.params["pos"], 3, 1, gcen), (pipe.params["feat"], 1, F3, None), (pipe.params["log_scale"], 1, 1, None),
           (pipe.params["offs"], 3, K3, None)]
    lay += [(pipe.opt_m[k], r, w, None) for k, r, w in (("feat", 1, F3), ("offs", 3, K3), ("log_scale", 1, 1))]
    lay += [(pipe.opt_v[k], r, w, None) for k, r, w in (("feat", 1, F3), ("offs", 3, K3), ("log_scale", 1, 1))]
    outs = [torch.empty(r * (A3 + n_new) * w, device=dev) for _, r, w, _ in lay]
    ins_bytes = sum(4 * r * w * (2 * A3 + n_new) + (4 * r * w * n_new if i is not None else 0) for _, r, w, i in lay)

    def insert_all():
        for (src, r, w, ins), dst in zip(lay, outs):
            binding.glam_insert_rows(src, dst, r, A3, w, at3, n_new, ins, nv if ins is not None else 0, 0.0,
                                     torch.cuda.current_stream())

    istep, ig = make_graph(torch, lambda: [insert_all() for _ in range(10)], True)
    t_ins = timed(torch, istep, 3, stream) / 10
    del ig, outs
    log(f"bench: growth bookkeeping {t_ins * 1e3:.1f} us ({len(lay)} arrays, {A3} + {n_new} anchors, "
        f"{ins_bytes / (t_ins * 1e-3) / 1e12:.2f} TB/s)")

    out.update({
        "flow_densification": {"workload": f"{npx} correspondences between two 1226x370 keyframes 1 m apart "
                                           "(0.5 px noise, 20% outliers)",
                               "us": round(t_epi * 1e3, 2), "kept": kept,
                               "correspondences_per_s": round(npx / (t_epi * 1e-3), 1)},
        "anchor_growth": {"workload": f"{nv} fused points (triangulated flow points, NaN where rejected, and "
                                      f"2000 tracked points), 1 mm voxels, onto {n_akeys} anchor voxels",
                          "us": round(t_vox * 1e3, 2), "new_voxels": n_new, "dropped": n_drop,
                          "points_per_s": round(nv / (t_vox * 1e-3), 1),
                          "bookkeeping_us": round(t_ins * 1e3, 2),
                          "bookkeeping_hbm_TBs": round(ins_bytes / (t_ins * 1e-3) / 1e12, 2)},
        "loop_closure": {"workload": f"{A3} anchors (K = {K3} offsets), {len(fixes)} corrected keyframes",
                         "us": round(t_def * 1e3, 2), "anchors_in_a_frustum": moved},
        "with_optimizer": {"workload": "config 3's four-view step followed by the Adam update",
                           "ms_per_step": round(t_opt, 4), "view_iterations_per_s": round(n_views * 1000.0 / t_opt, 2),
                           "adam_ms": round(t_adam, 4), "parameters": n_opt,
                           "adam_hbm_GBs": round(28.0 * n_opt / (t_adam * 1e-3) / 1e9, 1)},
    })
    del pipe, w4

    # a per-pixel loss: config 2 (20k anchors x 10 Gaussians, one 1226x370 view, L1), its
    # step with the forward, the loss and the compositing adjoint in one pass against the
    # same step through the three separate calls
    log("bench: config 2 (L1 loss): fused forward + loss + adjoint against the separate calls")
    s2 = synth.config("C2")
    fused_ms = {}
    for fuse in (True, False):
        p2 = Pipeline(s2, device=dev, tuning=tuning.schedule(tuning.DEFAULT), fuse_l1=fuse)
        p2.fit_capacity()
        p2.status.zero_()
        for _ in range(2):
            p2.step()
        f2step, f2g = make_step(torch, p2, True)
        fused_ms[fuse] = timed(torch, f2step, max(5, args.steps), stream)
        p2.check_status()
        del f2g, p2
    out["fused_l1"] = {"workload": "config 2: 20k anchors x 10 = 200k Gaussians, one 1226x370 view, L1 loss",
                       "fused_ms": round(fused_ms[True], 4), "separate_ms": round(fused_ms[False], 4),
                       "speedup": round(fused_ms[False] / fused_ms[True], 3),
                       "iterations_per_s_fused": round(1000.0 / fused_ms[True], 1)}
    log(f"bench: config 2 step {fused_ms[True]:.3f} ms fused, {fused_ms[False]:.3f} ms separate")

    evals4 = None
    if not args.no_batched:
        log("bench: config 4 (16 partitions x 4 views), batched vs plain")
        s4 = synth.config("C4")
        c4 = choose(s4)
        sched4 = tuning.schedule(c4)
        bp = Pipeline(s4, device=dev, tile=c4["tile"], tuning=sched4)
        bp.fit_capacity()
        bp.status.zero_()
        for _ in range(2):
            bp.step()
        bstep, bg = make_step(torch, bp, True)
        tb = timed(torch, bstep, max(3, args.steps // 4), stream)
        bp.check_status()
        bp.count_evaluations()
        bp.render()
        torch.cuda.synchronize()
        evals4 = [int(t.to(torch.int64).sum().item()) for t in bp.per_pixel(bp.n_eval)]
        bp.count_evaluations(False)
        # the plain form: each view its own launch sequence (one view's anchors and MLP
        # set, its own bins) with the compositing launched non-persistently (one wave per
        # (tile, quadrant) item in tile order, whole ranges), from the host; beside it the
        # same sequences from one graph, and the per-view sequences at the batched
        # (persistent) schedule
        def per_view(sched):
            ps = []
            for sub in split_views(s4):
                p = Pipeline(sub, device=dev, tile=c4["tile"], tuning=sched)
                p.fit_capacity()
                p.status.zero_()
                ps.append(p)
            return ps

        def run_all(ps):
            for p in ps:
                p.step()

        plains = per_view(dict(sched4, non_persistent=1))
        run_all(plains)
        tp = timed(torch, lambda: run_all(plains), max(2, args.steps // 8), stream)
        pstep, pg = make_graph(torch, lambda: run_all(plains), True)
        tpg = timed(torch, pstep, max(2, args.steps // 8), stream)
        for p in plains:
            p.check_status()
        del pg
        pers = per_view(sched4)
        run_all(pers)
        tpp = timed(torch, lambda: run_all(pers), max(2, args.steps // 8), stream)
        for p in pers:
            p.check_status()
        del pers
        out["batched_vs_plain"] = {"workload": "config 4: 16 partitions (log-uniform 20k-400k Gaussians) x 4 views "
                                               "1226x370, own MLPs",
                                   "views": bp.vt.n, "view_gaussians": int(bp.vt.n_gauss),
                                   "tile": c4["tile"], "schedule": sched4, "tuning": c4["source"],
                                   "batched_ms": round(tb, 3), "plain_ms": round(tp, 3),
                                   "plain_graph_ms": round(tpg, 3), "plain_persistent_ms": round(tpp, 3),
                                   "speedup": round(tp / tb, 3), "speedup_vs_plain_graph": round(tpg / tb, 3),
                                   "speedup_vs_plain_persistent": round(tpp / tb, 3),
                                   "batched_view_iterations_per_s": round(bp.vt.n * 1000.0 / tb, 1),
                                   "plain_view_iterations_per_s": round(bp.vt.n * 1000.0 / tp, 1),
                                   "plain_graph_view_iterations_per_s": round(bp.vt.n * 1000.0 / tpg, 1),
                                   "note": "plain: the 64 views as separate launch sequences from the host, their "
                                           "compositing launched non-persistently (one wave per tile quadrant); "
                                           "plain_graph: the same sequences replayed from one graph; "
                                           "plain_persistent: the per-view sequences at the batched schedule; "
                                           "batched: one graph replay of the batched step"}
        log(f"bench: batched {tb:.2f} ms, plain {tp:.2f} ms eager / {tpg:.2f} ms graph / {tpp:.2f} ms persistent, "
            f"speedup {tp / tb:.2f}")
        del bg, bp, plains

    if not args.no_config5:
        log("bench: config 5 (2 km path, 64 partitions x 8 views)")
        torch.cuda.reset_peak_memory_stats()
        s5 = synth.config("C5")
        c5 = choose(s5)
        sched5 = tuning.schedule(c5)
        p5 = Pipeline(s5, device=dev, tile=c5["tile"], tuning=sched5)
        need5 = p5.fit_capacity()
        p5.status.zero_()
        for _ in range(2):
            p5.step()
        step5, g5 = make_step(torch, p5, True)
        for _ in range(2):
            step5()
        t5 = timed(torch, step5, 3, stream)
        p5.check_status()
        del g5
        peak5 = round(torch.cuda.max_memory_allocated() / 2 ** 30, 2)
        n_views5, g5n, pix5, pairs5 = p5.vt.n, int(p5.vt.n_gauss), int(p5.vt.n_pix), int(need5)
        # the algorithm's work is counted at the 16x16 tiles of the paper's rasterizer
        # whatever tile edge the launches use (larger tiles lengthen every pixel's list,
        # and counting those walks would credit them as work): a pipeline at 16x16 tiles
        # counts the pairs, radix passes and Gaussian-pixel evaluations of this step
        if c5["tile"] != 16:
            del p5
            torch.cuda.empty_cache()
            p5 = Pipeline(s5, device=dev, tile=16)
            need5 = p5.fit_capacity()
            p5.status.zero_()
            p5.forward()
        p5.count_evaluations()
        p5.render()
        torch.cuda.synchronize()
        ev5_fwd = int(p5.n_eval.to(torch.int64).sum().item())
        ev5_bwd = int(p5.n_contrib.to(torch.int64).sum().item())
        p5.count_evaluations(False)
        p5.check_status()
        out["config5"] = {"workload": "config 5: 2 km path, 64 partitions (log-uniform 30k-300k Gaussians), "
                                      "8 views each at 1226x370 / 1280x384 / 1280x960",
                          "views": n_views5, "view_gaussians": g5n, "pixels": pix5,
                          "pairs": pairs5, "tile": c5["tile"], "schedule": sched5, "tuning": c5["source"],
                          "step_ms": round(t5, 2),
                          "view_iterations_per_s": round(n_views5 * 1000.0 / t5, 1), "launch": "hip graph",
                          "step_roofline": whole_step_roofline(p5, t5, need5, ev5_fwd, ev5_bwd),
                          "work_counted_at_tile": 16,
                          "peak_hbm_gib": peak5}
        log(f"bench: config 5 step {t5:.2f} ms (graph, {c5['tile']}x{c5['tile']} tiles), whole-step roofline "
            f"{out['config5']['step_roofline']['frac']:.3f} (work at 16x16 tiles)")
        del p5, s5

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * 262144, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.no_cpu:
        threads = oracle_threads()
        log(f"bench: CPU oracle baseline (config 3 view 0, {threads} threads)")
        out["cpu_baseline"] = cpu_baseline(scene, 0, threads)
        log("bench: CPU oracle at configs 1 and 2 (1 thread and all), config 4 sampled")
        out["cpu_baselines"] = cpu_baselines(threads, evals4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
