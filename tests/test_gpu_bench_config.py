"""The benchmark's own workloads in the benchmark's own launch configurations: config 3
(50k anchors x 10 offsets = 500k Gaussians, 1226x370, L1 + 0.2 (1 - SSIM)) as one
mapping iteration on view 0 alone (the headline) and as the four views in one step, each
at the tuner's stored choice for it (tile edge, long-tile threshold, workgroup widths and
counts, printed by the test), the whole step replayed from a HIP graph as the benchmark
times it.

Against the oracle, at full size and on every output: the tile assignment, sort order,
ranges and longest-first order bit for bit at that tile edge; every pixel, T and
contributor count stage-wise; the 2-D gradients of the compositing adjoint, the
projection adjoint and the anchor and MLP gradients stage-wise; and end to end, raw
inputs to the images, the loss and the anchor and MLP gradients (the same bars as the
16x16 parity tests).  The graph replay reproduces an eager step: bit for bit with
reproducible gradients, and to the order of the compositing adjoint's atomics without."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (AMB_STAGE, AMB_VALUE, GAMMA_E2E, GAMMA_STAGE, U32, check_anchor_grads, check_dgauss,
                      check_e2e_pixels, check_pixels, decode_grads_magnitude, e2e_grad_magnitude, gpu_splats,
                      grad_close, host, stage_render, view_image, view_pixels, view_slices)
from paper_2607_21416_amd import tuning
from paper_2607_21416_amd.pipeline import Pipeline
from test_gpu_parity import g2d_gradients

pytestmark = pytest.mark.gpu


WORKLOADS = {"view0": lambda: synth.one_view(synth.config("C3"), 0), "four_views": lambda: synth.config("C3")}


@pytest.fixture(scope="module", params=list(WORKLOADS))
def bench_case(request):
    scene = WORKLOADS[request.param]()
    choice = tuning.autotune(scene, device="cuda")  # the stored choice: nothing is measured
    assert choice["source"] == "stored"
    tile = choice["tile"]
    print(f"config 3 ({request.param}) at tile {tile}, schedule {tuning.schedule(choice)}", flush=True)
    pipe = Pipeline(scene, device="cuda", tile=tile, tuning=tuning.schedule(choice))
    pipe.fit_capacity()
    pipe.status.zero_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipe.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipe.step()
    for _ in range(3):
        pipe.image.fill_(-1.0)  # the replay must overwrite it
        g.replay()
    torch.cuda.synchronize()
    pipe.check_status()
    return scene, choice, pipe, host(pipe), g


def _view_inputs(h, sl):
    pr, gs = gpu_splats(h, sl)
    vals = h["vals"].astype(np.int64) - sl["g0"]
    ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
    return pr, gs, vals, ranges


def test_sort_bit_exact(bench_case):
    scene, choice, pipe, h, _ = bench_case
    tile = choice["tile"]
    sls = view_slices(pipe)
    G = h["ntiles"].shape[0]
    prect = np.zeros((4, G), np.int32)
    nt = np.zeros(G, np.int32)
    for sl in sls:
        g0, g1 = sl["g0"], sl["g1"]
        prect[:, g0:g1], nt[g0:g1] = oracle.rect_f32(h["uv"][0, g0:g1], h["uv"][1, g0:g1], h["ext"][0, g0:g1],
                                                     h["ext"][1, g0:g1], sl["W"], sl["H"], (tile, tile))
    assert np.array_equal(nt, h["ntiles"])
    gb = [sl["g0"] for sl in sls] + [sls[-1]["g1"]]
    ref = oracle.bin_sort(prect, nt, h["depth"].astype(np.float64), gb, scene["cams"], (tile, tile))
    # every visible view-Gaussian has a pair, and the views are the full-size ones (about
    # 0.14M of each view's 0.5M Gaussians visible; 0.59M pairs per view at 16x16 tiles,
    # 0.31M at 32x32)
    assert h["P"] == ref["P"] >= int((nt > 0).sum()) > 10 ** 5 * len(sls)
    assert np.array_equal(h["vals"], ref["vals"])
    assert np.array_equal((h["keys"] >> np.uint64(h["dbits"])).astype(np.int64), ref["tiles"].astype(np.int64))
    assert np.array_equal(h["ranges"], ref["ranges"])
    lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    long_min = 1 << choice["long_log2"]
    n_long = int((lens >= long_min).sum())
    assert n_long > 0 and int(pipe.status.cpu().numpy()[7]) == n_long
    order = pipe.order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(lens)))
    assert (lens[order[:n_long]] >= long_min).all() and (lens[order[n_long:]] < long_min).all()


def test_forward_stagewise(bench_case):
    scene, choice, pipe, h, _ = bench_case
    tile = choice["tile"]
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs, vals, ranges = _view_inputs(h, sl)
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v], tile=(tile, tile))
        check_pixels(view_image(h, sl), view_pixels(h, sl, "T_final"), view_pixels(h, sl, "n_contrib"), ref,
                     f"config 3 view {v}")


def test_backward_stagewise(bench_case):
    scene, choice, pipe, h, _ = bench_case
    tile = choice["tile"]
    sls = view_slices(pipe)
    dims = []
    for v, sl in enumerate(sls):
        pr, gs, vals, ranges = _view_inputs(h, sl)
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v], tile=(tile, tile))
        _, _, _, d = oracle.loss(view_image(h, sl).astype(np.float64), scene["targets"][v], scene["ssim_weight"])
        d[:, (ref["amb"] & (AMB_STAGE | oracle.AMB_CLAMP)) != 0] = 0.0
        dims.append(d)
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.backward(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    hb = host(pipe)
    acc = oracle.zero_grads(scene)
    dgs, scales = {}, {}
    for v, sl in enumerate(sls):
        pr, gs, vals, ranges = _view_inputs(h, sl)
        g2d = oracle.render_bwd(pr, gs, vals, ranges, scene["cams"][v], dims[v], tile=(tile, tile))
        got = g2d_gradients(hb["g2d"][sl["g0"]:sl["g1"]], h["conic"][:, sl["g0"]:sl["g1"]])
        for k, nm in enumerate(("u", "v", "A", "B", "C", "opacity", "r", "g", "b")):
            grad_close(got[k], g2d[k], name=f"config 3 view {v} d{nm}")
        gin = {k: hb["dec"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dec"]}
        dgp = oracle.project_bwd(gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got.astype(np.float64))
        dgv = {k: hb["dg"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dg"]}
        check_dgauss(dgv, dgp, gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got, f"config 3 view {v}")
        oracle.decode_bwd(scene, scene["cams"][v]["partition"], scene["cams"][v], dgv, acc)
        dgs[v], scales[v] = dgv, gin["scale"]
    check_anchor_grads(hb["pgrad"], acc, scene, dgs, scales, "config 3 anchor")


def test_end_to_end(bench_case):
    scene, choice, pipe, h, _ = bench_case
    fwd = oracle.forward(scene)
    dims = []
    for v, (sl, r) in enumerate(zip(view_slices(pipe), fwd)):
        check_e2e_pixels(view_image(h, sl), r, h, sl, scene["cams"][v], f"config 3 view {v}",
                         tile=(choice["tile"], choice["tile"]))
        assert h["loss"][v] == pytest.approx(r["loss"], rel=1e-4)
        d = r["dimage"].copy()
        d[:, (r["amb"] & (AMB_VALUE | oracle.AMB_CLAMP)) != 0] = 0.0
        dims.append(d)
    ref = oracle.backward(scene, fwd, dimages=dims)
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.backward(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    got = host(pipe)["pgrad"]
    mag = e2e_grad_magnitude(scene, fwd, dims)
    for k in ref:
        grad_close(got[k], ref[k], name=f"config 3 end-to-end d{k}", mag=mag[k], gamma=GAMMA_E2E)


def test_replay_equals_eager_step(bench_case):
    """The graph replay the benchmark times against an eager step.  Everything but the
    compositing adjoint is independent of the order of execution, so the forward, the
    sort, dL/dC and the losses agree bit for bit.  The adjoint's 2-D gradients are sums
    of FP32 atomics in whatever order the waves reach them, so they and the Gaussian
    gradients are compared in L2; the decode adjoint is deterministic and linear in its
    incoming Gaussian gradients dg, so per anchor and MLP element the two steps differ by
    at most M(|dg_replay - dg_eager|) + 2 GAMMA_STAGE u M(|dg|), M the magnitudes of the
    decode adjoint's terms (the difference carried through, plus each evaluation's own
    rounding)."""
    scene, choice, pipe, h, g = bench_case
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    e = host(pipe)
    for k in ("image", "T_final", "n_contrib", "dimage", "keys", "vals", "ranges"):
        assert np.array_equal(h[k], e[k]), k
    np.testing.assert_allclose(h["loss"], e["loss"], rtol=1e-5)

    def l2_rel(a, b):
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)

    assert l2_rel(h["g2d"], e["g2d"]) <= 1e-5
    for k in e["dg"]:
        assert l2_rel(h["dg"][k], e["dg"][k]) <= 1e-5, k
    d_abs, d_ref, scales = {}, {}, {}
    for v, sl in enumerate(view_slices(pipe)):
        cut = slice(sl["g0"], sl["g1"])
        d_abs[v] = {k: np.abs(h["dg"][k][..., cut].astype(np.float64) - e["dg"][k][..., cut]) for k in e["dg"]}
        d_ref[v] = {k: e["dg"][k][..., cut].astype(np.float64) for k in e["dg"]}
        scales[v] = e["dec"]["scale"][..., cut].astype(np.float64)
    m_diff = decode_grads_magnitude(scene, d_abs, scales)
    m_ref = decode_grads_magnitude(scene, d_ref, scales)
    worst = 0.0
    for k in e["pgrad"]:
        a, b = h["pgrad"][k].astype(np.float64), e["pgrad"][k].astype(np.float64)
        err = np.abs(a - b)
        bound = np.maximum(1e-5 * np.abs(b) + 1e-6 * np.abs(b).max(),
                           m_diff[k] * (1 + 1e-6) + 2 * GAMMA_STAGE * U32 * m_ref[k])
        bad = err > bound
        assert not bad.any(), (f"replay d{k}: {int(bad.sum())} of {bad.size} elements off; worst "
                               f"{err[bad].max():.3e} against {bound[bad][np.argmax(err[bad])]:.3e}")
        assert l2_rel(a, b) <= 1e-5, k
        worst = max(worst, float(np.max(err / np.maximum(bound, 1e-300))))
    print(f"replay against eager: largest anchor/MLP gradient difference {worst:.3f} of its bound", flush=True)


def test_replay_equals_eager_step_reproducible(bench_case):
    """With reproducible gradients (GLAM_DETERMINISTIC_GRADS: per-(pair, quadrant)
    partials and a fixed-order reduction in place of the atomics) nothing in the step
    depends on the order of execution, so the graph replay of the benchmark's step at its
    launch configuration equals an eager step bit for bit, gradients included."""
    scene, choice, _, _, _ = bench_case
    pipe = Pipeline(scene, device="cuda", tile=choice["tile"], tuning=tuning.schedule(choice), deterministic=True)
    pipe.fit_capacity()
    pipe.status.zero_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipe.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pipe.step()
    for _ in range(2):
        pipe.image.fill_(-1.0)
        graph.replay()
    torch.cuda.synchronize()
    pipe.check_status()
    h = host(pipe)
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    e = host(pipe)
    for k in ("image", "T_final", "n_contrib", "dimage", "keys", "vals", "ranges", "loss", "g2d"):
        assert np.array_equal(h[k], e[k]), k
    for grp in ("dg", "pgrad"):
        for k in e[grp]:
            assert np.array_equal(h[grp][k], e[grp][k]), (grp, k)
    del pipe, graph
    torch.cuda.empty_cache()
