"""The batched benchmark workload in its own launch configuration: config 4 (16
partitions of 2k-40k anchors, own MLP sets, 4 views each = 64 views at 1226x370) at the
tuner's stored choice for it (16x16 tiles, long tiles >= 2^12, 5/6 workgroups per CU),
the whole step replayed from a HIP graph.

Against the oracle: the sort over all 64 views (tile assignment, order, ranges and the
longest-first order) bit for bit; and on a sample of views from different partitions,
every pixel stage-wise, then the backward fed dL/dC on those views only (zero elsewhere):
their 2-D and Gaussian gradients stage-wise, and the anchor and MLP gradients of every
partition (zero where no sampled view looks) against the oracle's adjoint of the sampled
views."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (AMB_STAGE, check_anchor_grads, check_dgauss, check_pixels, gpu_splats, grad_close, host,
                      stage_render, view_image, view_pixels, view_slices)
from paper_2607_21416_amd import tuning
from paper_2607_21416_amd.pipeline import Pipeline
from test_gpu_parity import g2d_gradients

pytestmark = pytest.mark.gpu

SAMPLE = (0, 21, 42, 63)  # views of partitions 0, 5, 10 and 15


@pytest.fixture(scope="module")
def batched_case():
    scene = synth.config("C4")
    choice = tuning.autotune(scene, device="cuda")  # the stored choice: nothing is measured
    assert choice["source"] == "stored"
    tile = choice["tile"]
    print(f"config 4 at tile {tile}, schedule {tuning.schedule(choice)}", flush=True)
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
    for _ in range(2):
        pipe.image.fill_(-1.0)
        g.replay()
    torch.cuda.synchronize()
    pipe.check_status()
    assert len(scene["cams"]) == 64 and len({scene["cams"][v]["partition"] for v in SAMPLE}) == len(SAMPLE)
    return scene, choice, pipe, host(pipe)


def _view_inputs(h, sl):
    pr, gs = gpu_splats(h, sl)
    vals = h["vals"].astype(np.int64) - sl["g0"]
    ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
    return pr, gs, vals, ranges


def test_sort_bit_exact(batched_case):
    scene, choice, pipe, h = batched_case
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
    assert h["P"] == ref["P"]
    assert np.array_equal(h["vals"], ref["vals"])
    assert np.array_equal((h["keys"] >> np.uint64(h["dbits"])).astype(np.int64), ref["tiles"].astype(np.int64))
    assert np.array_equal(h["ranges"], ref["ranges"])
    lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    long_min = 1 << choice["long_log2"]
    n_long = int((lens >= long_min).sum())
    assert int(pipe.status.cpu().numpy()[7]) == n_long
    order = pipe.order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(lens)))
    assert (lens[order[:n_long]] >= long_min).all() and (lens[order[n_long:]] < long_min).all()


def test_sampled_views_forward_and_backward(batched_case):
    scene, choice, pipe, h = batched_case
    tile = choice["tile"]
    sls = view_slices(pipe)
    dims = [np.zeros((3, sl["H"], sl["W"])) for sl in sls]
    for v in SAMPLE:
        sl = sls[v]
        pr, gs, vals, ranges = _view_inputs(h, sl)
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v], tile=(tile, tile))
        check_pixels(view_image(h, sl), view_pixels(h, sl, "T_final"), view_pixels(h, sl, "n_contrib"), ref,
                     f"config 4 view {v}")
        _, _, _, d = oracle.loss(view_image(h, sl).astype(np.float64), scene["targets"][v], scene["ssim_weight"])
        d[:, (ref["amb"] & (AMB_STAGE | oracle.AMB_CLAMP)) != 0] = 0.0
        dims[v] = d
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.backward(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    hb = host(pipe)
    acc = oracle.zero_grads(scene)
    dgs, scales = {}, {}
    for v in SAMPLE:
        sl = sls[v]
        pr, gs, vals, ranges = _view_inputs(h, sl)
        g2d = oracle.render_bwd(pr, gs, vals, ranges, scene["cams"][v], dims[v], tile=(tile, tile))
        got = g2d_gradients(hb["g2d"][sl["g0"]:sl["g1"]], h["conic"][:, sl["g0"]:sl["g1"]])
        for k, nm in enumerate(("u", "v", "A", "B", "C", "opacity", "r", "g", "b")):
            grad_close(got[k], g2d[k], name=f"config 4 view {v} d{nm}")
        gin = {k: hb["dec"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dec"]}
        dgp = oracle.project_bwd(gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got.astype(np.float64))
        dgv = {k: hb["dg"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dg"]}
        check_dgauss(dgv, dgp, gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got, f"config 4 view {v}")
        oracle.decode_bwd(scene, scene["cams"][v]["partition"], scene["cams"][v], dgv, acc)
        dgs[v], scales[v] = dgv, gin["scale"]
    # views outside the sample got dL/dC = 0: their 2-D gradients vanish exactly
    others = np.ones(hb["g2d"].shape[0], bool)
    for v in SAMPLE:
        others[sls[v]["g0"]:sls[v]["g1"]] = False
    assert not hb["g2d"][others].any()
    check_anchor_grads(hb["pgrad"], acc, scene, dgs, scales, "config 4 anchor")
