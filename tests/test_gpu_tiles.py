"""The binning tile edge and the compositing schedule change the work decomposition,
never the result: with 8x8 and 32x32 tiles (one and sixteen 8x8 compositing quadrants
per tile) and non-default schedules (a low long-tile threshold, smaller persistent
grids, long tiles shared by workgroups of 8 and 16 waves, no persistent grid at all),
the tile assignment, sort order and ranges match the oracle's at that tile edge bit for
bit, the long tiles are counted and listed first, and the pixels and the 2-D gradients
match the oracle stage-wise (same bars as the 16x16 parity tests)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (AMB_STAGE, check_pixels, gpu_splats, grad_close, host, run, stage_render, view_image, view_pixels,
                      view_slices)
from test_gpu_parity import _masked_dimage, anchor_small, g2d_gradients, plain_dense, plain_ragged

pytestmark = pytest.mark.gpu

SCENES = {"plain_ragged": plain_ragged, "anchor_small": anchor_small, "plain_dense": plain_dense}
SCHEDULES = {
    "narrow": {"long_log2": 8, "fwd_blocks_per_cu": 3, "bwd_blocks_per_cu": 4},
    # every range of 128 entries or more walked by 16 waves: a round of up to 1024 entries,
    # chunks of 8..64, pixels that stop inside a round (plain_dense)
    "wide16": {"long_log2": 7, "fwd_group_waves": 16, "bwd_group_waves": 16},
    "wide8": {"long_log2": 8, "fwd_group_waves": 8, "fwd_blocks_per_cu": 1, "bwd_group_waves": 8,
              "bwd_blocks_per_cu": 2},
    # forward and backward at different widths
    "mixed": {"long_log2": 7, "fwd_group_waves": 16, "bwd_group_waves": 4},
    # no persistent grid: one wave per (tile, quadrant) item in tile order, whole ranges
    "direct": {"long_log2": 7, "non_persistent": 1},
}
CASES = ([(t, n, "narrow") for t in (8, 32) for n in SCENES] + [(16, n, "wide16") for n in SCENES]
         + [(t, "plain_dense", "wide8") for t in (8, 32)]
         + [(16, n, "mixed") for n in ("plain_dense", "anchor_small")]
         + [(t, n, "direct") for t in (8, 16, 32) for n in ("plain_dense", "anchor_small")])


@pytest.fixture(scope="module", params=CASES, ids=lambda p: f"tile{p[0]}-{p[1]}-{p[2]}")
def case(request):
    tile, name, sched = request.param
    scene = SCENES[name]()
    print(f"tile {tile}, {name}, schedule {SCHEDULES[sched]}", flush=True)
    pipe = run(scene, tile=tile, tuning=SCHEDULES[sched])
    return tile, name, scene, pipe, host(pipe), SCHEDULES[sched]


def test_bin_sort_bit_exact(case):
    tile, name, scene, pipe, h, sched = case
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
    n_long = int((lens >= 1 << sched["long_log2"]).sum())
    assert int(pipe.status.cpu().numpy()[7]) == n_long
    order = pipe.order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(lens)))
    assert (lens[order[:n_long]] >= 1 << sched["long_log2"]).all()
    assert (lens[order[n_long:]] < 1 << sched["long_log2"]).all()


def test_render_fwd_stagewise(case):
    tile, name, scene, pipe, h, sched = case
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v], tile=(tile, tile))
        check_pixels(view_image(h, sl), view_pixels(h, sl, "T_final"), view_pixels(h, sl, "n_contrib"), ref,
                     f"tile {tile} {name} view {v}", n_eval=view_pixels(h, sl, "n_eval"))


def test_composite_bwd_stagewise(case):
    tile, name, scene, pipe, h, sched = case
    dims = []
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v], tile=(tile, tile))
        _, _, _, d = oracle.loss(view_image(h, sl).astype(np.float64), scene["targets"][v], scene["ssim_weight"])
        d[:, (ref["amb"] & (AMB_STAGE | oracle.AMB_CLAMP)) != 0] = 0.0
        dims.append(d)
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.composite_bwd(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    g2d_gpu = pipe.g2d.cpu().numpy()
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        g2d = oracle.render_bwd(pr, gs, vals, ranges, scene["cams"][v], dims[v], tile=(tile, tile))
        got = g2d_gradients(g2d_gpu[sl["g0"]:sl["g1"]], h["conic"][:, sl["g0"]:sl["g1"]])
        for k, nm in enumerate(("u", "v", "A", "B", "C", "opacity", "r", "g", "b")):
            grad_close(got[k], g2d[k], name=f"tile {tile} {name} view {v} d{nm}")


def test_images_agree_across_tile_edges(case):
    # the image does not depend on the tile edge (opacity-aware footprints): the 16x16
    # default reproduces the same pixels except where a decision sits within rounding
    tile, name, scene, pipe, h, sched = case
    ref_pipe = run(scene)
    hr = host(ref_pipe)
    for v, sl in enumerate(view_slices(pipe)):
        fwd = oracle.forward(scene, views=[v])[0]
        ok = (fwd["amb"] & (AMB_STAGE | oracle.AMB_DEPTH)) == 0
        a, b = view_image(h, sl), view_image(hr, sl)
        assert np.abs(a - b)[:, ok].max() <= 2e-4


def test_autotuner_choice_is_valid_and_harmless():
    from paper_2607_21416_amd import tuning
    scene = anchor_small()
    choice = tuning.autotune(scene, iters=2, use_cache=False)
    assert choice["tile"] in tuning.TILES and choice["long_log2"] in tuning.LONG_LOG2
    s = tuning.schedule(choice)
    assert (s["fwd_group_waves"], s["fwd_blocks_per_cu"]) in tuning.FWD_GRIDS
    assert (s["bwd_group_waves"], s["bwd_blocks_per_cu"]) in tuning.BWD_GRIDS
    a = host(run(scene, tile=choice["tile"], tuning=tuning.schedule(choice)))
    b = host(run(scene))
    np.testing.assert_allclose(a["loss"], b["loss"], rtol=1e-5)
    for k in b["pgrad"]:
        grad_close(a["pgrad"][k], b["pgrad"][k], rel=1e-4, floor=1e-5, norm_rel=1e-4, name=f"tuned d{k}")
