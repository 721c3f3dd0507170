"""Parity of the HIP path with the FP64 oracle, stage by stage and end to end.

Stage-wise: each GPU stage's output is compared with the oracle's same stage fed the
GPU's own inputs to that stage, so that FP32-vs-FP64 differences upstream cannot move
a discrete decision: tile assignment, sort order and ranges bit-exact; pixels within
1e-4 absolute; gradients within 1e-3 relative (plus a floor of 1e-5 of the tensor's
largest entry for cancelling sums); decode within 1e-5 relative (plus 1e-5 of the
field's largest entry for cancelling dot products).
End to end: raw inputs -> pixels within 1e-4 and gradients within 1e-3, on pixels the
oracle does not flag as ambiguous (a threshold, stop or depth order within rounding).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (AMB_STAGE, AMB_VALUE, gpu_splats, grad_close, host, run, unpack_box, view_image, view_pixels,
                      view_slices)

pytestmark = pytest.mark.gpu


def plain_ragged():
    return synth.plain_scene(1011, 2000, 70, 45)


def plain_dense():
    # 20k faint Gaussians on 64x48: every tile's range holds 1000-4000 entries (the
    # workgroup path for long tiles) and about 40% of the pixels stop between entries
    # 1400 and 2400, i.e. inside its chunks and rounds
    s = synth.plain_scene(1015, 20000, 64, 48)
    s["logit"] = (s["logit"] - 1.8).astype(np.float32)
    return s


def anchor_small():
    # two partitions with uneven anchor counts, two views each, ragged 200x120 tiles
    return synth.anchor_scene(1012, [1500, 800], 2, W=200, H=120, fx=140.0, ssim_weight=0.2, bias_std=0.2)


def partition_without_anchors():
    # a partition whose only view has no anchors next to two populated ones
    return synth.anchor_scene(1013, [600, 0, 300], 1, W=96, H=64, fx=70.0, ssim_weight=0.2)


def partition_without_views():
    # the middle partition has anchors but no view: its gradients must be zero
    s = synth.anchor_scene(1014, [500, 400, 300], 1, W=96, H=64, fx=70.0, ssim_weight=0.2)
    keep = [i for i, c in enumerate(s["cams"]) if c["partition"] != 1]
    s["cams"] = [s["cams"][i] for i in keep]
    s["targets"] = [s["targets"][i] for i in keep]
    return s


# full-size workloads: config 2 (20k anchors, one 1226x370 view) and config 3 (50k
# anchors, four views, the benchmark's workload)
SCENES = {"C1": lambda: synth.config("C1"), "plain_ragged": plain_ragged, "plain_dense": plain_dense,
          "anchor_small": anchor_small,
          "empty_partition": partition_without_anchors, "viewless_partition": partition_without_views,
          "C2": lambda: synth.config("C2"),
          "C3": lambda: synth.config("C3")}


@pytest.fixture(scope="module", params=list(SCENES))
def case(request):
    scene = SCENES[request.param]()
    pipe = run(scene)
    return request.param, scene, pipe, host(pipe)


def g2d_gradients(g2d, conic):
    """The 2-D gradients d(u, v, A, B, C, opacity, r, g, b) [9][n] from the kernel's
    accumulators: moments m of dL/dpower and the conic (A, B, C), as the projection
    adjoint forms them: du = -(A m0 + B m1), dv = -(B m0 + C m1), dA = -m2/2, dB = -m3,
    dC = -m4/2."""
    m = g2d.T.astype(np.float64)
    A, B, C = conic.astype(np.float64)
    out = m.copy()
    out[0] = -(A * m[0] + B * m[1])
    out[1] = -(B * m[0] + C * m[1])
    out[2] = -0.5 * m[2]
    out[3] = -m[3]
    out[4] = -0.5 * m[4]
    return out


def oracle_gauss(scene, v):
    return oracle.view_gaussians(scene, v)


def _gpu_gaussians(scene, h, v, sl):
    """The Gaussians the GPU projected for view v: its own decode output in anchor
    mode (so the projection is compared stage-wise), the plain activation otherwise."""
    if scene["kind"] == "plain":
        return oracle_gauss(scene, v)
    return {k: h["dec"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in h["dec"]}


def test_project(case):
    name, scene, pipe, h = case
    for v, sl in enumerate(view_slices(pipe)):
        cam = scene["cams"][v]
        g0, g1 = sl["g0"], sl["g1"]
        if g1 == g0:
            continue
        gs = _gpu_gaussians(scene, h, v, sl)
        ref = oracle.project(gs, cam)
        vis_g = h["ntiles"][g0:g1] > 0
        vis_o = ref["ntiles"] > 0
        # visibility agrees except within rounding of the cull thresholds
        diff = vis_g != vis_o
        near = (np.abs(255 * gs["opacity"] - 1) < 1e-4) | (np.abs(ref["depth"] - 0.2) < 1e-5)
        assert not (diff & ~near).any()
        both = vis_g & vis_o
        for key in ("uv", "conic"):
            a = h[key][:, g0:g1][:, both].astype(np.float64)
            b = ref[key][:, both]
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-5 * np.abs(b).max(), err_msg=key)
        # the extent scales with sqrt(ln(255 opacity)): its relative rounding error grows
        # like (ulp of 255 opacity) / (2 ln(255 opacity)) as the opacity nears 1/255
        a = h["ext"][:, g0:g1][:, both].astype(np.float64)
        b = ref["ext"][:, both]
        lg = np.log(255.0 * gs["opacity"][both])
        tol = 1e-5 * np.abs(b) + 1e-5 * np.abs(b).max() + np.abs(b) * 1e-6 / np.maximum(lg, 1e-12)
        assert (np.abs(a - b) <= tol).all(), np.abs(a - b).max()
        np.testing.assert_allclose(h["depth"][g0:g1][both], ref["depth"][both], rtol=1e-6)
        # tile assignment bit-exact given the GPU's single-precision centre and extents
        prect, nt = oracle.rect_f32(h["uv"][0, g0:g1], h["uv"][1, g0:g1], h["ext"][0, g0:g1],
                                    h["ext"][1, g0:g1], sl["W"], sl["H"])
        assert np.array_equal(nt, h["ntiles"][g0:g1])
        box = unpack_box(h["splat"][g0:g1])
        assert np.array_equal(box[:, vis_g], prect[:, vis_g])


def test_bin_sort_bit_exact(case):
    name, scene, pipe, h = case
    sls = view_slices(pipe)
    G = h["ntiles"].shape[0]
    prect = np.zeros((4, G), np.int32)
    nt = np.zeros(G, np.int32)
    for sl in sls:
        g0, g1 = sl["g0"], sl["g1"]
        prect[:, g0:g1], nt[g0:g1] = oracle.rect_f32(h["uv"][0, g0:g1], h["uv"][1, g0:g1], h["ext"][0, g0:g1],
                                                     h["ext"][1, g0:g1], sl["W"], sl["H"])
    gb = [sl["g0"] for sl in sls] + [sls[-1]["g1"]]
    ref = oracle.bin_sort(prect, nt, h["depth"].astype(np.float64), gb, scene["cams"])
    assert h["P"] == ref["P"]
    assert np.array_equal(h["vals"], ref["vals"])
    assert np.array_equal((h["keys"] >> np.uint64(h["dbits"])).astype(np.int64), ref["tiles"].astype(np.int64))
    # the low bits are the depth key: bit pattern minus that of 0.2f, lossless
    dk = (h["keys"] & np.uint64((1 << h["dbits"]) - 1)).astype(np.uint64)
    want = h["depth"][h["vals"]].view(np.uint32).astype(np.uint64) - np.uint64(0x3E4CCCCD)
    assert np.array_equal(dk, want)
    assert np.array_equal(h["ranges"], ref["ranges"])
    # the long tiles (ranges of 1024+ entries) are counted and listed first in the order
    lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    n_long = int((lens >= 1024).sum())
    assert int(pipe.status.cpu().numpy()[7]) == n_long
    order = pipe.order.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(len(lens)))
    assert (lens[order[:n_long]] >= 1024).all() and (lens[order[n_long:]] < 1024).all()


def test_render_fwd_stagewise(case):
    name, scene, pipe, h = case
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = oracle.render_fwd(pr, gs, vals, ranges, scene["cams"][v])
        ok = (ref["amb"] & AMB_STAGE) == 0
        assert ok.mean() > 0.95
        img = view_image(h, sl)
        err = np.abs(img - ref["image"])[:, ok]
        assert err.max() <= 1e-4, err.max()
        assert np.abs(view_pixels(h, sl, "T_final") - ref["T_final"])[ok].max() <= 1e-4
        assert np.array_equal(view_pixels(h, sl, "n_contrib")[ok], ref["n_contrib"][ok])
        assert np.array_equal(view_pixels(h, sl, "n_eval")[ok], ref["n_eval"][ok])
        # ambiguous pixels stay within the loose bound
        assert np.abs(img - ref["image"]).max() <= 0.02 or (~ok).sum() > 0


def test_loss_kernel(case):
    name, scene, pipe, h = case
    for v, sl in enumerate(view_slices(pipe)):
        img = view_image(h, sl).astype(np.float64)
        L, _, _, dimg = oracle.loss(img, scene["targets"][v], scene["ssim_weight"])
        assert h["loss"][v] == pytest.approx(L, rel=1e-5)
        got = view_image(h, sl, "dimage")
        # L1 sign flips only where the FP32 image equals the target to rounding
        tie = np.abs(img - scene["targets"][v]) < 1e-6
        grad_close(got[~tie], dimg[~tie], rel=1e-3, floor=1e-4, name="dL/dC")


def _masked_dimage(h, scene, pipe):
    """The oracle's dL/dC of the GPU image with ambiguous pixels zeroed, per view."""
    out, amb_all = [], []
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = oracle.render_fwd(pr, gs, vals, ranges, scene["cams"][v])
        _, _, _, d = oracle.loss(view_image(h, sl).astype(np.float64), scene["targets"][v], scene["ssim_weight"])
        amb = (ref["amb"] & (AMB_STAGE | oracle.AMB_CLAMP)) != 0
        d[:, amb] = 0.0
        out.append(d)
        amb_all.append(amb)
    return out, amb_all


def test_backward_stagewise(case):
    name, scene, pipe, h = case
    dims, _ = _masked_dimage(h, scene, pipe)
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.backward(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    hb = host(pipe)
    sls = view_slices(pipe)
    acc = oracle.zero_grads(scene)
    for v, sl in enumerate(sls):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        g2d = oracle.render_bwd(pr, gs, vals, ranges, scene["cams"][v], dims[v])
        got = g2d_gradients(hb["g2d"][sl["g0"]:sl["g1"]], h["conic"][:, sl["g0"]:sl["g1"]])
        for k, nm in enumerate(("u", "v", "A", "B", "C", "opacity", "r", "g", "b")):
            grad_close(got[k], g2d[k], name=f"{name} view {v} d{nm}")
        # projection adjoint fed the GPU's 2-D gradients and (anchor mode) decoded Gaussians
        if scene["kind"] == "plain":
            gin = oracle.plain_activate(scene)
        else:
            gin = {k: hb["dec"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dec"]}
        dgp = oracle.project_bwd(gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got.astype(np.float64))
        if scene["kind"] == "plain":
            d = oracle.plain_activate_bwd(scene, dgp)
            for k in acc:
                acc[k] += d[k]
        else:
            for k, gk in (("mean", "mean"), ("scale", "scale"), ("quat", "quat"), ("opacity", "opacity"),
                          ("rgb", "rgb")):
                grad_close(hb["dg"][gk][..., sl["g0"]:sl["g1"]], dgp[k], name=f"{name} view {v} dgauss {k}")
            dgv = {k: hb["dg"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dg"]}
            oracle.decode_bwd(scene, scene["cams"][v]["partition"], scene["cams"][v], dgv, acc)
    if scene["kind"] == "plain":
        for k in acc:
            grad_close(hb["dg"][k], acc[k], name=f"{name} plain d{k}")
    else:
        for k in acc:
            grad_close(hb["pgrad"][k], acc[k], name=f"{name} anchor d{k}")


def test_decode_stagewise(case):
    name, scene, pipe, h = case
    if scene["kind"] == "plain":
        pytest.skip("plain scene has no decode")
    for v, sl in enumerate(view_slices(pipe)):
        ref = oracle.decode(scene, scene["cams"][v]["partition"], scene["cams"][v])
        assert ref["opacity"].shape[-1] == sl["g1"] - sl["g0"]
        if sl["g1"] == sl["g0"]:
            continue
        for k in ("mean", "scale", "quat", "opacity", "rgb"):
            got = h["dec"][k][..., sl["g0"]:sl["g1"]]
            np.testing.assert_allclose(got, ref[k], rtol=1e-5, atol=1e-5 * max(np.abs(ref[k]).max(), 1e-30),
                                       err_msg=k)


def test_end_to_end(case):
    name, scene, pipe, h = case
    fwd = oracle.forward(scene)
    dims = []
    for v, (sl, r) in enumerate(zip(view_slices(pipe), fwd)):
        ok = (r["amb"] & AMB_VALUE) == 0
        assert ok.mean() > 0.85
        img = view_image(h, sl)
        assert np.abs(img - r["image"])[:, ok].max() <= 1e-4
        assert h["loss"][v] == pytest.approx(r["loss"], rel=1e-4)
        d = r["dimage"].copy()
        d[:, (r["amb"] & (AMB_VALUE | oracle.AMB_CLAMP)) != 0] = 0.0
        dims.append(d)
    ref = oracle.backward(scene, fwd, dimages=dims)
    flat = np.concatenate([d.reshape(-1) for d in dims]).astype(np.float32)
    pipe.backward(dimage=torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    hb = host(pipe)
    got = hb["dg"] if scene["kind"] == "plain" else hb["pgrad"]
    for k in ref:
        grad_close(got[k], ref[k], rel=1e-3, floor=1e-5, name=f"{name} end-to-end d{k}")


def test_empty_and_overflow():
    # every Gaussian behind the camera: no pairs, background image, zero gradients
    s = synth.plain_scene(5, 100, 40, 30)
    s["mean"][2] = -5.0
    pipe = run(s)
    h = host(pipe)
    assert h["P"] == 0 and np.all(h["ranges"] == 0)
    assert np.all(h["image"] == 0) and np.all(h["T_final"] == 1) and np.all(h["n_contrib"] == 0)
    assert np.all(h["dg"]["mean"] == 0)
    # pair capacity overflow is reported, not written past
    s = synth.config("C1")
    from paper_2607_21416_amd.pipeline import Pipeline
    pipe = Pipeline(s, device="cuda", capacity=64)
    guard = pipe.keys.new_zeros(0)
    pipe.forward()
    torch.cuda.synchronize()
    st = pipe.status.cpu().numpy()
    assert st[0] == 3  # GLAM_ERR_CAPACITY
    assert pipe.pair_count() == oracle.forward(s)[0]["bins"]["P"]
    del guard
