"""Parity of the HIP path with the FP64 oracle, stage by stage and end to end.

Stage-wise: each GPU stage's output is compared with the oracle's same stage fed the
GPU's own inputs to that stage, so that FP32-vs-FP64 differences upstream cannot move
a discrete decision: tile assignment, sort order and ranges bit-exact; pixels within
1e-4 absolute off the pixels whose skip or stop decision lies within FP32 rounding of
its threshold (at most 0.5% of a view's pixels, each within 0.02); gradients within
1e-3 relative plus 1e-6 of the tensor's largest element; decoded values within 1e-5
relative plus the FP32 rounding bound of the MLP sums behind them; projected centres
and conics within the rounding bound of their own arithmetic.
End to end: raw inputs -> pixels within 1e-4 off the flagged pixels (a threshold, stop
or depth order within rounding), and every pixel, depth near-ties included, within 1e-4
of the oracle composited in the GPU's order off threshold and stop ambiguities;
gradients within 1e-3 relative plus 1e-6 of the largest.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2607_21416_amd.pipeline import Pipeline
from gpu_util import (AMB_STAGE, AMB_VALUE, DECODE_GAMMA, GAMMA_E2E, U32, check_anchor_grads, check_dgauss,
                      check_e2e_pixels, check_pixels, decode_magnitude, e2e_grad_magnitude, gpu_splats, grad_close,
                      host, projection_bounds, run, stage_render, unpack_box, view_image, view_pixels, view_slices)

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


def anchor_feat8():
    # the feature width the paper prints (F = 8), two partitions
    return synth.anchor_scene(1016, [900, 500], 2, W=160, H=100, fx=110.0, F=8, ssim_weight=0.2, bias_std=0.2)


def anchor_feat64():
    # a wide feature vector (F = 64): layer 1 runs over 17 K-steps
    return synth.anchor_scene(1017, [700, 400], 1, W=150, H=90, fx=100.0, F=64, ssim_weight=0.2, bias_std=0.2)


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
          "anchor_small": anchor_small, "anchor_feat8": anchor_feat8, "anchor_feat64": anchor_feat64,
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
        uvs, kappa = projection_bounds(gs, cam, ref)
        # centres: a few roundings (R mu + t, the division, fx x + cx) of their scale
        duv = np.abs(h["uv"][:, g0:g1][:, both].astype(np.float64) - ref["uv"][:, both])
        assert (duv <= 16 * U32 * uvs[:, both]).all(), np.max(duv / (16 * U32 * uvs[:, both]))
        # conics per element: A and C relative to themselves, B relative to sqrt(A C),
        # within 1e-5, widened by the determinant's condition where a c ~ b^2
        a = h["conic"][:, g0:g1][:, both].astype(np.float64)
        b = ref["conic"][:, both]
        scale = np.stack([np.abs(b[0]), np.sqrt(np.abs(b[0] * b[2])), np.abs(b[2])])
        rel = np.abs(a - b) / scale
        lim = 1e-5 + 64 * U32 * kappa[both]
        print(f"{name} view {v}: centre error / bound {np.max(duv / (16 * U32 * uvs[:, both])):.3f}, conic error / "
              f"bound {np.max(rel / lim):.3f} (largest relative {rel.max():.2e})", flush=True)
        assert (rel <= lim).all(), np.max(rel / lim)
        # the extent scales with sqrt(ln(255 opacity)): its relative rounding error grows
        # like (ulp of 255 opacity) / (2 ln(255 opacity)) as the opacity nears 1/255
        a = h["ext"][:, g0:g1][:, both].astype(np.float64)
        b = ref["ext"][:, both]
        lg = np.log(255.0 * gs["opacity"][both])
        tol = 1e-5 * np.abs(b) + np.abs(b) * 1e-6 / np.maximum(lg, 1e-12)
        assert (np.abs(a - b) <= tol).all(), np.abs(a - b).max()
        np.testing.assert_allclose(h["depth"][g0:g1][both], ref["depth"][both], rtol=1e-6)
        # tile assignment bit-exact given the GPU's single-precision centre and extents
        prect, nt = oracle.rect_f32(h["uv"][0, g0:g1], h["uv"][1, g0:g1], h["ext"][0, g0:g1],
                                    h["ext"][1, g0:g1], sl["W"], sl["H"])
        assert np.array_equal(nt, h["ntiles"][g0:g1])
        box = unpack_box(h["splat"][g0:g1])
        assert np.array_equal(box[:, vis_g], prect[:, vis_g])


def test_project_far_from_origin():
    # a scene moved rigidly 1.5 km from the origin under a yawed camera: the camera-frame
    # position is the small difference of world-frame terms of ~1,500 m, which a plain FP32
    # evaluation would leave with errors of ~1e-4 m; the centres must match the oracle's
    # projection of the same FP32 inputs within a few roundings of the camera-frame
    # coordinates alone (the bound test_project takes without the world terms)
    s = plain_ragged()
    a = np.radians(33.0)
    Rw = np.array([[np.cos(a), 0.0, np.sin(a)], [0.0, 1.0, 0.0], [-np.sin(a), 0.0, np.cos(a)]])
    c = np.array([1500.37, -2.19, 1498.81])
    cam = dict(s["cams"][0], R=Rw.astype(np.float32), t=(-Rw @ c).astype(np.float32))
    Rf = np.asarray(cam["R"], np.float64)
    s["mean"] = (Rf.T @ (s["mean"].astype(np.float64) - np.asarray(cam["t"], np.float64)[:, None])).astype(np.float32)
    s["cams"] = [cam]
    pipe = run(s)
    h = host(pipe)
    gs = oracle_gauss(s, 0)
    ref = oracle.project(gs, cam)
    both = (h["ntiles"] > 0) & (ref["ntiles"] > 0)
    assert both.sum() > 1000
    R, t = Rf, np.asarray(cam["t"], np.float64)
    tc = R @ np.asarray(gs["mean"], np.float64) + t[:, None]
    tz = np.where(ref["depth"] > 0.2, ref["depth"], 1.0)
    su = cam["fx"] * (np.abs(tc[0]) + np.abs(tc[0] / tz) * np.abs(tc[2])) / tz + np.abs(ref["uv"][0])
    sv = cam["fy"] * (np.abs(tc[1]) + np.abs(tc[1] / tz) * np.abs(tc[2])) / tz + np.abs(ref["uv"][1])
    duv = np.abs(h["uv"].astype(np.float64) - ref["uv"])[:, both]
    bound = 16 * U32 * np.stack([su, sv])[:, both]
    print(f"far from the origin: centre error / local bound {np.max(duv / bound):.3f}, largest {duv.max():.2e} px",
          flush=True)
    assert (duv <= bound).all()
    np.testing.assert_allclose(h["depth"][both], ref["depth"][both], rtol=1e-6)


def test_bin_sort_bit_exact(case):
    name, scene, pipe, h = case
    check_bins(scene, pipe, h)


def test_bin_sort_long_ranges():
    # 40k wide Gaussians over 48x40 pixels: six of the nine 16x16 tiles hold 8,400-14,000
    # pairs, each range spanning several of the sort's blocks, the other three
    # 5,000-6,500.  Scaling a scene about the camera leaves its image alone and changes the
    # depth keys' width: 24 bits at depths 0.2-0.75, 27 bits at 20-100.  The sort takes
    # 1024-key blocks up to 2^20 pairs of capacity and 2048-key blocks above: the last
    # case sorts the same pairs in a buffer of 2^21.
    for seed, k, capacity in ((1018, 0.075, None), (1019, 10.0, None), (1019, 10.0, 1 << 21)):
        s = synth.plain_scene(seed, 40000, 48, 40)
        s["mean"] = (s["mean"] * k).astype(np.float32)
        s["log_scale"] = (s["log_scale"] + np.log(k) + 0.8).astype(np.float32)
        if capacity is None:
            pipe = run(s)
        else:
            pipe = Pipeline(s, device="cuda", capacity=capacity)
            pipe.step()
            torch.cuda.synchronize()
            pipe.check_status()
            assert pipe.capacity == capacity
        h = host(pipe)
        lens = check_bins(s, pipe, h)
        print(f"seed {seed}, capacity {pipe.capacity}: {len(lens)} tiles, ranges {sorted(lens.tolist())}, "
              f"depth bits {h['dbits']}", flush=True)
        assert (lens > 8192).sum() >= 2 and ((lens > 1023) & (lens <= 8192)).any()


def check_bins(scene, pipe, h):
    """The GPU's binning against the oracle's, bit for bit; returns the range lengths."""
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
    return lens


def test_render_fwd_stagewise(case):
    name, scene, pipe, h = case
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v])
        check_pixels(view_image(h, sl), view_pixels(h, sl, "T_final"), view_pixels(h, sl, "n_contrib"), ref,
                     f"{name} view {v}", n_eval=view_pixels(h, sl, "n_eval"))


def test_loss_kernel(case):
    name, scene, pipe, h = case
    for v, sl in enumerate(view_slices(pipe)):
        img = view_image(h, sl).astype(np.float64)
        L, _, _, dimg = oracle.loss(img, scene["targets"][v], scene["ssim_weight"])
        assert h["loss"][v] == pytest.approx(L, rel=1e-5)
        got = view_image(h, sl, "dimage")
        # L1 sign flips only where the FP32 image equals the target to rounding
        tie = np.abs(img - scene["targets"][v]) < 1e-6
        grad_close(got[~tie], dimg[~tie], name="dL/dC")


def _masked_dimage(h, scene, pipe):
    """The oracle's dL/dC of the GPU image with ambiguous pixels zeroed, per view."""
    out, amb_all = [], []
    for v, sl in enumerate(view_slices(pipe)):
        pr, gs = gpu_splats(h, sl)
        vals = h["vals"].astype(np.int64) - sl["g0"]
        ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
        ref = stage_render(pr, gs, vals, ranges, scene["cams"][v])
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
    dgs, scales = {}, {}
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
            dgv = {k: hb["dg"][k][..., sl["g0"]:sl["g1"]].astype(np.float64) for k in hb["dg"]}
            check_dgauss(dgv, dgp, gin, scene["cams"][v], h["ntiles"][sl["g0"]:sl["g1"]], got, f"{name} view {v}")
            oracle.decode_bwd(scene, scene["cams"][v]["partition"], scene["cams"][v], dgv, acc)
            dgs[v], scales[v] = dgv, gin["scale"]
    if scene["kind"] == "plain":
        for k in acc:
            grad_close(hb["dg"][k], acc[k], name=f"{name} plain d{k}")
    else:
        check_anchor_grads(hb["pgrad"], acc, scene, dgs, scales, f"{name} anchor")


def test_decode_stagewise(case):
    name, scene, pipe, h = case
    if scene["kind"] == "plain":
        pytest.skip("plain scene has no decode")
    for v, sl in enumerate(view_slices(pipe)):
        ref = oracle.decode(scene, scene["cams"][v]["partition"], scene["cams"][v])
        assert ref["opacity"].shape[-1] == sl["g1"] - sl["g0"]
        if sl["g1"] == sl["g0"]:
            continue
        mag = decode_magnitude(scene, v)
        for k in ("mean", "scale", "quat", "opacity", "rgb"):
            got = h["dec"][k][..., sl["g0"]:sl["g1"]].astype(np.float64)
            lim = 1e-5 * np.abs(ref[k]) + DECODE_GAMMA * U32 * mag[k]
            err = np.abs(got - ref[k])
            print(f"{name} view {v} decode {k}: error / bound {np.max(err / lim):.3f}", flush=True)
            assert (err <= lim).all(), (k, np.max(err / lim))


def test_end_to_end(case):
    name, scene, pipe, h = case
    fwd = oracle.forward(scene)
    dims = []
    for v, (sl, r) in enumerate(zip(view_slices(pipe), fwd)):
        check_e2e_pixels(view_image(h, sl), r, h, sl, scene["cams"][v], f"{name} view {v}")
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
    mag = None if scene["kind"] == "plain" else e2e_grad_magnitude(scene, fwd, dims)
    for k in ref:
        grad_close(got[k], ref[k], name=f"{name} end-to-end d{k}", mag=None if mag is None else mag[k],
                   gamma=GAMMA_E2E)


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
    pipe = Pipeline(s, device="cuda", capacity=64)
    guard = pipe.keys.new_zeros(0)
    pipe.forward()
    torch.cuda.synchronize()
    st = pipe.status.cpu().numpy()
    assert st[0] == 3  # GLAM_ERR_CAPACITY
    assert pipe.pair_count() == oracle.forward(s)[0]["bins"]["P"]
    del guard
