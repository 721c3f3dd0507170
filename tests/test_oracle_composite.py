"""Pins of the oracle's compositing (Eq. 1, Sec. III-A) and of its tiling.

Closed forms (a lone Gaussian renders as its analytic projected 2-D Gaussian; the
hand-derived stacks in tests/golden/closed_forms.json), invariants (partition of unity,
non-increasing transmittance, occlusion by an opaque front), thresholds, and
brute-force per-pixel compositing without tiles, which the tiled oracle must equal
exactly in FP64 for any tile shape."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def splats(uv, cov, opacity, rgb, depth, W, H):
    """2-D splats given directly (centre, covariance), with the full image as their
    footprint box; conic from numpy's matrix inverse."""
    n = len(opacity)
    conic = np.zeros((3, n))
    for i, (a, b, c) in enumerate(cov):
        inv = np.linalg.inv(np.array([[a, b], [b, c]]))
        conic[:, i] = [inv[0, 0], inv[0, 1], inv[1, 1]]
    prect = np.array([[0] * n, [W - 1] * n, [0] * n, [H - 1] * n], np.int32)
    pr = dict(uv=np.array(uv, float).T.copy(), conic=conic, prect=prect, depth=np.array(depth, float),
              ntiles=np.full(n, 1, np.int32))
    gs = dict(opacity=np.array(opacity, float), rgb=np.array(rgb, float).T.copy())
    return pr, gs


def render_tiled(pr, gs, cm, tile=(16, 16), bg=(0.0, 0.0, 0.0)):
    G = len(gs["opacity"])
    tx = (cm["W"] + tile[0] - 1) // tile[0]
    ty = (cm["H"] + tile[1] - 1) // tile[1]
    nt = np.array([(pr["prect"][1, g] // tile[0] - pr["prect"][0, g] // tile[0] + 1) *
                   (pr["prect"][3, g] // tile[1] - pr["prect"][2, g] // tile[1] + 1)
                   if pr["prect"][0, g] <= pr["prect"][1, g] else 0 for g in range(G)])
    b = oracle.bin_sort(pr["prect"], nt, pr["depth"], [0, G], [cm], tile)
    assert b["ranges"].shape[0] == tx * ty
    return oracle.render_fwd(pr, gs, b["vals"], b["ranges"], cm, bg, tile)


def cam(W=64, H=48, f=60.0):
    return synth.camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)


def test_lone_gaussian_is_its_projected_2d_gaussian():
    rng = np.random.default_rng(1)
    cm = cam()
    for _ in range(20):
        g = dict(mean=np.array([[rng.uniform(-1, 1)], [rng.uniform(-0.7, 0.7)], [rng.uniform(2, 6)]]),
                 scale=np.exp(rng.normal(-2.0, 0.5, (3, 1))), quat=rng.normal(size=(4, 1)),
                 opacity=np.array([rng.uniform(0.02, 1.0)]), rgb=rng.uniform(0, 1, (3, 1)))
        g["quat"] /= np.linalg.norm(g["quat"])
        pr = oracle.project(g, cm)
        if pr["ntiles"][0] == 0:
            continue
        out = render_tiled(pr, g, cm)
        a, b, c = pr["cov2d"][:, 0]
        Sinv = np.linalg.inv(np.array([[a, b], [b, c]]))
        xs, ys = np.meshgrid(np.arange(64) + 0.5, np.arange(48) + 0.5)
        d = np.stack([xs - pr["uv"][0, 0], ys - pr["uv"][1, 0]], -1)
        dens = np.exp(-0.5 * np.einsum("hwi,ij,hwj->hw", d, Sinv, d))
        alpha = np.minimum(0.99, g["opacity"][0] * dens)
        alpha[alpha < 1 / 255] = 0.0
        for ch in range(3):
            np.testing.assert_allclose(out["image"][ch], g["rgb"][ch, 0] * alpha, atol=1e-12)
        np.testing.assert_allclose(out["T_final"], 1 - alpha, atol=1e-12)
        assert np.array_equal(out["n_contrib"] > 0, alpha > 0)


def test_golden_stacks():
    W, H = 32, 32
    cm = cam(W, H)
    for key in ("opaque_front_stack", "half_over_half"):
        gd = GOLD[key]
        n = len(gd["opacities_front_to_back"])
        # all centred on the centre of pixel (10, 12), broad footprints, depths 1, 2, ...
        pr, gs = splats([(10.5, 12.5)] * n, [(4.0, 0.3, 3.0)] * n, gd["opacities_front_to_back"],
                        gd["colours"], np.arange(1, n + 1) * 1.0, W, H)
        out = render_tiled(pr, gs, cm)
        np.testing.assert_allclose(out["image"][:, 12, 10], gd["pixel_colour"], atol=1e-15)
        assert out["T_final"][12, 10] == pytest.approx(gd["T_final"], abs=1e-16)
        assert out["n_contrib"][12, 10] == gd["n_contrib"]
        # value decisions unambiguous (a 0.99 opacity sits on the clamp kink, which only
        # matters for gradients)
        assert out["amb"][12, 10] & (oracle.AMB_ALPHA | oracle.AMB_T | oracle.AMB_DEPTH) == 0
    gd = GOLD["two_clamped_layers"]
    pr, gs = splats([(10.5, 12.5)] * 2, [(4.0, 0.0, 4.0)] * 2, gd["opacities_front_to_back"],
                    [(1, 1, 1)] * 2, [1.0, 2.0], W, H)
    out = render_tiled(pr, gs, cm)
    assert out["amb"][12, 10] & oracle.AMB_T


def test_occlusion_behind_stop_is_invisible():
    # Anything behind the stopping Gaussian cannot change the pixel, bit for bit.
    W, H = 32, 32
    cm = cam(W, H)
    base_op = [0.99, 0.98, 0.99]
    rng = np.random.default_rng(4)
    ref = None
    for trial in range(6):
        extra = rng.integers(0, 5)
        ops = base_op + list(rng.uniform(0.05, 1.0, extra))
        cols = [(1, 0, 0), (0, 1, 0), (0, 0, 1)] + [tuple(rng.uniform(0, 1, 3)) for _ in range(extra)]
        uvs = [(10.5, 12.5)] * 3 + [tuple(rng.uniform(5, 25, 2)) for _ in range(extra)]
        covs = [(4.0, 0.3, 3.0)] * 3 + [(rng.uniform(1, 9), 0.0, rng.uniform(1, 9)) for _ in range(extra)]
        pr, gs = splats(uvs, covs, ops, cols, [1.0, 2.0, 3.0] + list(rng.uniform(3.5, 9, extra)), W, H)
        out = render_tiled(pr, gs, cm)
        px = (out["image"][:, 12, 10].copy(), out["T_final"][12, 10], out["n_contrib"][12, 10])
        if ref is None:
            ref = px
        assert np.array_equal(px[0], ref[0]) and px[1] == ref[1] and px[2] == ref[2]


def test_thresholds_and_clamp():
    W, H = 16, 16
    cm = cam(W, H)
    for op, visible in ((1 / 255 - 1e-9, False), (1 / 255 + 1e-9, True)):
        pr, gs = splats([(8.5, 8.5)], [(2.0, 0.0, 2.0)], [op], [(1, 1, 1)], [1.0], W, H)
        out = render_tiled(pr, gs, cm)
        assert (out["image"][0] > 0).sum() == (1 if visible else 0)
        if visible:
            assert out["image"][0, 8, 8] == pytest.approx(op, rel=1e-12)
    pr, gs = splats([(8.5, 8.5)], [(2.0, 0.0, 2.0)], [1.0], [(1, 1, 1)], [1.0], W, H)
    out = render_tiled(pr, gs, cm)
    assert out["image"][0, 8, 8] == 0.99
    assert out["T_final"][8, 8] == pytest.approx(0.01, abs=1e-16)


def random_scene(seed, G, W=64, H=48):
    s = synth.plain_scene(seed, G, W, H)
    gs = oracle.plain_activate(s)
    return s, gs, s["cams"][0]


@pytest.mark.parametrize("seed,G", [(21, 50), (22, 200), (23, 120)])
def test_invariants(seed, G):
    s, gs, cm = random_scene(seed, G)
    gs["rgb"] = np.ones_like(gs["rgb"])  # white: C = 1 - T_final when bg = 0
    pr = oracle.project(gs, cm)
    out = render_tiled(pr, gs, cm)
    for ch in range(3):
        np.testing.assert_allclose(out["image"][ch], 1.0 - out["T_final"], atol=1e-14)
    assert np.all(out["T_final"] >= 1e-4) and np.all(out["T_final"] <= 1.0)
    # transmittance never increases: render growing depth-ordered prefixes
    order = np.argsort(pr["depth"], kind="stable")
    prev = np.ones((cm["H"], cm["W"]))
    for k in range(0, G + 1, max(1, G // 10)):
        keep = np.zeros(G, bool)
        keep[order[:k]] = True
        p2 = {key: (val.copy() if isinstance(val, np.ndarray) else val) for key, val in pr.items()}
        p2["prect"][:, ~keep] = np.array([[0], [-1], [0], [-1]])
        o = render_tiled(p2, gs, cm)
        assert np.all(o["T_final"] <= prev + 1e-15)
        prev = o["T_final"]


@pytest.mark.parametrize("seed,G", [(31, 20), (32, 100), (33, 200)])
def test_tiled_equals_brute_force(seed, G):
    s, gs, cm = random_scene(seed, G)
    pr = oracle.project(gs, cm)
    br = oracle.render_brute(pr, gs, cm)
    for tile in ((16, 16), (8, 8), (32, 16), (64, 48)):
        tl = render_tiled(pr, gs, cm, tile)
        assert np.array_equal(tl["image"], br["image"])
        assert np.array_equal(tl["T_final"], br["T_final"])


def test_tiled_equals_brute_force_config1_and_background():
    s = synth.config("C1")
    gs = oracle.plain_activate(s)
    cm = s["cams"][0]
    pr = oracle.project(gs, cm)
    bg = (0.2, 0.5, 0.9)
    br = oracle.render_brute(pr, gs, cm, bg)
    tl = render_tiled(pr, gs, cm, bg=bg)
    assert np.array_equal(tl["image"], br["image"])
    assert np.array_equal(tl["T_final"], br["T_final"])
    # background enters as T_final * bg
    nobg = render_tiled(pr, gs, cm)
    for ch in range(3):
        np.testing.assert_allclose(tl["image"][ch] - nobg["image"][ch], bg[ch] * nobg["T_final"], atol=1e-15)


def test_stop_rule_and_counts():
    # a deep stack of identical half-opaque layers: T halves each time, so the walk
    # composites 13 layers (T = 2^-13 = 1.2e-4) and stops at the 14th (6.1e-5)
    W, H = 16, 16
    cm = cam(W, H)
    n = 20
    pr, gs = splats([(8.5, 8.5)] * n, [(9.0, 0.0, 9.0)] * n, [0.5] * n, [(1, 1, 1)] * n,
                    np.arange(1, n + 1) * 1.0, W, H)
    out = render_tiled(pr, gs, cm)
    assert out["n_contrib"][8, 8] == 13
    assert out["n_eval"][8, 8] == 14
    assert out["T_final"][8, 8] == 2.0 ** -13
