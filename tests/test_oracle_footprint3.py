"""Pins of the oracle's second footprint rule, the 3-sigma square of the 3-D Gaussian
splatting lineage the paper builds on (Sec. II, Sec. III-A): a Gaussian is binned to
the tiles reached by the pixel centres within r = ceil(3 sqrt(lambda_max)) of its
centre, and is then a candidate at every pixel of those tiles.

Closed forms: r of an isotropic Gaussian; a lone Gaussian of opacity below
255^-1 e^4.5 renders exactly as with the opacity-aware box (nothing with alpha >= 1/255
lies beyond 3 sigma); one of higher opacity renders as c alpha inside its tiles and 0
outside them, so some pixels with alpha >= 1/255 are clipped and the image changes with
the tile edge."""
import math

import numpy as np

import oracle
import synth


def _lone(opacity, s=0.05, z=3.0, u=20.3, v=17.6, W=64, H=48, f=60.0):
    cm = synth.camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)
    g = dict(mean=np.array([[(u - W / 2) * z / f], [(v - H / 2) * z / f], [z]]), scale=np.full((3, 1), s),
             quat=np.array([[1.0], [0.0], [0.0], [0.0]]), opacity=np.array([opacity]), rgb=np.array([[0.8], [0.3], [0.5]]))
    return cm, g


def _render(cm, g, tile, footprint):
    pr = oracle.project(g, cm, tile=(tile, tile), footprint=footprint)
    b = oracle.bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, 1], [cm], (tile, tile))
    return pr, oracle.render_fwd(pr, g, b["vals"], b["ranges"], cm, tile=(tile, tile))


def _alpha_map(cm, g, pr):
    A, B, C = pr["conic"][:, 0]
    x = np.arange(cm["W"]) + 0.5
    y = np.arange(cm["H"]) + 0.5
    dx = pr["uv"][0, 0] - x[None, :]
    dy = pr["uv"][1, 0] - y[:, None]
    return np.minimum(0.99, g["opacity"][0] * np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy))


def test_radius_closed_form():
    # isotropic on the optical axis: Sigma2D = ((f s / z)^2 + 0.3) I, so lambda_max is
    # that and r = ceil(3 sqrt(lambda_max))
    for s, z in ((0.05, 3.0), (0.02, 7.0), (0.3, 2.5)):
        cm, g = _lone(0.5, s=s, z=z, u=32.0, v=24.0)
        pr = oracle.project(g, cm, footprint="3sigma")
        lam = (60.0 * s / z) ** 2 + 0.3
        assert pr["ext"][0, 0] == pr["ext"][1, 0] == math.ceil(3 * math.sqrt(lam))


def test_faint_gaussian_renders_as_with_the_exact_box():
    # opacity 0.3 < 255^-1 e^4.5: every pixel with alpha >= 1/255 is within 3 sigma
    cm, g = _lone(0.3)
    for tile in (8, 16, 32):
        _, r3 = _render(cm, g, tile, "3sigma")
        _, ro = _render(cm, g, tile, "opacity")
        assert np.array_equal(r3["image"], ro["image"])


def test_opaque_gaussian_is_clipped_at_its_tiles():
    # opacity 0.9: alpha >= 1/255 out to sqrt(2 ln(255 * 0.9)) = 3.3 sigma, beyond the
    # square; a wide Gaussian (sigma ~ 10 px) whose square ends at a tile boundary loses
    # the pixels with alpha >= 1/255 past it
    clipped = differs = 0
    for u in np.arange(5.0, 13.0, 0.5):
        cm, g = _lone(0.9, s=0.5, z=3.0, u=u)
        images = {}
        for tile in (8, 16):
            pr, r = _render(cm, g, tile, "3sigma")
            alpha = _alpha_map(cm, g, pr)
            x0, x1, y0, y1 = pr["prect"][:, 0]
            # the box is whole tiles (clipped to the image)
            assert x0 % tile == 0 and y0 % tile == 0
            assert (x1 + 1) % tile == 0 or x1 == cm["W"] - 1
            assert (y1 + 1) % tile == 0 or y1 == cm["H"] - 1
            inside = np.zeros_like(alpha, bool)
            inside[y0:y1 + 1, x0:x1 + 1] = True
            keep = inside & (alpha >= 1 / 255)
            want = np.where(keep[None], g["rgb"][:, 0][:, None, None] * alpha[None], 0.0)
            np.testing.assert_allclose(r["image"], want, rtol=0, atol=1e-15)
            if tile == 8 and ((alpha >= 1 / 255) & ~inside).any():
                clipped += 1
            images[tile] = r["image"]
        differs += not np.array_equal(images[8], images[16])
    assert clipped > 0 and differs > 0


def test_3sigma_tiling_equals_its_own_candidate_rule():
    # on a random scene the tiled 3-sigma render equals compositing every Gaussian whose
    # widened box holds the pixel, depth-sorted (the brute-force path with those boxes)
    s = synth.plain_scene(71, 150, 64, 48)
    gs = oracle.plain_activate(s)
    cm = s["cams"][0]
    for tile in (8, 16):
        pr = oracle.project(gs, cm, tile=(tile, tile), footprint="3sigma")
        b = oracle.bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, 150], [cm], (tile, tile))
        r = oracle.render_fwd(pr, gs, b["vals"], b["ranges"], cm, tile=(tile, tile))
        br = oracle.render_brute(pr, gs, cm)
        assert np.array_equal(r["image"], br["image"])
        # its tile counts follow from the square: tiles of [ceil(u - r - 1/2), floor(u + r - 1/2)]
        vis = pr["ntiles"] > 0
        u, v, ex = pr["uv"][0], pr["uv"][1], pr["ext"][0]
        lo_x = np.maximum(np.ceil(u - ex - 0.5), 0)
        hi_x = np.minimum(np.floor(u + ex - 0.5), cm["W"] - 1)
        lo_y = np.maximum(np.ceil(v - ex - 0.5), 0)
        hi_y = np.minimum(np.floor(v + ex - 0.5), cm["H"] - 1)
        nt = ((hi_x // tile - lo_x // tile + 1) * (hi_y // tile - lo_y // tile + 1)).astype(np.int64)
        assert np.array_equal(nt[vis], pr["ntiles"][vis])
