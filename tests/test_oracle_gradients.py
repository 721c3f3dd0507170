"""Pins of the oracle's analytic backward: central finite differences of the FP64
forward (h = 1e-6, differenced pixel by pixel and summed exactly, parameters whose +-h
perturbation flips a discrete decision rejected), the O(n^2) direct-formula adjoint of
Eq. 1, and the closed-form gradients of a lone Gaussian."""
import numpy as np
import pytest

import oracle
import synth


def _check_fd(scene, grads, names, n_per_name, seed, rel=1e-5):
    rng = np.random.default_rng(seed)
    checked = 0
    for name in names:
        g = grads[name]
        flat = np.abs(g).ravel()
        # stratified: half from the largest gradients, half uniformly among nonzero ones
        big = list(np.argsort(-flat)[: n_per_name // 2])
        nz = np.flatnonzero(flat > 1e-3 * flat.max())
        big += list(rng.choice(nz, size=min(len(nz), n_per_name - len(big)), replace=False))
        for fi in big:
            idx = np.unravel_index(int(fi), g.shape)
            fd, flipped = oracle.fd_gradient(scene, name, idx)
            if flipped:
                continue
            tol = rel * abs(fd) + 1e-6 * flat.max()
            assert abs(fd - g[idx]) <= tol, (name, idx, g[idx], fd)
            checked += 1
    assert checked >= len(names) * n_per_name * 0.75


def test_plain_gradients_match_finite_differences():
    s = synth.plain_scene(51, 300, 64, 48)
    L, fwd, grads = oracle.step(s)
    _check_fd(s, grads, ["mean", "log_scale", "quat", "logit", "rgb"], 8, 0)


def test_plain_gradients_with_background_and_ssim():
    s = synth.plain_scene(52, 200, 48, 40)
    s["ssim_weight"] = 0.2
    bg = (0.3, 0.6, 0.1)
    fwd = oracle.forward(s, bg=bg)
    grads = oracle.backward(s, fwd, bg=bg)
    rng = np.random.default_rng(2)
    for name in ["mean", "logit", "rgb"]:
        g = grads[name]
        for fi in np.argsort(-np.abs(g).ravel())[:4]:
            idx = np.unravel_index(int(fi), g.shape)
            orig = s[name][idx]
            vals = []
            for sgn in (1, -1):
                w = dict(s)
                w[name] = np.asarray(s[name], np.float64).copy()
                w[name][idx] = float(orig) + sgn * 1e-6
                vals.append(sum(r["loss"] for r in oracle.forward(w, bg=bg)))
            fd = (vals[0] - vals[1]) / 2e-6
            assert fd == pytest.approx(g[idx], rel=1e-4, abs=1e-9)


def test_anchor_gradients_match_finite_differences():
    s = synth.anchor_scene(53, [250, 180], 2, W=128, H=64, fx=80, ssim_weight=0.2, bias_std=0.3)
    L, fwd, grads = oracle.step(s)
    _check_fd(s, grads, ["feat", "offs", "log_scale", "mlp"], 8, 1)


def test_stored_T_adjoint_equals_direct_formula():
    # The backward with stored transmittances equals the O(n^2) term-by-term derivative
    # of Eq. 1 on small scenes.
    for seed, G in ((61, 40), (62, 120)):
        s = synth.plain_scene(seed, G, 48, 32)
        gs = oracle.plain_activate(s)
        cm = s["cams"][0]
        pr = oracle.project(gs, cm)
        b = oracle.bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, G], [cm])
        rng = np.random.default_rng(seed)
        dimg = rng.normal(size=(3, 32, 48))
        bg = (0.1, 0.2, 0.3)
        a = oracle.render_bwd(pr, gs, b["vals"], b["ranges"], cm, dimg, bg)
        d = oracle.render_brute_bwd(pr, gs, cm, dimg, bg)
        np.testing.assert_allclose(a, d, rtol=1e-9, atol=1e-12 * np.abs(d).max())


def test_lone_gaussian_closed_form_gradients():
    # dC/dc = alpha_p, dC/dopacity = c e^power, dC/dmean2d = -c alpha_p (A dx + B dy, B dx + C dy)
    W, H = 40, 30
    cm = synth.camera(np.eye(3), np.zeros(3), 50, 50, 20, 15, W, H)
    g = dict(mean=np.array([[0.1], [-0.05], [3.0]]), scale=np.array([[0.15], [0.1], [0.12]]),
             quat=np.array([[0.9], [0.1], [-0.3], [0.2]]), opacity=np.array([0.6]),
             rgb=np.array([[0.8], [0.3], [0.5]]))
    g["quat"] /= np.linalg.norm(g["quat"])
    pr = oracle.project(g, cm)
    b = oracle.bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, 1], [cm])
    for (x, y) in ((20, 13), (23, 17), (18, 12)):
        dimg = np.zeros((3, H, W))
        dimg[0, y, x] = 1.0  # red channel of one pixel
        g2d = oracle.render_bwd(pr, g, b["vals"], b["ranges"], cm, dimg)
        u, v = pr["uv"][:, 0]
        A, B, C = pr["conic"][:, 0]
        dx, dy = u - x - 0.5, v - y - 0.5
        ep = np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
        ap = 0.6 * ep
        assert ap > 1 / 255 and ap < 0.99
        assert g2d[6, 0] == pytest.approx(ap, rel=1e-12)
        assert g2d[7, 0] == 0 and g2d[8, 0] == 0
        assert g2d[5, 0] == pytest.approx(0.8 * ep, rel=1e-12)
        assert g2d[0, 0] == pytest.approx(-0.8 * ap * (A * dx + B * dy), rel=1e-12)
        assert g2d[1, 0] == pytest.approx(-0.8 * ap * (B * dx + C * dy), rel=1e-12)
