"""Pins of the oracle's finite-difference harness and of its plain activation.

The harness differentiates a piecewise-smooth loss: the skip threshold of Eq. 1
(alpha < 1/255), the stop rule, the depth order and the 0.99 clamp make it jump or
kink, and so do the ReLU gates of the decode MLPs (Eq. 2), the Jacobian clamp of the
projection and the L1 term of Eq. 3.  A central difference is only a check of the
analytic gradient when no such decision changes between -h and +h, so the harness
records all of them: these tests plant each kind of flip and check that it is
reported, that the flip really breaks the plain difference, and that the difference
taken with the decisions held at the unperturbed point (fd_gradient_frozen) still
equals the analytic gradient.

The plain activation (scale = e^s, q / |q|, sigmoid(logit)) is pinned by closed forms.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _skip_flip_scene():
    """Two Gaussians on a 16x16 view.  A (in front) has opacity ~0.048 and its alpha at
    pixel (11, 9) sits within rounding of the 1/255 skip threshold, three pixels right
    and one down of its centre; B (behind) covers that pixel and is the pixel's last
    contributor, so a flip of A's skip leaves the pixel's contributor count, its visit
    count, both footprint boxes and the sorted tile lists unchanged."""
    W = H = 16
    f = 60.0
    s = synth.plain_scene(7, 2, W, H, fx=f, fy=f)
    zA, zB = 4.0, 8.0
    sA = math.sqrt(1.7) * zA / f  # 2-D variance (f s / z)^2 + 0.3 = 2
    uA, vA = 8.5, 8.5
    uB, vB = 11.5, 9.5
    s["mean"] = np.array([[(uA - 8) * zA / f, (uB - 8) * zB / f], [(vA - 8) * zA / f, (vB - 8) * zB / f],
                          [zA, zB]], np.float32)
    s["log_scale"] = np.log(np.array([[sA, 0.3], [sA, 0.3], [sA, 0.3]])).astype(np.float32)
    s["quat"] = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]], np.float32)
    s["rgb"] = np.array([[0.9, 0.2], [0.1, 0.7], [0.4, 0.3]], np.float32)
    # A's logit: the float32 value whose alpha at pixel (11, 9) is nearest to 1/255
    gs = oracle.plain_activate(s)
    pr = oracle.project(gs, s["cams"][0])
    A_, B_, C_ = pr["conic"][:, 0]
    dx, dy = pr["uv"][0, 0] - 11.5, pr["uv"][1, 0] - 9.5
    power = -0.5 * (A_ * dx * dx + C_ * dy * dy) - B_ * dx * dy
    op = (1.0 / 255.0) / math.exp(power)
    s["logit"] = np.array([math.log(op / (1 - op)), 3.0], np.float32)
    return s


def _alpha_at(s, g, x, y):
    gs = oracle.plain_activate(s)
    pr = oracle.project(gs, s["cams"][0])
    A_, B_, C_ = pr["conic"][:, g]
    dx, dy = pr["uv"][0, g] - (x + 0.5), pr["uv"][1, g] - (y + 0.5)
    return gs["opacity"][g] * math.exp(-0.5 * (A_ * dx * dx + C_ * dy * dy) - B_ * dx * dy)


def test_skip_flip_before_the_last_contributor_is_detected():
    s = _skip_flip_scene()
    h = 1e-6
    # the threshold lies inside [logit - h, logit + h]
    lo, hi = (_alpha_at(synth_perturb(s, "logit", 0, d), 0, 11, 9) for d in (-h, h))
    assert lo < 1.0 / 255.0 <= hi
    # the decisions the earlier record held do not see it
    rec = []
    for d in (-h, h):
        r = oracle.forward(synth_perturb(s, "logit", 0, d))[0]
        rec.append((r["proj"]["prect"], r["bins"]["vals"], r["n_contrib"], r["n_eval"]))
    assert all(np.array_equal(a, b) for a, b in zip(*rec))
    # the composited lists do
    val, flipped, kinds = oracle.fd_gradient(s, "logit", (0,), h=h, detail=True)
    assert flipped and kinds["lists"] and not kinds["sign"] and not kinds["clamp"]
    # and the plain difference is off by the jump: (1/255) c T over 3 W H pixels / 2h
    _, _, grads = oracle.step(s)
    g = grads["logit"][0]
    assert abs(val - g) > 100 * abs(g)
    # with the decisions held at the unperturbed point the difference is the gradient
    fz = oracle.fd_gradient_frozen(s, "logit", (0,), h=h)
    assert fz == pytest.approx(g, rel=1e-6, abs=1e-12)


def synth_perturb(s, name, idx, d):
    w = dict(s)
    w[name] = np.asarray(s[name], np.float64).copy()
    w[name][idx] = float(s[name][idx]) + d
    return w


def test_no_flip_frozen_equals_plain_difference():
    s = synth.plain_scene(52, 200, 48, 40)
    _, _, grads = oracle.step(s)
    g = grads["mean"]
    for fi in np.argsort(-np.abs(g).ravel())[:3]:
        idx = np.unravel_index(int(fi), g.shape)
        val, flipped = oracle.fd_gradient(s, "mean", idx)
        if flipped:
            continue
        fz = oracle.fd_gradient_frozen(s, "mean", idx)
        assert fz == pytest.approx(val, rel=1e-7, abs=1e-13)
        assert fz == pytest.approx(g[idx], rel=1e-5)


def test_relu_flip_is_detected_and_frozen_difference_matches():
    s = synth.anchor_scene(53, [60], 1, W=96, H=64, fx=70, ssim_weight=0.2, bias_std=0.3)
    F, hid = s["F"], s["hidden"]
    cam = s["cams"][0]
    # anchor 0, opacity MLP, hidden unit 0: move the bias so that its pre-activation is
    # within rounding of zero
    R = np.asarray(cam["R"], np.float64)
    c = -R.T @ np.asarray(cam["t"], np.float64)
    d = s["pos"][:, 0].astype(np.float64) - c
    z = np.concatenate([s["feat"][0].astype(np.float64), d / np.linalg.norm(d), [np.linalg.norm(d)]])
    W1 = s["mlp"][0, :hid * (F + 4)].astype(np.float64).reshape(hid, F + 4)
    b_idx = hid * (F + 4)  # b1[0] of the opacity MLP
    mlp = s["mlp"].copy()
    mlp[0, b_idx] = np.float32(-(W1[0] @ z))
    s["mlp"] = mlp
    pre = W1[0] @ z + float(s["mlp"][0, b_idx])
    h = 1e-6
    assert abs(pre) < h
    val, flipped, kinds = oracle.fd_gradient(s, "mlp", (0, b_idx), h=h, detail=True)
    assert flipped and kinds["relu"]
    _, _, grads = oracle.step(s)
    fz = oracle.fd_gradient_frozen(s, "mlp", (0, b_idx), h=h)
    g = grads["mlp"][0, b_idx]
    assert fz == pytest.approx(g, rel=1e-5, abs=1e-6 * np.abs(grads["mlp"]).max())


def test_held_decisions_reproduce_the_free_forward():
    # imposing the decisions a forward pass took gives that same pass bit for bit
    s = synth.anchor_scene(54, [120], 1, W=96, H=64, fx=70, ssim_weight=0.2, bias_std=0.3)
    cam = s["cams"][0]
    gs = oracle.decode(s, 0, cam, want_relu=True)
    relu = gs.pop("relu")
    gs2 = oracle.decode(s, 0, cam, relu_in=relu)
    for k in gs:
        assert np.array_equal(gs[k], gs2[k])
    pr = oracle.project(gs, cam)
    pr2 = oracle.project(gs, cam, clamp_in=pr["clamp"])
    for k in ("uv", "conic", "depth", "ext", "prect"):
        assert np.array_equal(pr[k], pr2[k])
    G = gs["opacity"].shape[0]
    b = oracle.bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, G], [cam])
    r = oracle.render_fwd(pr, gs, b["vals"], b["ranges"], cam)
    lists = oracle.render_lists(pr, gs, b["vals"], b["ranges"], cam)
    fr = oracle.render_frozen(pr, gs, lists, cam)
    assert np.array_equal(fr["image"], r["image"]) and np.array_equal(fr["T_final"], r["T_final"])
    # list lengths: composited entries never exceed the contributor position
    n = np.diff(lists["offsets"]).reshape(cam["H"], cam["W"])
    assert (n <= r["n_contrib"]).all() and ((n == 0) == (r["n_contrib"] == 0)).all()


def test_jacobian_clamp_decision_recorded():
    # a Gaussian far left of the view (x/z below the low limit) and one inside it
    cm = synth.camera(np.eye(3), np.zeros(3), 60, 60, 32, 24, 64, 48)
    gs = dict(mean=np.array([[-8.0, 0.1], [0.0, 0.0], [4.0, 4.0]]), scale=np.full((3, 2), 0.05),
              quat=np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]]), opacity=np.array([0.5, 0.5]),
              rgb=np.full((3, 2), 0.5))
    pr = oracle.project(gs, cm)
    assert pr["clamp"].tolist() == [[1, 0], [0, 0]]
    # imposing "free" on the clamped one changes its conic (the Jacobian uses x/z itself)
    pr2 = oracle.project(gs, cm, clamp_in=np.zeros((2, 2), np.int8))
    assert not np.allclose(pr2["conic"][:, 0], pr["conic"][:, 0])
    assert np.array_equal(pr2["conic"][:, 1], pr["conic"][:, 1])


def test_l1_sign_held():
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (3, 20, 24))
    tgt = rng.uniform(0, 1, (3, 20, 24))
    L, lpx, _, _ = oracle.loss(img, tgt, 0.2)
    L2, lpx2, _, _ = oracle.loss(img, tgt, 0.2, l1_sign=np.sign(img - tgt))
    assert L == L2 and np.array_equal(lpx, lpx2)
    # the opposite signs give the L1 term's negative
    L3, _, _, _ = oracle.loss(img, tgt, 0.0, l1_sign=-np.sign(img - tgt))
    assert L3 == pytest.approx(-np.abs(img - tgt).mean(), rel=1e-12)


def test_plain_activation_closed_forms():
    # scale = e^s: e^0 = 1, e^{ln 2} = 2, e^{-1} = 1/e
    # quaternion: (1, 2, 2, 4) has norm 5; a zero quaternion stays zero (no NaN)
    # opacity: sigmoid(0) = 1/2, sigmoid(ln 3) = 3/4, sigmoid(-ln 3) = 1/4
    s = dict(mean=np.zeros((3, 3)), rgb=np.zeros((3, 3)),
             log_scale=np.array([[0.0, math.log(2.0), -1.0], [0.0, 0.0, 0.0], [math.log(2.0), -1.0, 0.0]]),
             quat=np.array([[1.0, 0.0, 3.0], [2.0, 0.0, 0.0], [2.0, 0.0, 4.0], [4.0, 0.0, 0.0]]),
             logit=np.array([0.0, math.log(3.0), -math.log(3.0)]))
    out = oracle.plain_activate(s)
    np.testing.assert_allclose(out["scale"], [[1.0, 2.0, 1 / math.e], [1.0, 1.0, 1.0], [2.0, 1 / math.e, 1.0]],
                               rtol=2e-16, atol=0)
    np.testing.assert_allclose(out["quat"][:, 0], [0.2, 0.4, 0.4, 0.8], rtol=1e-15)
    assert np.array_equal(out["quat"][:, 1], np.zeros(4))
    np.testing.assert_allclose(out["quat"][:, 2], [0.6, 0.0, 0.8, 0.0], rtol=1e-15)
    np.testing.assert_allclose(out["opacity"], [0.5, 0.75, 0.25], rtol=1e-15)
    assert out["opacity"][0] == 0.5
