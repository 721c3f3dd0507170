"""Pins of the oracle's tile binning and depth sort, its photometric loss (Eq. 3,
Sec. III-A) and its anchor decode (Eq. 2, Sec. III-A; Eq. 6, Sec. III-D).

Sort: per-tile brute force (every Gaussian whose tile box covers the tile, ordered by
(depth, index)).  Loss: identity and constant-image closed forms, an SSIM map built
from scipy's box filter, finite differences.  Decode: weight constructions that route
one MLP input to one output, a NumPy FP64 matmul, and the partition selection."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth


# ----------------------------------------------------------------------------------
# bin + sort
# ----------------------------------------------------------------------------------

def _brute_tiles(prect, depth, gbegin, cams, tile):
    tx, ty, base = oracle.tile_grid(cams, tile)
    lists = {}
    for k, cm in enumerate(cams):
        for t_y in range(ty[k]):
            for t_x in range(tx[k]):
                members = []
                for g in range(gbegin[k], gbegin[k + 1]):
                    x0, x1, y0, y1 = prect[:, g]
                    if x0 > x1:
                        continue
                    if x0 // tile[0] <= t_x <= x1 // tile[0] and y0 // tile[1] <= t_y <= y1 // tile[1]:
                        members.append((depth[g], g))
                lists[int(base[k] + t_y * tx[k] + t_x)] = [g for _, g in sorted(members)]
    return lists


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_bin_sort_matches_per_tile_brute_force(tile):
    cams, prs, gb = [], [], [0]
    for v, (seed, G, W, H) in enumerate([(41, 150, 64, 48), (42, 90, 70, 45)]):
        s = synth.plain_scene(seed, G, W, H)
        gs = oracle.plain_activate(s)
        pr = oracle.project(gs, s["cams"][0], tile)
        cams.append(s["cams"][0]); prs.append(pr); gb.append(gb[-1] + G)
    prect = np.concatenate([p["prect"] for p in prs], 1)
    depth = np.concatenate([p["depth"] for p in prs])
    # force exact depth ties so the index order decides
    depth[5] = depth[6] = depth[7]
    nt = np.concatenate([p["ntiles"] for p in prs])
    b = oracle.bin_sort(prect, nt, depth, gb, cams, tile)
    want = _brute_tiles(prect, depth, gb, cams, tile)
    assert b["P"] == sum(len(v) for v in want.values())
    for t, members in want.items():
        s0, s1 = b["ranges"][t]
        assert list(b["vals"][s0:s1]) == members, t
        assert np.all(b["tiles"][s0:s1] == t)


# ----------------------------------------------------------------------------------
# loss
# ----------------------------------------------------------------------------------

def test_loss_identity_and_l1():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (3, 20, 30))
    L, lpx, ssim, d = oracle.loss(x, x, 0.2)
    assert L == pytest.approx(0.0, abs=1e-14)
    np.testing.assert_allclose(ssim, 1.0, atol=1e-13)
    np.testing.assert_allclose(d, 0.0, atol=1e-14)
    y = rng.uniform(0, 1, (3, 20, 30))
    L, lpx, ssim, d = oracle.loss(x, y, 0.0)
    assert L == pytest.approx(np.abs(x - y).mean(), rel=1e-13)
    np.testing.assert_allclose(d, np.sign(x - y) / x.size, rtol=1e-13)
    assert lpx.sum() == pytest.approx(L, rel=1e-13)


def test_ssim_constant_images_closed_form():
    a, b = 0.3, 0.7
    x = np.full((3, 24, 24), a)
    y = np.full((3, 24, 24), b)
    _, _, ssim, _ = oracle.loss(x, y, 0.2)
    c1 = 0.01 ** 2
    # windows fully inside the image: variance and covariance vanish
    np.testing.assert_allclose(ssim[:, 5:-5, 5:-5], (2 * a * b + c1) / (a * a + b * b + c1), rtol=1e-10)


def test_ssim_map_matches_scipy_box_statistics():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (3, 19, 27))
    y = rng.uniform(0, 1, (3, 19, 27))
    _, _, ssim, _ = oracle.loss(x, y, 0.2)
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    box = lambda a: ndimage.uniform_filter(a, size=11, mode="constant", cval=0.0)
    for ch in range(3):
        mx, my = box(x[ch]), box(y[ch])
        vx = box(x[ch] ** 2) - mx ** 2
        vy = box(y[ch] ** 2) - my ** 2
        cxy = box(x[ch] * y[ch]) - mx * my
        want = (2 * mx * my + c1) * (2 * cxy + c2) / ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2))
        np.testing.assert_allclose(ssim[ch], want, rtol=1e-10, atol=1e-12)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, (3, 17, 23))
    y = rng.uniform(0, 1, (3, 17, 23))
    L, _, _, d = oracle.loss(x, y, 0.2)
    h = 1e-6
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (oracle.loss(xp, y, 0.2)[0] - oracle.loss(xm, y, 0.2)[0]) / (2 * h)
        assert fd == pytest.approx(d[idx], rel=1e-5, abs=1e-11)


# ----------------------------------------------------------------------------------
# decode
# ----------------------------------------------------------------------------------

def _layout(F, K, hidden):
    n_in = F + 4
    off, out = 0, {}
    for name, o in (("op", K), ("col", 3 * K), ("cov", 7 * K)):
        w1 = off; b1 = w1 + hidden * n_in; w2 = b1 + hidden; b2 = w2 + o * hidden
        out[name] = (w1, b1, w2, b2, o)
        off = b2 + o
    return out, off


def _tiny_scene(A=6, F=8, K=3, hidden=5, seed=0):
    rng = np.random.default_rng(seed)
    lay, P = _layout(F, K, hidden)
    assert P == oracle.mlp_param_count(F, K, hidden)
    R = synth._yaw(0.3)
    cm = synth.posed_camera([0.4, -0.2, 1.5], R, 100, 100, 50, 40, 100, 80)
    sc = dict(kind="anchor", F=F, K=K, hidden=hidden,
              pos=rng.uniform(-2, 2, (3, A)) + np.array([[0], [0], [6]]), feat=rng.normal(size=(A, F)),
              log_scale=rng.normal(-1, 0.3, A), offs=rng.normal(0, 0.1, (3, A * K)),
              part_begin=np.array([0, A], np.int32), mlp=np.zeros((1, P)), cams=[cm],
              targets=[np.zeros((3, 80, 100))], ssim_weight=0.0, opacity_mode="tanh")
    return sc, lay, cm


def test_decode_routes_distance_and_direction():
    # W1 copies delta (input F+3) and d_x (input F) into hidden units 0 and 1; W2 sends
    # them to opacity output j and colour output 3j+1.  Then opacity_j = tanh(w delta) and
    # colour = sigmoid(v d_x), with delta and d_x from the camera centre solved from
    # the pose independently.
    sc, lay, cm = _tiny_scene()
    F, K, hid = sc["F"], sc["K"], sc["hidden"]
    n_in = F + 4
    p = sc["mlp"][0]
    w1, b1, w2, b2, o = lay["op"]
    p[w1 + 0 * n_in + F + 3] = 1.0
    for j in range(K):
        p[w2 + j * hid + 0] = 0.1 * (j + 1)
    w1, b1, w2, b2, o = lay["col"]
    p[w1 + 1 * n_in + F] = 1.0
    p[b1 + 1] = 2.0  # keep the ReLU open: d_x >= -1
    for j in range(K):
        p[w2 + (3 * j + 1) * hid + 1] = 0.5 * (j + 1)
    out = oracle.decode(sc, 0, cm)
    R = cm["R"].astype(float); t = cm["t"].astype(float)
    xc = np.linalg.solve(R, -t)
    for a in range(sc["feat"].shape[0]):
        diff = sc["pos"][:, a] - xc
        delta = np.linalg.norm(diff)
        dxn = diff[0] / delta
        for j in range(K):
            g = a * K + j
            # (float32 storage leaves R orthogonal only to ~1e-8, hence rel 1e-7)
            assert out["opacity"][g] == pytest.approx(math.tanh(0.1 * (j + 1) * delta), rel=1e-7)
            assert out["rgb"][1, g] == pytest.approx(1 / (1 + math.exp(-0.5 * (j + 1) * (dxn + 2.0))), rel=1e-7)
            assert out["rgb"][0, g] == 0.5 and out["rgb"][2, g] == 0.5
            # zero covariance head: scale = e^s / 2, quaternion guarded to zero
            np.testing.assert_allclose(out["scale"][:, g], math.exp(sc["log_scale"][a]) / 2, rtol=1e-12)
            np.testing.assert_allclose(out["mean"][:, g],
                                       sc["pos"][:, a] + math.exp(sc["log_scale"][a]) * sc["offs"][:, g],
                                       rtol=1e-12)


def test_decode_matches_numpy_matmul():
    sc, lay, cm = _tiny_scene(A=9, F=8, K=4, hidden=7, seed=3)
    rng = np.random.default_rng(7)
    sc["mlp"] = rng.normal(0, 0.5, sc["mlp"].shape)
    F, K, hid = sc["F"], sc["K"], sc["hidden"]
    n_in = F + 4
    out = oracle.decode(sc, 0, cm)
    R = cm["R"].astype(float); t = cm["t"].astype(float)
    xc = -R.T @ t
    diff = sc["pos"].T - xc
    delta = np.linalg.norm(diff, axis=1, keepdims=True)
    Z = np.concatenate([sc["feat"], diff / delta, delta], 1)  # [A][F+4]
    p = sc["mlp"][0]
    Y = {}
    for name, (w1, b1, w2, b2, o) in lay.items():
        W1 = p[w1:b1].reshape(hid, n_in); W2 = p[w2:b2].reshape(o, hid)
        Y[name] = np.maximum(Z @ W1.T + p[b1:w2], 0.0) @ W2.T + p[b2:b2 + o]
    A = sc["feat"].shape[0]
    op = np.tanh(Y["op"]).reshape(A * K)
    col = 1 / (1 + np.exp(-Y["col"].reshape(A, K, 3)))
    cov = Y["cov"].reshape(A, K, 7)
    es = np.exp(sc["log_scale"])[:, None, None]
    scale = es / (1 + np.exp(-cov[..., :3]))
    q = cov[..., 3:] / np.linalg.norm(cov[..., 3:], axis=-1, keepdims=True)
    np.testing.assert_allclose(out["opacity"], op, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(out["rgb"], col.reshape(A * K, 3).T, rtol=1e-12)
    np.testing.assert_allclose(out["scale"], scale.reshape(A * K, 3).T, rtol=1e-12)
    np.testing.assert_allclose(out["quat"], q.reshape(A * K, 4).T, rtol=1e-10, atol=1e-14)
    # drop rule: non-positive tanh opacity never renders
    pr = oracle.project(out, cm)
    assert np.all(pr["ntiles"][out["opacity"] <= 0] == 0)
    assert (out["opacity"] <= 0).sum() > 0


def test_decode_uses_the_partition_of_the_view():
    # Eq. 6: a view of partition m decodes only partition m's anchors with theta_m.
    s = synth.anchor_scene(5, [30, 40], 1, W=96, H=48, fx=70, bias_std=0.2)
    a = oracle.decode(s, 1, s["cams"][1])
    s2 = dict(s)
    s2["mlp"] = s["mlp"].copy()
    s2["mlp"][0] = 0.0  # partition 0's weights do not matter to partition 1
    b = oracle.decode(s2, 1, s2["cams"][1])
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert a["opacity"].shape[0] == 40 * s["K"]
