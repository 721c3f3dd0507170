"""Pins of the oracle's projection and footprint (the projected 2-D Gaussian of
Sec. III-A, built by EWA splatting as in the 3DGS lineage the paper cites).

Each test checks the oracle against something other than its own formula: a closed
form, a finite-difference Jacobian of the pinhole map, a symmetry, or brute-force
evaluation of alpha around the footprint box."""
import math

import numpy as np
import pytest

import oracle
import synth


def gauss(mean, scale, quat, opacity=0.8, rgb=(1.0, 0.5, 0.25)):
    return dict(mean=np.array(mean, float).reshape(3, 1), scale=np.array(scale, float).reshape(3, 1),
                quat=np.array(quat, float).reshape(4, 1) / np.linalg.norm(quat),
                opacity=np.array([opacity], float), rgb=np.array(rgb, float).reshape(3, 1))


def cam(W=64, H=48, f=60.0, R=None, t=None, cx=None, cy=None):
    return synth.camera(np.eye(3) if R is None else R, np.zeros(3) if t is None else t, f, f,
                        W / 2 if cx is None else cx, H / 2 if cy is None else cy, W, H)


@pytest.mark.parametrize("z,s", [(2.0, 0.05), (5.0, 0.3), (9.0, 0.01)])
def test_isotropic_on_axis_closed_form(z, s):
    # An isotropic Gaussian on the optical axis: Sigma2D = ((f s / z)^2 + 0.3) I for any
    # rotation, centre at the principal point.
    rng = np.random.default_rng(3)
    for _ in range(5):
        q = rng.normal(size=4)
        g = gauss([0, 0, z], [s, s, s], q)
        pr = oracle.project(g, cam())
        expect = (60.0 * s / z) ** 2 + 0.3
        a, b, c = pr["cov2d"][:, 0]
        assert a == pytest.approx(expect, rel=1e-12)
        assert c == pytest.approx(expect, rel=1e-12)
        assert abs(b) < 1e-12 * expect
        assert pr["uv"][0, 0] == pytest.approx(32.0, abs=1e-12)
        assert pr["uv"][1, 0] == pytest.approx(24.0, abs=1e-12)
        assert pr["depth"][0] == pytest.approx(z)
        A, B, C = pr["conic"][:, 0]
        assert A == pytest.approx(1 / expect, rel=1e-12) and C == pytest.approx(1 / expect, rel=1e-12)


def _rotz(psi):
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def test_off_axis_matches_fd_jacobian():
    # Sigma2D = J Sigma J^T + 0.3 I with J the derivative of the pinhole map
    # (x, y, z) -> (fx x/z + cx, fy y/z + cy), taken here by central differences.
    rng = np.random.default_rng(5)
    R = synth._yaw(0.3) @ _rotz(0.2)
    t = np.array([0.1, -0.2, 0.5])
    cm = cam(W=200, H=120, f=150.0, R=R, t=t)
    R, t = cm["R"].astype(float), cm["t"].astype(float)  # the camera stores float32
    for _ in range(10):
        mu = np.array([rng.uniform(-1, 1), rng.uniform(-0.5, 0.5), rng.uniform(3, 8)])
        s = np.exp(rng.normal(-2, 0.5, 3))
        q = rng.normal(size=4)
        g = gauss(mu, s, q)
        pr = oracle.project(g, cm)
        tc = R @ mu + t

        def pin(p):
            return np.array([150.0 * p[0] / p[2] + 100.0, 150.0 * p[1] / p[2] + 60.0])

        h = 1e-6
        J = np.stack([(pin(tc + h * e) - pin(tc - h * e)) / (2 * h) for e in np.eye(3)], 1)
        qn = q / np.linalg.norm(q)
        w, x, y, z = qn
        Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Sig = Rq @ np.diag(s ** 2) @ Rq.T
        S2 = J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov2d"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(pr["uv"][:, 0], pin(tc), rtol=1e-13)
        # conic is the inverse of Sigma2D
        A, B, C = pr["conic"][:, 0]
        np.testing.assert_allclose(np.array([[A, B], [B, C]]) @ S2, np.eye(2), atol=1e-6)


def test_rotation_matrix_is_a_rotation_of_the_scale_axes():
    # Rotating the Gaussian by 90 degrees about its z axis while swapping the x and y
    # scales leaves the covariance, and so the projection, unchanged.
    rng = np.random.default_rng(8)
    for _ in range(5):
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        s = np.exp(rng.normal(-1.5, 0.4, 3))
        r90 = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])  # (w,x,y,z)
        w1, x1, y1, z1 = q; w2, x2, y2, z2 = r90
        q2 = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                       w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
        mu = [0.3, -0.2, 4.0]
        a = oracle.project(gauss(mu, s, q), cam())
        b = oracle.project(gauss(mu, [s[1], s[0], s[2]], q2), cam())
        np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-10, atol=1e-12)
        # the same quaternion negated is the same rotation
        c = oracle.project(gauss(mu, s, -q), cam())
        np.testing.assert_allclose(a["cov2d"], c["cov2d"], rtol=1e-12)


def test_camera_pose_equals_moving_the_world():
    # A world->camera pose (R, t) gives the same projection as applying it to the
    # Gaussian by hand and using the identity camera.
    rng = np.random.default_rng(11)
    R = synth._yaw(-0.4) @ _rotz(0.1)
    t = np.array([0.3, 0.1, 1.0])
    cm = cam(R=R, t=t)
    R, t = cm["R"].astype(float), cm["t"].astype(float)
    for _ in range(5):
        mu = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(2, 6)])
        s = np.exp(rng.normal(-2, 0.3, 3))
        q = rng.normal(size=4); q /= np.linalg.norm(q)
        w, x, y, z = q
        Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        M = R @ Rq  # rotation of the moved Gaussian
        # quaternion of M (Shepperd's method, valid for any rotation)
        tr = np.trace(M)
        if tr > 0:
            S = math.sqrt(tr + 1.0) * 2
            qm = [0.25 * S, (M[2, 1] - M[1, 2]) / S, (M[0, 2] - M[2, 0]) / S, (M[1, 0] - M[0, 1]) / S]
        else:
            i = int(np.argmax(np.diag(M)))
            j, k = (i + 1) % 3, (i + 2) % 3
            S = math.sqrt(1.0 + M[i, i] - M[j, j] - M[k, k]) * 2
            qm = [0.0] * 4
            qm[0] = (M[k, j] - M[j, k]) / S
            qm[1 + i] = 0.25 * S
            qm[1 + j] = (M[j, i] + M[i, j]) / S
            qm[1 + k] = (M[k, i] + M[i, k]) / S
        a = oracle.project(gauss(mu, s, q), cm)
        b = oracle.project(gauss(R @ mu + t, s, qm), cam())
        # float32 storage leaves R orthogonal to ~1e-7 only
        np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-6)
        np.testing.assert_allclose(a["uv"], b["uv"], rtol=1e-12)
        assert a["depth"][0] == pytest.approx(b["depth"][0])


def test_near_plane_and_opacity_cull():
    g = gauss([0, 0, 0.2], [0.1] * 3, [1, 0, 0, 0])
    assert oracle.project(g, cam())["ntiles"][0] == 0  # z <= 0.2
    g = gauss([0, 0, 0.2 + 1e-9], [0.1] * 3, [1, 0, 0, 0])
    assert oracle.project(g, cam())["ntiles"][0] > 0
    g = gauss([0, 0, 3], [0.1] * 3, [1, 0, 0, 0], opacity=1.0 / 255.0)
    assert oracle.project(g, cam())["ntiles"][0] == 0  # 255 alpha <= 1
    # just above the threshold the footprint shrinks to the pixel under the centre
    g = gauss([0.025, 0.025, 3], [0.1] * 3, [1, 0, 0, 0], opacity=1.0 / 255.0 + 1e-9)
    pr = oracle.project(g, cam())
    assert pr["ntiles"][0] == 1 and tuple(pr["prect"][:, 0]) == (32, 32, 24, 24)
    g = gauss([0.0, 0.0, 3], [0.1] * 3, [1, 0, 0, 0], opacity=1.0 / 255.0 + 1e-9)
    assert oracle.project(g, cam())["ntiles"][0] == 0  # centre between pixel centres
    g = gauss([50, 0, 3], [0.1] * 3, [1, 0, 0, 0])  # far outside the image
    assert oracle.project(g, cam())["ntiles"][0] == 0


def test_jacobian_clamp_limits():
    # Far off-screen the Jacobian uses x/z clamped to (1.15 W - cx)/fx, so Sigma2D equals
    # that of the same Gaussian moved sideways onto the clamp line (same depth), up to the
    # dependence of J on x only through the clamp.
    g1 = gauss([6.0, 0.0, 2.0], [0.2, 0.1, 0.3], [0.9, 0.1, 0.2, 0.3])
    lim = (1.15 * 64 - 32) / 60.0
    g2 = gauss([lim * 2.0, 0.0, 2.0], [0.2, 0.1, 0.3], [0.9, 0.1, 0.2, 0.3])
    a = oracle.project(g1, cam())
    b = oracle.project(g2, cam())
    np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-12)


def test_footprint_box_is_conservative_and_tight():
    # Outside the box every pixel has alpha < 1/255; the box is the smallest integer box
    # holding the continuous ellipse alpha(p) = 1/255 (checked on a fine sub-pixel grid).
    rng = np.random.default_rng(2)
    cm = cam(W=96, H=80, f=70.0)
    for _ in range(40):
        mu = [rng.uniform(-1.5, 1.5), rng.uniform(-1.2, 1.2), rng.uniform(2, 6)]
        s = np.exp(rng.normal(-2.0, 0.6, 3))
        q = rng.normal(size=4)
        op = rng.uniform(0.01, 0.999)
        g = gauss(mu, s, q, op)
        pr = oracle.project(g, cm)
        if pr["ntiles"][0] == 0:
            continue
        x0, x1, y0, y1 = pr["prect"][:, 0]
        u, v = pr["uv"][:, 0]
        A, B, C = pr["conic"][:, 0]
        xs, ys = np.meshgrid(np.arange(96) + 0.5, np.arange(80) + 0.5)
        dx, dy = u - xs, v - ys
        alpha = np.minimum(0.99, op * np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy))
        inside = (xs >= x0) & (xs <= x1 + 1) & (ys >= y0) & (ys <= y1 + 1)
        assert np.all(alpha[~inside] < 1 / 255)
        # tightness: the level-set ellipse reaches each unclamped side of the box within a
        # pixel (sample the continuous alpha around the extreme points)
        ex, ey = pr["ext"][:, 0]
        kappa = 2 * math.log(255 * op)
        assert ex == pytest.approx(math.sqrt(kappa * pr["cov2d"][0, 0]))
        assert ey == pytest.approx(math.sqrt(kappa * pr["cov2d"][2, 0]))


def test_rect_f32_matches_fp64_rule_away_from_edges():
    # The single-precision box rule agrees with the FP64 rule whenever the box edges are
    # not within rounding of an integer.
    rng = np.random.default_rng(9)
    n = 2000
    u = rng.uniform(-30, 230, n); v = rng.uniform(-30, 130, n)
    ex = rng.uniform(0, 40, n); ey = rng.uniform(0, 40, n)
    ex[::17] = -1.0
    prect, nt = oracle.rect_f32(u, v, ex, ey, 200, 100)
    for i in range(n):
        if ex[i] < 0:
            assert nt[i] == 0
            continue
        u32, v32, ex32, ey32 = (np.float32(a[i]) for a in (u, v, ex, ey))
        lo = math.ceil(float(u32) - float(ex32) - 0.5); hi = math.floor(float(u32) + float(ex32) - 0.5)
        ly = math.ceil(float(v32) - float(ey32) - 0.5); hy = math.floor(float(v32) + float(ey32) - 0.5)
        near = min(abs(x - round(x)) for x in (float(u32) - float(ex32) - 0.5, float(u32) + float(ex32) - 0.5,
                                               float(v32) - float(ey32) - 0.5, float(v32) + float(ey32) - 0.5))
        if near < 1e-4:
            continue
        lo, hi, ly, hy = max(lo, 0), min(hi, 199), max(ly, 0), min(hy, 99)
        if lo > hi or ly > hy:
            assert nt[i] == 0
        else:
            assert tuple(prect[:, i]) == (lo, hi, ly, hy)
            assert nt[i] == (hi // 16 - lo // 16 + 1) * (hy // 16 - ly // 16 + 1)
