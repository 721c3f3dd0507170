"""Pins of the flow-densification oracle (Eq. 5): the fundamental matrix built from the
two projection matrices, the residual filter and the triangulation."""
import numpy as np

import synth
from oracle import epipolar as E


def _exact(seed=1, n=400, baseline=1.0):
    c1, c2, x1, x2, pts, _ = synth.flow_pairs(seed, n, baseline=baseline)
    # exact double-precision projections (the synth output is rounded to float32)
    h = []
    for c in (c1, c2):
        y = c["R"].astype(np.float64) @ pts + c["t"].astype(np.float64)[:, None]
        h.append(np.stack([c["fx"] * y[0] / y[2] + c["cx"], c["fy"] * y[1] / y[2] + c["cy"]]))
    return c1, c2, h[0], h[1], pts


def test_exact_correspondences_have_zero_residual_and_triangulate_exactly():
    c1, c2, x1, x2, pts = _exact()
    r, keep, X, _ = E.filter_triangulate(c1, c2, x1, x2, 1e-6)
    assert r.max() < 1e-10 and keep.all()
    np.testing.assert_allclose(X, pts, rtol=1e-8, atol=1e-8)


def test_fundamental_is_rank_two_with_the_epipoles_as_null_vectors():
    c1, c2, *_ = _exact()
    F = E.fundamental(c1, c2)
    s = np.linalg.svd(F, compute_uv=False)
    assert s[2] < 1e-12 * s[0]
    P1, P2 = E.projection(c1), E.projection(c2)
    C1 = np.append(-c1["R"].astype(np.float64).T @ c1["t"].astype(np.float64), 1.0)
    C2 = np.append(-c2["R"].astype(np.float64).T @ c2["t"].astype(np.float64), 1.0)
    e1, e2 = P1 @ C2, P2 @ C1
    assert np.linalg.norm(F @ e1) < 1e-12 * np.linalg.norm(e1)
    assert np.linalg.norm(F.T @ e2) < 1e-12 * np.linalg.norm(e2)


def _orthonormal(c):
    # the closed form below needs R^T = R^-1 exactly: project R onto the rotations
    u, _, vt = np.linalg.svd(np.asarray(c["R"], np.float64))
    return dict(c, R=u @ vt, t=np.asarray(c["t"], np.float64))


def test_fundamental_equals_the_essential_matrix_construction():
    c1, c2, *_ = _exact(seed=3, baseline=2.5)
    c1, c2 = _orthonormal(c1), _orthonormal(c2)
    R1, t1 = c1["R"].astype(np.float64), c1["t"].astype(np.float64)
    R2, t2 = c2["R"].astype(np.float64), c2["t"].astype(np.float64)
    R, t = R2 @ R1.T, t2 - R2 @ R1.T @ t1  # pose of camera 2 relative to camera 1
    tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
    K1 = np.array([[c1["fx"], 0, c1["cx"]], [0, c1["fy"], c1["cy"]], [0, 0, 1.0]])
    K2 = np.array([[c2["fx"], 0, c2["cx"]], [0, c2["fy"], c2["cy"]], [0, 0, 1.0]])
    G = np.linalg.inv(K2).T @ tx @ R @ np.linalg.inv(K1)
    G = G / np.linalg.norm(G)
    G = G if G.flat[np.argmax(np.abs(G))] > 0 else -G
    np.testing.assert_allclose(E.fundamental(c1, c2), G, atol=1e-12)


def test_residual_of_a_pair_moved_off_its_epipolar_line():
    c1, c2, x1, x2, _ = _exact(seed=4, n=50)
    F = E.fundamental(c1, c2)
    h1 = np.vstack([x1, np.ones(50)])
    line = F @ h1  # epipolar lines in image 2
    nrm = np.linalg.norm(line[:2], axis=0)
    d = np.linspace(-3.0, 3.0, 50)
    moved = x2 + d * line[:2] / nrm  # d pixels along the line normal
    r, keep, _, _ = E.filter_triangulate(c1, c2, x1, moved, 1e-3)
    np.testing.assert_allclose(r, np.abs(d) * nrm, rtol=1e-6, atol=1e-12)
    assert np.array_equal(keep, np.abs(d) * nrm < 1e-3)
