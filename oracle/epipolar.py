"""FP64 oracle of the flow-densification geometry (Eq. 5): the epipolar filter of
two-view correspondences and the triangulation of the retained ones.

TEST INFRASTRUCTURE ONLY (see the package docstring).

F = [e2]x P2 P1^+ with P = K [R | t], e2 = P2 C1 (C1 the first camera centre, the right
null vector of P1) and P1^+ the Moore-Penrose pseudo-inverse (numpy.linalg.pinv); scaled
to unit Frobenius norm with its largest-magnitude entry positive.  The residual of
x1 <-> x2 is |x2^T F x1| on homogeneous pixel coordinates; a pair is retained when it is
below tau.  Retained pairs are triangulated by linear least squares (numpy.linalg.lstsq)
on the four DLT rows in normalised image coordinates with X = (X, Y, Z, 1).

Pinned by tests/test_oracle_epipolar.py: F of exact correspondences of known 3-D points
gives residuals at rounding level and F has rank 2 with e2 and e1 as its null vectors;
F equals, up to scale, the essential-matrix construction K2^-T [t]x R K1^-1 of the
relative pose; exact correspondences triangulate to their 3-D points; a pair displaced
off its epipolar line has the residual of the line distance times the line's scale.
"""
from __future__ import annotations

import numpy as np


def projection(cam: dict) -> np.ndarray:
    K = np.array([[cam["fx"], 0.0, cam["cx"]], [0.0, cam["fy"], cam["cy"]], [0.0, 0.0, 1.0]])
    Rt = np.hstack([np.asarray(cam["R"], np.float64).reshape(3, 3), np.asarray(cam["t"], np.float64).reshape(3, 1)])
    return K @ Rt


def fundamental(cam1: dict, cam2: dict) -> np.ndarray:
    P1, P2 = projection(cam1), projection(cam2)
    R1 = np.asarray(cam1["R"], np.float64).reshape(3, 3)
    C1 = np.append(-R1.T @ np.asarray(cam1["t"], np.float64), 1.0)
    e2 = P2 @ C1
    S = np.array([[0.0, -e2[2], e2[1]], [e2[2], 0.0, -e2[0]], [-e2[1], e2[0], 0.0]])
    F = S @ P2 @ np.linalg.pinv(P1)
    F = F / np.linalg.norm(F)
    big = F.flat[np.argmax(np.abs(F))]
    return F if big > 0 else -F


def filter_triangulate(cam1: dict, cam2: dict, x1, x2, tau: float):
    """x1, x2 [2][N] pixel coordinates.  Returns residual [N], keep [N] (bool), X [3][N]
    (NaN where not kept), and near [N]: residuals within a relative 1e-9 of tau."""
    F = fundamental(cam1, cam2)
    x1 = np.asarray(x1, np.float64)
    x2 = np.asarray(x2, np.float64)
    n = x1.shape[1]
    h1 = np.vstack([x1, np.ones(n)])
    h2 = np.vstack([x2, np.ones(n)])
    r = np.abs(np.einsum("in,ij,jn->n", h2, F, h1))
    keep = r < tau
    X = np.full((3, n), np.nan)
    Rt1 = np.hstack([np.asarray(cam1["R"], np.float64).reshape(3, 3), np.asarray(cam1["t"], np.float64).reshape(3, 1)])
    Rt2 = np.hstack([np.asarray(cam2["R"], np.float64).reshape(3, 3), np.asarray(cam2["t"], np.float64).reshape(3, 1)])
    for i in np.nonzero(keep)[0]:
        a1, b1 = (x1[0, i] - cam1["cx"]) / cam1["fx"], (x1[1, i] - cam1["cy"]) / cam1["fy"]
        a2, b2 = (x2[0, i] - cam2["cx"]) / cam2["fx"], (x2[1, i] - cam2["cy"]) / cam2["fy"]
        A = np.array([a1 * Rt1[2] - Rt1[0], b1 * Rt1[2] - Rt1[1], a2 * Rt2[2] - Rt2[0], b2 * Rt2[2] - Rt2[1]])
        X[:, i] = np.linalg.lstsq(A[:, :3], -A[:, 3], rcond=None)[0]
    near = np.abs(r - tau) <= 1e-9 * max(tau, 1e-300)
    return r, keep, X, near
