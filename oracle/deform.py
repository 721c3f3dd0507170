"""FP64 oracle of the loop-closure deformation of the anchor grid (Eq. 7).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For each corrected keyframe i with world->camera poses T_old,i and T_new,i, the
correction dT_i = T_new,i^-1 T_old,i is applied to the anchors of keyframe i's old view
frustum (depth in [near, far] in the old camera frame, projection inside the image).
Readings where the paper is silent: an anchor in several frusta follows the keyframe
whose old camera centre is nearest (ties to the lower index); the anchor's offsets
rotate with it.  Pinned by tests/test_oracle_deform.py: a correction that changes nothing
moves nothing, a pure translation of the camera shifts its anchors by the opposite
world translation, every moved anchor keeps its camera-frame coordinates in its owner
keyframe (T_new x' = T_old x), anchors outside every frustum stay, and the owner is the
brute-force nearest frustum holding the anchor.
"""
from __future__ import annotations

import numpy as np


def _pose(R, t):
    T = np.eye(4)
    T[:3, :3] = np.asarray(R, np.float64).reshape(3, 3)
    T[:3, 3] = np.asarray(t, np.float64)
    return T


def deform(pos, offs, K: int, fixes: list, near: float, far: float):
    """pos [3][A], offs [3][A*K]; fixes: dicts with R_old, t_old, R_new, t_new, fx, fy, cx,
    cy, W, H.  Returns (new pos, new offs, owner [A], ambiguous [A]): ambiguous marks
    anchors whose frustum membership or nearest keyframe is decided within rounding."""
    x = np.asarray(pos, np.float64)
    A = x.shape[1]
    owner = np.full(A, -1, np.int64)
    best = np.full(A, np.inf)
    second = np.full(A, np.inf)
    amb = np.zeros(A, bool)
    for i, f in enumerate(fixes):
        To = _pose(f["R_old"], f["t_old"])
        y = To[:3, :3] @ x + To[:3, 3:4]
        z = y[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = f["fx"] * y[0] / z + f["cx"]
            v = f["fy"] * y[1] / z + f["cy"]
        inside = (z >= near) & (z <= far) & (u >= 0) & (u < f["W"]) & (v >= 0) & (v < f["H"])
        # membership decided within rounding: any frustum plane within a relative 1e-5
        m = 1e-5
        near_edge = ((np.abs(z - near) < m * near) | (np.abs(z - far) < m * far) |
                     (np.abs(u) < m * f["W"]) | (np.abs(u - f["W"]) < m * f["W"]) |
                     (np.abs(v) < m * f["H"]) | (np.abs(v - f["H"]) < m * f["H"])) & (z > 0)
        amb |= near_edge
        d2 = (y * y).sum(0)
        closer = inside & (d2 < best)
        second = np.where(closer, best, np.where(inside, np.minimum(second, d2), second))
        best = np.where(closer, d2, best)
        owner = np.where(closer, i, owner)
    with np.errstate(invalid="ignore"):
        amb |= np.isfinite(second) & (np.abs(second - best) <= 1e-5 * best)
    newx = x.copy()
    o = np.asarray(offs, np.float64).reshape(3, A, K).copy()
    for i, f in enumerate(fixes):
        sel = owner == i
        if not sel.any():
            continue
        dT = np.linalg.inv(_pose(f["R_new"], f["t_new"])) @ _pose(f["R_old"], f["t_old"])
        newx[:, sel] = dT[:3, :3] @ x[:, sel] + dT[:3, 3:4]
        o[:, sel, :] = np.einsum("rc,cak->rak", dT[:3, :3], o[:, sel, :])
    return newx, o.reshape(3, A * K), owner, amb
