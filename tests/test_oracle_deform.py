"""Pins of the loop-closure deformation oracle (Eq. 7)."""
import numpy as np

import synth
from oracle.deform import deform


def _anchors(seed, A, K=3):
    rng = np.random.default_rng(seed)
    vox = synth.corridor_voxels(z1=40.0)
    pos = vox[np.sort(rng.choice(len(vox), A, replace=False))].T.copy()
    offs = rng.normal(0, 0.1, (3, A * K))
    return pos, offs


def test_a_correction_that_changes_nothing_moves_nothing():
    pos, offs = _anchors(1, 500)
    fixes = synth.loop_fixes(2, 6)
    for f in fixes:
        f["R_new"], f["t_new"] = f["R_old"], f["t_old"]
    x, o, owner, _ = deform(pos, offs, 3, fixes, 0.2, 80.0)
    assert (owner >= 0).sum() > 100
    np.testing.assert_allclose(x, pos, atol=1e-6)
    np.testing.assert_allclose(o, offs, atol=1e-6)


def test_camera_translation_shifts_its_anchors_the_opposite_way():
    pos, offs = _anchors(3, 500)
    fixes = synth.loop_fixes(4, 1)
    d = np.array([0.05, -0.02, 0.1])
    fixes[0]["R_new"] = fixes[0]["R_old"]
    fixes[0]["t_new"] = fixes[0]["t_old"] + d
    x, o, owner, _ = deform(pos, offs, 3, fixes, 0.2, 80.0)
    sel = owner == 0
    assert sel.sum() > 50
    R = np.asarray(fixes[0]["R_old"], np.float64)
    np.testing.assert_allclose(x[:, sel], pos[:, sel] - (R.T @ d)[:, None], atol=1e-9)
    np.testing.assert_allclose(x[:, ~sel], pos[:, ~sel], atol=0)
    np.testing.assert_allclose(o, offs, atol=1e-12)  # no rotation, offsets stay


def test_moved_anchors_keep_their_camera_frame_coordinates():
    pos, offs = _anchors(5, 800)
    fixes = synth.loop_fixes(6, 8, rot_deg=3.0, trans_m=0.3)
    x, o, owner, _ = deform(pos, offs, 3, fixes, 0.2, 80.0)
    assert (owner >= 0).sum() > 200
    for i, f in enumerate(fixes):
        sel = owner == i
        Ro, to = np.asarray(f["R_old"], np.float64), np.asarray(f["t_old"], np.float64)
        Rn, tn = np.asarray(f["R_new"], np.float64), np.asarray(f["t_new"], np.float64)
        np.testing.assert_allclose(Rn @ x[:, sel] + tn[:, None], Ro @ pos[:, sel] + to[:, None], atol=1e-9)
        # offsets rotate with the anchor: lengths kept, and R_new o' == R_old o
        oo = offs.reshape(3, -1, 3)[:, sel, :].reshape(3, -1)
        on = o.reshape(3, -1, 3)[:, sel, :].reshape(3, -1)
        np.testing.assert_allclose(Rn @ on, Ro @ oo, atol=1e-9)


def test_owner_is_the_nearest_frustum_by_brute_force():
    pos, offs = _anchors(7, 300)
    fixes = synth.loop_fixes(8, 5, spacing=2.0)
    _, _, owner, _ = deform(pos, offs, 3, fixes, 0.2, 30.0)
    for a in range(pos.shape[1]):
        best, bd = -1, np.inf
        for i, f in enumerate(fixes):
            y = np.asarray(f["R_old"], np.float64) @ pos[:, a] + np.asarray(f["t_old"], np.float64)
            if not (0.2 <= y[2] <= 30.0):
                continue
            u, v = f["fx"] * y[0] / y[2] + f["cx"], f["fy"] * y[1] / y[2] + f["cy"]
            if not (0 <= u < f["W"] and 0 <= v < f["H"]):
                continue
            d = float(y @ y)
            if d < bd:
                best, bd = i, d
        assert owner[a] == best
