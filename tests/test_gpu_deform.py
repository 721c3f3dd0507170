"""Loop-closure deformation on the GPU against the FP64 oracle: owners bit-exact away
from decisions taken within rounding (a frustum plane or a near tie of distances), the
moved positions and rotated offsets within FP32 rounding of the scene scale."""
import numpy as np
import pytest
import torch

import synth
from oracle.deform import deform
from paper_2607_21416_amd import binding as B

pytestmark = pytest.mark.gpu


def _fix_table(fixes):
    arr = (B.KeyframeFix * len(fixes))()
    for i, f in enumerate(fixes):
        c = arr[i].before
        for k in range(9):
            c.R[k] = float(np.asarray(f["R_old"]).ravel()[k])
            arr[i].R_new[k] = float(np.asarray(f["R_new"]).ravel()[k])
        for k in range(3):
            c.t[k] = float(f["t_old"][k])
            arr[i].t_new[k] = float(f["t_new"][k])
        c.fx, c.fy, c.cx, c.cy, c.width, c.height = f["fx"], f["fy"], f["cx"], f["cy"], f["W"], f["H"]
    raw = np.frombuffer(bytes(arr), np.uint8).copy()
    return torch.from_numpy(raw).cuda()


@pytest.mark.parametrize("A,K,n_fix,far", [(20000, 10, 12, 80.0), (3001, 4, 1, 30.0), (5, 2, 0, 50.0),
                                           (50000, 10, 40, 60.0)])
def test_deform_against_oracle(A, K, n_fix, far):
    rng = np.random.default_rng(A + n_fix)
    vox = synth.corridor_voxels()
    pos = vox[np.sort(rng.choice(len(vox), A, replace=False))].T.astype(np.float32)
    offs = rng.normal(0, 0.1, (3, A * K)).astype(np.float32)
    fixes = synth.loop_fixes(A + 1, n_fix, spacing=2.0, rot_deg=2.0, trans_m=0.2)
    dpos, doffs = torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(offs.copy()).cuda()
    owner = torch.empty(A, dtype=torch.int32, device="cuda")
    table = _fix_table(fixes) if n_fix else torch.zeros(16, dtype=torch.uint8, device="cuda")
    B.glam_deform_anchors(dpos, doffs, A, K, table, n_fix, 0.2, far, owner, None)
    torch.cuda.synchronize()
    x, o, own, amb = deform(pos.astype(np.float64), offs.astype(np.float64), K, fixes, 0.2, far)
    got_owner = owner.cpu().numpy().astype(np.int64)
    ok = ~amb
    assert np.array_equal(got_owner[ok], own[ok])
    if n_fix:
        assert (own >= 0).sum() > A // 10
    # FP32 rounding of a rigid motion of coordinates up to ~80 m
    same = ok & (got_owner == own)
    np.testing.assert_allclose(dpos.cpu().numpy()[:, same], x[:, same], atol=2e-5 * 80, rtol=0)
    o_same = np.repeat(same, K)
    np.testing.assert_allclose(doffs.cpu().numpy()[:, o_same], o[:, o_same], atol=2e-6, rtol=0)
