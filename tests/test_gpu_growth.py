"""Anchor growth end to end (Eq. 4 with its bookkeeping): a keyframe's cloud is
voxelised against one partition's anchors on the GPU, the new anchors are inserted at
the end of that partition, and the grown pipeline is checked against the oracle's
growth (parameters, partition offsets and optimiser moments bit for bit), against a
pipeline built directly from the oracle's grown scene (same images bit for bit), and
against the oracle's render of the grown scene."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import check_e2e_pixels, grad_close, host, run, view_image, view_slices
from oracle import voxel as V
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu


def lib_new_voxels(points, eps, existing_points):
    """The library's new voxels of `points` against the voxels of `existing_points`:
    (centres device tensor [3][capacity], count, capacity)."""
    def call(pts, ex, n_ex):
        n = pts.shape[1]
        new = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        cen = torch.empty((3, max(n, 1)), device="cuda")
        mer = torch.empty(n_ex + max(n, 1), dtype=torch.int64, device="cuda")
        cnt = torch.empty(2, dtype=torch.int64, device="cuda")
        wsb = B.glam_voxelize_workspace_bytes(n)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        B.glam_voxelize(torch.from_numpy(np.ascontiguousarray(pts)).cuda(), n, eps, ex, n_ex, new, cen, max(n, 1), mer,
                        cnt, ws, wsb, None)
        torch.cuda.synchronize()
        m = int(cnt[0].item())
        return new, cen, mer, m

    _, _, have, m_have = call(existing_points, None, 0)
    _, cen, _, m = call(points, have, m_have)
    return cen, m, cen.shape[1]


@pytest.mark.parametrize("part", [0, 1])
def test_growth_end_to_end(part):
    eps = 0.2
    scene = synth.anchor_scene(2031, [900, 600], 2, W=160, H=96, fx=110.0, ssim_weight=0.2)
    pb = scene["part_begin"]
    pipe = Pipeline(scene, device="cuda")
    pipe.init_optimizer()
    rng = np.random.default_rng(7 + part)
    mom = {}
    for k in ("feat", "offs", "log_scale"):
        m = rng.normal(size=tuple(pipe.opt_m[k].shape)).astype(np.float32)
        v = rng.uniform(0, 1, size=tuple(pipe.opt_v[k].shape)).astype(np.float32)
        pipe.opt_m[k].copy_(torch.from_numpy(m))
        pipe.opt_v[k].copy_(torch.from_numpy(v))
        mom[k] = (m, v)
    cloud = synth.fused_points(2032 + part, 3000, nan_frac=0.1)
    own = scene["pos"][:, pb[part]:pb[part + 1]]
    print(f"growth: partition {part}", flush=True)
    cen, m, stride = lib_new_voxels(cloud, eps, own)
    pipe.grow_anchors(cen, m, part, eps, centres_stride=stride)
    torch.cuda.synchronize()
    # the oracle's growth of the same inputs
    _, _, have, _ = V.voxelize(own, eps)
    new, want_cen, _, _ = V.voxelize(cloud, eps, have)
    assert m == len(new) > 20
    pos2, feat2, ls2, offs2, pb2 = V.grow_anchors(scene["pos"], scene["feat"], scene["log_scale"], scene["offs"], pb,
                                                  part, want_cen, eps)
    got = {k: pipe.params[k].cpu().numpy() for k in ("pos", "feat", "log_scale", "offs")}
    for k, want in (("pos", pos2), ("feat", feat2), ("log_scale", ls2), ("offs", offs2)):
        assert np.array_equal(got[k], want), k
    assert pipe.part_begin.tolist() == pb2.tolist() and pipe.anchors.A == pos2.shape[1]
    # the moments move with their anchors; the new anchors' are zero
    K = scene["K"]
    at = int(pb[part + 1])
    for k, (mm, vv) in mom.items():
        for got_t, old in ((pipe.opt_m[k], mm), (pipe.opt_v[k], vv)):
            if k == "offs":
                want = np.concatenate([old[:, :at * K], np.zeros((3, m * K), np.float32), old[:, at * K:]], axis=1)
            else:
                want = np.concatenate([old[:at], np.zeros((m,) + old.shape[1:], np.float32), old[at:]], axis=0)
            assert np.array_equal(got_t.cpu().numpy(), want), k
    # the grown pipeline renders the grown scene: bit for bit as a pipeline built from the
    # oracle's grown scene, and within tolerance of the oracle
    grown = dict(scene, pos=pos2, feat=feat2, log_scale=ls2, offs=offs2, part_begin=pb2.astype(np.int32))
    pipe.fit_capacity()
    pipe.status.zero_()
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    h = host(pipe)
    fresh = host(run(grown))
    assert np.array_equal(h["image"], fresh["image"]) and np.array_equal(h["n_contrib"], fresh["n_contrib"])
    np.testing.assert_allclose(h["loss"], fresh["loss"], rtol=1e-6)
    for k in fresh["pgrad"]:
        grad_close(h["pgrad"][k], fresh["pgrad"][k], rel=1e-5, floor=1e-6, norm_rel=1e-5, name=f"grown d{k}")
    fwd = oracle.forward(grown)
    for v, (sl, r) in enumerate(zip(view_slices(pipe), fwd)):
        # a new anchor's K Gaussians all start at its centre (zero offsets): exact depth
        # ties, whose order the oracle flags as ambiguous, cover much of the image; the
        # GPU's order is checked on them instead
        check_e2e_pixels(view_image(h, sl), r, h, sl, grown["cams"][v], f"grown view {v}", depth_max=0.7)
    # the optimiser's groups follow the grown tensors
    before = pipe.params["feat"].clone()
    pipe.adam_step()
    torch.cuda.synchronize()
    moved = (pipe.params["feat"] != before).any(dim=1).cpu().numpy()
    touched = (pipe.pgrad["feat"] != 0).any(dim=1).cpu().numpy()
    assert touched.any() and moved[touched].all()


def test_growth_of_nothing_and_bad_partition():
    scene = synth.anchor_scene(2041, [300, 200], 1, W=96, H=64, fx=70.0)
    pipe = Pipeline(scene, device="cuda")
    before = {k: v.clone() for k, v in pipe.params.items()}
    pipe.grow_anchors(torch.zeros((3, 4), device="cuda"), 0, 0, 0.2)
    assert all(torch.equal(before[k], pipe.params[k]) for k in before)
    with pytest.raises(ValueError):
        pipe.grow_anchors(torch.zeros((3, 4), device="cuda"), 2, 5, 0.2)
