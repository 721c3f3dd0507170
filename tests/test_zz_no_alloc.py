"""glam_loss_noalloc (the loss for callers that cannot allocate: its partial sums in
the library's per-device scratch) against glam_loss with a caller workspace, through
the C ABI: two calls in a row, the second on a smaller view table, each bit-identical to
glam_loss on the same inputs (same kernels); and a view table whose partial sums would
not fit the scratch is rejected before anything is launched."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import Pipeline, ViewTable

pytestmark = pytest.mark.gpu


def _forward(scene):
    pipe = Pipeline(scene, device="cuda")
    pipe.fit_capacity()
    pipe.status.zero_()
    pipe.forward()
    torch.cuda.synchronize()
    pipe.check_status()
    return pipe


def _both(pipe):
    s = torch.cuda.current_stream()
    n = pipe.vt.n
    d_ref, d_na = torch.full_like(pipe.dimage, 7.0), torch.full_like(pipe.dimage, -7.0)
    l_ref, l_na = torch.full((n,), 7.0, device="cuda"), torch.full((n,), -7.0, device="cuda")
    t_ref, t_na = torch.full((1,), 7.0, device="cuda"), torch.full((1,), -7.0, device="cuda")
    B.glam_loss(pipe.vt.views, pipe.image, pipe.target, pipe.ssim_weight, d_ref, l_ref, t_ref, pipe.ws_loss,
                pipe.ws_loss.numel(), s)
    B.glam_loss_noalloc(pipe.vt.views, pipe.image, pipe.target, pipe.ssim_weight, d_na, l_na, t_na, s)
    torch.cuda.synchronize()
    for a, b in ((d_ref, d_na), (l_ref, l_na), (t_ref, t_na)):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    return l_na.cpu().numpy()


def test_noalloc_loss_matches_the_workspace_call_twice():
    big = _forward(synth.config("C3"))                       # 4 views of 1226x370, SSIM
    print(f"no-alloc loss: config 3, {big.vt.n} views", flush=True)
    l1 = _both(big)
    assert np.isfinite(l1).all() and (l1 > 0).all()
    small = _forward(synth.plain_scene(1011, 2000, 70, 45))  # one ragged 70x45 view
    small.ssim_weight = 0.2
    print("no-alloc loss: ragged 70x45 view", flush=True)
    l2 = _both(small)
    assert l2.shape == (1,) and np.isfinite(l2).all()


def test_noalloc_loss_rejects_a_view_table_beyond_its_scratch():
    # 1,500 views of 1226x370: 1,500 x 468 tiles x 3 channels x 8 bytes > 16 MiB
    cams = [synth.camera(np.eye(3), np.zeros(3), 718, 718, 613, 185, 1226, 370) for _ in range(1500)]
    vt = ViewTable(cams, "cuda", plain_G=1)
    assert B.glam_loss_workspace_bytes(vt.views) > B.GLAM_LOSS_SCRATCH_BYTES
    fake = C.c_void_p(0x100000)
    st = B.load().glam_loss_noalloc(B.ref(vt.views), fake, fake, C.c_float(0.2), fake, fake, None, None)
    assert st == B.GLAM_ERR_WORKSPACE
