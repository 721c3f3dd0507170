"""The forward, the L1 loss and the compositing adjoint in one pass (glam_render_fused_l1)
against the three separate calls (glam_render_fwd, glam_loss with no SSIM term,
glam_composite_bwd), on the GPU through the C ABI: for scenes with a per-pixel L1 loss
(Eq. 3 without its SSIM term), the step that takes the fused pass gives the same image,
transmittance, contributor counts and dL/dC bit for bit (the same forward and loss
arithmetic), the same per-view losses to the rounding of their sums, and the same 2-D,
Gaussian and anchor/MLP gradients to FP32 rounding (floating-point atomics in both).
The end-to-end parity tests run the fused pass against the oracle, since the pipeline's
step takes it for these scenes."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import grad_close, host
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import Pipeline
from test_gpu_parity import plain_dense, plain_ragged

pytestmark = pytest.mark.gpu

CASES = {
    "C1": (lambda: synth.config("C1"), None),
    "plain_ragged": (plain_ragged, None),
    # ranges of 1000-4000 entries: long tiles walked by whole workgroups, forward and back
    "plain_dense": (plain_dense, None),
    "plain_dense_wide8": (plain_dense, {"long_log2": 7, "fwd_group_waves": 8, "fwd_blocks_per_cu": 2,
                                        "bwd_group_waves": 8, "bwd_blocks_per_cu": 2}),
    "plain_dense_wide16": (plain_dense, {"long_log2": 8, "fwd_group_waves": 16, "bwd_group_waves": 16}),
    "anchor_two_parts": (lambda: synth.anchor_scene(1021, [1500, 800], 2, W=200, H=120, fx=140.0, bias_std=0.2),
                         None),
    "C2": (lambda: synth.config("C2"), None),
}


def _pipe(scene, sched, fuse):
    pipe = Pipeline(scene, device="cuda", tuning=sched, fuse_l1=fuse)
    pipe.fit_capacity()
    pipe.status.zero_()
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    return pipe


@pytest.mark.parametrize("name", list(CASES))
def test_fused_l1_step_equals_separate_calls(name):
    make, sched = CASES[name]
    scene = make()
    assert scene.get("ssim_weight", 0.0) == 0.0
    a = _pipe(scene, sched, True)
    b = _pipe(scene, sched, False)
    assert a.fuse_l1 and not b.fuse_l1
    ha, hb = host(a), host(b)
    for k in ("image", "T_final", "n_contrib", "dimage"):
        assert np.array_equal(ha[k], hb[k]), k
    np.testing.assert_allclose(ha["loss"], hb["loss"], rtol=2e-6)
    np.testing.assert_allclose(a.loss_total.cpu().numpy(), b.loss_total.cpu().numpy(), rtol=2e-6)
    assert np.all(ha["loss"] > 0)
    grad_close(ha["g2d"], hb["g2d"], name=f"{name} fused g2d")
    grads_a = a.dg if a.plain else a.pgrad
    grads_b = b.dg if b.plain else b.pgrad
    for k in grads_a:
        grad_close(grads_a[k].cpu().numpy(), grads_b[k].cpu().numpy(), name=f"{name} fused d{k}")
    print(f"{name}: losses {ha['loss']}, {a.vt.n_gauss} view-Gaussians", flush=True)


def test_fused_l1_rejects_bad_arguments():
    scene = plain_ragged()
    pipe = _pipe(scene, None, True)
    lib = B.load()
    args = [B.ref(pipe.proj), B.ref(pipe.bins), B.ref(pipe.vt.views), B.ref(pipe.bg), B.ref(pipe.target),
            B.ref(pipe.image), B.ref(pipe.T_final), B.ref(pipe.n_contrib), B.ref(pipe.dimage), B.ref(pipe.loss),
            B.ref(pipe.loss_total), B.ref(pipe.g2d), B.ref(pipe.ws_fused)]
    need = B.glam_render_fused_l1_workspace_bytes(pipe.vt.views)
    assert 0 < need <= pipe.ws_fused.numel()
    assert lib.glam_render_fused_l1(*args, need - 1, None) == B.GLAM_ERR_WORKSPACE
    bad = list(args)
    bad[8] = None  # dL/dC is required
    assert lib.glam_render_fused_l1(*bad, need, None) == B.GLAM_ERR_INVALID_ARG
