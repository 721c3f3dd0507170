"""The torch.autograd.Function wrappers: images = GlamRender(params) and
loss = GlamLoss(images) give, through loss.backward(), the same parameter gradients as
the pipeline's own step (which the parity tests pin to the oracle); a scaled loss scales
them, and a torch operation between the two (a pixel mask) reaches the render's adjoint
as its incoming dL/dC."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import grad_close
from paper_2607_21416_amd.pipeline import GlamLoss, GlamRender, Pipeline

pytestmark = pytest.mark.gpu

SCENES = {
    "anchor": lambda: synth.anchor_scene(2051, [700, 500], 2, W=128, H=80, fx=90.0, ssim_weight=0.2),
    "plain": lambda: synth.plain_scene(2052, 1200, 96, 64),
}


def _setup(name):
    pipe = Pipeline(SCENES[name](), device="cuda")
    pipe.fit_capacity()
    pipe.status.zero_()
    keys = ("mean", "log_scale", "quat", "logit", "rgb") if pipe.plain else ("feat", "offs", "log_scale", "mlp")
    return pipe, keys


def _reference(pipe, keys):
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    src = pipe.dg if pipe.plain else pipe.pgrad
    return {k: src[k].cpu().numpy().copy() for k in keys}, pipe.loss.sum().item()


@pytest.mark.parametrize("name", list(SCENES))
def test_autograd_matches_pipeline_step(name):
    pipe, keys = _setup(name)
    want, want_loss = _reference(pipe, keys)
    params = [pipe.params[k].requires_grad_(True) for k in keys]
    try:
        image = GlamRender.apply(pipe, *params)
        loss = GlamLoss.apply(pipe, image)
        assert loss.item() == pytest.approx(want_loss, rel=1e-6)
        loss.backward()
        torch.cuda.synchronize()
        for k, p in zip(keys, params):
            # the same kernels; the atomic sums of gradients run in a run-dependent order, which
            # moves cancelling elements (quaternions) by a few 1e-4: the parity bar per element
            grad_close(p.grad.cpu().numpy(), want[k], rel=1e-3, floor=1e-5, norm_rel=1e-4, name=f"{name} autograd d{k}")
        # a scaled loss scales the gradients
        for p in params:
            p.grad = None
        image = GlamRender.apply(pipe, *params)
        (3.0 * GlamLoss.apply(pipe, image)).backward()
        torch.cuda.synchronize()
        for k, p in zip(keys, params):
            # 3 dL/dC is not exact in FP32 and the sums run in another order
            grad_close(p.grad.cpu().numpy(), 3.0 * want[k], rel=1e-3, floor=1e-5, norm_rel=1e-4,
                       name=f"{name} scaled d{k}")
    finally:
        for p in params:
            p.requires_grad_(False)
            p.grad = None


@pytest.mark.parametrize("name", list(SCENES))
def test_torch_op_between_render_and_loss(name):
    pipe, keys = _setup(name)
    params = [pipe.params[k].requires_grad_(True) for k in keys]
    try:
        mask = (torch.rand(pipe.image.shape, generator=torch.Generator().manual_seed(7)) > 0.3).float().cuda()
        image = GlamRender.apply(pipe, *params)
        loss = GlamLoss.apply(pipe, image * mask)
        loss.backward()
        torch.cuda.synchronize()
        got = {k: p.grad.cpu().numpy().copy() for k, p in zip(keys, params)}
        # the same adjoint fed the masked dL/dC directly
        dimage = (pipe.dimage * mask).contiguous()
        pipe.forward()
        pipe.backward(dimage=dimage)
        torch.cuda.synchronize()
        src = pipe.dg if pipe.plain else pipe.pgrad
        for k in keys:
            ref = src[k].cpu().numpy()
            assert np.abs(ref).max() > 0
            grad_close(got[k], ref, rel=1e-3, floor=1e-5, norm_rel=1e-4, name=f"{name} masked d{k}")
    finally:
        for p in params:
            p.requires_grad_(False)
            p.grad = None
