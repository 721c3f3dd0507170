"""The optimiser step on the GPU against the FP64 oracle: several groups in one launch
(ragged lengths, an empty group, periodic per-segment learning rates), three steps in a
row; and the pipeline's step after a real backward."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import run
from oracle import optim
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import ADAM, ADAM_LR_ANCHOR

pytestmark = pytest.mark.gpu


def _group(p, g, m, v, period, ends, lrs):
    a = B.AdamGroup()
    a.param, a.grad, a.m, a.v = p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr()
    a.n, a.period, a.n_seg = p.numel(), period, len(ends)
    for j, (e, lr) in enumerate(zip(ends, lrs)):
        a.seg_end[j], a.lr[j] = e, lr
    return a


def test_adam_groups_against_oracle():
    rng = np.random.default_rng(11)
    specs = [(1000, 1, [1], [0.01]), (4099, 1, [1], [0.003]), (0, 1, [1], [0.1]), (3, 1, [1], [0.5]),
             (7182 * 3 + 5, 7182, [2394, 4788, 7182], [0.002, 0.008, 0.004]), (64, 16, [4, 9, 13, 16],
                                                                              [0.1, 0.2, 0.3, 0.4])]
    host, dev = [], []
    for n, period, ends, lrs in specs:
        p = rng.normal(size=n).astype(np.float32)
        m = (rng.normal(size=n) * 0.1).astype(np.float32)
        v = (rng.uniform(0, 1, n) * 0.01).astype(np.float32)
        host.append([p.astype(np.float64), m.astype(np.float64), v.astype(np.float64), period, ends, lrs])
        dev.append([torch.from_numpy(x).cuda() for x in (p, m, v)] + [torch.empty(max(n, 1), device="cuda")])
    # the ABI takes the hyper-parameters in single precision: the oracle gets the same
    # values (rounded to FP32, then promoted exactly)
    b1, b2, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8))
    for t in range(1, 4):
        groups = (B.AdamGroup * len(specs))()
        for i, ((n, period, ends, lrs), (pd, md, vd, gd)) in enumerate(zip(specs, dev)):
            g = (rng.normal(size=n) * 10.0 ** rng.uniform(-4, 1, n)).astype(np.float32)
            gd[:n] = torch.from_numpy(g).cuda()
            host[i].append(g.astype(np.float64))
            groups[i] = _group(pd, gd, md, vd, period, ends, lrs)
        B.glam_adam_step(groups, len(specs), t, b1, b2, eps, None)
        torch.cuda.synchronize()
        for i, (n, period, ends, lrs) in enumerate(specs):
            p0, m0, v0 = host[i][:3]
            lr = optim.segment_lr(n, period, ends, lrs)
            g = host[i].pop()
            p, m, v = optim.adam_step(p0, g, m0, v0, t, lr, b1, b2, eps)
            pd, md, vd, _ = dev[i]
            # FP32: the moments to a few ulp of their terms (m can cancel); the parameter to
            # a few ulp of itself plus a few ulp of the update (a handful of roundings)
            err_m = np.abs(md.cpu().numpy() - m)
            assert (err_m <= 1e-6 * (b1 * np.abs(m0) + (1 - b1) * np.abs(g)) + 1e-30).all(), err_m.max()
            np.testing.assert_allclose(vd.cpu().numpy(), v, rtol=1e-5, atol=1e-15)
            err = np.abs(pd.cpu().numpy() - p)
            assert (err <= 2e-6 * np.abs(p) + 4e-6 * np.abs(p - p0) + 1e-12).all(), err.max()
            # continue from the GPU's own state, as the next step will
            host[i][:3] = [x.cpu().numpy().astype(np.float64) for x in (pd, md, vd)]


def test_pipeline_step_after_backward():
    scene = synth.anchor_scene(21, [600, 300], 2, W=96, H=64, fx=70.0, ssim_weight=0.2)
    pipe = run(scene)
    before = {k: pipe.params[k].cpu().numpy().astype(np.float64) for k in ADAM_LR_ANCHOR}
    grads = {k: pipe.pgrad[k].cpu().numpy().astype(np.float64) for k in ADAM_LR_ANCHOR}
    pipe.adam_step()
    torch.cuda.synchronize()
    for k in ADAM_LR_ANCHOR:
        if k == "mlp":
            P = before[k].shape[1]
            F, K, h = scene["F"], scene["K"], scene["hidden"]
            e0 = h * (F + 4) + h + K * h + K
            e1 = e0 + h * (F + 4) + h + 3 * K * h + 3 * K
            lr = optim.segment_lr(before[k].size, P, [e0, e1, P], ADAM_LR_ANCHOR[k]).reshape(before[k].shape)
        else:
            lr = ADAM_LR_ANCHOR[k]
        b1, b2, eps = (float(np.float32(ADAM[x])) for x in ("beta1", "beta2", "eps"))
        want, _, _ = optim.adam_step(before[k], grads[k], 0 * before[k], 0 * before[k], 1, lr, b1, b2, eps)
        got = pipe.params[k].cpu().numpy()
        err = np.abs(got - want)
        assert (err <= 2e-6 * np.abs(want) + 4e-6 * np.abs(want - before[k]) + 1e-12).all(), (k, err.max())
