"""The benchmark's launch configuration: the whole step captured in one HIP graph.

Every replay must reproduce the eager step (images, transmittance, contributor counts
and sort bit for bit; the loss and the gradients, which are summed with atomics in a
run-dependent order, to 1e-5), with eager work of the program between replays, and
the work queues and device status must come back clean after each replay."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import grad_close, host
from paper_2607_21416_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu


def snapshot(pipe):
    h = host(pipe)
    return {k: h[k] for k in ("image", "T_final", "n_contrib", "keys", "vals", "ranges", "loss")} | {
        "grads": h["pgrad"] if not pipe.plain else h["dg"]}


def check_same(a, b, what):
    for k in ("image", "T_final", "n_contrib", "keys", "vals", "ranges"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"
    np.testing.assert_allclose(a["loss"], b["loss"], rtol=1e-5, err_msg=what)
    for k in a["grads"]:
        grad_close(a["grads"][k], b["grads"][k], rel=1e-5, floor=1e-6, norm_rel=1e-5, name=f"{what} d{k}")


@pytest.mark.parametrize("name", ["anchor", "plain"])
def test_graph_replays_match_eager(name):
    if name == "anchor":
        scene = synth.anchor_scene(2021, [1200, 700], 2, W=160, H=96, fx=110.0, ssim_weight=0.2)
    else:
        scene = synth.plain_scene(2022, 1500, 96, 64)
    pipe = Pipeline(scene, device="cuda")
    pipe.fit_capacity()
    pipe.status.zero_()
    pipe.step()
    torch.cuda.synchronize()
    ref = snapshot(pipe)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipe.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        pipe.step()
    torch.cuda.synchronize()
    for r in range(4):
        pipe.image.fill_(-1.0)  # eager work between replays; the replay must overwrite it
        pipe.g2d.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        pipe.check_status()
        assert int(pipe.queue.abs().sum().item()) == 0, "work queue not reset"
        check_same(snapshot(pipe), ref, f"replay {r}")
        pipe.step()
        torch.cuda.synchronize()
        check_same(snapshot(pipe), ref, f"eager after replay {r}")
