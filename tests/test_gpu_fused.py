"""The fused decode + projection launch (glam_decode_project) against the two separate
calls: decoded Gaussians and every projected output bit for bit, for both opacity
activations, several partitions and every tile edge (the tile count depends on it)."""
import numpy as np
import pytest
import torch

import synth
from paper_2607_21416_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu


def snap(pipe):
    out = {f"dec_{k}": v.clone() for k, v in pipe.dec.items()}
    out.update({f"proj_{k}": v.clone() for k, v in pipe.proj_t.items()})
    return out


@pytest.mark.parametrize("tile,sigmoid", [(16, False), (8, True), (32, False)])
def test_fused_equals_separate(tile, sigmoid):
    scene = synth.anchor_scene(3101 + tile, [1500, 900, 400], 2, W=200, H=120, fx=140.0, bias_std=0.3)
    if sigmoid:
        scene["opacity_mode"] = "sigmoid"
    pipe = Pipeline(scene, device="cuda", tile=tile)
    print(f"fused decode+project: tile {tile}, sigmoid {sigmoid}", flush=True)
    for t in list(pipe.dec.values()) + list(pipe.proj_t.values()):
        t.fill_(7 if t.dtype == torch.int32 else float("nan"))
    pipe.decode()
    pipe.project()
    torch.cuda.synchronize()
    a = snap(pipe)
    for t in list(pipe.dec.values()) + list(pipe.proj_t.values()):
        t.fill_(-3 if t.dtype == torch.int32 else 123.0)
    pipe.decode_project()
    torch.cuda.synchronize()
    b = snap(pipe)
    vis = a["proj_ntiles"] > 0
    assert vis.any() and (~vis).any()
    for k in a:
        x, y = a[k], b[k]
        if k == "proj_splat":  # the record is written for visible Gaussians only
            x, y = x[vis], y[vis]
        assert torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y), k
