"""Config 3's gradients against finite differences: 64 parameters of the benchmark's
workload, stratified as 16 MLP weights and biases, 16 anchor features, 16 offsets and
16 log-scales (half the largest gradients of each kind, half drawn at random among the
non-negligible ones).  Their gradient of view 0's loss, computed on the GPU in the
benchmark's launch configuration (stored tile edge and schedule), is compared with the
FP64 oracle's central finite difference (h = 1e-6, differenced pixel by pixel and
summed exactly), and the oracle's own analytic gradient with the same difference.

The loss is piecewise smooth: the skip threshold, the stop rule, the depth order and the
0.99 clamp of Eq. 1, the ReLU gates of Eq. 2 / Eq. 6, the Jacobian clamp and the L1 term
jump or kink.  The oracle records every one of those decisions at -h and +h.  Where
none changes, the plain difference is the reference.  Where one does (a weight of an MLP
moves all 500k Gaussians, and some pixel's alpha then crosses 1/255 somewhere in its
list), the plain difference straddles a jump and the reference is the difference taken
with every decision held at the unperturbed point (the derivative of the piece the
parameters sit on, which the adjoint computes); both counts are printed."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import view_slices
from paper_2607_21416_amd import tuning
from paper_2607_21416_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu

COUNTS = {"mlp": 16, "feat": 16, "offs": 16, "log_scale": 16}  # 64 parameters


@pytest.mark.timeout(900)
def test_view0_gradients_match_finite_differences():
    scene = synth.config("C3")
    choice = tuning.autotune(scene, device="cuda")
    pipe = Pipeline(scene, device="cuda", tile=choice["tile"], tuning=tuning.schedule(choice))
    pipe.fit_capacity()
    pipe.status.zero_()
    pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    # the loss of view 0 only: its dL/dC, zero on the other views
    sl = view_slices(pipe)[0]
    dim = torch.zeros_like(pipe.dimage)
    n0 = 3 * sl["W"] * sl["H"]
    dim[3 * sl["p0"]:3 * sl["p0"] + n0] = pipe.dimage[3 * sl["p0"]:3 * sl["p0"] + n0]
    pipe.backward(dimage=dim)
    torch.cuda.synchronize()
    grads = {k: v.cpu().numpy().astype(np.float64) for k, v in pipe.pgrad.items()}
    # the oracle's analytic gradient of the same loss, and its decision record
    fwd = oracle.forward(scene, [0])
    ref = oracle.backward(scene, fwd)
    _, base = oracle.loss_maps(scene, [0])
    rng = np.random.default_rng(3003)
    checked = frozen = 0
    worst_gpu = worst_orc = 0.0
    t0 = time.time()
    for name, count in COUNTS.items():
        g = grads[name]
        flat = np.abs(g).ravel()
        gmax = flat.max()
        picks = list(np.argsort(-flat)[: count // 2])
        nz = np.setdiff1d(np.flatnonzero(flat > 1e-3 * gmax), picks)
        picks += list(rng.choice(nz, size=min(len(nz), count - len(picks)), replace=False))
        assert len(picks) == count
        for fi in picks:
            idx = np.unravel_index(int(fi), g.shape)
            fd, flipped = oracle.fd_gradient(scene, name, idx, h=1e-6, views=[0])
            if flipped:
                fd = oracle.fd_gradient_frozen(scene, name, idx, h=1e-6, views=[0], decisions=base)
                frozen += 1
            # the oracle's adjoint against its own difference (FP64 both)
            bound_o = 1e-5 * abs(fd) + 1e-9 * np.abs(ref[name]).max()
            assert abs(ref[name][idx] - fd) <= bound_o, (name, idx, ref[name][idx], fd, flipped)
            worst_orc = max(worst_orc, abs(ref[name][idx] - fd) / bound_o)
            # the GPU's gradient against it: 1e-3 relative, with a floor of 1e-6 of the
            # tensor's largest gradient for elements that are small differences
            tol = 1e-3 * abs(fd) + 1e-6 * gmax
            assert abs(g[idx] - fd) <= tol, (name, idx, g[idx], fd, flipped)
            worst_gpu = max(worst_gpu, abs(g[idx] - fd) / tol)
            checked += 1
        print(f"fd {name}: {checked} checked so far ({frozen} with decisions held: a decision flips "
              f"between -h and +h), largest error / bound: GPU {worst_gpu:.3f}, oracle {worst_orc:.3f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    assert checked == sum(COUNTS.values())
