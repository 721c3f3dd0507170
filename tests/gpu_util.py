"""Helpers shared by the GPU parity tests: run the HIP pipeline, pull its stage
outputs to the host, and feed them to the FP64 oracle stage by stage."""
import numpy as np
import torch

import oracle
from paper_2607_21416_amd.pipeline import Pipeline

# flags that mark a pixel whose value depends on a decision taken within rounding: a
# threshold, the stop test, or (end to end only) the depth order of a near-tie
AMB_VALUE = oracle.AMB_ALPHA | oracle.AMB_T | oracle.AMB_DEPTH
# stage-wise the oracle composites in the GPU's own order, so depth ties cannot matter
AMB_STAGE = oracle.AMB_ALPHA | oracle.AMB_T


def run(scene, steps=1, tile=16, tuning=None):
    pipe = Pipeline(scene, device="cuda", tile=tile, tuning=tuning)
    pipe.count_evaluations()
    pipe.fit_capacity()
    pipe.status.zero_()
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    pipe.check_status()
    return pipe


def host(pipe):
    """Everything the GPU computed, as numpy arrays."""
    h = {k: v.cpu().numpy() for k, v in pipe.proj_t.items()}
    st = pipe.status.cpu().numpy()
    P = int(np.uint32(st[1]))
    dbits = int(st[4])
    keys = pipe.keys[:P].cpu().numpy().view(np.uint64)
    h.update(P=P, dbits=dbits, keys=keys, vals=pipe.vals[:P].cpu().numpy(),
             ranges=pipe.ranges.cpu().numpy().reshape(-1, 2).astype(np.int64),
             image=pipe.image.cpu().numpy(), T_final=pipe.T_final.cpu().numpy(),
             n_contrib=pipe.n_contrib.cpu().numpy(), dimage=pipe.dimage.cpu().numpy(),
             n_eval=None if pipe.n_eval is None else pipe.n_eval.cpu().numpy(),
             loss=pipe.loss.cpu().numpy(), g2d=pipe.g2d.cpu().numpy())
    if not pipe.plain:
        h["dec"] = {k: v.cpu().numpy() for k, v in pipe.dec.items()}
        h["pgrad"] = {k: v.cpu().numpy() for k, v in pipe.pgrad.items()}
    h["dg"] = {k: v.cpu().numpy() for k, v in pipe.dg.items()}
    return h


def unpack_box(splat):
    bx = splat[:, 9].view(np.uint32)
    by = splat[:, 10].view(np.uint32)
    return np.stack([bx & 0xFFFF, bx >> 16, by & 0xFFFF, by >> 16]).astype(np.int32)


def view_slices(pipe):
    vt = pipe.vt
    out = []
    for i in range(vt.n):
        vi = vt.info[i]
        out.append(dict(g0=int(vi.g_begin), g1=int(vi.g_begin + vi.g_count), p0=int(vi.pix_begin),
                        t0=int(vi.tile_begin), nt=int(vi.tiles_x * vi.tiles_y), W=int(vi.cam.width),
                        H=int(vi.cam.height)))
    return out


def gpu_splats(h, sl):
    """The GPU's projected splats of one view, in the oracle's layout."""
    g0, g1 = sl["g0"], sl["g1"]
    sp = h["splat"][g0:g1]
    vis = h["ntiles"][g0:g1] > 0
    prect = unpack_box(sp)
    prect[:, ~vis] = np.array([[0], [-1], [0], [-1]])
    pr = dict(uv=h["uv"][:, g0:g1].astype(np.float64), conic=h["conic"][:, g0:g1].astype(np.float64),
              depth=h["depth"][g0:g1].astype(np.float64), prect=prect, ntiles=h["ntiles"][g0:g1])
    gs = dict(opacity=sp[:, 5].astype(np.float64), rgb=sp[:, 6:9].T.astype(np.float64))
    return pr, gs


def view_image(h, sl, key="image"):
    p0, W, H = sl["p0"], sl["W"], sl["H"]
    return h[key][3 * p0:3 * p0 + 3 * W * H].reshape(3, H, W)


def view_pixels(h, sl, key):
    p0, W, H = sl["p0"], sl["W"], sl["H"]
    return h[key][p0:p0 + W * H].reshape(H, W)


def grad_close(g, ref, rel=1e-3, floor=1e-5, norm_rel=1e-3, name=""):
    """Per element |g - ref| <= rel |ref| + floor max|ref|, and relative L2 error.

    The floor is the cancellation allowance of an FP32 sum: an element that is the
    small difference of many large per-pixel terms carries an absolute error of a few
    ulp of those terms, which the largest element of the tensor bounds."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    assert g.shape == ref.shape, (name, g.shape, ref.shape)
    if ref.size == 0:
        return
    scale = np.abs(ref).max()
    if scale == 0:
        assert np.abs(g).max() == 0, name
        return
    err = np.abs(g - ref)
    bad = err > rel * np.abs(ref) + floor * scale
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} elements off; worst "
                           f"{err[bad].max():.3e} at ref {ref[bad][np.argmax(err[bad])]:.3e} (max|ref| {scale:.3e})")
    nr = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
    assert nr <= norm_rel, f"{name}: relative L2 error {nr:.3e}"
