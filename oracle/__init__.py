"""FP64 CPU oracle of the anchor-decoded Gaussian-splatting render.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's CPU-baseline leg
are the only callers.  The library product never imports this package.

A thin ctypes wrapper over `liboracle.so` (plain C++17 loops in double precision,
oracle_geometry.cpp and oracle_raster.cpp) plus the composition of its stages into a
full mapping step: decode (Eq. 2, Eq. 6) -> projection -> tile binning and depth sort
-> compositing (Eq. 1) -> loss (Eq. 3) -> analytic backward.  Inputs are the float32
arrays of the `synth` module promoted exactly to float64.

Parity pins: every function here is checked by tests/test_oracle_*.py against closed
forms, invariants, brute force, a NumPy matmul and finite differences.  The readings
that no such pin can fix (MLP activations, partition semantics, footprint rule, loss
weights and window) are "parity unpinned": they are the oracle's stated definitions.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

TILE = (16, 16)
AMB_ALPHA, AMB_T, AMB_DEPTH, AMB_CLAMP = 1, 2, 4, 8
OPACITY_MODE = {"tanh": 0, "sigmoid": 1}

_lib = None


class Cam(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("W", C.c_int32), ("H", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_loss.restype = C.c_double
        _lib.orc_loss_signed.restype = C.c_double
        _lib.orc_mlp_param_count.restype = C.c_int
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_render_lists.restype = C.c_void_p
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


DEFAULT_MARGINS = dict(alpha=1e-6, T=1e-8, depth=1e-6, clamp=1e-6)


def set_margins(alpha=1e-6, T=1e-8, depth=1e-6, clamp=1e-6) -> None:
    """Widths of the ambiguity windows behind the AMB_* flags (see orc_set_margins)."""
    lib().orc_set_margins(C.c_double(alpha), C.c_double(T), C.c_double(depth), C.c_double(clamp))


class margins:
    """Context manager: ambiguity windows of the given widths, defaults restored after."""

    def __init__(self, **kw):
        self.kw = dict(DEFAULT_MARGINS, **kw)

    def __enter__(self):
        set_margins(**self.kw)
        return self

    def __exit__(self, *exc):
        set_margins(**DEFAULT_MARGINS)
        return False


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def cam_struct(cam: dict) -> Cam:
    c = Cam()
    R = np.asarray(cam["R"], np.float64).ravel()
    t = np.asarray(cam["t"], np.float64).ravel()
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    c.W, c.H = int(cam["W"]), int(cam["H"])
    return c


def _d(a):
    return np.ascontiguousarray(a, np.float64)


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i(x):
    return C.c_int(int(x))


# ----------------------------------------------------------------------------------
# Geometry stages
# ----------------------------------------------------------------------------------

def mlp_param_count(F, K, hidden=32):
    return lib().orc_mlp_param_count(F, K, hidden)


def decode(scene: dict, m: int, cam: dict, relu_in=None, want_relu: bool = False) -> dict:
    """Anchors of partition m decoded for camera `cam` (Eq. 2 and Eq. 6).  With
    want_relu the ReLU decisions [A][3][hidden] come back as out["relu"]; relu_in holds
    them fixed (finite-difference checks)."""
    a0, a1 = int(scene["part_begin"][m]), int(scene["part_begin"][m + 1])
    A, F, K, hid = a1 - a0, scene["F"], scene["K"], scene["hidden"]
    pos = _d(scene["pos"][:, a0:a1])
    feat = _d(scene["feat"][a0:a1])
    ls = _d(scene["log_scale"][a0:a1])
    offs = _d(scene["offs"][:, a0 * K:a1 * K])
    mlp = _d(scene["mlp"][m])
    G = A * K
    out = dict(mean=np.zeros((3, G)), scale=np.zeros((3, G)), quat=np.zeros((4, G)),
               opacity=np.zeros(G), rgb=np.zeros((3, G)))
    cs = cam_struct(cam)
    rin = None if relu_in is None else np.ascontiguousarray(relu_in, np.uint8)
    rout = np.zeros((A, 3, hid), np.uint8) if want_relu else None
    lib().orc_decode_ex(_i(A), _i(F), _i(K), _i(hid), _p(pos), _p(feat), _p(ls), _p(offs), _p(mlp),
                        C.byref(cs), _i(OPACITY_MODE[scene["opacity_mode"]]), _p(out["mean"]),
                        _p(out["scale"]), _p(out["quat"]), _p(out["opacity"]), _p(out["rgb"]),
                        None if rin is None else _p(rin), None if rout is None else _p(rout))
    if want_relu:
        out["relu"] = rout
    return out


def decode_bwd(scene: dict, m: int, cam: dict, dg: dict, acc: dict) -> None:
    """Accumulates the decode adjoint of one view into acc (dfeat, doffs, dlog_scale,
    dmlp over the whole scene)."""
    a0, a1 = int(scene["part_begin"][m]), int(scene["part_begin"][m + 1])
    A, F, K, hid = a1 - a0, scene["F"], scene["K"], scene["hidden"]
    pos = _d(scene["pos"][:, a0:a1])
    feat = _d(scene["feat"][a0:a1])
    ls = _d(scene["log_scale"][a0:a1])
    offs = _d(scene["offs"][:, a0 * K:a1 * K])
    mlp = _d(scene["mlp"][m])
    dfeat = np.zeros((A, F)); doffs = np.zeros((3, A * K)); dls = np.zeros(A)
    dmlp = np.zeros(mlp.size)
    cs = cam_struct(cam)
    lib().orc_decode_bwd(_i(A), _i(F), _i(K), _i(hid), _p(pos), _p(feat), _p(ls), _p(offs),
                         _p(mlp), C.byref(cs), _i(OPACITY_MODE[scene["opacity_mode"]]),
                         _p(_d(dg["mean"])), _p(_d(dg["scale"])), _p(_d(dg["quat"])),
                         _p(_d(dg["opacity"])), _p(_d(dg["rgb"])), _p(dfeat), _p(doffs), _p(dls),
                         _p(dmlp))
    acc["feat"][a0:a1] += dfeat
    acc["offs"][:, a0 * K:a1 * K] += doffs
    acc["log_scale"][a0:a1] += dls
    acc["mlp"][m] += dmlp


def plain_activate(scene: dict) -> dict:
    G = scene["mean"].shape[1]
    out = dict(mean=_d(scene["mean"]), scale=np.zeros((3, G)), quat=np.zeros((4, G)),
               opacity=np.zeros(G), rgb=_d(scene["rgb"]))
    lib().orc_plain_activate(_i(G), _p(_d(scene["log_scale"])), _p(_d(scene["quat"])),
                             _p(_d(scene["logit"])), _p(out["scale"]), _p(out["quat"]),
                             _p(out["opacity"]))
    return out


def plain_activate_bwd(scene: dict, dg: dict) -> dict:
    G = scene["mean"].shape[1]
    out = dict(mean=_d(dg["mean"]).copy(), log_scale=np.zeros((3, G)), quat=np.zeros((4, G)),
               logit=np.zeros(G), rgb=_d(dg["rgb"]).copy())
    lib().orc_plain_activate_bwd(_i(G), _p(_d(scene["log_scale"])), _p(_d(scene["quat"])),
                                 _p(_d(scene["logit"])), _p(_d(dg["scale"])),
                                 _p(_d(dg["quat"])), _p(_d(dg["opacity"])), _p(out["log_scale"]),
                                 _p(out["quat"]), _p(out["logit"]))
    return out


FOOTPRINT = {"opacity": 0, "3sigma": 1}


def project(gs: dict, cam: dict, tile=TILE, clamp_in=None, footprint: str = "opacity") -> dict:
    """Projection and footprint; out["clamp"][G][2] holds the Jacobian clamp decision
    per axis (0 free, 1 low limit, 2 high limit); clamp_in holds it fixed.  footprint:
    "opacity" (the alpha >= 1/255 box) or "3sigma" (the lineage's tile-granular square,
    see orc_project_ex)."""
    G = gs["opacity"].shape[0]
    out = dict(uv=np.zeros((2, G)), conic=np.zeros((3, G)), cov2d=np.zeros((3, G)),
               depth=np.zeros(G), ext=np.zeros((2, G)), prect=np.zeros((4, G), np.int32),
               ntiles=np.zeros(G, np.int32), clamp=np.zeros((G, 2), np.int8))
    cs = cam_struct(cam)
    cin = None if clamp_in is None else np.ascontiguousarray(clamp_in, np.int8)
    lib().orc_project_ex(_i(G), _p(_d(gs["mean"])), _p(_d(gs["scale"])), _p(_d(gs["quat"])),
                         _p(_d(gs["opacity"])), C.byref(cs), _i(tile[0]), _i(tile[1]),
                         _p(out["uv"]), _p(out["conic"]), _p(out["cov2d"]), _p(out["depth"]),
                         _p(out["ext"]), _p(out["prect"]), _p(out["ntiles"]),
                         None if cin is None else _p(cin), _p(out["clamp"]), _i(FOOTPRINT[footprint]))
    return out


def project_bwd(gs: dict, cam: dict, ntiles: np.ndarray, g2d: np.ndarray) -> dict:
    G = gs["opacity"].shape[0]
    out = dict(mean=np.zeros((3, G)), scale=np.zeros((3, G)), quat=np.zeros((4, G)),
               opacity=np.zeros(G), rgb=np.zeros((3, G)))
    cs = cam_struct(cam)
    lib().orc_project_bwd(_i(G), _p(_d(gs["mean"])), _p(_d(gs["scale"])), _p(_d(gs["quat"])),
                          _p(_d(gs["opacity"])), C.byref(cs),
                          _p(np.ascontiguousarray(ntiles, np.int32)), _p(_d(g2d)),
                          _p(out["mean"]), _p(out["scale"]), _p(out["quat"]), _p(out["opacity"]),
                          _p(out["rgb"]))
    return out


def rect_f32(u, v, ex, ey, W, H, tile=TILE):
    """Footprint boxes and tile counts from single-precision centres and half extents,
    with the same single-precision operations as a GPU (stage-wise tile assignment)."""
    f = lambda a: np.ascontiguousarray(a, np.float32)
    u, v, ex, ey = f(u), f(v), f(ex), f(ey)
    G = u.shape[0]
    prect = np.zeros((4, G), np.int32)
    nt = np.zeros(G, np.int32)
    lib().orc_rect_f32(_i(G), _p(u), _p(v), _p(ex), _p(ey), _i(W), _i(H), _i(tile[0]),
                       _i(tile[1]), _p(prect), _p(nt))
    return prect, nt


def tile_grid(cams, tile=TILE):
    tx = np.array([(c["W"] + tile[0] - 1) // tile[0] for c in cams], np.int32)
    ty = np.array([(c["H"] + tile[1] - 1) // tile[1] for c in cams], np.int32)
    base = np.concatenate([[0], np.cumsum(tx.astype(np.int64) * ty)]).astype(np.int64)
    return tx, ty, base


def bin_sort(prect: np.ndarray, ntiles: np.ndarray, depth: np.ndarray, gbegin, cams, tile=TILE):
    """Stable (tile, depth) sort of the duplicated pairs of all views.  Returns global
    tile ids, Gaussian ids (global) and ranges[T][2]."""
    G = prect.shape[1]
    tx, ty, base = tile_grid(cams, tile)
    P = int(np.asarray(ntiles, np.int64).sum())
    T = int(base[-1])
    tiles = np.zeros(P, np.int32)
    vals = np.zeros(P, np.int32)
    ranges = np.zeros((T, 2), np.int64)
    gb = np.ascontiguousarray(gbegin, np.int64)
    lib().orc_bin_sort(_i(len(cams)), _p(gb), _p(tx), _p(ty), _p(base), _i(tile[0]), _i(tile[1]),
                       _p(np.ascontiguousarray(prect, np.int32)), _p(_d(depth)), C.c_int64(G),
                       C.c_int64(T), _p(tiles), _p(vals), _p(ranges))
    return dict(tiles=tiles, vals=vals, ranges=ranges, tile_base=base, P=P)


# ----------------------------------------------------------------------------------
# Raster stages (one view, view-local arrays)
# ----------------------------------------------------------------------------------

def _splats(pr: dict, gs: dict):
    return (_d(pr["uv"]), _d(pr["conic"]), _d(gs["opacity"]), _d(gs["rgb"]),
            np.ascontiguousarray(pr["prect"], np.int32), _d(pr["depth"]))


def render_fwd(pr: dict, gs: dict, vals, ranges, cam, bg=(0.0, 0.0, 0.0), tile=TILE) -> dict:
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, prect, depth = _splats(pr, gs)
    out = dict(image=np.zeros((3, H, W)), T_final=np.zeros((H, W)),
               n_contrib=np.zeros((H, W), np.int32), n_eval=np.zeros((H, W), np.int32),
               amb=np.zeros((H, W), np.uint8))
    lib().orc_render_fwd(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _p(prect), _p(depth),
                         _p(np.ascontiguousarray(vals, np.int32)),
                         _p(np.ascontiguousarray(ranges, np.int64)), _i(W), _i(H), _i(tile[0]),
                         _i(tile[1]), _p(_d(bg)), _p(out["image"]), _p(out["T_final"]),
                         _p(out["n_contrib"]), _p(out["n_eval"]), _p(out["amb"]))
    return out


def render_bwd(pr: dict, gs: dict, vals, ranges, cam, dimage, bg=(0.0, 0.0, 0.0), tile=TILE):
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, prect, depth = _splats(pr, gs)
    g2d = np.zeros((9, G))
    lib().orc_render_bwd(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _p(prect), _p(depth),
                         _p(np.ascontiguousarray(vals, np.int32)),
                         _p(np.ascontiguousarray(ranges, np.int64)), _i(W), _i(H), _i(tile[0]),
                         _i(tile[1]), _p(_d(bg)), _p(_d(dimage)), _p(g2d))
    return g2d


def render_bwd_magnitude(pr: dict, gs: dict, vals, ranges, cam, dimage, bg=(0.0, 0.0, 0.0), tile=TILE):
    """Per element of render_bwd's output [9][G], the sum of the magnitudes of the terms
    it is a sum of: an FP32 evaluation of the element is within a modest multiple of
    2^-24 times this of the exact value."""
    lib().orc_set_magnitude_mode(1)
    try:
        return render_bwd(pr, gs, vals, ranges, cam, dimage, bg, tile)
    finally:
        lib().orc_set_magnitude_mode(0)


def render_lists(pr: dict, gs: dict, vals, ranges, cam, tile=TILE) -> dict:
    """Every pixel's composited list (Gaussians that took part, front to back, and
    whether each alpha was clamped): offsets[H*W+1], ids[], clamped[]."""
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, prect, depth = _splats(pr, gs)
    v = np.ascontiguousarray(vals, np.int32)
    r = np.ascontiguousarray(ranges, np.int64)
    total = C.c_int64(0)
    handle = lib().orc_render_lists(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _p(prect), _p(depth), _p(v),
                                    _p(r), _i(W), _i(H), _i(tile[0]), _i(tile[1]), C.byref(total))
    n = int(total.value)
    offsets = np.zeros(W * H + 1, np.int64)
    ids = np.zeros(max(n, 1), np.int32)
    clamped = np.zeros(max(n, 1), np.uint8)
    lib().orc_render_lists_take(C.c_void_p(handle), _p(offsets), _p(ids), _p(clamped))
    return dict(offsets=offsets, ids=ids[:n], clamped=clamped[:n])


def render_frozen(pr: dict, gs: dict, lists: dict, cam, bg=(0.0, 0.0, 0.0)) -> dict:
    """Eq. 1 over fixed composited lists (see render_lists)."""
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, _, _ = _splats(pr, gs)
    out = dict(image=np.zeros((3, H, W)), T_final=np.zeros((H, W)))
    ids = np.ascontiguousarray(lists["ids"], np.int32)
    cl = np.ascontiguousarray(lists["clamped"], np.uint8)
    if ids.size == 0:
        ids, cl = np.zeros(1, np.int32), np.zeros(1, np.uint8)
    lib().orc_render_frozen(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _i(W), _i(H), _p(_d(bg)),
                            _p(np.ascontiguousarray(lists["offsets"], np.int64)), _p(ids), _p(cl),
                            _p(out["image"]), _p(out["T_final"]))
    return out


def render_brute(pr: dict, gs: dict, cam, bg=(0.0, 0.0, 0.0)) -> dict:
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, prect, depth = _splats(pr, gs)
    out = dict(image=np.zeros((3, H, W)), T_final=np.zeros((H, W)),
               n_contrib=np.zeros((H, W), np.int32), amb=np.zeros((H, W), np.uint8))
    lib().orc_render_brute(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _p(prect), _p(depth), _i(W),
                           _i(H), _p(_d(bg)), _p(out["image"]), _p(out["T_final"]),
                           _p(out["n_contrib"]), _p(out["amb"]))
    return out


def render_brute_bwd(pr: dict, gs: dict, cam, dimage, bg=(0.0, 0.0, 0.0)):
    W, H = cam["W"], cam["H"]
    G = gs["opacity"].shape[0]
    uv, con, op, rgb, prect, depth = _splats(pr, gs)
    g2d = np.zeros((9, G))
    lib().orc_render_brute_bwd(_i(G), _p(uv), _p(con), _p(op), _p(rgb), _p(prect), _p(depth),
                               _i(W), _i(H), _p(_d(bg)), _p(_d(dimage)), _p(g2d))
    return g2d


def loss(image, target, w_ssim: float, l1_sign=None):
    """Eq. 3 for one view: (L, per-pixel terms, SSIM map, dL/dC).  l1_sign [3][H][W]
    holds the sign of each L1 term fixed (finite-difference checks)."""
    image, target = _d(image), _d(target)
    _, H, W = image.shape
    loss_px = np.zeros((H, W))
    ssim = np.zeros((3, H, W))
    dimage = np.zeros((3, H, W))
    sg = None if l1_sign is None else _d(l1_sign)
    L = lib().orc_loss_signed(_i(W), _i(H), _p(image), _p(target), C.c_double(w_ssim),
                              None if sg is None else _p(sg), _p(loss_px), _p(ssim), _p(dimage))
    return L, loss_px, ssim, dimage


# ----------------------------------------------------------------------------------
# Whole step
# ----------------------------------------------------------------------------------

def view_gaussians(scene: dict, v: int) -> dict:
    cam = scene["cams"][v]
    if scene["kind"] == "plain":
        return plain_activate(scene)
    return decode(scene, cam["partition"], cam)


def forward(scene: dict, views=None, tile=TILE, bg=(0.0, 0.0, 0.0), want_loss=True,
            footprint: str = "opacity") -> list:
    """Forward pass of every view (FP64 end to end).  Returns one dict per view with
    the decoded Gaussians, projection, bins, render outputs and loss terms."""
    views = range(len(scene["cams"])) if views is None else views
    out = []
    for v in views:
        cam = scene["cams"][v]
        gs = view_gaussians(scene, v)
        pr = project(gs, cam, tile, footprint=footprint)
        G = gs["opacity"].shape[0]
        b = bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, G], [cam], tile)
        r = render_fwd(pr, gs, b["vals"], b["ranges"], cam, bg, tile)
        rec = dict(view=v, gs=gs, proj=pr, bins=b, **r)
        if want_loss:
            L, lpx, ssim, dimg = loss(r["image"], scene["targets"][v], scene["ssim_weight"])
            rec.update(loss=L, loss_px=lpx, ssim=ssim, dimage=dimg)
        out.append(rec)
    return out


def zero_grads(scene: dict) -> dict:
    if scene["kind"] == "plain":
        G = scene["mean"].shape[1]
        return dict(mean=np.zeros((3, G)), log_scale=np.zeros((3, G)), quat=np.zeros((4, G)),
                    logit=np.zeros(G), rgb=np.zeros((3, G)))
    A, F, K = scene["feat"].shape[0], scene["F"], scene["K"]
    return dict(feat=np.zeros((A, F)), offs=np.zeros((3, A * K)), log_scale=np.zeros(A),
                mlp=np.zeros(scene["mlp"].shape))


def backward(scene: dict, fwd: list, tile=TILE, bg=(0.0, 0.0, 0.0), dimages=None) -> dict:
    """Analytic gradients of the total loss (sum of the per-view losses) with respect
    to the trainable parameters: anchor features, offsets, log-scales and MLP weights
    (anchor scenes) or mean, log-scale, quaternion, opacity logit and colour (plain)."""
    acc = zero_grads(scene)
    for i, rec in enumerate(fwd):
        v = rec["view"]
        cam = scene["cams"][v]
        dimage = rec["dimage"] if dimages is None else dimages[i]
        g2d = render_bwd(rec["proj"], rec["gs"], rec["bins"]["vals"], rec["bins"]["ranges"], cam,
                         dimage, bg, tile)
        rec["g2d"] = g2d
        dg = project_bwd(rec["gs"], cam, rec["proj"]["ntiles"], g2d)
        rec["dgauss"] = dg
        if scene["kind"] == "plain":
            d = plain_activate_bwd(scene, dg)
            for k in acc:
                acc[k] += d[k]
        else:
            decode_bwd(scene, cam["partition"], cam, dg, acc)
    return acc


def step(scene: dict, tile=TILE, bg=(0.0, 0.0, 0.0)):
    fwd = forward(scene, tile=tile, bg=bg)
    grads = backward(scene, fwd, tile, bg)
    return sum(r["loss"] for r in fwd), fwd, grads


def _decisions(scene: dict, views, tile, bg):
    """Forward pass of the given views recording every discrete decision it takes: the
    ReLU gates of the decode, the Jacobian clamps of the projection, each pixel's
    composited list (candidate set, depth order, skips, stop, 0.99 clamps) and the sign
    of each L1 term.  Returns the per-pixel loss terms and the decisions, per view."""
    maps, dec = [], []
    for v in views:
        cam = scene["cams"][v]
        if scene["kind"] == "plain":
            gs, relu = plain_activate(scene), None
        else:
            gs = decode(scene, cam["partition"], cam, want_relu=True)
            relu = gs.pop("relu")
        pr = project(gs, cam, tile)
        G = gs["opacity"].shape[0]
        b = bin_sort(pr["prect"], pr["ntiles"], pr["depth"], [0, G], [cam], tile)
        lists = render_lists(pr, gs, b["vals"], b["ranges"], cam, tile)
        img = render_frozen(pr, gs, lists, cam, bg)["image"]
        sign = np.sign(img - _d(scene["targets"][v]))
        _, lpx, _, _ = loss(img, scene["targets"][v], scene["ssim_weight"], sign)
        maps.append(lpx)
        dec.append(dict(relu=relu, clamp=pr["clamp"], lists=lists, sign=sign))
    return maps, dec


def _frozen_maps(scene: dict, views, dec, bg):
    """Per-pixel loss terms with every discrete decision held at `dec` (from
    _decisions): the smooth function whose derivative the analytic adjoint computes."""
    maps = []
    for v, d in zip(views, dec):
        cam = scene["cams"][v]
        if scene["kind"] == "plain":
            gs = plain_activate(scene)
        else:
            gs = decode(scene, cam["partition"], cam, relu_in=d["relu"])
        pr = project(gs, cam, clamp_in=d["clamp"])
        img = render_frozen(pr, gs, d["lists"], cam, bg)["image"]
        _, lpx, _, _ = loss(img, scene["targets"][v], scene["ssim_weight"], d["sign"])
        maps.append(lpx)
    return maps


def _same_decisions(a: list, b: list) -> dict:
    """Which kinds of decision differ between two records of _decisions."""
    out = dict(relu=False, clamp=False, lists=False, sign=False)
    for x, y in zip(a, b):
        if x["relu"] is not None and not np.array_equal(x["relu"], y["relu"]):
            out["relu"] = True
        if not np.array_equal(x["clamp"], y["clamp"]):
            out["clamp"] = True
        lx, ly = x["lists"], y["lists"]
        if not (np.array_equal(lx["offsets"], ly["offsets"]) and np.array_equal(lx["ids"], ly["ids"])
                and np.array_equal(lx["clamped"], ly["clamped"])):
            out["lists"] = True
        if not np.array_equal(x["sign"], y["sign"]):
            out["sign"] = True
    return out


def loss_maps(scene: dict, views=None, tile=TILE, bg=(0.0, 0.0, 0.0)):
    """Per-pixel loss terms of each view (they sum to the total loss), plus the record
    of every discrete decision of the forward pass (see _decisions) for flip detection."""
    views = list(range(len(scene["cams"]))) if views is None else list(views)
    return _decisions(scene, views, tile, bg)


def _perturbed(scene: dict, name: str, index, value: float) -> dict:
    work = dict(scene)
    arr = np.asarray(scene[name], np.float64).copy()
    arr[index] = value
    work[name] = arr
    return work


def _difference(mp, mm, h):
    """Sum over pixels of the per-pixel differences (exact summation: math.fsum), / 2h."""
    terms = []
    for a, b in zip(mp, mm):
        diff = (a - b).ravel()
        terms.extend(diff[diff != 0.0].tolist())
    return math.fsum(terms) / (2.0 * h)


def fd_gradient(scene: dict, name: str, index, h: float = 1e-6, views=None, tile=TILE,
                detail: bool = False):
    """Central finite difference of the total loss with respect to scene[name][index],
    differenced pixel by pixel and summed exactly (math.fsum) so that the FP64 rounding
    of two large global sums does not swamp the signal.  Returns (value, flipped): flipped
    says that some discrete decision of the forward pass (ReLU gate, Jacobian clamp, any
    pixel's composited list: candidates, order, skip of an entry anywhere in it, stop,
    0.99 clamp; or an L1 sign) differs between +h and -h, in which case the quotient
    straddles a jump or kink of the loss.  With detail, a third value names the kinds of
    decision that flipped."""
    views = list(range(len(scene["cams"]))) if views is None else list(views)
    orig = float(scene[name][index])
    mp, dp = _decisions(_perturbed(scene, name, index, orig + h), views, tile, (0.0, 0.0, 0.0))
    mm, dm = _decisions(_perturbed(scene, name, index, orig - h), views, tile, (0.0, 0.0, 0.0))
    kinds = _same_decisions(dp, dm)
    flipped = any(kinds.values())
    val = _difference(mp, mm, h)
    return (val, flipped, kinds) if detail else (val, flipped)


def fd_gradient_frozen(scene: dict, name: str, index, h: float = 1e-6, views=None, tile=TILE,
                       decisions=None):
    """Central finite difference of the total loss with every discrete decision of the
    forward pass held at its value at the unperturbed parameters (the ReLU gates, the
    Jacobian clamps, each pixel's composited list with its clamps, the L1 signs): the
    derivative of the piece of the piecewise-smooth loss on which the parameters sit,
    which is what the analytic adjoint computes.  Equal to fd_gradient where nothing
    flips; where something does, it still checks the adjoint's arithmetic.  decisions:
    the record of loss_maps(scene, views, tile) at the unperturbed parameters, if the
    caller already has it."""
    views = list(range(len(scene["cams"]))) if views is None else list(views)
    orig = float(scene[name][index])
    dec = decisions if decisions is not None else _decisions(scene, views, tile, (0.0, 0.0, 0.0))[1]
    mp = _frozen_maps(_perturbed(scene, name, index, orig + h), views, dec, (0.0, 0.0, 0.0))
    mm = _frozen_maps(_perturbed(scene, name, index, orig - h), views, dec, (0.0, 0.0, 0.0))
    return _difference(mp, mm, h)
