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
# Stage-wise the oracle is fed the kernel's own FP32 centres and conics, so the only
# difference in an alpha is the kernel's FP32 evaluation of the exponent (a few ulp of
# |exponent| <= log2(255) ~ 8, i.e. ~1.5e-6 relative) and of 2^x: the skip window is
# 1e-5 relative to the 1/255 threshold (~7x that).  The stop window: T after a hundred
# FP32 updates is within ~1e-5 relative, 1e-9 absolute at 1e-4; 1e-8 is kept.
STAGE_MARGINS = dict(alpha=1e-5 / 255.0, T=1e-8, clamp=1e-6)
# Largest flagged fraction of a view's pixels (measured: at most 0.06% with these
# windows on config 3, 0.3% on the 20k-faint-Gaussian scene) and the bound on a
# flagged pixel's error (one skip flip moves a pixel by at most about (1/255) c T).
STAGE_FLAG_MAX = 0.005
FLAGGED_ERR_MAX = 0.02
U32 = 2.0 ** -24


def stage_render(pr, gs, vals, ranges, cam, tile=(16, 16)):
    """The oracle's compositing of the GPU's splats and lists, ambiguity windows sized
    to the FP32 evaluation of alpha (STAGE_MARGINS)."""
    with oracle.margins(**STAGE_MARGINS):
        return oracle.render_fwd(pr, gs, vals, ranges, cam, tile=tile)


def check_pixels(img, T, n_contrib, ref, label, n_eval=None, mask_bits=AMB_STAGE, flag_max=STAGE_FLAG_MAX):
    """Pixels against the oracle: unflagged within 1e-4 (and the contributor and visit
    counts exact), the flagged fraction below flag_max and flagged pixels within
    FLAGGED_ERR_MAX.  Returns the flagged fraction (printed)."""
    flag = (ref["amb"] & mask_bits) != 0
    err = np.abs(img - ref["image"])
    frac = float(flag.mean())
    print(f"{label}: {flag.sum()} flagged pixels ({frac:.2e}), largest error unflagged "
          f"{err[:, ~flag].max() if (~flag).any() else 0:.2e}, flagged {err[:, flag].max() if flag.any() else 0:.2e}",
          flush=True)
    assert frac <= flag_max, (label, frac)
    ok = ~flag
    assert err[:, ok].max() <= 1e-4, (label, err[:, ok].max())
    if flag.any():
        assert err[:, flag].max() <= FLAGGED_ERR_MAX, (label, err[:, flag].max())
    if T is not None:
        assert np.abs(T - ref["T_final"])[ok].max() <= 1e-4
    if n_contrib is not None:
        assert np.array_equal(n_contrib[ok], ref["n_contrib"][ok]), label
    if n_eval is not None:
        assert np.array_equal(n_eval[ok], ref["n_eval"][ok]), label
    return frac


def run(scene, steps=1, tile=16, tuning=None, **kw):
    pipe = Pipeline(scene, device="cuda", tile=tile, tuning=tuning, **kw)
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


def grad_close(g, ref, rel=1e-3, floor=1e-6, norm_rel=1e-3, name="", mag=None, gamma=None):
    """Per element |g - ref| <= rel |ref| + floor max|ref| (the gradient bar: 1e-3
    relative with a floor of 1e-6 of the tensor's largest element for near-zero sums),
    and relative L2 error <= norm_rel.  With mag (the sum of the magnitudes of the terms
    each element is formed from) an element may instead lie within gamma u mag,
    u = 2^-24: the rounding bound of an FP32 evaluation of that sum, for elements that
    are small differences of large terms; how many need it is printed."""
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
    if mag is not None and bad.any():
        mag = np.asarray(mag, np.float64)
        # a sum is no larger than the sum of its terms' magnitudes
        assert (np.abs(ref) <= mag * (1 + 1e-9) + 1e-300).all(), f"{name}: magnitude below the value"
        within = err <= gamma * U32 * mag
        print(f"{name}: {int(bad.sum())} of {bad.size} elements within the rounding bound only "
              f"(largest error / bound {float(np.max(err[bad] / np.maximum(gamma * U32 * mag[bad], 1e-300))):.3f})",
              flush=True)
        bad &= ~within
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} elements off; worst "
                           f"{err[bad].max():.3e} at ref {ref[bad][np.argmax(err[bad])]:.3e} (max|ref| {scale:.3e})")
    nr = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)
    assert nr <= norm_rel, f"{name}: relative L2 error {nr:.3e}"


# End to end the oracle's own decode and projection in FP64 are compared: centres
# differ by ~1e-4 px, so alphas near 1/255 by ~1e-6 absolute (the default windows), and
# FP32 depths (relative error ~3e-7) cannot order entries closer than ~1e-6 relative.
# Depth near-ties are frequent on long lists: with ~300 entries taking part per pixel over
# tens of metres, about one pixel in twenty has a pair closer than 1e-6 of its depth.
# Those pixels are checked against the oracle composited in the GPU's order (a valid
# order for such a pair), where only the threshold and stop windows remain.  Each
# evaluated entry has about the same small chance of an alpha inside the 1/255 window,
# so the flagged fraction grows with the evaluations per pixel: measured 1.3e-5 per
# evaluation on the 20k-faint-Gaussian scene (1,900 evaluations per pixel, 2.4% of its
# pixels), under 1% on the anchor scenes; the bound is the larger of 1% and 2e-5 per
# mean evaluation.
E2E_ORDER_FLAG_MAX = 0.01
E2E_ORDER_FLAG_PER_EVAL = 2e-5
E2E_DEPTH_FLAG_MAX = 0.12


def check_e2e_pixels(img, rec, h, sl, cam, label, tile=(16, 16), depth_max=E2E_DEPTH_FLAG_MAX):
    """A view's GPU image end to end: against the oracle's own render off every flagged
    pixel, and against the oracle's FP64 splats composited along the GPU's sorted lists
    off threshold and stop ambiguities only."""
    flag = (rec["amb"] & AMB_VALUE) != 0
    err = np.abs(img - rec["image"])
    depth_frac = float(((rec["amb"] & oracle.AMB_DEPTH) != 0).mean())
    assert err[:, ~flag].max() <= 1e-4, (label, err[:, ~flag].max())
    assert depth_frac <= depth_max, (label, depth_frac)
    vals = h["vals"].astype(np.int64) - sl["g0"]
    ranges = h["ranges"][sl["t0"]:sl["t0"] + sl["nt"]]
    gpu_order = oracle.render_fwd(rec["proj"], rec["gs"], vals, ranges, cam, tile=tile)
    oflag = (gpu_order["amb"] & AMB_STAGE) != 0
    oerr = np.abs(img - gpu_order["image"])
    ofrac = float(oflag.mean())
    order_max = max(E2E_ORDER_FLAG_MAX, E2E_ORDER_FLAG_PER_EVAL * float(rec["n_eval"].mean()))
    print(f"{label}: end to end, {flag.mean():.2e} of pixels flagged ({depth_frac:.2e} depth near-ties); in the "
          f"GPU's order {ofrac:.2e} flagged, largest error unflagged {oerr[:, ~oflag].max():.2e}, flagged "
          f"{oerr[:, oflag].max() if oflag.any() else 0:.2e} (flagged bound {order_max:.2e})", flush=True)
    assert ofrac <= order_max, (label, ofrac, order_max)
    assert oerr[:, ~oflag].max() <= 1e-4, (label, oerr[:, ~oflag].max())
    if oflag.any():
        assert oerr[:, oflag].max() <= FLAGGED_ERR_MAX, (label, oerr[:, oflag].max())


def _mlp_layers(flat, F, K, hidden):
    out, o = [], 0
    for n_out in (K, 3 * K, 7 * K):
        W1 = flat[o:o + hidden * (F + 4)].reshape(hidden, F + 4); o += hidden * (F + 4)
        b1 = flat[o:o + hidden]; o += hidden
        W2 = flat[o:o + n_out * hidden].reshape(n_out, hidden); o += n_out * hidden
        b2 = flat[o:o + n_out]; o += n_out
        out.append((W1, b1, W2, b2))
    return out


# Longest chain of FP32 roundings behind a decoded value: layer 1 sums 36 terms, layer
# 2 sums 32, the activation and its own rounding a few more.
DECODE_GAMMA = 36 + 32 + 8


def decode_magnitude(scene, v):
    """Per decoded output of view v (layout of oracle.decode), the scale M of its
    rounding error: an FP32 evaluation lies within DECODE_GAMMA u M of the exact value.
    M carries the sums of the magnitudes of the MLP's terms (|W1| |z| + |b1| through the
    ReLU, then |W2| and |b2|) through each activation's derivative, plus the value's own
    magnitude (its last rounding and the activation function's error)."""
    cam = scene["cams"][v]
    m = cam["partition"]
    F, K, hid = scene["F"], scene["K"], scene["hidden"]
    a0, a1 = int(scene["part_begin"][m]), int(scene["part_begin"][m + 1])
    A = a1 - a0
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    c = -R.T @ np.asarray(cam["t"], np.float64)
    d = scene["pos"][:, a0:a1].astype(np.float64).T - c
    dist = np.linalg.norm(d, axis=1, keepdims=True)
    Z = np.concatenate([scene["feat"][a0:a1].astype(np.float64), d / dist, dist], axis=1)
    es = np.exp(scene["log_scale"][a0:a1].astype(np.float64))[:, None]
    ys, ms = [], []
    for W1, b1, W2, b2 in _mlp_layers(scene["mlp"][m].astype(np.float64), F, K, hid):
        pre = Z @ W1.T + b1
        mask = pre > 0
        Hm = (np.abs(Z) @ np.abs(W1).T + np.abs(b1)) * mask
        ys.append((pre * mask) @ W2.T + b2)
        ms.append(Hm @ np.abs(W2).T + np.abs(b2))
    yo, mo = ys[0], ms[0]
    if scene["opacity_mode"] == "sigmoid":
        sg = 1 / (1 + np.exp(-yo))
        m_op = sg * (1 - sg) * mo + sg
    else:
        th = np.tanh(yo)
        m_op = (1 - th * th) * mo + np.abs(th)
    yc, mc = ys[1].reshape(A, K, 3), ms[1].reshape(A, K, 3)
    sg = 1 / (1 + np.exp(-yc))
    m_rgb = sg * (1 - sg) * mc + sg
    yv, mv = ys[2].reshape(A, K, 7), ms[2].reshape(A, K, 7)
    sg = 1 / (1 + np.exp(-yv[..., :3]))
    m_scale = es[..., None] * (sg * (1 - sg) * mv[..., :3] + 2 * sg)
    q = yv[..., 3:]
    nr = np.linalg.norm(q, axis=-1, keepdims=True)
    qh = np.abs(q) / nr
    m_quat = (mv[..., 3:] + qh * np.sum(qh * mv[..., 3:], axis=-1, keepdims=True)) / nr + qh
    offs = np.abs(scene["offs"][:, a0 * K:a1 * K].astype(np.float64)).reshape(3, A, K)
    m_mean = np.abs(scene["pos"][:, a0:a1].astype(np.float64))[:, :, None] + 2 * es[None, :, :] * offs
    G = A * K
    return {"opacity": m_op.reshape(G), "rgb": m_rgb.transpose(2, 0, 1).reshape(3, G),
            "scale": m_scale.transpose(2, 0, 1).reshape(3, G), "quat": m_quat.transpose(2, 0, 1).reshape(4, G),
            "mean": m_mean.reshape(3, G)}


def projection_bounds(gs, cam, ref):
    """Per visible view-Gaussian, the scale of the FP32 rounding error of its projected
    centre and conic, from the FP64 quantities of the oracle's projection `ref` of the
    Gaussians gs (oracle layout).
    Centre: u = fx tx / tz + cx with t = R mu + t_cw; the sums behind tx and tz carry
    |R| |mu| + |t_cw|, so u's error scale is fx (that of tx + |tx / tz| that of tz) / tz
    + |u|.  Conic: (c, -b, a) / (a c - b^2): its relative error scale is the condition
    of the determinant, (a c + b^2) / (a c - b^2), times the depth of the product chain
    behind a, b, c.  Returns (uv_scale [2][G], conic_rel_scale [G])."""
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    mu = np.asarray(gs["mean"], np.float64)
    mag = np.abs(R) @ np.abs(mu) + np.abs(t)[:, None]
    tz = np.where(ref["depth"] > 0.2, ref["depth"], 1.0)
    tx, ty = R[0] @ mu + t[0], R[1] @ mu + t[1]
    su = cam["fx"] * (mag[0] + np.abs(tx / tz) * mag[2]) / tz + np.abs(ref["uv"][0])
    sv = cam["fy"] * (mag[1] + np.abs(ty / tz) * mag[2]) / tz + np.abs(ref["uv"][1])
    a, b, c = ref["cov2d"]
    det = a * c - b * b
    kappa = np.where(det > 0, (a * c + b * b) / np.where(det > 0, det, 1.0), 1.0)
    return np.stack([su, sv]), kappa


def _mlp_dy_magnitude(i, y, ym, g, es, A, K, opacity_mode):
    """Magnitude of the decode adjoint's incoming output gradients dY of MLP i (the
    activation adjoints), each carrying the forward output's own error scale ym through
    the activation's second derivative."""
    if i == 0:
        dop = np.abs(g["opacity"].reshape(A, K))
        if opacity_mode == "sigmoid":
            sg = 1 / (1 + np.exp(-y))
            return dop * sg * (1 - sg) * (1 + np.abs(1 - 2 * sg) * ym)
        al = np.tanh(y)
        return np.where(al > 0, dop * (1 - al * al) * (1 + 2 * np.abs(al) * ym), 0.0)
    if i == 1:
        pg = np.abs(g["rgb"].reshape(3, A, K).transpose(1, 2, 0).reshape(A, 3 * K))
        sg = 1 / (1 + np.exp(-y))
        return pg * sg * (1 - sg) * (1 + np.abs(1 - 2 * sg) * ym)
    yk, ymk = y.reshape(A, K, 7), ym.reshape(A, K, 7)
    mYk = np.zeros((A, K, 7))
    dsc = np.abs(g["scale"].reshape(3, A, K).transpose(1, 2, 0))
    sg = 1 / (1 + np.exp(-yk[..., :3]))
    mYk[..., :3] = dsc * es[..., None] * sg * (1 - sg) * (1 + np.abs(1 - 2 * sg) * ymk[..., :3])
    q = yk[..., 3:]
    nr = np.linalg.norm(q, axis=-1, keepdims=True)
    qh = np.abs(q / nr)
    pq = np.abs(g["quat"].reshape(4, A, K).transpose(1, 2, 0))
    mYk[..., 3:] = ((pq + qh * np.sum(qh * pq, axis=-1, keepdims=True)) / nr
                    + 3 * np.linalg.norm(pq, axis=-1, keepdims=True)
                    * np.linalg.norm(ymk[..., 3:], axis=-1, keepdims=True) / nr ** 2)
    return mYk.reshape(A, 7 * K)


def decode_grad_magnitude(scene, v, dg):
    """For the anchors of view v's partition: per element of the decode adjoint's
    outputs (features [A][F], log-scales [A], offsets [3][A K], the partition's packed MLP
    gradients [P]), the sum of the magnitudes of the terms this view contributes to it,
    forward values included (each decoded output's own error scale carried through the
    derivative of its activation).  An FP32 evaluation is within a small multiple of
    2^-24 times this of the exact value.  dg: this view's incoming Gaussian gradients
    ([3][G], [4][G], [G], ...).  Returns (partition, a0, a1, dict)."""
    cam = scene["cams"][v]
    m = cam["partition"]
    F, K, hid = scene["F"], scene["K"], scene["hidden"]
    a0, a1 = int(scene["part_begin"][m]), int(scene["part_begin"][m + 1])
    A = a1 - a0
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    c = -R.T @ np.asarray(cam["t"], np.float64)
    d = scene["pos"][:, a0:a1].astype(np.float64).T - c
    dist = np.linalg.norm(d, axis=1, keepdims=True)
    Z = np.concatenate([scene["feat"][a0:a1].astype(np.float64), d / dist, dist], axis=1)
    es = np.exp(scene["log_scale"][a0:a1].astype(np.float64))[:, None]
    g = {k: np.asarray(x, np.float64) for k, x in dg.items()}
    feat = np.zeros((A, F))
    mlp = []
    for i, (W1, b1, W2, b2) in enumerate(_mlp_layers(scene["mlp"][m].astype(np.float64), F, K, hid)):
        pre = Z @ W1.T + b1
        mask = pre > 0
        Hm = (np.abs(Z) @ np.abs(W1).T + np.abs(b1)) * mask
        y = (pre * mask) @ W2.T + b2
        ym = Hm @ np.abs(W2).T + np.abs(b2)
        mY = _mlp_dy_magnitude(i, y, ym, g, es, A, K, scene["opacity_mode"])
        dP = (mY @ np.abs(W2)) * mask
        feat += (dP @ np.abs(W1))[:, :F]
        mlp += [(dP.T @ np.abs(Z)).ravel(), dP.sum(0), (mY.T @ Hm).ravel(), mY.sum(0)]
    # log-scale: e^{s_a} times the scales' sigmoids and the offsets, each K times
    dsc = np.abs(g["scale"]).reshape(3, A, K)
    dmu = np.abs(g["mean"]).reshape(3, A, K)
    offs = np.abs(scene["offs"][:, a0 * K:a1 * K].astype(np.float64)).reshape(3, A, K)
    scl = np.asarray(dg.get("scale_value", np.zeros((3, A * K))), np.float64).reshape(3, A, K)
    ls = (dsc * np.abs(scl)).sum((0, 2)) + (es[:, 0][None, :, None] * offs * dmu).sum((0, 2))
    return m, a0, a1, {"feat": feat, "mlp": np.concatenate(mlp), "log_scale": ls,
                       "offs": (es[:, 0][None, :, None] * dmu).reshape(3, A * K)}


def decode_grads_magnitude(scene, dgs, scales=None):
    """decode_grad_magnitude summed over the views whose incoming Gaussian gradients are
    given (dgs: view -> dg), in the layout of oracle.zero_grads(scene).  scales: view ->
    the decoded scales of that view ([3][G]), for the log-scale term."""
    acc = {k: np.zeros_like(x) for k, x in zip(("feat", "offs", "log_scale", "mlp"),
                                                (np.zeros((scene["feat"].shape[0], scene["F"])),
                                                 np.zeros((3, scene["feat"].shape[0] * scene["K"])),
                                                 np.zeros(scene["feat"].shape[0]), np.zeros(scene["mlp"].shape)))}
    K = scene["K"]
    for v, dg in dgs.items():
        dgv = dict(dg)
        if scales is not None:
            dgv["scale_value"] = scales[v]
        m, a0, a1, mg = decode_grad_magnitude(scene, v, dgv)
        acc["feat"][a0:a1] += mg["feat"]
        acc["log_scale"][a0:a1] += mg["log_scale"]
        acc["offs"][:, a0 * K:a1 * K] += mg["offs"]
        acc["mlp"][m] += mg["mlp"]
    return acc


def project_bwd_magnitude(gs, cam, ntiles, g2d):
    """Per view-Gaussian, the magnitudes of the terms the projection adjoint forms each
    of d(mean[3], scale[3], quat[4], opacity, rgb[3]) from, for the 2-D gradients g2d
    [9][G] (every factor by its absolute value; the factors that divide by the 2-D
    covariance's determinant a c - b^2 carry its condition (a c + b^2) / (a c - b^2),
    the relative error of that determinant in units of the rounding unit)."""
    G = gs["opacity"].shape[0]
    mu = np.asarray(gs["mean"], np.float64)
    s = np.asarray(gs["scale"], np.float64)
    q = np.asarray(gs["quat"], np.float64)
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = R @ mu + np.asarray(cam["t"], np.float64)[:, None]
    tx, ty, tz = t
    vis = (ntiles > 0) & (tz > 0.2)
    tz = np.where(vis, tz, 1.0)
    fx, fy, cx, cy, W, H = cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["W"], cam["H"]
    lxl, lxh = (-cx - 0.15 * W) / fx, (1.15 * W - cx) / fx
    lyl, lyh = (-cy - 0.15 * H) / fy, (1.15 * H - cy) / fy
    xt = np.clip(tx / tz, lxl, lxh) * tz
    yt = np.clip(ty / tz, lyl, lyh) * tz
    J = np.zeros((G, 2, 3))
    J[:, 0, 0], J[:, 0, 2] = fx / tz, -fx * xt / tz ** 2
    J[:, 1, 1], J[:, 1, 2] = fy / tz, -fy * yt / tz ** 2
    w, x, y, z = q
    Rq = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                   2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1).reshape(G, 3, 3)
    N = Rq * s.T[:, None, :]
    Sig = N @ N.transpose(0, 2, 1)
    M = J @ R
    S2 = M @ Sig @ M.transpose(0, 2, 1)
    a, b, c = S2[:, 0, 0] + 0.3, 0.5 * (S2[:, 0, 1] + S2[:, 1, 0]), S2[:, 1, 1] + 0.3
    det = a * c - b * b
    det = np.where(det > 0, det, 1.0)
    kap = 1 + 2 * (a * c + b * b) / det
    g = np.abs(np.asarray(g2d, np.float64))
    d2 = det * det
    da = kap * (g[2] * c * c + g[3] * np.abs(b) * c + g[4] * b * b) / d2
    db = kap * (g[2] * 2 * np.abs(b) * c + g[3] * (a * c + b * b) + g[4] * 2 * a * np.abs(b)) / d2
    dc = kap * (g[2] * b * b + g[3] * a * np.abs(b) + g[4] * a * a) / d2
    G2 = np.stack([np.stack([da, 0.5 * db], -1), np.stack([0.5 * db, dc], -1)], -2)
    aM, aSig, aR, aN, aRq = np.abs(M), np.abs(Sig), np.abs(R), np.abs(N), np.abs(Rq)
    dSig = aM.transpose(0, 2, 1) @ G2 @ aM
    dM = 2 * G2 @ aM @ aSig
    dJ = dM @ aR.T
    dt0 = g[0] * fx / tz + dJ[:, 0, 2] * fx / tz ** 2
    dt1 = g[1] * fy / tz + dJ[:, 1, 2] * fy / tz ** 2
    dt2 = ((g[0] * fx * np.abs(tx) + g[1] * fy * np.abs(ty)) / tz ** 2 + (dJ[:, 0, 0] * fx + dJ[:, 1, 1] * fy) / tz ** 2
           + 2 * (dJ[:, 0, 2] * fx * np.abs(xt) + dJ[:, 1, 2] * fy * np.abs(yt)) / tz ** 3
           + (dJ[:, 0, 2] * fx * np.abs(xt) + dJ[:, 1, 2] * fy * np.abs(yt)) / tz ** 3)
    dt = np.stack([dt0, dt1, dt2])
    dmean = aR.T @ dt
    dN = 2 * dSig @ aN
    dscale = (dN * aRq).sum(1).T
    dRq = (dN * s.T[:, None, :]).reshape(G, 9)
    aw, ax, ay, az = np.abs(q)
    d_ = dRq.T
    dq = 2 * np.stack([
        az * d_[1] + ay * d_[2] + az * d_[3] + ax * d_[5] + ay * d_[6] + ax * d_[7],
        ay * d_[1] + az * d_[2] + ay * d_[3] + 2 * ax * d_[4] + aw * d_[5] + az * d_[6] + aw * d_[7] + 2 * ax * d_[8],
        2 * ay * d_[0] + ax * d_[1] + aw * d_[2] + ax * d_[3] + az * d_[5] + aw * d_[6] + az * d_[7] + 2 * ay * d_[8],
        2 * az * d_[0] + aw * d_[1] + ax * d_[2] + aw * d_[3] + 2 * az * d_[4] + ay * d_[5] + ax * d_[6] + ay * d_[7]])
    out = {"mean": dmean, "scale": dscale, "quat": dq, "opacity": g[5], "rgb": g[6:9]}
    for k in ("mean", "scale", "quat"):
        out[k] = np.where(vis[None, :], out[k], 0.0)
    return out


# Rounding allowances, in units of u = 2^-24 times an element's magnitude M (the sum of
# the magnitudes of the terms it is formed from), for elements that are small
# differences of large terms: stage-wise the kernels evaluate the same sums as the
# oracle in another order, a few roundings per term (gamma 16); end to end every term
# also carries the FP32 forward pass's relative differences (centres ~1e-7 relative,
# alphas near the footprint edge ~1e-5), gamma 256 (1.5e-5 relative to M).
GAMMA_STAGE = 16
GAMMA_E2E = 256


def check_dgauss(got_dg, dgp, gin, cam, ntiles, g2d, label):
    """Projection adjoint stage-wise: the GPU's Gaussian gradients (fed its own 2-D
    gradients g2d [9][G]) against the oracle's dgp."""
    mag = project_bwd_magnitude(gin, cam, ntiles, g2d)
    for k in ("mean", "scale", "quat", "opacity", "rgb"):
        grad_close(got_dg[k], dgp[k], name=f"{label} dgauss {k}", mag=mag[k], gamma=GAMMA_STAGE)


def check_anchor_grads(got, ref, scene, dgs, scales, label, gamma=GAMMA_STAGE):
    """Decode adjoint: the GPU's anchor and MLP gradients against the oracle's, the
    rounding allowance from the magnitudes of the views' terms (dgs: view -> the Gaussian
    gradients fed to the decode adjoint; scales: view -> decoded scales)."""
    mag = decode_grads_magnitude(scene, dgs, scales)
    for k in ref:
        grad_close(got[k], ref[k], name=f"{label} d{k}", mag=mag[k], gamma=gamma)


def e2e_grad_magnitude(scene, fwd, dims):
    """End to end: per anchor and MLP gradient element the magnitudes of the per-pixel
    terms it is formed from, carried through the whole adjoint chain (compositing, then
    projection, then decode)."""
    dgs, scales = {}, {}
    for r, d in zip(fwd, dims):
        v = r["view"]
        cam = scene["cams"][v]
        g2m = oracle.render_bwd_magnitude(r["proj"], r["gs"], r["bins"]["vals"], r["bins"]["ranges"], cam, d)
        dgs[v] = project_bwd_magnitude(r["gs"], cam, r["proj"]["ntiles"], g2m)
        scales[v] = r["gs"]["scale"]
    return decode_grads_magnitude(scene, dgs, scales)
