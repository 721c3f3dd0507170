"""ctypes binding of libglam.so: the C ABI of include/glam.h, same names, argument
marshalling only.  Every computation happens in the HIP kernels behind these calls.

Loading fails loudly (ImportError) when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglam.so")

GLAM_OK, GLAM_ERR_INVALID_ARG, GLAM_ERR_WORKSPACE, GLAM_ERR_CAPACITY, GLAM_ERR_HIP, GLAM_ERR_UNSUPPORTED = range(6)
GLAM_PLAIN = 1
GLAM_OPACITY_SIGMOID = 2
GLAM_FOOTPRINT_3SIGMA = 4
GLAM_DETERMINISTIC_GRADS = 8
GLAM_RETURN_INTERMEDIATES = 16
GLAM_QUEUE_WORDS = 1088

EXPORTS = [
    "glam_status_string", "glam_mlp_param_count", "glam_views_build", "glam_bin_sort_workspace_bytes",
    "glam_render_fused_l1_workspace_bytes", "glam_render_fused_l1",
    "glam_decode", "glam_project", "glam_bin_sort", "glam_render_fwd", "glam_loss_workspace_bytes", "glam_loss",
    "glam_composite_bwd", "glam_project_bwd", "glam_decode_bwd_workspace_bytes", "glam_decode_bwd",
    "glam_render_bwd", "glam_adam_step", "glam_sample_keyframes", "glam_deform_anchors",
    "glam_epipolar_triangulate", "glam_voxelize_workspace_bytes", "glam_voxelize",
    "glam_insert_rows", "glam_decode_project", "glam_render_bwd_workspace_bytes", "glam_loss_noalloc",
]
GLAM_LOSS_SCRATCH_BYTES = 16 << 20
GLAM_ADAM_MAX_GROUPS = 16


class GlamError(RuntimeError):
    def __init__(self, call, status):
        super().__init__(f"{call} failed: {status_string(status)} ({status})")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("partition", C.c_int32), ("reserved", C.c_int32)]


class ViewInfo(C.Structure):
    _fields_ = [("cam", Camera), ("g_begin", C.c_int64), ("g_count", C.c_int64), ("pix_begin", C.c_int64),
                ("tile_begin", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("anchor_begin", C.c_int32), ("anchor_count", C.c_int32), ("reserved", C.c_int32)]


class Views(C.Structure):
    _fields_ = [("host", C.c_void_p), ("dev", C.c_void_p), ("n", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("reserved", C.c_int32), ("n_gauss", C.c_int64), ("n_pix", C.c_int64),
                ("n_tiles", C.c_int64)]


class Anchors(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("feat", C.c_void_p), ("log_scale", C.c_void_p), ("offs", C.c_void_p),
                ("A", C.c_int32), ("F", C.c_int32), ("K", C.c_int32), ("hidden", C.c_int32)]


class Gaussians(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("rgb", C.c_void_p), ("n", C.c_int64)]


class Projected(C.Structure):
    _fields_ = [("uv", C.c_void_p), ("conic", C.c_void_p), ("depth", C.c_void_p), ("ext", C.c_void_p),
                ("ntiles", C.c_void_p), ("splat", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("long_log2", C.c_int32), ("fwd_blocks_per_cu", C.c_int32), ("bwd_blocks_per_cu", C.c_int32),
                ("fwd_group_waves", C.c_int32), ("bwd_group_waves", C.c_int32), ("non_persistent", C.c_int32),
                ("reserved", C.c_int32 * 2)]


SCHEDULE_KEYS = ("long_log2", "fwd_blocks_per_cu", "bwd_blocks_per_cu", "fwd_group_waves", "bwd_group_waves",
                 "non_persistent")


def make_tuning(schedule: dict | None) -> Tuning:
    """glam_tuning from a schedule dict (missing keys: 0, the built-in default)."""
    return Tuning(*(int((schedule or {}).get(k, 0)) for k in SCHEDULE_KEYS))


class Bins(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("vals", C.c_void_p), ("ranges", C.c_void_p), ("capacity", C.c_int64),
                ("status", C.c_void_p), ("order", C.c_void_p), ("queue", C.c_void_p), ("tuning", Tuning),
                ("pair_begin", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("g2d", C.c_void_p), ("dgauss", Gaussians), ("dfeat", C.c_void_p), ("doffs", C.c_void_p),
                ("dlog_scale", C.c_void_p), ("dmlp", C.c_void_p), ("d2d", C.c_void_p)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("period", C.c_int32), ("n_seg", C.c_int32), ("seg_end", C.c_int32 * 4),
                ("lr", C.c_float * 4)]


class KeyframeFix(C.Structure):
    _fields_ = [("before", Camera), ("R_new", C.c_float * 9), ("t_new", C.c_float * 3)]


_lib = None


def load():
    """Loads libglam.so; raises ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                          "python paper_2607_21416_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, SZ, F32, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_float, C.c_uint32
    sig = {
        "glam_status_string": (C.c_char_p, [I32]),
        "glam_mlp_param_count": (I32, [I32, I32, I32]),
        "glam_views_build": (I32, [P, I32, P, I32, I32, I64, I32, I32, P, P]),
        "glam_bin_sort_workspace_bytes": (SZ, [P, I64]),
        "glam_decode": (I32, [P, P, I32, P, U32, P, P]),
        "glam_project": (I32, [P, P, U32, P, P]),
        "glam_bin_sort": (I32, [P, P, P, P, SZ, P]),
        "glam_render_fwd": (I32, [P, P, P, P, P, P, P, P, P]),
        "glam_loss_workspace_bytes": (SZ, [P]),
        "glam_loss": (I32, [P, P, P, F32, P, P, P, P, SZ, P]),
        "glam_composite_bwd": (I32, [P, P, P, P, P, P, P, P, P]),
        "glam_render_fused_l1_workspace_bytes": (SZ, [P]),
        "glam_render_fused_l1": (I32, [P, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P]),
        "glam_project_bwd": (I32, [P, P, P, U32, P, P, P]),
        "glam_decode_bwd_workspace_bytes": (SZ, [P, P, I32]),
        "glam_decode_bwd": (I32, [P, P, I32, P, U32, P, P, P, P, P, P, SZ, P]),
        "glam_render_bwd": (I32, [P, P, P, P, P, P, P, P, P, P, I32, U32, P, P, SZ, P]),
        "glam_adam_step": (I32, [P, I32, I32, F32, F32, F32, P]),
        "glam_sample_keyframes": (I32, [I32, I32, F32, I32, C.c_uint64, C.c_uint64, P]),
        "glam_deform_anchors": (I32, [P, P, I32, I32, P, I32, F32, F32, P, P]),
        "glam_epipolar_triangulate": (I32, [P, P, P, P, I64, F32, P, P, P, P]),
        "glam_voxelize_workspace_bytes": (SZ, [I64]),
        "glam_voxelize": (I32, [P, I64, F32, P, I64, P, P, I64, P, P, P, SZ, P]),
        "glam_insert_rows": (I32, [P, P, I32, I64, I32, I64, I64, P, I64, F32, P]),
        "glam_decode_project": (I32, [P, P, I32, P, U32, P, P, P]),
        "glam_render_bwd_workspace_bytes": (SZ, [P, P, I32, I64, U32]),
        "glam_loss_noalloc": (I32, [P, P, P, F32, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().glam_status_string(int(s)).decode()


def _check(name, status):
    if status != GLAM_OK:
        raise GlamError(name, status)
    return status


def ref(x):
    """Pointer argument: a ctypes structure (by reference), a torch tensor (its data
    pointer), a numpy array, an int address or None."""
    if x is None:
        return None
    if isinstance(x, C.c_void_p):
        return x
    if isinstance(x, (C.Structure, C.Array)):
        return C.cast(C.byref(x), C.c_void_p)
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return C.c_void_p(x.ctypes.data)
    return C.c_void_p(int(x))


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return C.c_void_p(s.cuda_stream)
    return C.c_void_p(int(s))


# ----------------------------------------------------------------------------------
# The ABI, one function per exported symbol
# ----------------------------------------------------------------------------------

def glam_mlp_param_count(F, K, hidden=32):
    return load().glam_mlp_param_count(F, K, hidden)


def glam_views_build(cams, n_views, part_begin, n_parts, K, plain_G, tile_w, tile_h, info, views):
    return _check("glam_views_build", load().glam_views_build(ref(cams), n_views, ref(part_begin), n_parts, K,
                                                              plain_G, tile_w, tile_h, ref(info), ref(views)))


def glam_bin_sort_workspace_bytes(views, capacity):
    return load().glam_bin_sort_workspace_bytes(ref(views), capacity)


def glam_decode(anchors, mlp, n_parts, views, flags, out, stream):
    return _check("glam_decode", load().glam_decode(ref(anchors), ref(mlp), n_parts, ref(views), flags, ref(out),
                                                    _stream(stream)))


def glam_project(gauss, views, flags, out, stream):
    return _check("glam_project", load().glam_project(ref(gauss), ref(views), flags, ref(out), _stream(stream)))


def glam_bin_sort(proj, views, bins, ws, ws_bytes, stream):
    return _check("glam_bin_sort", load().glam_bin_sort(ref(proj), ref(views), ref(bins), ref(ws), ws_bytes,
                                                        _stream(stream)))


def glam_render_fwd(proj, bins, views, bg, image, T_final, n_contrib, n_eval, stream):
    return _check("glam_render_fwd", load().glam_render_fwd(ref(proj), ref(bins), ref(views), ref(bg), ref(image),
                                                            ref(T_final), ref(n_contrib), ref(n_eval),
                                                            _stream(stream)))


def glam_loss_workspace_bytes(views):
    return load().glam_loss_workspace_bytes(ref(views))


def glam_loss(views, image, target, w_ssim, dimage, loss, total, ws, ws_bytes, stream):
    return _check("glam_loss", load().glam_loss(ref(views), ref(image), ref(target), float(w_ssim), ref(dimage),
                                                ref(loss), ref(total), ref(ws), ws_bytes, _stream(stream)))


def glam_loss_noalloc(views, image, target, w_ssim, dimage, loss, total, stream):
    return _check("glam_loss_noalloc", load().glam_loss_noalloc(ref(views), ref(image), ref(target), float(w_ssim),
                                                                ref(dimage), ref(loss), ref(total), _stream(stream)))


def glam_composite_bwd(proj, bins, views, bg, T_final, n_contrib, dimage, g2d, stream):
    return _check("glam_composite_bwd",
                  load().glam_composite_bwd(ref(proj), ref(bins), ref(views), ref(bg), ref(T_final), ref(n_contrib),
                                            ref(dimage), ref(g2d), _stream(stream)))


def glam_render_fused_l1_workspace_bytes(views):
    return load().glam_render_fused_l1_workspace_bytes(ref(views))


def glam_render_fused_l1(proj, bins, views, bg, target, image, T_final, n_contrib, dimage, loss, total, g2d, ws,
                         ws_bytes, stream):
    return _check("glam_render_fused_l1",
                  load().glam_render_fused_l1(ref(proj), ref(bins), ref(views), ref(bg), ref(target), ref(image),
                                              ref(T_final), ref(n_contrib), ref(dimage), ref(loss), ref(total),
                                              ref(g2d), ref(ws), ws_bytes, _stream(stream)))


def glam_project_bwd(gauss, proj, views, flags, g2d, dgauss, stream):
    return _check("glam_project_bwd", load().glam_project_bwd(ref(gauss), ref(proj), ref(views), flags, ref(g2d),
                                                              ref(dgauss), _stream(stream)))


def glam_decode_bwd_workspace_bytes(anchors, views, n_parts):
    return load().glam_decode_bwd_workspace_bytes(ref(anchors), ref(views), n_parts)


def glam_decode_bwd(anchors, mlp, n_parts, views, flags, dgauss, dfeat, doffs, dlog_scale, dmlp, ws, ws_bytes,
                    stream):
    return _check("glam_decode_bwd",
                  load().glam_decode_bwd(ref(anchors), ref(mlp), n_parts, ref(views), flags, ref(dgauss), ref(dfeat),
                                         ref(doffs), ref(dlog_scale), ref(dmlp), ref(ws), ws_bytes,
                                         _stream(stream)))


def glam_render_bwd_workspace_bytes(anchors, views, n_parts, capacity, flags):
    return load().glam_render_bwd_workspace_bytes(ref(anchors), ref(views), n_parts, capacity, flags)


def glam_render_bwd(proj, bins, views, bg, T_final, n_contrib, dimage, gauss, anchors, mlp, n_parts, flags, grads,
                    ws, ws_bytes, stream):
    return _check("glam_render_bwd",
                  load().glam_render_bwd(ref(proj), ref(bins), ref(views), ref(bg), ref(T_final), ref(n_contrib),
                                         ref(dimage), ref(gauss), ref(anchors), ref(mlp), n_parts, flags, ref(grads),
                                         ref(ws), ws_bytes, _stream(stream)))


def glam_adam_step(groups, n_groups, step, beta1, beta2, eps, stream):
    return _check("glam_adam_step", load().glam_adam_step(ref(groups), n_groups, step, float(beta1), float(beta2),
                                                          float(eps), _stream(stream)))


def glam_sample_keyframes(n_keyframes, k_recent, p_recent, count, seed, counter):
    """Returns the count sampled keyframe indices (numpy int32)."""
    out = np.zeros(max(count, 1), np.int32)
    _check("glam_sample_keyframes", load().glam_sample_keyframes(n_keyframes, k_recent, float(p_recent), count,
                                                                 C.c_uint64(seed), C.c_uint64(counter), ref(out)))
    return out[:count]


def glam_deform_anchors(pos, offs, A, K, fixes, n_fix, near, far, owner, stream):
    return _check("glam_deform_anchors", load().glam_deform_anchors(ref(pos), ref(offs), A, K, ref(fixes), n_fix,
                                                                    float(near), float(far), ref(owner),
                                                                    _stream(stream)))


def glam_epipolar_triangulate(cam1, cam2, x1, x2, n, tau, residual, keep, X, stream):
    return _check("glam_epipolar_triangulate",
                  load().glam_epipolar_triangulate(ref(cam1), ref(cam2), ref(x1), ref(x2), n, float(tau),
                                                   ref(residual), ref(keep), ref(X), _stream(stream)))


def glam_voxelize_workspace_bytes(n_points):
    return load().glam_voxelize_workspace_bytes(n_points)


def glam_voxelize(points, n_points, eps, existing, n_existing, new_keys, new_centres, capacity, merged, counts,
                  workspace, workspace_bytes, stream):
    return _check("glam_voxelize",
                  load().glam_voxelize(ref(points), n_points, float(eps), ref(existing), n_existing, ref(new_keys),
                                       ref(new_centres), capacity, ref(merged), ref(counts), ref(workspace),
                                       workspace_bytes, _stream(stream)))


def glam_insert_rows(src, dst, rows, n_old, width, at, n_new, ins, ins_stride, fill, stream):
    return _check("glam_insert_rows", load().glam_insert_rows(ref(src), ref(dst), rows, n_old, width, at, n_new,
                                                              ref(ins), ins_stride, float(fill), _stream(stream)))


def glam_decode_project(anchors, mlp, n_parts, views, flags, out, proj, stream):
    return _check("glam_decode_project", load().glam_decode_project(ref(anchors), ref(mlp), n_parts, ref(views),
                                                                    flags, ref(out), ref(proj), _stream(stream)))
