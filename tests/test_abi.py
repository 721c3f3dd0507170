"""The C ABI library on the host: it loads, exports every function include/glam.h
declares, builds view tables, and rejects bad arguments before any launch (no GPU is
touched by these tests)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import camera_array

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "glam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?(glam_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_param_count_matches_oracle():
    assert B.glam_mlp_param_count(32, 10, 32) == 7182 == oracle.mlp_param_count(32, 10, 32)
    assert B.glam_mlp_param_count(16, 4, 32) == oracle.mlp_param_count(16, 4, 32)


def _build(cams, part_begin=None, K=0, plain_G=0, tile=(16, 16)):
    arr = camera_array(cams)
    info = (B.ViewInfo * len(cams))()
    views = B.Views()
    pb = None if part_begin is None else np.ascontiguousarray(part_begin, np.int32)
    st = B.load().glam_views_build(B.ref(arr), len(cams), B.ref(pb), 0 if pb is None else len(pb) - 1, K, plain_G,
                                   tile[0], tile[1], B.ref(info), B.ref(views))
    return st, info, views


def test_views_build_tile_edges():
    cams = [synth.camera(np.eye(3), np.zeros(3), 50, 50, 10, 10, 70, 45)]
    for t, grid in ((8, (9, 6)), (16, (5, 3)), (32, (3, 2))):
        st, info, views = _build(cams, None, 0, 10, (t, t))
        assert st == B.GLAM_OK and (info[0].tiles_x, info[0].tiles_y) == grid and views.n_tiles == grid[0] * grid[1]
        assert views.tile_w == views.tile_h == t
    for t in ((12, 12), (16, 32), (64, 64), (4, 4)):
        assert _build(cams, None, 0, 10, t)[0] == B.GLAM_ERR_UNSUPPORTED


def test_schedule_out_of_range_is_rejected():
    lib = B.load()
    s = synth.plain_scene(1, 10, 32, 32)
    st, info, views = _build(s["cams"], None, 0, 10)
    fake = 0x100000
    views.host = C.cast(info, C.c_void_p)
    views.dev = fake
    proj = B.Projected(fake, fake, fake, fake, fake, fake)
    need = lib.glam_bin_sort_workspace_bytes(B.ref(views), 1000)
    bad_sched = [dict(long_log2=5), dict(long_log2=25), dict(fwd_blocks_per_cu=6), dict(bwd_blocks_per_cu=7),
                 dict(fwd_blocks_per_cu=-1), dict(fwd_group_waves=12), dict(bwd_group_waves=2),
                 dict(fwd_group_waves=16, fwd_blocks_per_cu=2), dict(bwd_group_waves=8, bwd_blocks_per_cu=3),
                 dict(fwd_group_waves=-4), dict(non_persistent=2), dict(non_persistent=-1)]
    reserved = B.make_tuning(None)
    reserved.reserved[1] = 1
    for bad in [B.make_tuning(d) for d in bad_sched] + [reserved]:
        bins = B.Bins(fake, fake, fake, 1000, fake, fake, fake, bad)
        assert lib.glam_bin_sort(B.ref(proj), B.ref(views), B.ref(bins), C.c_void_p(fake), need,
                                 None) == B.GLAM_ERR_INVALID_ARG
        assert lib.glam_render_fwd(B.ref(proj), B.ref(bins), B.ref(views), None, C.c_void_p(fake),
                                   C.c_void_p(fake), C.c_void_p(fake), None, None) == B.GLAM_ERR_INVALID_ARG


def test_views_build_offsets():
    s = synth.anchor_scene(3, [100, 50, 75], 2, W=70, H=45, fx=50)
    st, info, views = _build(s["cams"], s["part_begin"], s["K"])
    assert st == B.GLAM_OK
    g = p = t = 0
    for i, cam in enumerate(s["cams"]):
        vi = info[i]
        m = cam["partition"]
        assert vi.g_begin == g and vi.pix_begin == p and vi.tile_begin == t
        assert vi.tiles_x == 5 and vi.tiles_y == 3  # ceil(70/16), ceil(45/16): ragged edges
        assert vi.anchor_begin == s["part_begin"][m]
        assert vi.anchor_count == s["part_begin"][m + 1] - s["part_begin"][m]
        assert vi.g_count == vi.anchor_count * s["K"]
        g += vi.g_count; p += 70 * 45; t += 15
    assert (views.n, views.n_gauss, views.n_pix, views.n_tiles) == (6, g, p, t)
    st, info, views = _build(s["cams"][:2], None, 0, 123)
    assert st == B.GLAM_OK and views.n_gauss == 246 and info[1].g_begin == 123


def test_views_build_rejects_bad_input():
    cams = [synth.camera(np.eye(3), np.zeros(3), 50, 50, 10, 10, 20, 20)]
    assert _build(cams, None, 0, 0)[0] == B.GLAM_ERR_INVALID_ARG           # no Gaussians
    bad = dict(cams[0], W=0)
    assert _build([bad], None, 0, 10)[0] == B.GLAM_ERR_INVALID_ARG         # empty image
    bad = dict(cams[0], partition=3)
    assert _build([bad], [0, 5], 10)[0] == B.GLAM_ERR_INVALID_ARG         # no such partition


def test_calls_reject_before_launch():
    lib = B.load()
    s = synth.plain_scene(1, 10, 32, 32)
    st, info, views = _build(s["cams"], None, 0, 10)
    fake = 0x100000  # aligned, never dereferenced: validation fails first
    views.host = C.cast(info, C.c_void_p)
    views.dev = fake
    g = B.Gaussians(fake, fake, fake, fake, fake, 10)
    proj_null = B.Projected(fake, None, fake, fake, fake, fake)
    assert lib.glam_project(B.ref(g), B.ref(views), B.GLAM_PLAIN, B.ref(proj_null), None) == B.GLAM_ERR_INVALID_ARG
    proj = B.Projected(fake, fake, fake, fake, fake, fake + 4)  # misaligned
    assert lib.glam_project(B.ref(g), B.ref(views), B.GLAM_PLAIN, B.ref(proj), None) == B.GLAM_ERR_INVALID_ARG
    proj = B.Projected(fake, fake, fake, fake, fake, fake)
    g_wrong = B.Gaussians(fake, fake, fake, fake, fake, 11)  # plain G must match the view table
    assert lib.glam_project(B.ref(g_wrong), B.ref(views), B.GLAM_PLAIN, B.ref(proj), None) == B.GLAM_ERR_INVALID_ARG
    bins = B.Bins(fake, fake, fake, 1000, fake, fake, fake)
    need = lib.glam_bin_sort_workspace_bytes(B.ref(views), 1000)
    assert need > 12000
    assert lib.glam_bin_sort(B.ref(proj), B.ref(views), B.ref(bins), C.c_void_p(fake), need - 1,
                             None) == B.GLAM_ERR_WORKSPACE
    bins0 = B.Bins(fake, fake, fake, 0, fake, fake, fake)
    assert lib.glam_bin_sort(B.ref(proj), B.ref(views), B.ref(bins0), C.c_void_p(fake), need,
                             None) == B.GLAM_ERR_INVALID_ARG
    # anchor decode: unsupported feature width / offset count
    sa = synth.anchor_scene(2, [20], 1, W=32, H=32, fx=30, F=8, K=3)
    st, info2, views2 = _build(sa["cams"], sa["part_begin"], 3)
    views2.host = C.cast(info2, C.c_void_p)
    views2.dev = fake
    an = B.Anchors(fake, fake, fake, fake, 20, 8, 3, 32)
    out = B.Gaussians(fake, fake, fake, fake, fake, views2.n_gauss)
    assert lib.glam_decode(B.ref(an), C.c_void_p(fake), 1, B.ref(views2), 0, B.ref(out), None) == B.GLAM_ERR_UNSUPPORTED
    an_bad = B.Anchors(fake, fake, fake, fake, 20, 8, 3, 16)  # hidden width other than 32
    assert lib.glam_decode(B.ref(an_bad), C.c_void_p(fake), 1, B.ref(views2), 0, B.ref(out),
                           None) == B.GLAM_ERR_INVALID_ARG
    assert lib.glam_decode(B.ref(an), C.c_void_p(fake), 0, B.ref(views2), 0, B.ref(out),
                           None) == B.GLAM_ERR_INVALID_ARG  # partition 0 needs one MLP set
    assert B.status_string(B.GLAM_ERR_CAPACITY) == "pair capacity exceeded"


def test_voxelize_rejects_before_launch():
    lib = B.load()
    fake = 0x100000  # aligned, never dereferenced: validation fails first
    need = lib.glam_voxelize_workspace_bytes(100000)
    assert need >= 100000 * 20 and lib.glam_voxelize_workspace_bytes(200000) > need
    assert lib.glam_voxelize_workspace_bytes(-1) == 0 and lib.glam_voxelize_workspace_bytes((1 << 31) + 1) == 0
    P = C.c_void_p

    def call(n=100000, eps=0.001, existing=fake, n_existing=10, new=fake, cen=fake, cap=1000, merged=fake,
             counts=fake, ws=fake, wsb=need):
        return lib.glam_voxelize(P(fake), n, eps, P(existing) if existing else None, n_existing,
                                 P(new) if new else None, P(cen) if cen else None, cap,
                                 P(merged) if merged else None, P(counts) if counts else None,
                                 P(ws) if ws else None, wsb, None)

    assert call(eps=0.0) == B.GLAM_ERR_INVALID_ARG
    assert call(eps=float("nan")) == B.GLAM_ERR_INVALID_ARG
    assert call(eps=float("inf")) == B.GLAM_ERR_INVALID_ARG
    assert call(n=-1) == B.GLAM_ERR_INVALID_ARG
    assert call(cap=-1) == B.GLAM_ERR_INVALID_ARG
    assert call(counts=None) == B.GLAM_ERR_INVALID_ARG
    assert call(existing=None) == B.GLAM_ERR_INVALID_ARG
    assert call(new=fake + 8) == B.GLAM_ERR_INVALID_ARG
    assert call(cen=None) == B.GLAM_ERR_INVALID_ARG
    assert call(merged=fake + 4) == B.GLAM_ERR_INVALID_ARG
    assert call(n=(1 << 31) + 1, wsb=1 << 40) == B.GLAM_ERR_UNSUPPORTED
    assert call(wsb=need - 1) == B.GLAM_ERR_WORKSPACE
    assert call(ws=None) == B.GLAM_ERR_WORKSPACE


def test_insert_rows_rejects_before_launch():
    lib = B.load()
    fake = 0x100000
    P = C.c_void_p
    ok = dict(src=fake, dst=fake + (1 << 24), rows=3, n_old=100, width=2, at=50, n_new=10, ins=None, stride=0)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.glam_insert_rows(P(a["src"]) if a["src"] else None, P(a["dst"]) if a["dst"] else None, a["rows"],
                                    a["n_old"], a["width"], a["at"], a["n_new"], P(a["ins"]) if a["ins"] else None,
                                    a["stride"], 0.0, None)

    assert call(at=101) == B.GLAM_ERR_INVALID_ARG  # beyond the end
    assert call(at=-1) == B.GLAM_ERR_INVALID_ARG
    assert call(rows=70000) == B.GLAM_ERR_INVALID_ARG
    assert call(dst=fake + 16) == B.GLAM_ERR_INVALID_ARG  # overlaps the source
    assert call(dst=fake + (1 << 24) + 4) == B.GLAM_ERR_INVALID_ARG  # misaligned
    assert call(ins=fake + (1 << 26), stride=19) == B.GLAM_ERR_INVALID_ARG  # rows of ins shorter than 20
    assert call(src=None) == B.GLAM_ERR_INVALID_ARG
    assert call(n_old=1 << 30, at=0, width=4) == B.GLAM_ERR_UNSUPPORTED


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libglam.so"))
    with pytest.raises(ImportError):
        B.load()


def test_backward_modes_validated_before_launch():
    lib = B.load()
    fake = 0x100000  # aligned, never dereferenced: validation fails first
    P = C.c_void_p
    s = synth.plain_scene(1, 10, 32, 32)
    st, info, views = _build(s["cams"], None, 0, 10)
    views.host = C.cast(info, C.c_void_p)
    views.dev = fake
    g = B.Gaussians(fake, fake, fake, fake, fake, 10)
    proj = B.Projected(fake, fake, fake, fake, fake, fake)
    plain = B.GLAM_PLAIN
    det = plain | B.GLAM_DETERMINISTIC_GRADS
    inter = plain | B.GLAM_RETURN_INTERMEDIATES
    # workspace: none in plain mode, the reproducible partials (36 B per pair and 8x8
    # quadrant) with the flag, unknown flags give 0
    assert lib.glam_render_bwd_workspace_bytes(None, B.ref(views), 0, 1000, plain) == 0
    w16 = lib.glam_render_bwd_workspace_bytes(None, B.ref(views), 0, 1000, det)
    assert w16 >= 1000 * 4 * 36
    assert lib.glam_render_bwd_workspace_bytes(None, B.ref(views), 0, 1000, det | (1 << 20)) == 0
    st8, info8, views8 = _build(s["cams"], None, 0, 10, (8, 8))
    assert lib.glam_render_bwd_workspace_bytes(None, B.ref(views8), 0, 1000, det) < w16
    # an anchor scene adds the decode adjoint's workspace in front
    sa = synth.anchor_scene(2, [20], 1, W=32, H=32, fx=30)
    sta, infoa, viewsa = _build(sa["cams"], sa["part_begin"], sa["K"])
    an = B.Anchors(fake, fake, fake, fake, 20, 32, 10, 32)
    # size queries read the host table: none given, no size
    assert lib.glam_render_bwd_workspace_bytes(B.ref(an), B.ref(viewsa), 1, 1000, 0) == 0
    assert lib.glam_decode_bwd_workspace_bytes(B.ref(an), B.ref(viewsa), 1) == 0
    assert lib.glam_loss_workspace_bytes(B.ref(viewsa)) == 0
    viewsa.host = C.cast(infoa, C.c_void_p)
    wa = lib.glam_render_bwd_workspace_bytes(B.ref(an), B.ref(viewsa), 1, 1000, 0)
    assert wa >= lib.glam_decode_bwd_workspace_bytes(B.ref(an), B.ref(viewsa), 1) > 0
    assert lib.glam_render_bwd_workspace_bytes(B.ref(an), B.ref(viewsa), 1, 1000, B.GLAM_DETERMINISTIC_GRADS) > wa
    dg = B.Gaussians(fake, fake, fake, fake, fake, 10)

    def call(flags, pair_begin=fake, d2d=fake, ws=fake, wsb=w16):
        bins = B.Bins(fake, fake, fake, 1000, fake, fake, fake, B.Tuning(0, 0, 0, 0), pair_begin)
        grads = B.Grads(fake, dg, None, None, None, None, d2d)
        return lib.glam_render_bwd(B.ref(proj), B.ref(bins), B.ref(views), None, P(fake), P(fake), P(fake), B.ref(g),
                                   None, None, 0, flags, B.ref(grads), P(ws) if ws else None, wsb, None)

    assert call(det, pair_begin=None) == B.GLAM_ERR_INVALID_ARG   # needs the bin sort's pair offsets
    assert call(det, pair_begin=fake + 4) == B.GLAM_ERR_INVALID_ARG
    assert call(det, wsb=w16 - 1) == B.GLAM_ERR_WORKSPACE
    assert call(inter, d2d=None) == B.GLAM_ERR_INVALID_ARG         # needs the d2d buffer
    assert call(plain | (1 << 9)) == B.GLAM_ERR_INVALID_ARG       # unknown flag
    # forward calls take no backward-only flag
    assert lib.glam_project(B.ref(g), B.ref(views), det, B.ref(proj), None) == B.GLAM_ERR_INVALID_ARG
    assert lib.glam_project(B.ref(g), B.ref(views), inter, B.ref(proj), None) == B.GLAM_ERR_INVALID_ARG
    # the loss total, when given, must be aligned
    ws = lib.glam_loss_workspace_bytes(B.ref(views))
    assert lib.glam_loss(B.ref(views), P(fake), P(fake), C.c_float(0.0), P(fake), P(fake), P(fake + 4), P(fake), ws,
                         None) == B.GLAM_ERR_INVALID_ARG
