"""The calls of a keyframe's update (optimiser step, loop-closure deformation, epipolar
filter and triangulation, voxelisation and growth) captured in a HIP graph, as the
benchmark times them: every replay reproduces the eager call bit for bit, with eager
work between replays that overwrites outputs, workspace and (for the in-place calls)
restores the inputs."""
import numpy as np
import pytest
import torch

import synth
from oracle import voxel as V
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import camera_array

pytestmark = pytest.mark.gpu


def capture(fn):
    """fn(stream) captured into a graph after one warm-up call on a side stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn(torch.cuda.current_stream())
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn(torch.cuda.current_stream())
    torch.cuda.synchronize()
    return g


def test_voxelize_graph_replays():
    eps = 0.002
    cloud = synth.fused_points(71, 60000, nan_frac=0.2, far_frac=0.01, far=(1 << 21) * eps)
    _, _, have, _ = V.voxelize(synth.fused_points(72, 30000), eps)
    n, ne = cloud.shape[1], len(have)
    pts = torch.from_numpy(cloud).cuda()
    ex = torch.from_numpy(have.view(np.int64).copy()).cuda()
    new = torch.empty(n, dtype=torch.int64, device="cuda")
    cen = torch.empty((3, n), device="cuda")
    mer = torch.empty(ne + n, dtype=torch.int64, device="cuda")
    cnt = torch.empty(2, dtype=torch.int64, device="cuda")
    wsb = B.glam_voxelize_workspace_bytes(n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def call(stream):
        B.glam_voxelize(pts, n, eps, ex, ne, new, cen, n, mer, cnt, ws, wsb, stream)

    print("voxelize eager", flush=True)
    call(None)
    torch.cuda.synchronize()
    m = int(cnt[0].item())
    ref = (new[:m].clone(), cen[:, :m].clone(), mer[:ne + m].clone(), cnt.clone())
    g = capture(call)
    for r in range(3):
        print(f"voxelize replay {r}", flush=True)
        new.fill_(-1)
        cen.fill_(float("nan"))
        mer.fill_(-1)
        cnt.fill_(-7)
        ws.fill_(0xA5)  # nothing may rely on a cleared workspace
        g.replay()
        torch.cuda.synchronize()
        got = (new[:m], cen[:, :m], mer[:ne + m], cnt)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {r}"


def test_epipolar_graph_replays():
    n = 100000
    c1, c2, x1, x2, _, _ = synth.flow_pairs(73, n, baseline=1.0, noise_px=0.5, outlier_frac=0.2)
    cams = camera_array([c1, c2])
    d1, d2 = torch.from_numpy(np.ascontiguousarray(x1)).cuda(), torch.from_numpy(np.ascontiguousarray(x2)).cuda()
    res = torch.empty(n, device="cuda")
    keep = torch.empty(n, dtype=torch.int32, device="cuda")
    X = torch.empty((3, n), device="cuda")

    def call(stream):
        B.glam_epipolar_triangulate(cams[0], cams[1], d1, d2, n, 0.05, res, keep, X, stream)

    print("epipolar eager", flush=True)
    call(None)
    torch.cuda.synchronize()
    ref = (res.clone(), keep.clone(), X.clone())
    g = capture(call)
    for r in range(3):
        print(f"epipolar replay {r}", flush=True)
        res.fill_(-1.0)
        keep.fill_(7)
        X.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, ref[0]) and torch.equal(keep, ref[1])
        assert torch.equal(torch.nan_to_num(X, nan=123.0), torch.nan_to_num(ref[2], nan=123.0))


def test_deform_graph_replays():
    rng = np.random.default_rng(74)
    A, K = 20000, 10
    vox = synth.corridor_voxels()
    pos0 = torch.from_numpy(vox[np.sort(rng.choice(len(vox), A, replace=False))].T.astype(np.float32).copy()).cuda()
    offs0 = torch.from_numpy(rng.normal(0, 0.1, (3, A * K)).astype(np.float32)).cuda()
    fixes = synth.loop_fixes(75, 12, spacing=2.0, rot_deg=2.0, trans_m=0.2)
    arr = (B.KeyframeFix * len(fixes))()
    for i, f in enumerate(fixes):
        c = arr[i].before
        for k in range(9):
            c.R[k] = float(np.asarray(f["R_old"]).ravel()[k])
            arr[i].R_new[k] = float(np.asarray(f["R_new"]).ravel()[k])
        for k in range(3):
            c.t[k] = float(f["t_old"][k])
            arr[i].t_new[k] = float(f["t_new"][k])
        c.fx, c.fy, c.cx, c.cy, c.width, c.height = f["fx"], f["fy"], f["cx"], f["cy"], f["W"], f["H"]
    table = torch.from_numpy(np.frombuffer(bytes(arr), np.uint8).copy()).cuda()
    pos, offs = pos0.clone(), offs0.clone()
    owner = torch.empty(A, dtype=torch.int32, device="cuda")

    def call(stream):
        B.glam_deform_anchors(pos, offs, A, K, table, len(fixes), 0.2, 80.0, owner, stream)

    print("deform eager", flush=True)
    call(None)
    torch.cuda.synchronize()
    ref = (pos.clone(), offs.clone(), owner.clone())
    assert int((ref[2] >= 0).sum().item()) > A // 4
    g = capture(call)
    for r in range(3):
        print(f"deform replay {r}", flush=True)
        pos.copy_(pos0)  # the call updates in place: each replay starts from the same anchors
        offs.copy_(offs0)
        owner.fill_(-5)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(pos, ref[0]) and torch.equal(offs, ref[1]) and torch.equal(owner, ref[2])


def test_adam_graph_replays():
    rng = np.random.default_rng(76)
    sizes = [(5000, 1, [1], [0.01]), (7182 * 2, 7182, [2394, 4788, 7182], [0.002, 0.008, 0.004]), (77, 1, [1], [0.1])]
    state0, state, groups = [], [], (B.AdamGroup * len(sizes))()
    for i, (n, period, ends, lrs) in enumerate(sizes):
        t0 = [torch.from_numpy(x.astype(np.float32)).cuda() for x in
              (rng.normal(size=n), rng.normal(size=n), rng.normal(size=n) * 0.1, rng.uniform(0, 0.01, n))]
        t = [x.clone() for x in t0]
        state0.append(t0)
        state.append(t)
        a = B.AdamGroup()
        a.param, a.grad, a.m, a.v = t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), t[3].data_ptr()
        a.n, a.period, a.n_seg = n, period, len(ends)
        for j, (e, lr) in enumerate(zip(ends, lrs)):
            a.seg_end[j], a.lr[j] = e, lr
        groups[i] = a

    def call(stream):
        B.glam_adam_step(groups, len(sizes), 5, 0.9, 0.999, 1e-15, stream)

    print("adam eager", flush=True)
    call(None)
    torch.cuda.synchronize()
    ref = [[x.clone() for x in t] for t in state]
    g = capture(call)
    for r in range(3):
        print(f"adam replay {r}", flush=True)
        for t, t0 in zip(state, state0):
            for x, x0 in zip(t, t0):
                x.copy_(x0)
        g.replay()
        torch.cuda.synchronize()
        for t, rt in zip(state, ref):
            for x, y in zip(t, rt):
                assert torch.equal(x, y), f"replay {r}"
