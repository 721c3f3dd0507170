"""One mapping step on the GPU: decode -> project -> bin/sort -> composite -> loss ->
backward, through the C ABI.  PyTorch only provides device memory and the stream.

`Pipeline` owns every device buffer of a scene (inputs, intermediates, outputs,
workspaces), so a step allocates nothing and its launch sequence can be replayed or
captured in a HIP graph.  `GlamRender` / `GlamLoss` expose the same calls as
torch.autograd.Functions.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import binding as B

TILE = 16  # default tile edge (8, 16 and 32 are built)

# Adam settings of the optimiser step (the paper names none; these are the defaults of
# the anchor-based Gaussian-splatting lineage it builds on): learning rates per
# parameter group, the MLP sets per MLP (opacity, colour, covariance).
ADAM = dict(beta1=0.9, beta2=0.999, eps=1e-15)
ADAM_LR_ANCHOR = {"feat": 0.0075, "offs": 0.01, "log_scale": 0.007, "mlp": (0.002, 0.008, 0.004)}
ADAM_LR_PLAIN = {"mean": 0.00016, "log_scale": 0.005, "quat": 0.001, "logit": 0.05, "rgb": 0.0025}


def camera_array(cams) -> "C.Array":
    arr = (B.Camera * len(cams))()
    for i, c in enumerate(cams):
        R = np.asarray(c["R"], np.float32).ravel()
        t = np.asarray(c["t"], np.float32).ravel()
        for k in range(9):
            arr[i].R[k] = float(R[k])
        for k in range(3):
            arr[i].t[k] = float(t[k])
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = (float(c[k]) for k in ("fx", "fy", "cx", "cy"))
        arr[i].width, arr[i].height = int(c["W"]), int(c["H"])
        arr[i].partition = int(c.get("partition", 0))
    return arr


def _f32(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)


class ViewTable:
    """Host and device copies of the per-view offsets (glam_views_build)."""

    def __init__(self, cams, device, part_begin=None, K=0, plain_G=0, tile=TILE):
        self.cams = camera_array(cams)
        self.tile = int(tile)
        n = len(cams)
        self.info = (B.ViewInfo * n)()
        self.views = B.Views()
        if part_begin is not None:
            pb = np.ascontiguousarray(part_begin, np.int32)
            self._pb = pb
            B.glam_views_build(self.cams, n, pb, len(pb) - 1, K, 0, self.tile, self.tile, self.info, self.views)
        else:
            B.glam_views_build(self.cams, n, None, 0, 0, plain_G, self.tile, self.tile, self.info, self.views)
        raw = np.frombuffer(bytes(self.info), dtype=np.uint8).copy()
        self.dev_bytes = torch.from_numpy(raw).to(device)
        self.views.host = C.cast(self.info, C.c_void_p)
        self.views.dev = self.dev_bytes.data_ptr()
        self.n = n

    @property
    def n_gauss(self):
        return self.views.n_gauss

    @property
    def n_pix(self):
        return self.views.n_pix

    @property
    def n_tiles(self):
        return self.views.n_tiles

    def pix_slices(self):
        return [(int(self.info[i].pix_begin), int(self.info[i].cam.width), int(self.info[i].cam.height))
                for i in range(self.n)]


class Pipeline:
    """Device buffers and launch sequence of one scene (see the synth module for the
    scene dictionaries)."""

    def __init__(self, scene: dict, device="cuda", capacity: int | None = None, bg=(0.0, 0.0, 0.0),
                 tile: int = TILE, tuning: dict | None = None, footprint: str = "opacity",
                 deterministic: bool = False, intermediates: bool = False, fuse_l1: bool = True):
        """tile: binning tile edge (8, 16 or 32); tuning: the compositing schedule
        (long_log2, fwd/bwd_blocks_per_cu, fwd/bwd_group_waves; missing or 0 = default);
        footprint: "opacity" (the exact alpha >= 1/255 box) or "3sigma" (the lineage's
        tile-granular 3-sigma square); deterministic: reproducible gradients (no
        floating-point atomics in the compositing adjoint); intermediates: the backward
        also writes the 2-D gradients d(u, v, A, B, C, opacity, rgb) to self.d2d;
        fuse_l1: with a per-pixel L1 loss (no SSIM term), step() composites, takes the loss
        and walks the compositing adjoint in one pass (glam_render_fused_l1)."""
        self.device = torch.device(device)
        dev = self.device
        self.scene = scene
        self.tuning = B.make_tuning(tuning)
        self.plain = scene["kind"] == "plain"
        self.flags = B.GLAM_PLAIN if self.plain else 0
        if not self.plain and scene.get("opacity_mode", "tanh") == "sigmoid":
            self.flags |= B.GLAM_OPACITY_SIGMOID
        if footprint not in ("opacity", "3sigma"):
            raise ValueError(f"footprint {footprint!r}: 'opacity' or '3sigma'")
        if footprint == "3sigma":
            self.flags |= B.GLAM_FOOTPRINT_3SIGMA
        self.deterministic = bool(deterministic)
        self.intermediates = bool(intermediates)
        self.bflags = self.flags | (B.GLAM_DETERMINISTIC_GRADS if self.deterministic else 0) | (
            B.GLAM_RETURN_INTERMEDIATES if self.intermediates else 0)
        self.generation = 0  # forward passes run so far (GlamRender checks it)
        self.ssim_weight = float(scene.get("ssim_weight", 0.0))
        cams = scene["cams"]
        self.tile = int(tile)
        if self.plain:
            G = scene["mean"].shape[1]
            self.vt = ViewTable(cams, dev, plain_G=G, tile=tile)
            self.params = {k: _f32(scene[k], dev) for k in ("mean", "log_scale", "quat", "logit", "rgb")}
            self.gauss = B.Gaussians(self.params["mean"].data_ptr(), self.params["log_scale"].data_ptr(),
                                     self.params["quat"].data_ptr(), self.params["logit"].data_ptr(),
                                     self.params["rgb"].data_ptr(), G)
            self.n_parts = 0
        else:
            self.params = {k: _f32(scene[k], dev) for k in ("pos", "feat", "log_scale", "offs", "mlp")}
            self.part_begin = np.asarray(scene["part_begin"], np.int64).copy()
            self.n_parts = scene["mlp"].shape[0]
            self._anchor_views()
        npix = self.vt.n_pix
        self.image = torch.empty(3 * npix, device=dev)
        self.T_final = torch.empty(npix, device=dev)
        self.n_contrib = torch.empty(npix, device=dev, dtype=torch.int32)
        self.n_eval = None
        self.target = torch.cat([_f32(t, dev).reshape(-1) for t in scene["targets"]])
        self.dimage = torch.empty(3 * npix, device=dev)
        self.loss = torch.empty(self.vt.n, device=dev)
        self.loss_total = torch.empty(1, device=dev)
        self.bg = torch.zeros(4, device=dev)
        self.bg[:3] = torch.tensor(bg, dtype=torch.float32)
        self.ws_loss = torch.empty(B.glam_loss_workspace_bytes(self.vt.views), device=dev, dtype=torch.uint8)
        self.fuse_l1 = bool(fuse_l1) and self.ssim_weight == 0.0 and not self.deterministic and not self.intermediates
        if self.fuse_l1:
            self.ws_fused = torch.empty(max(256, B.glam_render_fused_l1_workspace_bytes(self.vt.views)), device=dev,
                                        dtype=torch.uint8)
        self.status = torch.zeros(8, device=dev, dtype=torch.int32)
        self._alloc_gauss_buffers(capacity)

    def _anchor_views(self):
        """View table, anchor descriptor and decoded-Gaussian buffers for the current
        anchors and partition ranges."""
        dev = self.device
        F, K = self.scene["F"], self.scene["K"]
        self.vt = ViewTable(self.scene["cams"], dev, part_begin=self.part_begin, K=K, tile=self.tile)
        A = self.params["feat"].shape[0]
        self.anchors = B.Anchors(self.params["pos"].data_ptr(), self.params["feat"].data_ptr(),
                                 self.params["log_scale"].data_ptr(), self.params["offs"].data_ptr(), A, F, K,
                                 self.scene["hidden"])
        n = self.vt.n_gauss
        self.dec = {k: torch.empty((r, n) if r > 1 else (n,), device=dev, dtype=torch.float32)
                    for k, r in (("mean", 3), ("scale", 3), ("quat", 4), ("opacity", 1), ("rgb", 3))}
        self.gauss = B.Gaussians(*(self.dec[k].data_ptr() for k in ("mean", "scale", "quat", "opacity", "rgb")), n)

    def _alloc_gauss_buffers(self, capacity: int | None):
        """Buffers sized by the view-Gaussian count: projection, pairs, gradients and the
        decode adjoint's workspace."""
        dev = self.device
        n = self.vt.n_gauss
        self.proj_t = dict(uv=torch.empty((2, n), device=dev), conic=torch.empty((3, n), device=dev),
                           depth=torch.empty(n, device=dev), ext=torch.empty((2, n), device=dev),
                           ntiles=torch.empty(n, device=dev, dtype=torch.int32),
                           splat=torch.empty((n, 12), device=dev))
        self.proj = B.Projected(*(self.proj_t[k].data_ptr() for k in ("uv", "conic", "depth", "ext", "ntiles",
                                                                     "splat")))
        self.pair_begin = torch.empty(max(n, 1), device=dev, dtype=torch.int32) if self.deterministic else None
        # gradients
        self.g2d = torch.empty((n, 9), device=dev)
        self.d2d = torch.empty((9, n), device=dev) if self.intermediates else None
        d2d = self.d2d.data_ptr() if self.intermediates else None
        if self.plain:
            G = self.gauss.n
            self.dg = {k: torch.empty((r, G) if r > 1 else (G,), device=dev)
                       for k, r in (("mean", 3), ("log_scale", 3), ("quat", 4), ("logit", 1), ("rgb", 3))}
            dgs = B.Gaussians(*(self.dg[k].data_ptr() for k in ("mean", "log_scale", "quat", "logit", "rgb")), G)
            self.dgs = dgs
            self.grads = B.Grads(self.g2d.data_ptr(), dgs, None, None, None, None, d2d)
        else:
            self.dg = {k: torch.empty((r, n) if r > 1 else (n,), device=dev)
                       for k, r in (("mean", 3), ("scale", 3), ("quat", 4), ("opacity", 1), ("rgb", 3))}
            dgs = B.Gaussians(*(self.dg[k].data_ptr() for k in ("mean", "scale", "quat", "opacity", "rgb")), n)
            self.dgs = dgs
            p = self.params
            self.pgrad = {k: torch.empty_like(p[k]) for k in ("feat", "offs", "log_scale", "mlp")}
            self.grads = B.Grads(self.g2d.data_ptr(), dgs, self.pgrad["feat"].data_ptr(),
                                 self.pgrad["offs"].data_ptr(), self.pgrad["log_scale"].data_ptr(),
                                 self.pgrad["mlp"].data_ptr(), d2d)
        self._alloc_bins(capacity if capacity else max(1024, 4 * n))

    # ------------------------------------------------------------------------------
    def grow_anchors(self, centres, n_new: int, partition: int, eps: float, centres_stride: int | None = None):
        """Anchor growth at a keyframe (Eq. 4 and its bookkeeping): n_new anchors at the
        voxel centres (device rows x, y, z of centres_stride floats each, by default
        centres.shape[1]; glam_voxelize's new_centres with its capacity as stride) join
        `partition`, inserted at the end of its range of every per-anchor array, as
        anchors created from points: zero features and offsets, log-scale ln(eps), zero
        Adam moments.  Later partitions' ranges shift; the view table and every buffer
        sized by the view-Gaussian count are rebuilt (the pair capacity keeps its slack
        rule through fit_capacity).  Runs on the current stream."""
        if self.plain:
            raise ValueError("anchor growth needs an anchor scene")
        n_new = int(n_new)
        if n_new <= 0:
            return
        if not 0 <= partition < self.n_parts:
            raise ValueError(f"partition {partition} out of range [0, {self.n_parts})")
        s = self.stream()
        A, F, K = self.anchors.A, self.anchors.F, self.anchors.K
        at = int(self.part_begin[partition + 1])
        stride = int(centres.shape[1] if centres_stride is None else centres_stride)
        ln_eps = math.log(float(np.float32(eps)))
        layout = {"pos": (3, 1), "feat": (1, F), "log_scale": (1, 1), "offs": (3, K)}

        def grow(t, name, ins=None, fill=0.0):
            rows, width = layout[name]
            if name == "feat":
                out = t.new_empty((A + n_new, F))
            elif rows == 1:
                out = t.new_empty(A + n_new)
            else:
                out = t.new_empty((3, (A + n_new) * width))
            B.glam_insert_rows(t, out, rows, A, width, at, n_new, ins, stride if ins is not None else 0, fill, s)
            return out

        self.params["pos"] = grow(self.params["pos"], "pos", centres)
        self.params["feat"] = grow(self.params["feat"], "feat")
        self.params["log_scale"] = grow(self.params["log_scale"], "log_scale", fill=ln_eps)
        self.params["offs"] = grow(self.params["offs"], "offs")
        if hasattr(self, "opt_m"):
            for k in ("feat", "offs", "log_scale"):
                self.opt_m[k] = grow(self.opt_m[k], k)
                self.opt_v[k] = grow(self.opt_v[k], k)
        self.part_begin[partition + 1:] += n_new
        self._anchor_views()
        self._alloc_gauss_buffers(None)
        if hasattr(self, "opt_groups"):
            self.opt_groups = self._adam_groups()

    # ------------------------------------------------------------------------------
    def _alloc_bins(self, capacity: int):
        dev = self.device
        self.capacity = int(capacity)
        self.keys = torch.empty(self.capacity, device=dev, dtype=torch.int64)
        self.vals = torch.empty(self.capacity, device=dev, dtype=torch.int32)
        self.ranges = torch.empty(2 * self.vt.n_tiles, device=dev, dtype=torch.int32)
        self.order = torch.empty(self.vt.n_tiles, device=dev, dtype=torch.int32)
        self.queue = torch.zeros(B.GLAM_QUEUE_WORDS, device=dev, dtype=torch.int32)
        self.bins = B.Bins(self.keys.data_ptr(), self.vals.data_ptr(), self.ranges.data_ptr(), self.capacity,
                           self.status.data_ptr(), self.order.data_ptr(), self.queue.data_ptr(), self.tuning,
                           self.pair_begin.data_ptr() if self.pair_begin is not None else None)
        nb = B.glam_bin_sort_workspace_bytes(self.vt.views, self.capacity)
        self.ws_sort = torch.empty(nb, device=dev, dtype=torch.uint8)
        # the backward's workspace: the decode adjoint's and, when reproducible, the
        # per-(pair, quadrant) partials, which scale with the pair capacity
        nb = B.glam_render_bwd_workspace_bytes(None if self.plain else self.anchors, self.vt.views, self.n_parts,
                                               self.capacity, self.bflags)
        self.ws_dec = torch.empty(max(256, nb), device=dev, dtype=torch.uint8)

    # ------------------------------------------------------------------------------
    def init_optimizer(self):
        """Adam state (zeroed moments) and the parameter groups of glam_adam_step: the
        anchors' features, offsets and log-scales and the MLP sets (one group, a segment
        per MLP), or the plain Gaussians' parameters.  Anchor positions stay fixed."""
        names = list(ADAM_LR_PLAIN) if self.plain else list(ADAM_LR_ANCHOR)
        self.opt_m = {k: torch.zeros_like(self.params[k]) for k in names}
        self.opt_v = {k: torch.zeros_like(self.params[k]) for k in names}
        self.opt_t = 0
        self.opt_groups = self._adam_groups()

    def _adam_groups(self):
        """glam_adam_step's parameter groups over the current parameter, gradient and
        moment tensors."""
        if self.plain:
            names, lrs = list(ADAM_LR_PLAIN), ADAM_LR_PLAIN
            grads = {"mean": self.dg["mean"], "log_scale": self.dg["log_scale"], "quat": self.dg["quat"],
                     "logit": self.dg["logit"], "rgb": self.dg["rgb"]}
        else:
            names, lrs = list(ADAM_LR_ANCHOR), ADAM_LR_ANCHOR
            grads = self.pgrad
        groups = (B.AdamGroup * len(names))()
        for i, k in enumerate(names):
            g = groups[i]
            g.param, g.grad = self.params[k].data_ptr(), grads[k].data_ptr()
            g.m, g.v = self.opt_m[k].data_ptr(), self.opt_v[k].data_ptr()
            g.n = self.params[k].numel()
            if k == "mlp":
                P = self.params[k].shape[1]
                F, K = self.scene["F"], self.scene["K"]
                n_in, h = F + 4, self.scene["hidden"]
                ends = []
                for out in (K, 3 * K, 7 * K):
                    ends.append((ends[-1] if ends else 0) + h * n_in + h + out * h + out)
                assert ends[-1] == P
                g.period, g.n_seg = P, 3
                for j in range(3):
                    g.seg_end[j], g.lr[j] = ends[j], lrs[k][j]
            else:
                g.period, g.n_seg = 1, 1  # one learning rate for the whole array
                g.seg_end[0], g.lr[0] = 1, lrs[k]
        return groups

    def adam_step(self, s=None, step: int | None = None):
        """The optimiser step after a backward (step number: the next one by default)."""
        if not hasattr(self, "opt_groups"):
            self.init_optimizer()
        self.opt_t = self.opt_t + 1 if step is None else int(step)
        B.glam_adam_step(self.opt_groups, len(self.opt_groups), self.opt_t, ADAM["beta1"], ADAM["beta2"],
                         ADAM["eps"], s or self.stream())

    def set_tuning(self, tuning: dict | None):
        """Changes the compositing schedule (takes effect from the next bin_sort)."""
        self.tuning = B.make_tuning(tuning)
        self.bins.tuning = self.tuning

    def stream(self):
        return torch.cuda.current_stream(self.device)

    # ------------------------------------------------------------------------------
    def decode(self, s=None):
        if not self.plain:
            B.glam_decode(self.anchors, self.params["mlp"], self.n_parts, self.vt.views, self.flags, self.gauss,
                          s or self.stream())

    def decode_project(self, s=None):
        """decode() and project() in one launch (anchor scenes; plain scenes project)."""
        if self.plain:
            self.project(s)
        else:
            B.glam_decode_project(self.anchors, self.params["mlp"], self.n_parts, self.vt.views, self.flags,
                                  self.gauss, self.proj, s or self.stream())

    def project(self, s=None):
        B.glam_project(self.gauss, self.vt.views, self.flags, self.proj, s or self.stream())

    def bin_sort(self, s=None):
        B.glam_bin_sort(self.proj, self.vt.views, self.bins, self.ws_sort, self.ws_sort.numel(), s or self.stream())

    def render(self, s=None):
        B.glam_render_fwd(self.proj, self.bins, self.vt.views, self.bg, self.image, self.T_final, self.n_contrib,
                          self.n_eval, s or self.stream())

    def count_evaluations(self, on: bool = True):
        """Makes render() also write per-pixel evaluation counts (self.n_eval)."""
        self.n_eval = torch.zeros(self.vt.n_pix, device=self.device, dtype=torch.int32) if on else None

    def compute_loss(self, s=None):
        B.glam_loss(self.vt.views, self.image, self.target, self.ssim_weight, self.dimage, self.loss, self.loss_total,
                    self.ws_loss, self.ws_loss.numel(), s or self.stream())

    def backward(self, s=None, dimage=None):
        B.glam_render_bwd(self.proj, self.bins, self.vt.views, self.bg, self.T_final, self.n_contrib,
                          self.dimage if dimage is None else dimage, self.gauss,
                          None if self.plain else self.anchors, None if self.plain else self.params["mlp"],
                          self.n_parts, self.bflags, self.grads, self.ws_dec, self.ws_dec.numel(), s or self.stream())

    def composite_bwd(self, s=None, dimage=None):
        B.glam_composite_bwd(self.proj, self.bins, self.vt.views, self.bg, self.T_final, self.n_contrib,
                             self.dimage if dimage is None else dimage, self.g2d, s or self.stream())

    def project_bwd(self, s=None):
        B.glam_project_bwd(self.gauss, self.proj, self.vt.views, self.flags, self.g2d, self.dgs, s or self.stream())

    def decode_bwd(self, s=None):
        if not self.plain:
            g = self.pgrad
            B.glam_decode_bwd(self.anchors, self.params["mlp"], self.n_parts, self.vt.views, self.flags, self.dgs,
                              g["feat"], g["offs"], g["log_scale"], g["mlp"], self.ws_dec, self.ws_dec.numel(),
                              s or self.stream())

    def forward(self, s=None):
        self.decode_project(s)
        self.bin_sort(s)
        self.render(s)
        self.compute_loss(s)
        self.generation += 1

    def fused_l1(self, s=None):
        """Forward compositing, the L1 loss and the compositing adjoint in one pass."""
        B.glam_render_fused_l1(self.proj, self.bins, self.vt.views, self.bg, self.target, self.image, self.T_final,
                               self.n_contrib, self.dimage, self.loss, self.loss_total, self.g2d, self.ws_fused,
                               self.ws_fused.numel(), s or self.stream())

    def step(self, s=None):
        if not self.fuse_l1 or self.n_eval is not None:
            self.forward(s)
            self.backward(s)
            return
        self.decode_project(s)
        self.bin_sort(s)
        self.fused_l1(s)
        self.generation += 1
        self.project_bwd(s)
        self.decode_bwd(s)

    # ------------------------------------------------------------------------------
    def pair_count(self) -> int:
        st = self.status.cpu().numpy()
        return int(np.uint32(st[2])) | (int(np.uint32(st[3])) << 32)

    def check_status(self):
        st = self.status.cpu().numpy()
        if st[0] != 0:
            raise B.GlamError("device status", int(st[0]))

    def fit_capacity(self, slack: float = 1.25):
        """Runs the forward up to the sort once and sizes the pair buffers to the
        required count times `slack` (one synchronising sizing pass; buffers more than
        twice that size are shrunk, since the sort's grids scale with the capacity)."""
        self.decode_project()
        self.bin_sort()
        torch.cuda.synchronize(self.device)
        need = self.pair_count()
        if need > self.capacity or self.capacity > 2 * slack * max(need, 1024):
            self.status.zero_()
            self._alloc_bins(max(1024, int(need * slack)))
        return need

    def images(self):
        out = []
        for pb, W, H in self.vt.pix_slices():
            out.append(self.image[3 * pb:3 * pb + 3 * W * H].view(3, H, W))
        return out

    def per_pixel(self, t):
        return [t[pb:pb + W * H].view(H, W) for pb, W, H in self.vt.pix_slices()]


class GlamRender(torch.autograd.Function):
    """images = render(params); backward runs the reverse compositing, projection and
    decode adjoints.  params: (feat, offs, log_scale, mlp) in anchor mode or (mean,
    log_scale, quat, logit, rgb) in plain mode; they must be the tensors the Pipeline
    holds (the kernels read them in place), and the backward must run before the
    Pipeline renders again (it reads the forward's stored per-pixel state)."""

    NAMES = {True: ("mean", "log_scale", "quat", "logit", "rgb"), False: ("feat", "offs", "log_scale", "mlp")}

    @staticmethod
    def forward(ctx, pipe: Pipeline, *params):
        names = GlamRender.NAMES[pipe.plain]
        if len(params) != len(names) or any(p.data_ptr() != pipe.params[k].data_ptr() for p, k in zip(params, names)):
            raise ValueError(f"GlamRender takes the Pipeline's own parameter tensors {names}")
        pipe.decode_project()
        pipe.bin_sort()
        pipe.render()
        pipe.generation += 1
        ctx.pipe = pipe
        ctx.generation = pipe.generation
        return pipe.image.clone()

    @staticmethod
    def backward(ctx, dimage):
        pipe = ctx.pipe
        if pipe.generation != ctx.generation:
            raise RuntimeError("the Pipeline rendered again after this forward; its stored state is gone")
        pipe.backward(dimage=dimage.contiguous())
        if pipe.plain:
            g = tuple(pipe.dg[k].clone() for k in ("mean", "log_scale", "quat", "logit", "rgb"))
        else:
            g = tuple(pipe.pgrad[k].clone() for k in ("feat", "offs", "log_scale", "mlp"))
        return (None,) + g


class GlamLoss(torch.autograd.Function):
    """Sum over views of L1 + w (1 - SSIM) (Eq. 3); dL/dimage comes from the loss kernel."""

    @staticmethod
    def forward(ctx, pipe: Pipeline, image):
        pipe.image.copy_(image)
        pipe.compute_loss()
        ctx.pipe = pipe
        return pipe.loss_total[0].clone()

    @staticmethod
    def backward(ctx, g):
        return None, ctx.pipe.dimage * g
