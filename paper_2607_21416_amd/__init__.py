"""MI355X (gfx950) hot path of a Gaussian mapping backend: anchor-MLP decode, EWA
projection, tile binning and depth sort, front-to-back compositing, the L1 + SSIM loss
and the backward of all of these, as hand-written HIP kernels behind the C ABI of
include/glam.h.

binding   ctypes binding of the C ABI (same names as the header)
pipeline  device buffers + launch sequence of one step; torch.autograd.Functions
"""
from . import binding  # noqa: F401
