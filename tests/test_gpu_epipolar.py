"""The epipolar filter and triangulation on the GPU against the FP64 oracle: retained
pairs bit-exact away from residuals within rounding of the threshold, residuals to FP32
rounding, triangulated points to FP32 rounding of their coordinates."""
import numpy as np
import pytest
import torch

import synth
from oracle import epipolar as E
from paper_2607_21416_amd import binding as B
from paper_2607_21416_amd.pipeline import camera_array

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,noise,outliers,baseline,q", [(100000, 0.5, 0.2, 1.0, 60), (1001, 0.0, 0.0, 2.0, 100),
                                                          (4096, 2.0, 0.5, 0.5, 30), (0, 0.0, 0.0, 1.0, 50)])
def test_epipolar_against_oracle(n, noise, outliers, baseline, q):
    c1, c2, x1, x2, pts, bad = synth.flow_pairs(n + 7, max(n, 1), baseline=baseline, noise_px=noise,
                                                outlier_frac=outliers)
    x1, x2 = x1[:, :n], x2[:, :n]
    r_ref, _, _, _ = E.filter_triangulate(c1, c2, x1, x2, 0.0)
    tau = float(np.float32(np.percentile(r_ref, q) * 1.0000001 if n else 1.0))
    r_ref, keep_ref, X_ref, near = E.filter_triangulate(c1, c2, x1, x2, tau)
    cams = camera_array([c1, c2])
    d1, d2 = torch.from_numpy(np.ascontiguousarray(x1)).cuda(), torch.from_numpy(np.ascontiguousarray(x2)).cuda()
    res = torch.empty(max(n, 1), device="cuda")
    keep = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    X = torch.empty((3, max(n, 1)), device="cuda")
    B.glam_epipolar_triangulate(cams[0], cams[1], d1, d2, n, tau, res, keep, X, None)
    torch.cuda.synchronize()
    if n == 0:
        return
    res, keep, X = res.cpu().numpy()[:n], keep.cpu().numpy()[:n].astype(bool), X.cpu().numpy()[:, :n]
    # FP64 residual rounded to FP32; its terms (pixel coordinates times unit-norm F) are
    # up to ~1e3, so a cancelling sum carries an absolute error of a few 1e-13
    np.testing.assert_allclose(res, r_ref, rtol=1e-6, atol=1e-12)
    ok = ~near
    singular = keep_ref & ~keep & ok
    assert singular.sum() <= max(2, n // 10000)  # near-singular normal equations declined
    assert np.array_equal(keep[ok & ~singular], keep_ref[ok & ~singular])
    both = keep & keep_ref
    assert both.sum() > 0.25 * n * q / 100
    scale = np.maximum(np.abs(X_ref[:, both]), 1.0)
    assert (np.abs(X[:, both] - X_ref[:, both]) <= 2e-6 * scale * 10).all()
    assert np.isnan(X[:, ~keep]).all()

