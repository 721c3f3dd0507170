"""bench.py on the CPU: more than one GPU is refused with a message before anything is
initialised, and the whole-step roofline sums each stage's ideal time from the stated
per-unit work at the published peaks."""
import os
import subprocess
import sys
import types

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                       env=dict(os.environ, **env), timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_whole_step_roofline_arithmetic():
    info = [types.SimpleNamespace(anchor_count=100000) for _ in range(2)]
    status = torch.zeros(8, dtype=torch.int32)
    status[6] = 5
    pipe = types.SimpleNamespace(status=status, anchors=types.SimpleNamespace(A=100000),
                                 vt=types.SimpleNamespace(n=2, info=info, n_gauss=2000000, n_pix=5000000))
    ms = 1.0
    r = bench.whole_step_roofline(pipe, ms, pairs=3000000, evals_fwd=10 ** 10, evals_bwd=8 * 10 ** 9)
    # published peaks: HBM 8 TB/s, FP32 matrix cores 157.3 TFLOP/s, FP32 VALU issue
    # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-op slots per second
    hbm, mfma = 8e12, 157.3e12
    alu = 256 * 4 * 16 * 2.4e9
    want = (max(200000 * 13952 / mfma, (100000 * 264 + 2000000 * 96) / hbm)     # decode + projection
            + 3000000 * (24 + 5 * 24) / hbm                                     # bin + sort, 5 passes
            + 10 ** 10 * 22 / alu                                               # forward: 18 VALU + exp (4)
            + 5000000 * 36 / hbm                                                # loss
            + 8 * 10 ** 9 * 53 / alu                                            # backward: 45 + exp + rcp
            + 2000000 * 132 / hbm                                               # projection adjoint
            + max(200000 * 27904 / mfma, (100000 * 264 + 2000000 * 56) / hbm))  # decode adjoint
    assert r["ideal_ms"] == pytest.approx(want * 1e3, rel=1e-3)
    assert r["frac"] == pytest.approx(want * 1e3 / ms, rel=1e-3)
    assert r["units"]["radix_passes"] == 5 and r["units"]["anchor_views"] == 200000
    # per-kernel fractions: each stage's ideal time over its own measured time
    st = {k: 0.5 for k in ("decode_project", "bin_sort", "render_fwd", "loss", "composite_bwd", "project_bwd",
                           "decode_bwd")}
    ceil = {"hbm_copy_TBs": 4.0, "fma_TFLOPs": 78.6 / 2, "mfma_fp32_TFLOPs": 100.0}
    kr = bench.kernel_rooflines(pipe, st, 3000000, 10 ** 10, 8 * 10 ** 9, ceil)
    assert kr["composite_bwd"]["bound"] == "alu"
    assert kr["composite_bwd"]["frac"] == pytest.approx(8 * 10 ** 9 * 53 / alu / 0.5e-3, rel=1e-3)
    assert kr["composite_bwd"]["frac_measured_ceiling"] == pytest.approx(2 * kr["composite_bwd"]["frac"], rel=1e-3)
    assert kr["loss"]["bound"] == "hbm" and kr["loss"]["frac"] == pytest.approx(5000000 * 36 / hbm / 0.5e-3, rel=1e-3)
    assert kr["loss"]["frac_measured_ceiling"] == pytest.approx(2 * kr["loss"]["frac"], rel=1e-3)
