"""Pins of the optimiser-step oracle (Adam) and of the keyframe sampler, and the host
sampler of the library against the oracle (both are host code, no GPU)."""
import numpy as np
import pytest
import torch

from oracle import optim
from paper_2607_21416_amd import binding as B


# Philox4x32-10 known-answer vectors published with the generator's definition (Salmon
# et al., SC 2011): (counter, key) -> output words
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(optim.philox4x32_10(ctr, key)) == want


def test_sampler_fraction_and_uniformity():
    n, k, p, count = 120, 25, 0.7, 40000
    idx = optim.sample_keyframes(n, k, p, count, seed=77, counter=0)
    assert idx.min() >= 0 and idx.max() < n
    recent = idx >= n - k
    # binomial: 0.7 +- 5 standard deviations
    sd = np.sqrt(p * (1 - p) / count)
    assert abs(recent.mean() - p) < 5 * sd
    # within each class every keyframe is about equally likely (loose chi-square bound)
    for sel, m in ((idx[recent], k), (idx[~recent], n - k)):
        h = np.bincount(sel - sel.min(), minlength=m)[:m]
        e = len(sel) / m
        chi2 = ((h - e) ** 2 / e).sum()
        assert chi2 < m + 8 * np.sqrt(2 * m)


def test_sampler_edge_cases():
    # fewer keyframes than the recent window: uniform over all of them
    idx = optim.sample_keyframes(10, 25, 0.7, 5000, seed=3, counter=11)
    assert set(np.unique(idx)) == set(range(10))
    # p = 1: only recent keyframes; p = 0: only older ones
    assert (optim.sample_keyframes(60, 25, 1.0, 2000, 5, 0) >= 35).all()
    assert (optim.sample_keyframes(60, 25, 0.0, 2000, 5, 0) < 35).all()
    # reproducible from (seed, counter), and draws are independent of how they are batched
    a = optim.sample_keyframes(60, 25, 0.7, 100, 9, 1000)
    b = np.concatenate([optim.sample_keyframes(60, 25, 0.7, 40, 9, 1000),
                        optim.sample_keyframes(60, 25, 0.7, 60, 9, 1040)])
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n,k,p,seed,counter", [(120, 25, 0.7, 1, 0), (26, 25, 0.7, 2, 5), (25, 25, 0.3, 3, 1 << 40),
                                                (1000, 1, 0.5, (1 << 63) + 12345, 77), (7, 3, 0.999, 4, 0)])
def test_library_sampler_matches_oracle(n, k, p, seed, counter):
    got = B.glam_sample_keyframes(n, k, p, 3000, seed, counter)
    want = optim.sample_keyframes(n, k, p, 3000, seed, counter)
    assert np.array_equal(got.astype(np.int64), want)


def test_library_sampler_rejects_bad_input():
    with pytest.raises(B.GlamError):
        B.glam_sample_keyframes(0, 25, 0.7, 10, 1, 0)
    with pytest.raises(B.GlamError):
        B.glam_sample_keyframes(10, 25, 1.5, 10, 1, 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.normal(size=1000)
    g = rng.normal(size=1000) * 10.0 ** rng.uniform(-6, 2, 1000)
    lr, eps = 0.01, 1e-15
    p1, m1, v1 = optim.adam_step(p, g, np.zeros(1000), np.zeros(1000), 1, lr, eps=eps)
    # m_hat = g and v_hat = g^2 after one step: the move is lr |g| / (|g| + eps) against sign(g)
    np.testing.assert_allclose(p - p1, lr * np.sign(g) * np.abs(g) / (np.abs(g) + eps), rtol=1e-12, atol=0)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_closed_form():
    rng = np.random.default_rng(6)
    g = rng.normal(size=200)
    p0 = rng.normal(size=200)
    p, m, v = p0, np.zeros(200), np.zeros(200)
    lr = 0.003
    for t in range(1, 8):
        p, m, v = optim.adam_step(p, g, m, v, t, lr, eps=1e-15)
        # bias-corrected moments of a constant gradient are g and g^2 at every step
        np.testing.assert_allclose(m / (1 - 0.9 ** t), g, rtol=1e-12)
        np.testing.assert_allclose(v / (1 - 0.999 ** t), g * g, rtol=1e-11)
    np.testing.assert_allclose(p0 - p, 7 * lr * np.sign(g), rtol=1e-9)


def test_adam_matches_torch_reference():
    rng = np.random.default_rng(7)
    n = 500
    p0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * 10.0 ** rng.uniform(-3, 1, n) for _ in range(5)]
    lr, b1, b2, eps = 0.02, 0.85, 0.99, 1e-8
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0, np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, 1):
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = optim.adam_step(p, g, m, v, t, lr, b1, b2, eps)
        np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_segment_learning_rates():
    lr = optim.segment_lr(10, 4, [1, 3, 4], [1.0, 2.0, 3.0])
    assert lr.tolist() == [1, 2, 2, 3, 1, 2, 2, 3, 1, 2]
