"""FP64 oracle of the optimiser step of a mapping iteration and of its keyframe sampler.

TEST INFRASTRUCTURE ONLY (see the package docstring).

- Adam (Kingma & Ba, ICLR 2015, Algorithm 1, with the epsilon added to the square root
  of the bias-corrected second moment): elementwise, written out in float64.  Pinned by
  tests/test_oracle_optim.py against its closed forms (the first step moves every
  parameter by lr |g| / (|g| + eps) against the gradient's sign; under a constant
  gradient the bias-corrected moments equal g and g^2 at every step) and against
  torch.optim.Adam in float64.
- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
  3", SC 2011): the counter-based generator the sampler draws from, written from its
  published definition (ten rounds of two 32x32 -> 64-bit products, the Weyl key
  schedule).  Pinned by the known-answer vectors published with the definition.
- The keyframe sampler of a training iteration (the paper draws from the 25 most recent
  keyframes with probability 0.7 and from the older ones with 0.3): per draw, the first
  Philox word decides recent or old (recent when below p 2^32), the second picks the
  keyframe uniformly by a 32x32-bit multiply-high.  Pinned by the binomial fraction of
  recent draws and per-keyframe uniformity over many draws.
"""
from __future__ import annotations

import math

import numpy as np

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_M32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Four 32-bit output words of Philox4x32 with ten rounds."""
    c = [int(x) & _M32 for x in ctr]
    k = [int(x) & _M32 for x in key]
    for r in range(10):
        if r > 0:
            k = [(k[0] + PHILOX_W[0]) & _M32, (k[1] + PHILOX_W[1]) & _M32]
        p0 = PHILOX_M[0] * c[0]
        p1 = PHILOX_M[1] * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k[0], p1 & _M32, (p0 >> 32) ^ c[3] ^ k[1], p0 & _M32]
    return c


def sample_keyframes(n: int, k_recent: int, p_recent: float, count: int, seed: int, counter: int):
    """Keyframe indices (0 = oldest) of `count` draws at counters counter, counter + 1, ..."""
    key = (seed & _M32, (seed >> 32) & _M32)
    thr = min(max(math.floor(float(np.float32(p_recent)) * 2.0 ** 32), 0), 2 ** 32)
    out = np.zeros(count, np.int64)
    for j in range(count):
        c = counter + j
        w = philox4x32_10((c & _M32, (c >> 32) & _M32, 0, 0), key)
        if n <= k_recent:
            out[j] = (w[1] * n) >> 32
        elif w[0] < thr:
            out[j] = n - k_recent + ((w[1] * k_recent) >> 32)
        else:
            out[j] = (w[1] * (n - k_recent)) >> 32
    return out


def adam_step(param, grad, m, v, t: int, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step in float64 (returns new param, m, v; inputs unchanged).  lr may be a
    scalar or an array of per-element learning rates."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m1 = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v1 = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** t)
    vh = v1 / (1.0 - beta2 ** t)
    return p - np.asarray(lr, np.float64) * mh / (np.sqrt(vh) + eps), m1, v1


def segment_lr(n: int, period: int, seg_end, lrs):
    """Per-element learning rates of a group whose rate is periodic in the index."""
    r = np.arange(n) % period
    out = np.empty(n, np.float64)
    lo = 0
    for end, lr in zip(seg_end, lrs):
        out[(r >= lo) & (r < end)] = lr
        lo = end
    return out
