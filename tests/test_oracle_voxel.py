"""Pins of the voxelisation and growth oracle (Eq. 4): brute force with exact rational
quotients, lattice recovery, ties to even, geometric invariants, set identities of the
growth step and the key order."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import voxel as V


def _brute_voxels(points, eps):
    """Voxels as integer triples: the exact quotient p / eps rounded to FP32 (a correctly
    rounded double rounded once more to FP32, innocuous for a quotient of FP32 values),
    then Python's round(), which takes ties to the even neighbour."""
    out, dropped = set(), 0
    e = Fraction(float(np.float32(eps)))
    for j in range(points.shape[1]):
        k = []
        for a in range(3):
            p = float(points[a, j])
            if p != p:
                k = None
                break
            q = float(np.float32(float(Fraction(p) / e)))
            r = round(q)
            if not (-(1 << 20) <= r < (1 << 20)):
                k = None
                break
            k.append(r)
        if k is None:
            dropped += 1
        else:
            out.add(tuple(k))
    return out, dropped


@pytest.mark.parametrize("seed,n,eps", [(1, 300, 0.001), (2, 400, 0.05), (3, 200, 0.2), (4, 300, 0.37)])
def test_brute_force_small_clouds(seed, n, eps):
    pts = synth.fused_points(seed, n, dup_frac=0.4, dup_jitter=eps / 3, nan_frac=0.05, far_frac=0.02,
                             far=(1 << 21) * eps)
    want, dropped = _brute_voxels(pts, eps)
    new, cen, grown, d = V.voxelize(pts, eps)
    got = {tuple(t) for t in V.unpack(new).T.tolist()}
    assert got == want and d == dropped
    assert np.array_equal(new, grown)
    # fewer voxels than kept points: the duplicates collapse
    assert len(want) < n - dropped


def test_lattice_recovery():
    rng = np.random.default_rng(9)
    eps = 0.01
    lattice = rng.integers(-5000, 5000, (3, 500))
    idx = rng.integers(0, 500, 3000)
    pts = lattice[:, idx] * eps + rng.uniform(-0.45 * eps, 0.45 * eps, (3, 3000))
    new, cen, _, dropped = V.voxelize(pts.astype(np.float32), eps)
    want = sorted({tuple(lattice[:, j]) for j in idx.tolist()})
    assert dropped == 0
    assert [tuple(t) for t in V.unpack(new).T.tolist()] == want


def test_ties_to_even():
    # eps a power of two: p / eps is exact, half-integers are true ties
    eps = 0.5
    p = np.array([[0.25, 0.75, -0.25, -0.75, 1.25, 1.75]] * 3, np.float32)
    k, dropped = V.quantise(p, eps)
    assert dropped == 0
    assert k[0].tolist() == [0, 2, 0, -2, 2, 4]


def test_half_voxel_and_occupancy():
    eps = 0.003
    pts = synth.fused_points(5, 20000, nan_frac=0.1)
    new, cen, _, dropped = V.voxelize(pts, eps)
    ok = ~np.isnan(pts).any(0)
    assert dropped == int((~ok).sum())
    p = pts[:, ok].astype(np.float64)
    k, _ = V.quantise(pts[:, ok], eps)
    # each point is within half a voxel (plus FP32 rounding) of its voxel's centre
    c = k.astype(np.float64) * eps
    assert np.abs(p - c).max() <= 0.5 * eps * (1 + 1e-4) + 1e-5
    # every voxel holds a point, and every point's voxel is listed
    assert set(V.pack(k).tolist()) == set(new.tolist())


def test_centres_are_fixed_points():
    pts = synth.fused_points(6, 5000)
    for eps in (0.001, 0.01, 0.2):
        new, cen, _, _ = V.voxelize(pts, eps)
        again, cen2, _, dropped = V.voxelize(cen, eps)
        assert dropped == 0 and np.array_equal(again, new) and np.array_equal(cen2, cen)


def test_growth_is_set_difference_and_union():
    eps = 0.02
    a = synth.fused_points(7, 4000)
    b = synth.fused_points(8, 4000)
    _, _, have, _ = V.voxelize(a, eps)
    new, _, grown, _ = V.voxelize(b, eps, existing=have)
    _, _, both, _ = V.voxelize(np.concatenate([a, b], axis=1), eps)
    assert len(np.intersect1d(new, have)) == 0
    assert np.array_equal(grown, both)
    assert np.array_equal(np.union1d(have, new), both)
    # nothing is new when the cloud adds no voxel
    new2, _, grown2, _ = V.voxelize(a, eps, existing=both)
    assert len(new2) == 0 and np.array_equal(grown2, both)


def test_key_order_is_lexicographic():
    rng = np.random.default_rng(10)
    k = rng.integers(-(1 << 20), 1 << 20, (3, 2000))
    k[:, :10] = [[-(1 << 20)], [(1 << 20) - 1], [0]]
    keys = V.pack(k)
    order = sorted(range(k.shape[1]), key=lambda j: tuple(k[:, j].tolist()))
    # keys taken in (x, y, z) tuple order are ascending
    assert all(int(keys[a]) <= int(keys[b]) for a, b in zip(order, order[1:]))
    assert np.array_equal(V.unpack(keys), k)


def test_range_limits():
    eps = 1.0
    lim = float(1 << 20)
    p = np.array([[-lim, lim - 1, lim - 0.5, lim, -lim - 0.5, -lim - 0.6, np.nan, np.inf]] + [[0.0] * 8] * 2,
                 np.float32)
    k, dropped = V.quantise(p, eps)
    # -2^20 and 2^20 - 1 are kept; 2^20 - 0.5 rounds to 2^20 (even) and is dropped;
    # -2^20 - 0.5 rounds to -2^20 (even) and is kept; -2^20 - 0.6 and NaN and inf are dropped
    assert k[0].tolist() == [-(1 << 20), (1 << 20) - 1, -(1 << 20)]
    assert dropped == 5


def test_empty_and_all_dropped():
    new, cen, grown, dropped = V.voxelize(np.zeros((3, 0), np.float32), 0.1)
    assert len(new) == 0 and cen.shape == (3, 0) and dropped == 0
    new, cen, grown, dropped = V.voxelize(np.full((3, 5), np.nan, np.float32), 0.1, existing=np.array([7], np.uint64))
    assert len(new) == 0 and dropped == 5 and grown.tolist() == [7]


def test_fp32_decision_at_near_ties():
    # points whose exact quotient p / eps is not a half-integer but whose FP32 quotient
    # is one: the FP32 decision (ties to even) differs from rounding the exact quotient
    eps = np.float32(0.1)
    cand = []
    for k in range(500, 900):
        base = np.float32((k + 0.5) * float(eps))
        for d in range(-3, 4):
            p = np.nextafter(base, np.float32(np.inf * d), dtype=np.float32) if d else base
            for _ in range(abs(d) - 1):
                p = np.nextafter(p, np.float32(np.inf * d), dtype=np.float32)
            q32 = np.float32(p) / eps
            exact = Fraction(float(p)) / Fraction(float(eps))
            if q32 == np.floor(q32) + 0.5 and exact != Fraction(int(np.floor(q32))) + Fraction(1, 2):
                cand.append(float(p))
    assert len(cand) >= 20
    pts = np.array([cand] * 3, np.float32)
    want, dropped = _brute_voxels(pts, float(eps))
    k, d = V.quantise(pts, float(eps))
    assert d == dropped == 0
    assert {tuple(t) for t in k.T.tolist()} == want
    # rounding the exact quotient instead would move some of them
    exact_k = [round(Fraction(c) / Fraction(float(eps))) for c in cand]
    assert exact_k != k[0].tolist()


def test_growth_bookkeeping():
    rng = np.random.default_rng(12)
    A, F, K = 40, 5, 3
    part_begin = [0, 15, 15, 32, 40]  # an empty partition too
    pos = rng.normal(size=(3, A)).astype(np.float32)
    feat = rng.normal(size=(A, F)).astype(np.float32)
    ls = rng.normal(size=A).astype(np.float32)
    offs = rng.normal(size=(3, A * K)).astype(np.float32)
    cen = rng.normal(size=(3, 6)).astype(np.float32)
    for part in range(4):
        pos2, feat2, ls2, offs2, pb = V.grow_anchors(pos, feat, ls, offs, part_begin, part, cen, 0.25)
        at = part_begin[part + 1]
        assert pb.tolist() == [b + (6 if i > part else 0) for i, b in enumerate(part_begin)]
        # every old anchor keeps its values (and its K offsets) at its new index
        new_idx = [a if a < at else a + 6 for a in range(A)]
        assert np.array_equal(pos2[:, new_idx], pos) and np.array_equal(feat2[new_idx], feat)
        assert np.array_equal(ls2[new_idx], ls)
        o2 = offs2.reshape(3, A + 6, K)
        assert np.array_equal(o2[:, new_idx], offs.reshape(3, A, K))
        # the new anchors close the partition's range, initialised from the points
        assert np.array_equal(pos2[:, at:at + 6], cen)
        assert (feat2[at:at + 6] == 0).all() and (o2[:, at:at + 6] == 0).all()
        assert np.allclose(ls2[at:at + 6], np.log(0.25), rtol=1e-7)
        # partition ranges: same anchors per partition, plus the new ones in `part`
        for q in range(4):
            old = pos[:, part_begin[q]:part_begin[q + 1]]
            got = pos2[:, pb[q]:pb[q + 1]]
            want = np.concatenate([old, cen], axis=1) if q == part else old
            assert np.array_equal(got, want)
