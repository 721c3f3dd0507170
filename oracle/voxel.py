"""Oracle of anchor voxelisation and growth (Eq. 4, Sec. III-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The fused point cloud P (tracked points and triangulated flow points) is snapped to the
grid of voxel size eps; the anchors are the unique voxels, V = {round(P / eps)} eps.
Growth at a keyframe keeps the voxels that are not anchors yet.  Written as that
definition: per point and axis the quotient p / eps in FP32 (the precision of the
positions; NumPy's float32 division is IEEE correctly rounded) rounded to the nearest
integer with ties to even (np.rint), then set operations on the integer triples.

Interface format (shared with the library's declaration, not arithmetic of the method):
k must lie in [-2^20, 2^20) on every axis, else the point is dropped (NaN coordinates
too); a voxel is identified by the 63-bit key (k_x + 2^20) << 42 | (k_y + 2^20) << 21 |
(k_z + 2^20), whose order is the lexicographic order of (k_x, k_y, k_z); its centre is the
FP32 product k eps.

Pins (tests/test_oracle_voxel.py): brute force with exact rational quotients
(fractions.Fraction) and Python's ties-to-even round() on small clouds; points jittered
around known lattice points recover exactly those lattice points; ties at half-integers
go to the even neighbour; every point lies within half a voxel of its voxel's centre
and every voxel holds a point; re-voxelising the centres is the identity; growth is a
set difference whose union with the existing keys equals the voxels of the union of
the clouds; keys sort as (x, y, z) tuples.  grow_anchors (the bookkeeping) is pinned by
its invariants (old anchors keep their values, offsets and partition; the new ones
close their partition's range; offsets shift); the new anchors' initial values (zero
features and offsets, log-scale ln eps) are a stated definition: parity unpinned.
"""
from __future__ import annotations

import math

import numpy as np

KEY_BITS = 21
KEY_OFF = 1 << (KEY_BITS - 1)
_MASK = (1 << KEY_BITS) - 1


def quantise(points, eps):
    """Integer voxel coordinates [3][m] (int64) of the points [3][n] that are kept, and
    the number dropped (out of range or NaN)."""
    p = np.asarray(points, np.float32)
    q = np.rint(p / np.float32(eps))  # float32 quotient, nearest integer, ties to even
    with np.errstate(invalid="ignore"):
        ok = np.all((q >= -KEY_OFF) & (q < KEY_OFF), axis=0)
    return q[:, ok].astype(np.int64), int((~ok).sum())


def pack(k):
    """Keys (uint64) of integer voxel coordinates [3][m]."""
    k = np.asarray(k, np.int64)
    u = (k + KEY_OFF).astype(np.uint64)
    return (u[0] << np.uint64(2 * KEY_BITS)) | (u[1] << np.uint64(KEY_BITS)) | u[2]


def unpack(keys):
    """Integer voxel coordinates [3][m] of keys."""
    u = np.asarray(keys, np.uint64)
    m = np.uint64(_MASK)
    return np.stack([(u >> np.uint64(2 * KEY_BITS)) & m, (u >> np.uint64(KEY_BITS)) & m, u & m]).astype(np.int64) - KEY_OFF


def centres(keys, eps):
    """Voxel centres [3][m] float32: k eps as an FP32 product."""
    return unpack(keys).astype(np.float32) * np.float32(eps)


def voxelize(points, eps, existing=None):
    """Eq. 4 and the growth step.  Returns (new keys ascending, their centres [3][m],
    the ascending key set after growth, number of dropped points)."""
    k, dropped = quantise(points, eps)
    voxels = set(pack(k).tolist())                       # the unique voxels of the cloud
    have = set() if existing is None else set(np.asarray(existing, np.uint64).tolist())
    new = np.array(sorted(voxels - have), np.uint64)
    grown = np.array(sorted(voxels | have), np.uint64)
    return new, centres(new, eps), grown, dropped


def grow_anchors(pos, feat, log_scale, offs, part_begin, partition, centres, eps):
    """Growth bookkeeping (Sec. III-A with the partitions of Eq. 6): the new anchors at
    the voxel centres [3][n] join `partition`, inserted at the end of its range of the
    partition-grouped arrays pos [3][A], feat [A][F], log_scale [A], offs [3][A*K];
    initialised as an anchor created from points (zero features and offsets, log-scale
    ln(eps)).  Returns the grown arrays and the shifted partition offsets."""
    c = np.asarray(centres, np.float32)
    n = c.shape[1]
    A = pos.shape[1]
    K = offs.shape[1] // A if A else 0
    at = int(part_begin[partition + 1])
    F = feat.shape[1]
    pos2 = np.concatenate([pos[:, :at], c, pos[:, at:]], axis=1)
    feat2 = np.concatenate([feat[:at], np.zeros((n, F), feat.dtype), feat[at:]], axis=0)
    ln_eps = np.float32(math.log(float(np.float32(eps))))  # natural log in double, rounded once
    ls2 = np.concatenate([log_scale[:at], np.full(n, ln_eps, log_scale.dtype), log_scale[at:]])
    offs2 = np.concatenate([offs[:, :at * K], np.zeros((3, n * K), offs.dtype), offs[:, at * K:]], axis=1)
    pb = np.asarray(part_begin, np.int64).copy()
    pb[partition + 1:] += n
    return pos2, feat2, ls2, offs2, pb
