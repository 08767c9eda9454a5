"""Pins for the oracle's Morton keys (tree cubes of the oct-tree, paper Sec. 2.1).

Checked against an independent brute-force construction (binary strings interleaved by
hand), a de-interleave round trip, and the level-k prefix identity
key >> 3(21-k) == floor(x * fl(2^k / L)).
"""
import numpy as np
import pytest

import dzs_ics
import oracle


def _brute_key(x, y, z, L):
    s = 2.0 ** 21 / L
    idx = []
    for v in (x, y, z):
        i = int(np.floor(v * s))
        idx.append(min(max(i, 0), 2 ** 21 - 1))
    bx, by, bz = (format(i, "021b") for i in idx)
    # most significant digit first: (x_j, y_j, z_j) for j = 20 .. 0
    return int("".join(a + b + c for a, b, c in zip(bx, by, bz)), 2)


def _deinterleave(key):
    ix = iy = iz = 0
    for j in range(21):
        ix |= ((key >> (3 * j + 2)) & 1) << j
        iy |= ((key >> (3 * j + 1)) & 1) << j
        iz |= ((key >> (3 * j)) & 1) << j
    return ix, iy, iz


@pytest.mark.parametrize("L", [100.0, 256.0, 1000.0, 3.0])
def test_keys_match_bruteforce(L):
    ps = dzs_ics.uniform_random(500, L, seed=11)
    keys = oracle.morton_keys(ps.x, ps.y, ps.z, L)
    for i in range(ps.n):
        assert int(keys[i]) == _brute_key(ps.x[i], ps.y[i], ps.z[i], L)


def test_keys_edges_and_roundtrip():
    L = 100.0
    xs = np.array([0.0, np.nextafter(L, 0), L * 0.5, np.nextafter(L * 0.5, 0), 1e-300, 37.25])
    ys = np.array([np.nextafter(L, 0), 0.0, 12.5, 99.999, 50.0, 0.0])
    zs = np.array([50.0, 50.0, np.nextafter(L, 0), 0.0, 0.0, 88.0])
    keys = oracle.morton_keys(xs, ys, zs, L)
    s = 2.0 ** 21 / L
    for i in range(xs.size):
        assert int(keys[i]) == _brute_key(xs[i], ys[i], zs[i], L)
        ix, iy, iz = _deinterleave(int(keys[i]))
        for v, got in zip((xs[i], ys[i], zs[i]), (ix, iy, iz)):
            assert got == min(int(np.floor(v * s)), 2 ** 21 - 1)
    # the top corner cell is the last key
    assert int(keys[0]) < 2 ** 63


def test_level_prefix_is_floor_of_scaled_position():
    L = 256.0
    ps = dzs_ics.clustered_random(4000, L, seed=3)
    keys = oracle.morton_keys(ps.x, ps.y, ps.z, L)
    for k in (0, 1, 3, 7, 12, 21):
        pre = keys >> np.uint64(3 * (21 - k))
        sk = 2.0 ** k / L
        cx = np.minimum(np.floor(ps.x * sk), 2 ** k - 1).astype(np.int64)
        cy = np.minimum(np.floor(ps.y * sk), 2 ** k - 1).astype(np.int64)
        cz = np.minimum(np.floor(ps.z * sk), 2 ** k - 1).astype(np.int64)
        for i in range(0, ps.n, 7):
            ix, iy, iz = _deinterleave(int(pre[i]))
            assert (ix, iy, iz) == (cx[i], cy[i], cz[i])


def test_keys_sorted_order_is_octree_preorder():
    """Sorting by key visits octants depth-first: each level-k cube is one contiguous run."""
    L = 64.0
    ps = dzs_ics.clustered_random(3000, L, seed=5)
    keys = np.sort(oracle.morton_keys(ps.x, ps.y, ps.z, L))
    for k in (1, 2, 4, 6):
        pre = keys >> np.uint64(3 * (21 - k))
        change = np.nonzero(np.diff(pre))[0]
        runs = np.split(pre, change + 1)
        firsts = [r[0] for r in runs]
        assert len(set(firsts)) == len(firsts)  # no cube appears in two runs
