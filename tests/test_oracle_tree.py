"""Pins of the oracle's octree, Morton keys and interaction lists.

Checks: hand-computed keys, containment invariants, O(cells^2) brute-force
enumeration of the near and far lists (written independently here from the
separation rule), list symmetry, the paper's structural constants and closed
forms for the number of M2L pairs in a full grid.
"""
import itertools
import json
import os

import numpy as np
import pytest

from paper_1206_0115_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def decode(keys, bits):
    keys = np.asarray(keys, dtype=np.uint64)
    c = np.zeros((len(keys), 3), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            c[:, d] |= ((keys >> np.uint64(3 * b + d)) & np.uint64(1)).astype(np.int64) << b
    return c


def test_octant_centre_keys(orc):
    # 8 points at the octant centres of a cube; h = 2 gives one leaf per
    # octant and key = xbit + 2*ybit + 4*zbit
    pts = np.array([[x, y, z] for z in (0.25, 0.75) for y in (0.25, 0.75)
                    for x in (0.25, 0.75)])
    order = np.random.default_rng(1).permutation(8)
    t = orc.Tree(pts[order], 2)
    keys = t.keys()
    assert list(keys) == list(range(8))
    # the particle with key k is the k-th octant centre
    np.testing.assert_array_equal(pts[order][t.perm()], pts)


def test_hand_computed_key(orc):
    # box fixed to [0,1]^3 by two corner points; h = 3 (4 leaves per side);
    # (0.3, 0.6, 0.9) -> k = (1, 2, 3) -> bits: b0: x=1,z=1 -> 1+4; b1: y=1,z=1 -> 16+32
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.3, 0.6, 0.9]])
    t = orc.Tree(pts, 3)
    keys = t.keys()
    perm = t.perm()
    assert keys[list(perm).index(2)] == 53
    assert keys[list(perm).index(0)] == 0
    assert keys[list(perm).index(1)] == 63  # top corner clamps to k = 3 in every dim


@pytest.mark.parametrize("kind,n,h", [("cube", 3000, 4), ("sphere", 4000, 5), ("cube", 100, 6)])
def test_sort_csr_and_containment(orc, kind, n, h):
    pos, q = inputs.make(kind, n, 11)
    t = orc.Tree(pos, h)
    keys, perm, start = t.keys(), t.perm(), t.leaf_start()
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.all(keys[1:] >= keys[:-1])
    same = keys[1:] == keys[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])  # ties by original index
    assert start[0] == 0 and start[-1] == n and np.all(np.diff(start) > 0)
    lk = keys[start[:-1]]
    assert np.all(lk[1:] > lk[:-1])
    np.testing.assert_array_equal(lk, t.cell_keys(h - 1))
    # every particle lies inside its leaf box
    w = t.L / 2 ** (h - 1)
    c = decode(keys, h - 1)
    x = pos[perm]
    lo = t.lo + c * w
    assert np.all(x >= lo - 1e-12) and np.all(x <= lo + w + 1e-12)
    # bounding cube: anchored at the per-axis minimum, side = max extent
    np.testing.assert_array_equal(t.lo, pos.min(axis=0))
    assert t.L == (pos.max(axis=0) - pos.min(axis=0)).max()
    # coarser levels are the unique shifted leaf keys
    for lv in range(h - 1):
        np.testing.assert_array_equal(t.cell_keys(lv),
                                      np.unique(lk >> np.uint64(3 * (h - 1 - lv))))


def brute_lists(keys_level, level):
    c = decode(keys_level, level)
    d = np.abs(c[:, None, :] - c[None, :, :]).max(axis=2)
    dp = np.abs((c[:, None, :] >> 1) - (c[None, :, :] >> 1)).max(axis=2)
    near = d <= 1
    far = (dp <= 1) & (d >= 2)
    return near, far


def csr_to_dense(off, idx, n):
    m = np.zeros((n, n), dtype=bool)
    for a in range(n):
        m[a, idx[off[a]:off[a + 1]]] = True
    return m


@pytest.mark.parametrize("kind,n,h", [("cube", 2000, 4), ("sphere", 3000, 5), ("cube", 800, 5)])
def test_lists_against_brute_force(orc, kind, n, h):
    pos, _ = inputs.make(kind, n, 21)
    t = orc.Tree(pos, h)
    off, idx = t.near()
    lk = t.cell_keys(h - 1)
    near, _ = brute_lists(lk, h - 1)
    assert np.array_equal(csr_to_dense(off, idx, t.n_leaf), near)
    for a in range(t.n_leaf):  # ascending index = ascending key
        assert np.all(np.diff(idx[off[a]:off[a + 1]]) > 0)
    assert np.diff(off).max() <= GOLD["near_cells_max"]["value"]
    for lv in range(2, h):
        foff, fidx = t.far(lv)
        _, far = brute_lists(t.cell_keys(lv), lv)
        dense = csr_to_dense(foff, fidx, t.ncell[lv])
        assert np.array_equal(dense, far)
        assert np.array_equal(dense, dense.T)  # B in far(A) <=> A in far(B)
        assert np.diff(foff).max() <= GOLD["far_cells_max"]["value"]
        for a in range(t.ncell[lv]):
            assert np.all(np.diff(fidx[foff[a]:foff[a + 1]]) > 0)


def full_grid(h):
    s = 2 ** (h - 1)
    g = (np.stack(np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij"),
                  -1).reshape(-1, 3) + 0.5) / s
    return g


def test_full_grid_pair_counts(orc):
    # one particle per leaf of a height-5 tree: every cell of every level is
    # present.  Per dimension the sum over cells of the candidate count is
    # 4 (3(n/2) - 2) = 6n - 8 and of the adjacent count 3n - 2, so the number
    # of M2L pairs at a level with n cells per side is (6n-8)^3 - (3n-2)^3.
    h = 5
    t = orc.Tree(full_grid(h), h)
    expect = {2: 3096, 3: 53352, 4: 584136}
    for lv in range(2, h):
        n = 2 ** lv
        off, idx = t.far(lv)
        assert off[-1] == (6 * n - 8) ** 3 - (3 * n - 2) ** 3 == expect[lv]
        # from level 3 on, interior cells have exactly the paper's 189 far cells
        if lv >= 3:
            assert np.diff(off).max() == GOLD["far_cells_max"]["value"]
    noff, _ = t.near()
    n = 2 ** (h - 1)
    assert noff[-1] == (3 * n - 2) ** 3
    assert np.diff(noff).max() == GOLD["near_cells_max"]["value"]


def test_316_offsets_in_16_classes(orc):
    h = 5
    t = orc.Tree(full_grid(h), h)
    lv = 4
    c = decode(t.cell_keys(lv), lv)
    off, idx = t.far(lv)
    offs = set()
    for a in range(t.ncell[lv]):
        for b in idx[off[a]:off[a + 1]]:
            offs.add(tuple(c[b] - c[a]))
    assert len(offs) == GOLD["m2l_offsets"]["value"]
    # orbits under the 48 axis permutations and reflections of the cube
    group = [(p, s) for p in itertools.permutations(range(3))
             for s in itertools.product((1, -1), repeat=3)]
    assert len(group) == 48
    seen, classes = set(), []
    for o in sorted(offs):
        if o in seen:
            continue
        orbit = {tuple(s[d] * o[p[d]] for d in range(3)) for p, s in group}
        assert orbit <= offs
        seen |= orbit
        classes.append(len(orbit))
    assert len(classes) == GOLD["m2l_canonical"]["value"]
    assert sum(classes) == 316
    assert sorted(classes) == sorted([6, 24, 24, 12, 24, 8, 6, 24, 24, 24, 48, 24, 12, 24, 24, 8])
    # every child parity sees exactly 189 offsets
    for p in itertools.product((0, 1), repeat=3):
        cnt = sum(1 for o in offs if all(-2 - p[d] <= o[d] <= 3 - p[d] for d in range(3)))
        assert cnt == 189


def test_invalid_inputs_rejected(orc):
    with pytest.raises(ValueError):
        orc.Tree(np.array([[0.0, np.nan, 0.0]]), 3)
    with pytest.raises(ValueError):
        orc.Tree(np.zeros((4, 3)), 0)
    t = orc.Tree(np.zeros((4, 3)), 3)  # all coincident: L := 1, one leaf
    assert t.L == 1.0 and t.n_leaf == 1
