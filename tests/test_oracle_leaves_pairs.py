"""Pins for the oracle's octree leaves (sec. 3.2-3.3) and near leaf pairs
(sec. 3.3, N-to-M leaf pairs within the short range).

Leaves: they partition the key-sorted particles into contiguous runs; each
is an octree node (one key prefix, inside one aligned cube); each holds at
most leaf_max particles unless it is a single grid cell; each is maximal
(its parent node holds more than leaf_max).  Parents are recounted here by
binary search on the sorted keys, not by the oracle's recursion.

Pairs: coverage is checked against particle-level brute force in FP64 (every
pair with s < r_cut appears with the right leaves and periodic shift), plus
the symmetry (A, B, s) <-> (B, A, -s), the presence of every (A, A, 0), and a
geometric upper bound showing the list is not simply everything.
"""
import numpy as np
import pytest

from workloads import BoxParams, mixture, rng_for


def leaf_of_particle(lv, n):
    owner = np.zeros(n, dtype=np.int64)
    for a, (b0, c) in enumerate(zip(lv["begin"], lv["count"])):
        owner[b0:b0 + c] = a
    return owner


@pytest.mark.parametrize("n,leaf_max,frac", [(3000, 32, 0.5), (5000, 8, 0.8), (40, 32, 0.0), (1, 32, 0.0)])
def test_leaf_invariants(oracle_mod, n, leaf_max, frac):
    rng = np.random.default_rng(n)
    L, b = 50.0, 21
    pos = mixture(rng, n, L, frac, max(1, n // 400))
    st = oracle_mod.structure(pos, BoxParams(L=L, rs=1.0, rcut=4.5, eps=0.01, leaf_max=leaf_max))
    sk, lv = st["sorted_keys"], st["leaves"]
    # contiguous partition
    assert lv["begin"][0] == 0
    assert np.array_equal(lv["begin"][1:], (lv["begin"] + lv["count"])[:-1])
    assert lv["count"].sum() == n
    for a in range(lv["begin"].size):
        b0, c, lev = lv["begin"][a], lv["count"][a], lv["level"][a]
        keys = sk[b0:b0 + c]
        sh = np.uint64(3 * (b - lev))
        pre = keys >> sh if lev > 0 else np.zeros_like(keys)
        assert (pre == lv["prefix"][a]).all()
        assert c <= leaf_max or lev == b
        # the node is exactly this run: no neighbour shares the prefix
        if lev > 0:
            if b0 > 0:
                assert (sk[b0 - 1] >> sh) != lv["prefix"][a]
            if b0 + c < n:
                assert (sk[b0 + c] >> sh) != lv["prefix"][a]
        # maximality: the parent node holds more than leaf_max
        if lev > 0:
            psh = np.uint64(3 * (b - lev + 1))
            ppre = keys[0] >> psh if lev > 1 else np.uint64(0)
            allp = sk >> psh if lev > 1 else np.zeros_like(sk)
            assert np.count_nonzero(allp == ppre) > leaf_max
        # AABB is tight and inside the node cube
        q = st["q_sorted"][:, b0:b0 + c].astype(np.int64)
        assert np.array_equal(st["lo"][:, a], q.min(axis=1))
        assert np.array_equal(st["hi"][:, a], q.max(axis=1) + 1)
        side = 1 << (b - lev)
        assert ((q.min(axis=1) // side) == (q.max(axis=1) // side)).all()


def test_leaves_small_and_empty(oracle_mod):
    lv = oracle_mod.leaves(np.zeros(0, dtype=np.uint64), 21, 32)
    assert lv["begin"].size == 0
    lv = oracle_mod.leaves(np.arange(32, dtype=np.uint64), 21, 32)
    assert lv["begin"].tolist() == [0] and lv["level"].tolist() == [0]


def test_duplicate_positions_make_deep_fat_leaf(oracle_mod):
    L = 10.0
    pos = np.concatenate([np.full((3, 100), 3.3), np.random.default_rng(0).random((3, 50)) * L], axis=1)
    st = oracle_mod.structure(pos, BoxParams(L=L, rs=0.5, rcut=2.25, eps=0.0, leaf_max=16))
    lv = st["leaves"]
    fat = np.flatnonzero(lv["count"] > 16)
    assert fat.size == 1 and lv["level"][fat[0]] == 21 and lv["count"][fat[0]] == 100


def shift_of_pair(xi, xj, L):
    """Periodic shift s with x_j + s L - x_i the minimum image, per axis."""
    d = xj - xi
    return -np.round(d / L).astype(np.int64)


@pytest.mark.parametrize("n,L,rcut,frac", [(2500, 40.0, 6.0, 0.5), (1200, 30.0, 14.0, 0.3)])
def test_pair_coverage_symmetry_bound(oracle_mod, n, L, rcut, frac):
    rng = np.random.default_rng(int(L))
    pos = mixture(rng, n, L, frac, 3)
    p = BoxParams(L=L, rs=rcut / 4.5, rcut=rcut, eps=0.01, leaf_max=16)
    st = oracle_mod.structure(pos, p)
    lo, hi = st["lo"], st["hi"]
    row_ptr, src, code = oracle_mod.near_pairs(lo, hi, L, rcut)
    m = lo.shape[1]
    listed = set()
    for a in range(m):
        for k in range(row_ptr[a], row_ptr[a + 1]):
            listed.add((a, int(src[k]), int(code[k])))
    # rows are sorted by (source, code)
    for a in range(m):
        seg = list(zip(src[row_ptr[a]:row_ptr[a + 1]].tolist(), code[row_ptr[a]:row_ptr[a + 1]].tolist()))
        assert seg == sorted(seg)
        assert (a, a, 13) in listed
    for (a, bb, c) in listed:
        assert (bb, a, 26 - c) in listed
    # particle-level coverage in FP64
    ps = pos[:, st["perm"]]
    ps = ps - L * np.floor(ps / L)
    owner = leaf_of_particle(st["leaves"], n)
    d = ps[:, None, :] - ps[:, :, None]
    sh = -np.round(d / L)
    d = d + sh * L
    s2 = (d * d).sum(axis=0)
    ii, jj = np.nonzero(s2 < rcut * rcut)
    for i, j in zip(ii.tolist(), jj.tolist()):
        sx, sy, sz = (int(v) for v in sh[:, i, j])
        c = 9 * (sx + 1) + 3 * (sy + 1) + (sz + 1)
        assert (owner[i], owner[j], c) in listed, (i, j)
    # not everything: listed boxes are within r + sqrt(3) grid units
    W = 1 << 21
    r = rcut * W / L
    for (a, bb, c) in list(listed)[:5000]:
        sg = np.array([c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1])
        gap = np.maximum(0, np.maximum(lo[:, bb] + sg * W - hi[:, a], lo[:, a] - hi[:, bb] - sg * W)).astype(float)
        assert np.sqrt((gap ** 2).sum()) < r + 1.0


def test_pair_rows_subset(oracle_mod):
    rng = rng_for(99)
    pos = rng.random((3, 600)) * 20.0
    p = BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01, leaf_max=8)
    st = oracle_mod.structure(pos, p)
    rp, src, code = oracle_mod.near_pairs(st["lo"], st["hi"], p.L, p.rcut)
    rows = np.array([3, 0, 7])
    rp2, src2, code2 = oracle_mod.near_pairs(st["lo"], st["hi"], p.L, p.rcut, rows=rows)
    for t, a in enumerate(rows):
        assert np.array_equal(src2[rp2[t]:rp2[t + 1]], src[rp[a]:rp[a + 1]])
        assert np.array_equal(code2[rp2[t]:rp2[t + 1]], code[rp[a]:rp[a + 1]])
