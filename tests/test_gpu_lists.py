"""GPU test of the source lists the FP32 PP kernel reads (pp_plan_lists_export).

The lists are the N-to-M leaf pairs of the dual tree traversal (sec. 3.3)
gathered per target block, in ranges of whole consecutive leaves at one
periodic shift.  Against the oracle (keys, sort, leaves, leaf boxes and the
FP64 in-cut neighbours, none of them from the library) every case checks:

* the key order is the oracle's and the blocks are a valid partition:
  consecutive runs of at most 64 particles inside one 64-particle chunk,
  with the integer box of the oracle's cells of their particles, no wider
  than floor(2 r_cut 2^b / L) cells per axis;
* every range is a run of whole oracle leaves, the ranges tile the block's
  list in order, and the (leaf, shift) pairs of a block are exactly the
  brute-force set of leaves whose box passes the integer near-pair test
  sum_k gap_k^2 < T against the block's box, each once;
* expanded to particles, a block's list holds every FP64 in-cut neighbour
  of each of its targets exactly once (one dropped source or one duplicated
  source fails), and every listed source passes the integer test.
"""
import math

import numpy as np
import pytest

import workloads as W
from workloads import BoxParams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHIFTS = np.array([(c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1) for c in range(27)], dtype=np.int64)


@pytest.fixture(scope="module")
def pp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09824_amd as m
    return m


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def edge_positions(L, rng, n=600):
    pos = rng.random((3, n)) * L
    pos[:, 0] = 0.0
    pos[:, 1] = L - 1e-12
    pos[:, 2] = -1e-300
    pos[:, 3] = L
    pos[:, 4] = 3.5 * L
    pos[:, 5] = -0.75 * L
    pos[:, 6] = L / 2
    return pos


def case(name):
    if name == "cfg1":
        b = W.make_config(1)
        return b.pos, b.params
    if name == "clustered":
        rng = np.random.Generator(np.random.PCG64(11))
        return W.mixture(rng, 20000, 80.0, 0.8, 15), BoxParams(L=80.0, rs=1.0, rcut=4.5, eps=0.02, leaf_max=8)
    if name == "duplicates":
        rng = np.random.default_rng(5)
        pos = np.concatenate([np.full((3, 300), 12.25), rng.random((3, 3000)) * 40.0], axis=1)
        return pos, BoxParams(L=40.0, rs=1.0, rcut=4.5, eps=0.0, leaf_max=16)
    if name == "edge-wrap":
        return edge_positions(37.5, np.random.default_rng(12)), BoxParams(L=37.5, rs=1.0, rcut=4.5, eps=0.01, leaf_max=8)
    if name == "bits4":
        rng = np.random.Generator(np.random.PCG64(9))
        return W.mixture(rng, 3000, 30.0, 0.7, 3), BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.01, key_bits=4)
    raise KeyError(name)


def gap2(blo, bhi, llo, lhi, W_):
    """Integer near-pair test quantity of a block box against every leaf box
    and every shift: [27, nleaf] int64."""
    sh = SHIFTS[:, :, None] * W_                                  # [27, 3, 1]
    g1 = llo[None] + sh - bhi[None, :, None]
    g2 = blo[None, :, None] - lhi[None] - sh
    g = np.maximum(np.maximum(g1, g2), 0)
    return (g * g).sum(axis=1)


@pytest.mark.parametrize("name", ["cfg1", "clustered", "duplicates", "edge-wrap", "bits4"])
def test_kernel_lists_cover_every_neighbour_once(pp, oracle_mod, name):
    pos, p = case(name)
    n = pos.shape[1]
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    plan = pp.Plan(p, n)
    plan.accel(dev(pos, torch.float64), dev(mass, torch.float32))
    lists = plan.export_lists()

    st = oracle_mod.structure(pos, p)
    perm = st["perm"]
    assert np.array_equal(lists["perm"].astype(np.int64), perm)
    q = st["q_sorted"].astype(np.int64)                          # cells, key order
    lbeg = st["leaves"]["begin"]
    lend = lbeg + st["leaves"]["count"]
    llo, lhi = st["lo"], st["hi"]
    W_ = 1 << p.key_bits
    r = p.rcut * W_ / p.L
    T = math.ceil(r * r)
    emax = math.floor(2.0 * p.rcut * W_ / p.L)

    # blocks: a partition of the key order into valid runs
    bs, bc = lists["bstart"].astype(np.int64), lists["bcount"].astype(np.int64)
    nb = bs.size
    assert bs[0] == 0 and np.array_equal(bs[1:], (bs + bc)[:-1]) and bs[-1] + bc[-1] == n
    assert np.all((bc >= 1) & (bc <= 64))
    assert np.all(bs // 64 == (bs + bc - 1) // 64)
    for b in range(nb):
        qb = q[:, bs[b]:bs[b] + bc[b]]
        assert np.array_equal(lists["blo"][:, b], qb.min(axis=1)), b
        assert np.array_equal(lists["bhi"][:, b], qb.max(axis=1) + 1), b
    assert np.all(lists["bhi"].astype(np.int64) - lists["blo"] <= emax)

    # the oracle's in-cut neighbours of every target, keyed (source, shift)
    rp, nbr, code = oracle_mod.neighbours(pos, p)
    leaf_of_begin = {int(v): i for i, v in enumerate(lbeg)}
    leaf_of_end = {int(v): i for i, v in enumerate(lend)}
    roff, rbeg, rpre, rcode = lists["roff"], lists["rbeg"], lists["rpre"], lists["rcode"]
    slen = lists["slen"].astype(np.int64)
    for b in range(nb):
        r0, r1 = int(roff[b]), int(roff[b + 1])
        pre = np.append(rpre[r0:r1].astype(np.int64), slen[b])
        ln = np.diff(pre)
        assert r1 == r0 or (pre[0] == 0 and np.all(ln > 0)), b
        # ranges of whole leaves -> the block's (leaf, shift) set
        pairs = []
        for k in range(r1 - r0):
            a0, a1 = int(rbeg[r0 + k]), int(rbeg[r0 + k]) + int(ln[k])
            assert a0 in leaf_of_begin and a1 in leaf_of_end, (b, k)
            for leaf in range(leaf_of_begin[a0], leaf_of_end[a1] + 1):
                pairs.append(leaf * 27 + int(rcode[r0 + k]))
        pairs = np.array(pairs, dtype=np.int64)
        assert np.unique(pairs).size == pairs.size, b
        g = gap2(lists["blo"][:, b].astype(np.int64), lists["bhi"][:, b].astype(np.int64), llo, lhi, W_)
        want = np.nonzero((g < T).T.reshape(-1))[0]               # leaf * 27 + code, ascending
        assert np.array_equal(np.sort(pairs), want), b
        # particles: every neighbour of every target listed exactly once
        src = np.concatenate([np.arange(int(rbeg[r0 + k]), int(rbeg[r0 + k]) + int(ln[k]))
                              for k in range(r1 - r0)]) if r1 > r0 else np.zeros(0, np.int64)
        cod = np.repeat(rcode[r0:r1].astype(np.int64), ln)
        keys = perm[src] * 27 + cod
        assert np.unique(keys).size == keys.size, b
        tgt = perm[bs[b]:bs[b] + bc[b]]
        need = np.concatenate([nbr[rp[i]:rp[i + 1]] * 27 + code[rp[i]:rp[i + 1]] for i in tgt])
        assert np.all(np.isin(need, keys)), b
