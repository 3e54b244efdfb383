"""Pins for the oracle's Peano-Hilbert keys (sec. 4.1, a 2^(3b) grid).

The paper prints no key values, so the specific curve is a reading (the
Skilling construction, x most significant); these tests pin that the
oracle's map IS a Hilbert curve of that orientation:
  * bijection onto [0, 8^b) (exhaustive for b <= 5),
  * consecutive keys are face-adjacent cells (the defining property of a
    Hilbert curve; a Morton order or a transposed digit fails it),
  * every 3l-bit key prefix is one aligned cube of side 2^(b-l) (what makes
    octree nodes contiguous, sec. 3.2),
  * the first level visits the octants in reflected binary Gray-code order
    with x as the most significant bit,
  * quantisation: cell boundaries, wrapping and clamping.
"""
import itertools

import numpy as np
import pytest


def all_cells(b):
    c = np.array(list(itertools.product(range(1 << b), repeat=3)), dtype=np.float64).T
    return c


@pytest.mark.parametrize("b", [1, 2, 3, 4, 5])
def test_bijection_adjacency_prefix_cubes(oracle_mod, b):
    cells = all_cells(b)
    L = float(1 << b)
    keys = oracle_mod.hilbert_keys(cells + 0.5, L, b)
    assert sorted(keys.tolist()) == list(range(8 ** b))
    order = np.argsort(keys)
    walk = cells[:, order].astype(np.int64)
    steps = np.abs(np.diff(walk, axis=1)).sum(axis=0)
    assert (steps == 1).all()
    for lev in range(1, b + 1):
        pre = keys >> np.uint64(3 * (b - lev))
        cube = cells.astype(np.int64) >> (b - lev)
        for p in np.unique(pre):
            sel = pre == p
            assert (cube[:, sel] == cube[:, sel][:, :1]).all()
    # decode inverts encode
    q = oracle_mod.hilbert_decode(keys, b)
    assert np.array_equal(q, cells.astype(np.uint32))


def test_top_level_is_gray_code(oracle_mod):
    q = oracle_mod.hilbert_decode(np.arange(8, dtype=np.uint64), 1)
    gray = [k ^ (k >> 1) for k in range(8)]
    assert [(int(q[0, k]) << 2) | (int(q[1, k]) << 1) | int(q[2, k]) for k in range(8)] == gray


def test_21_bit_random_walk_adjacency_and_roundtrip(oracle_mod):
    rng = np.random.default_rng(2)
    b = 21
    k0 = rng.integers(0, 8 ** b - 1, 300, dtype=np.uint64)
    q0 = oracle_mod.hilbert_decode(k0, b).astype(np.int64)
    q1 = oracle_mod.hilbert_decode(k0 + np.uint64(1), b).astype(np.int64)
    assert (np.abs(q1 - q0).sum(axis=0) == 1).all()
    L = 1000.0
    pos = (q0 + 0.5) * (L / 2 ** b)
    assert np.array_equal(oracle_mod.hilbert_keys(pos, L, b), k0)


def test_quantisation_wrap_and_clamp(oracle_mod):
    L, b = 100.0, 21
    W = 1 << b
    pos = np.array([[0.0, 50.0, L - 1e-12, -1e-300, L, 2.5 * L, -0.25 * L]] * 3)
    q = oracle_mod.quantise(pos, L, b)
    assert q[0].tolist() == [0, W // 2, W - 1, W - 1, 0, W // 2, 3 * W // 4]
    # keys of wrapped positions equal keys of the originals (the tiny negative
    # wraps to L itself, which is clamped into the last cell, so skip it)
    keep = [0, 1, 2, 4, 5, 6]
    k = oracle_mod.hilbert_keys(pos[:, keep], L, b)
    kw = oracle_mod.hilbert_keys(pos[:, keep] - L * np.floor(pos[:, keep] / L), L, b)
    assert np.array_equal(k, kw)
