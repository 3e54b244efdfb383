"""Pins of the monopole tree oracle (oracle/tree.py) against what the
mathematics fixes, independent of its own formulas:

* with acceptance off the walk must reach every pair: the result is the
  direct pair sum of the C oracle and the pair count is its count;
* a monopole about the centre of mass has no dipole term, so for two tight
  clusters the monopole error falls with the square of the cluster size
  (a wrong mass, a wrong centre or a dropped shift breaks the ratio);
* the relative test of sec. 3.1 switches at G M B^2 / r^4 = alpha |a|,
  with B and r measured here from the clusters' extents, not from the
  oracle's integer boxes.
"""
import numpy as np

import oracle
from oracle import tree
from workloads import BoxParams
import workloads as W

# Two clusters of 64 particles, each inside its own cell of side L / 32
# (so the key order keeps each cluster contiguous and every 64-particle
# block and level-2 node is one whole cluster with leaf_max = 1).
L = 100.0
CELL5 = L / 32
CA = np.array([8.5, 8.5, 8.5]) * CELL5
CB = np.array([9.5, 8.5, 8.5]) * CELL5
P = BoxParams(L=L, rs=1.5, rcut=4.5 * 1.5, eps=1e-3, leaf_max=1)


def clusters(delta, seed=7):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.5, 0.5, (3, 128))
    pos = np.empty((3, 128))
    pos[:, :64] = CA[:, None] + delta * u[:, :64]
    pos[:, 64:] = CB[:, None] + delta * u[:, 64:]
    mass = rng.uniform(0.5, 1.5, 128).astype(np.float32).astype(np.float64)
    return pos, mass


def test_acceptance_off_is_the_pair_sum():
    rng = np.random.default_rng(11)
    Lb = 40.0
    pos = W.mixture(rng, 3000, Lb, 0.6, 5)
    p = BoxParams(L=Lb, rs=1.2, rcut=5.4, eps=0.02, leaf_max=4)
    mass = rng.uniform(0.5, 1.5, 3000)
    ref = oracle.accel(pos, mass, p)
    got = tree.monopole_accel(pos, mass, p, theta=0.0)
    assert got["n_mono_pairs"] == 0
    assert got["n_pp_pairs"] == int(ref["n_inter"].sum())
    err = np.abs(got["acc"] - ref["acc"]).max() / np.abs(ref["acc"]).max()
    assert err <= 1e-12, err


def monopole_error(delta):
    pos, mass = clusters(delta)
    ref = oracle.accel(pos, mass, P)["acc"]
    got = tree.monopole_accel(pos, mass, P, theta=0.5)
    assert got["n_mono_pairs"] == 128          # each cluster is a monopole for the other
    return np.linalg.norm(got["acc"] - ref, axis=0).max()


def test_monopole_error_is_second_order_in_node_size():
    e = [monopole_error(d) for d in (0.4, 0.2, 0.1)]
    assert 3.3 < e[0] / e[1] < 4.7 and 3.3 < e[1] / e[2] < 4.7, e


def test_relative_criterion_threshold():
    delta = 0.3
    pos, mass = clusters(delta)
    a0 = 2.5
    acc_ref = np.zeros((3, 128))
    acc_ref[1] = a0                               # |a| = a0 for every target
    # threshold alpha* = G M B^2 / (r^4 |a|) of each cluster seen from the
    # other, from the clusters' extents (the integer boxes agree to a cell)
    gap = pos[0, 64:].min() - pos[0, :64].max()
    thr = []
    for src in (slice(0, 64), slice(64, 128)):
        M = mass[src].sum()
        B = (pos[:, src].max(1) - pos[:, src].min(1)).max()
        thr.append(P.G * M * B * B / (gap ** 4 * a0))
    worst, lo = max(thr), min(thr)
    on = tree.monopole_accel(pos, mass, P, theta=0.0, alpha=1.05 * worst, acc_ref=acc_ref)
    off = tree.monopole_accel(pos, mass, P, theta=0.0, alpha=0.95 * lo, acc_ref=acc_ref)
    assert on["n_mono_pairs"] == 128 and off["n_mono_pairs"] == 0
    # with a geometric test that rejects, the relative one alone cannot accept
    both = tree.monopole_accel(pos, mass, P, theta=0.05, alpha=1.05 * worst, acc_ref=acc_ref)
    assert both["n_mono_pairs"] == 0
    # |a| is the block's smallest: one slow target rejects its whole block
    acc_ref[1, 5] = a0 * 1e-3
    one = tree.monopole_accel(pos, mass, P, theta=0.0, alpha=1.05 * worst, acc_ref=acc_ref)
    assert one["n_mono_pairs"] == 64
