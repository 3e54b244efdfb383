"""Pins of the dual-tree-traversal oracle (oracle/tree.py) against what the
paper's definitions and the mathematics fix, independent of its code:

* with both acceptance tests off the walk must reach every pair: the result
  is the direct pair sum of the C oracle and the pair count is its count;
  the tree's leaves are the C oracle's leaves;
* the geometric test of sec. 3.3 switches where theta1 = (A + B) / R crosses
  theta, with A, B the cube sides and R the distance of the cube centres
  known from how the clusters were placed: a test of theta2 alone, R taken
  as the gap between the cubes or between the centres of mass, or sides
  taken from the particles' extent would switch elsewhere; the same holds
  across the periodic boundary;
* a monopole about the centre of mass has no dipole term, so for two tight
  clusters the monopole error falls with the square of the cluster size (a
  wrong mass, a wrong centre or a dropped shift breaks the ratio);
* the relative test of sec. 3.1 switches at G M l^2 / s^4 = alpha |a| for the
  worst target of the leaf, with s measured here from the positions and l
  the cube side by construction; one slow target holds its whole leaf back.
"""
import numpy as np

import oracle
from oracle import tree
from workloads import BoxParams
import workloads as W

L = 100.0
C5 = L / 32                     # side of a level-5 cube


def in_cube(rng, idx, n, frac=0.5, offset=(0.0, 0.0, 0.0)):
    """n points inside the level-5 cube idx, within the central `frac` of
    its side, moved by `offset` (in cube sides)."""
    u = rng.uniform(-0.5, 0.5, (3, n)) * frac
    c = (np.asarray(idx, dtype=np.float64) + 0.5 + np.asarray(offset))[:, None]
    return (c + u) * C5


def two_clusters(k=7, n=8, seed=3, wrap=False):
    """Cluster A in cube (8, 8, 8) (or (2, 8, 8) with wrap), cluster B k cubes
    further along x (through the boundary with wrap), each with one filler
    particle in a sibling cube so that every level-5 cube is its own leaf at
    leaf_max = n.  B is pushed towards +x inside its cube (its centre of mass
    is not the cube centre)."""
    rng = np.random.default_rng(seed)
    ia = 2 if wrap else 8
    ib = (ia - k) % 32 if wrap else ia + k
    A = in_cube(rng, (ia, 8, 8), n)
    B = in_cube(rng, (ib, 8, 8), n, offset=(0.2, 0.0, 0.0))
    fa = in_cube(rng, (ia ^ 1, 9, 9), 1)
    fb = in_cube(rng, (ib ^ 1, 9, 9), 1)
    pos = np.concatenate([A, B, fa, fb], axis=1)
    mass = rng.uniform(0.5, 1.5, pos.shape[1])
    return pos, mass


P2 = BoxParams(L=L, rs=6.0, rcut=27.0, eps=1e-3, leaf_max=8)


def leaf_of(tr, particle):
    """The tree leaf holding input particle `particle`."""
    k = int(np.nonzero(tr.order == particle)[0][0])
    for i in tr.leaves():
        nd = tr.nodes[i]
        if nd.begin <= k < nd.end:
            return i
    raise AssertionError


def pair_accepted(res, a, b):
    return any(x == a and y == b for x, y, _ in res["accepted"])


def test_acceptance_off_is_the_pair_sum():
    rng = np.random.default_rng(11)
    Lb = 40.0
    pos = W.mixture(rng, 3000, Lb, 0.6, 5)
    p = BoxParams(L=Lb, rs=1.2, rcut=5.4, eps=0.02, leaf_max=4)
    mass = rng.uniform(0.5, 1.5, 3000)
    ref = oracle.accel(pos, mass, p)
    got = tree.dtt_accel(pos, mass, p)
    assert got["n_mono_pairs"] == 0 and not got["accepted"]
    assert got["n_pp_pairs"] == int(ref["n_inter"].sum())
    err = np.abs(got["acc"] - ref["acc"]).max() / np.abs(ref["acc"]).max()
    assert err <= 1e-12, err
    tr = got["tree"]
    lv = oracle.leaves(tr.keys, p.key_bits, p.leaf_max)
    assert np.array_equal([tr.nodes[i].begin for i in tr.leaves()], lv["begin"])
    assert np.array_equal([tr.nodes[i].end - tr.nodes[i].begin for i in tr.leaves()], lv["count"])


def test_leaves_sit_in_their_cubes():
    pos, mass = two_clusters()
    tr = tree.Tree(pos, mass, P2)
    a, b = leaf_of(tr, 0), leaf_of(tr, 8)
    for i, idx in ((a, (8, 8, 8)), (b, (15, 8, 8))):
        nd = tr.nodes[i]
        assert nd.level == 5 and nd.end - nd.begin == 8
        assert np.allclose(nd.flo, np.asarray(idx) * C5) and np.isclose(nd.width, C5)


def theta_star():
    return 2.0 * C5 / (7 * C5)       # (A + B) / R with R = 7 cube sides between the centres


def test_theta_threshold_from_cube_geometry():
    pos, mass = two_clusters()
    tr = tree.Tree(pos, mass, P2)
    a, b = leaf_of(tr, 0), leaf_of(tr, 8)
    th = theta_star()
    # theta2 = B / (R - A) = 1/6 and the gap-based (A + B) / gap = 1/3 lie on
    # either side of theta1 = 2/7: only theta1 switches between these two
    on = tree.dtt_accel(pos, mass, P2, theta=th * 1.001, tree=tr)
    off = tree.dtt_accel(pos, mass, P2, theta=th * 0.999, tree=tr)
    assert pair_accepted(on, a, b) and pair_accepted(on, b, a)
    assert not pair_accepted(off, a, b) and not pair_accepted(off, b, a)
    # the centre of mass of B lies 0.2 cube sides beyond its cube centre, so a
    # distance between centres of mass would switch at 2 / 7.2 < 0.999 theta*
    # (rejected above) ; the clusters span half a cube, so sides from the
    # particles' extent would switch at 1 / 7 (also rejected above)
    th1, th2 = tree.opening_angles(tr, a, b, (0, 0, 0))
    assert np.isclose(th1, th) and np.isclose(th2, 1.0 / 6.0)


def test_theta_threshold_across_the_boundary():
    pos, mass = two_clusters(wrap=True)
    tr = tree.Tree(pos, mass, P2)
    a, b = leaf_of(tr, 0), leaf_of(tr, 8)
    th = theta_star()
    on = tree.dtt_accel(pos, mass, P2, theta=th * 1.001, tree=tr)
    off = tree.dtt_accel(pos, mass, P2, theta=th * 0.999, tree=tr)
    shifts = {s for x, y, s in on["accepted"] if x == a and y == b}
    assert shifts == {(-1, 0, 0)}
    assert not pair_accepted(off, a, b)
    # the accepted monopole acts from B's image: the change it makes to A's
    # targets is small against the force B's particles exert on them
    assert_monopole_close(pos, mass, on, off)


def assert_monopole_close(pos, mass, on, off, tol=0.05):
    """(on - off) on cluster A's targets is the monopole's force minus the
    exact force of B's particles; compare it with that exact force, from the
    C oracle as the sum over A and B minus the sum over A alone."""
    ab = oracle.accel(pos[:, :16], mass[:16], P2)["acc"][:, :8]
    a_only = oracle.accel(pos[:, :8], mass[:8], P2)["acc"]
    fb = ab - a_only
    diff = on["acc"][:, :8] - off["acc"][:, :8]
    e = np.linalg.norm(diff, axis=0) / np.linalg.norm(fb, axis=0)
    assert e.max() < tol, e


def test_acceptance_keeps_the_force_close():
    """Accepting B for A replaces B's particles by one particle at their
    centre of mass: the targets of A see nearly the same force from B."""
    pos, mass = two_clusters()
    tr = tree.Tree(pos, mass, P2)
    on = tree.dtt_accel(pos, mass, P2, theta=theta_star() * 1.001, tree=tr)
    off = tree.dtt_accel(pos, mass, P2, theta=theta_star() * 0.999, tree=tr)
    assert on["n_mono_pairs"] >= 16
    assert_monopole_close(pos, mass, on, off)


# Two clusters of 64 particles in level-5 cubes whose centres are three cube
# sides apart (theta1 = 2/3), with a filler beside each (leaf_max = 64), well
# inside the cut: theta = 0.7 accepts each for the other at every cluster
# size below.
PS = BoxParams(L=L, rs=2.8, rcut=4.5 * 2.8, eps=1e-3, leaf_max=64)


def shrinking_clusters(delta, seed=7):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.5, 0.5, (3, 128))
    ca = (np.array([8.5, 8.5, 8.5]) * C5)[:, None]
    cb = (np.array([11.5, 8.5, 8.5]) * C5)[:, None]
    pos = np.concatenate([ca + delta * u[:, :64], cb + delta * u[:, 64:],
                          in_cube(rng, (9, 9, 9), 1), in_cube(rng, (10, 9, 9), 1)], axis=1)
    mass = rng.uniform(0.5, 1.5, 130)
    return pos, mass


def monopole_error(delta):
    pos, mass = shrinking_clusters(delta)
    ref = oracle.accel(pos, mass, PS)["acc"]
    got = tree.dtt_accel(pos, mass, PS, theta=0.7)
    tr = got["tree"]
    a, b = leaf_of(tr, 0), leaf_of(tr, 64)
    assert pair_accepted(got, a, b) and pair_accepted(got, b, a)
    return np.linalg.norm(got["acc"][:, :128] - ref[:, :128], axis=0).max()


def test_monopole_error_is_second_order_in_cluster_size():
    e = [monopole_error(d) for d in (0.8, 0.4, 0.2)]
    assert 3.3 < e[0] / e[1] < 4.7 and 3.3 < e[1] / e[2] < 4.7, e


def test_relative_criterion_threshold():
    pos, mass = two_clusters()
    tr = tree.Tree(pos, mass, P2)
    a, b = leaf_of(tr, 0), leaf_of(tr, 8)
    a0 = 2.5
    acc_ref = np.zeros((3, pos.shape[1]))
    acc_ref[1] = a0                               # |a| = a0 for every target
    # threshold alpha* = max over A's targets of G M l^2 / (s^4 |a|): M the
    # mass of B, l its cube side, s the target's distance to B's centre of mass
    mB = mass[8:16]
    com = (pos[:, 8:16] * mB).sum(axis=1) / mB.sum()
    s = np.linalg.norm(pos[:, :8] - com[:, None], axis=0)
    thr = (P2.G * mB.sum() * C5 ** 2 / (s ** 4 * a0)).max()
    on = tree.dtt_accel(pos, mass, P2, alpha=1.001 * thr, acc_ref=acc_ref, tree=tr)
    off = tree.dtt_accel(pos, mass, P2, alpha=0.999 * thr, acc_ref=acc_ref, tree=tr)
    assert pair_accepted(on, a, b) and not pair_accepted(off, a, b)
    # with a geometric test that rejects, the relative one alone cannot accept
    both = tree.dtt_accel(pos, mass, P2, theta=0.05, alpha=1.001 * thr, acc_ref=acc_ref, tree=tr)
    assert not pair_accepted(both, a, b)
    # every target of A must pass: one slow target holds the leaf back
    acc_ref[1, 3] = a0 * 1e-3
    one = tree.dtt_accel(pos, mass, P2, alpha=1.001 * thr, acc_ref=acc_ref, tree=tr)
    assert not pair_accepted(one, a, b)


def test_nodes_holding_the_target_are_never_taken():
    """With huge acceptance parameters only nodes apart from the target leaf
    are taken: never the leaf itself or one of its ancestors."""
    rng = np.random.default_rng(5)
    pos = W.mixture(rng, 800, 30.0, 0.5, 3)
    p = BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.01, leaf_max=4)
    mass = rng.uniform(0.5, 1.5, 800)
    got = tree.dtt_accel(pos, mass, p, alpha=1e30, acc_ref=np.ones((3, 800)))
    tr = got["tree"]
    assert got["accepted"]
    for a, b, s in got["accepted"]:
        assert s != (0, 0, 0) or not tr.contains(b, a)
