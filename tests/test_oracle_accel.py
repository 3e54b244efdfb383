"""Pins for the oracle's direct short-range sum.

What fixes each property (none of them is a retyped copy of the oracle):
  * two-body closed form evaluated at 50 digits with mpmath, at every
    orientation and across the periodic boundary (sign, index, image,
    softening, which mass enters);
  * the textbook limits: r_s -> infinity gives Plummer-softened Newton,
    and eps = 0 gives G m / s^2;
  * the hard cut at r_cut (sec. 3.1): a pair just inside counts, just
    outside does not;
  * Newton's third law: sum_i m_i a_i = 0;
  * a perfect cubic lattice feels no force; one displaced particle feels a
    force along its displacement, balanced by the lattice;
  * translation, axis-permutation and mirror invariance;
  * reduction to a textbook routine: with r_s -> infinity and r_cut just
    under L/2 the sum is the minimum-image Plummer direct sum, computed here
    by a separate vectorised numpy loop;
  * pair counts equal a numpy brute-force count;
  * the pair-magnitude sum (the scale of the condition-robust error) is
    |a| for two bodies, twice one pair's magnitude for a target midway
    between two equal masses (whose force cancels), and never below |a|.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from workloads import BoxParams, lattice


def P(L=10.0, rs=0.5, rcut=None, eps=0.01, G=1.0):
    return BoxParams(L=L, rs=rs, rcut=4.5 * rs if rcut is None else rcut, eps=eps, G=G)


def two_body_ref(d, m_src, p):
    mp.mp.dps = 50
    s2 = sum(mp.mpf(float(c)) ** 2 for c in d)
    if s2 >= mp.mpf(p.rcut) ** 2:
        return np.zeros(3)
    se = mp.sqrt(s2 + mp.mpf(p.eps) ** 2)
    x = se / (2 * mp.mpf(p.rs))
    g = mp.erfc(x) + 2 * x / mp.sqrt(mp.pi) * mp.exp(-x * x)
    f = mp.mpf(p.G) * mp.mpf(float(m_src)) * g / se ** 3
    return np.array([float(f * mp.mpf(float(c))) for c in d])


def test_two_body_closed_form_all_orientations(oracle_mod):
    rng = np.random.default_rng(1)
    p = P()
    for trial in range(60):
        s = rng.uniform(0.02, 0.999 * p.rcut)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        x0 = rng.uniform(0, p.L, 3)
        if trial % 3 == 0:           # force the pair across the periodic boundary
            x0[trial % 3] = p.L - 0.3 * s
        x1 = np.mod(x0 + s * u, p.L)
        pos = np.stack([x0, x1], axis=1)
        mass = np.array([0.7, 1.9])
        r = oracle_mod.accel(pos, mass, p)
        d = s * u                   # separation x1 - x0 at the minimum image
        # use the separation the oracle sees after wrapping (exact in FP64 up to rounding of x1)
        dd = x1 - x0
        dd -= p.L * np.round(dd / p.L)
        ref0 = two_body_ref(dd, mass[1], p)
        ref1 = two_body_ref(-dd, mass[0], p)
        assert np.allclose(r["acc"][:, 0], ref0, rtol=1e-13, atol=0), (trial, r["acc"][:, 0], ref0)
        assert np.allclose(r["acc"][:, 1], ref1, rtol=1e-13, atol=0)
        # attractive: particle 0 is pulled toward particle 1
        assert np.dot(r["acc"][:, 0], d) > 0
        assert r["n_inter"].tolist() == [1, 1]


def test_textbook_limits(oracle_mod):
    # r_s huge: g -> 1, Plummer softened Newton
    p = P(L=10.0, rs=1e9, rcut=4.0, eps=0.05, G=2.0)
    pos = np.array([[1.0, 1.0 + 1.5], [2.0, 2.0], [3.0, 3.0]])
    r = oracle_mod.accel(pos, np.array([1.0, 3.0]), p)
    s = 1.5
    assert math.isclose(r["acc"][0, 0], 2.0 * 3.0 * s / (s * s + 0.05 ** 2) ** 1.5, rel_tol=1e-14)
    # and eps = 0: Newton G m / s^2
    p0 = P(L=10.0, rs=1e9, rcut=4.0, eps=0.0, G=1.0)
    r0 = oracle_mod.accel(pos, np.array([1.0, 3.0]), p0)
    assert math.isclose(r0["acc"][0, 0], 3.0 / s ** 2, rel_tol=1e-14)
    assert math.isclose(r0["acc"][0, 1], -1.0 / s ** 2, rel_tol=1e-14)


def test_hard_cut(oracle_mod):
    p = P(L=10.0, rs=0.5)
    for s, inside in [(p.rcut * (1 - 1e-9), True), (p.rcut * (1 + 1e-9), False), (p.rcut, False)]:
        pos = np.array([[1.0, 1.0 + s], [5.0, 5.0], [5.0, 5.0]])
        r = oracle_mod.accel(pos, np.ones(2), p)
        assert (r["acc"][0, 0] > 0) == inside
        assert r["n_inter"][0] == int(inside)
        assert r["n_band"][0] == 1        # all three sit inside the 2^-20 band


def test_coincident_pair_eps_zero_is_zero(oracle_mod):
    p = P(eps=0.0)
    pos = np.array([[1.0, 1.0, 1.5], [2.0, 2.0, 2.0], [3.0, 3.0, 3.0]])
    r = oracle_mod.accel(pos, np.ones(3), p)
    assert np.all(np.isfinite(r["acc"]))
    assert math.isclose(r["acc"][0, 0], r["acc"][0, 1])   # each feels only the third particle


def test_momentum_conservation(oracle_mod):
    rng = np.random.default_rng(7)
    p = P(L=20.0, rs=0.8)
    n = 1500
    pos = rng.random((3, n)) * p.L
    pos[:, :500] = np.mod(3.0 + 0.8 * rng.standard_normal((3, 500)), p.L)   # a clump
    mass = rng.uniform(0.5, 2.0, n)
    r = oracle_mod.accel(pos, mass, p)
    net = (r["acc"] * mass).sum(axis=1)
    scale = (np.linalg.norm(r["acc"], axis=0) * mass).sum()
    assert np.linalg.norm(net) / scale < 1e-13


def test_lattice_is_force_free_and_displacement(oracle_mod):
    L, ns = 8.0, 8
    p = P(L=L, rs=0.6, eps=0.02)      # r_cut = 2.7 < L/2
    pos = lattice(ns, L)
    r = oracle_mod.accel(pos, np.ones(pos.shape[1]), p)
    unit = 1.0 / (L / ns) ** 2
    assert np.abs(r["acc"]).max() < 1e-12 * unit
    k = 100
    delta = np.array([0.05, 0.0, 0.0])
    pos2 = pos.copy()
    pos2[:, k] += delta
    r2 = oracle_mod.accel(pos2, np.ones(pos.shape[1]), p)
    a = r2["acc"][:, k]
    assert a[0] > 1e-6 * unit                       # pulled further along +x
    assert abs(a[1]) < 1e-12 * unit and abs(a[2]) < 1e-12 * unit
    rest = np.delete(r2["acc"], k, axis=1).sum(axis=1)
    assert np.allclose(rest, -a, rtol=1e-10, atol=1e-12 * unit)


def test_translation_permutation_mirror(oracle_mod):
    rng = np.random.default_rng(3)
    p = P(L=16.0, rs=0.7)
    n = 800
    pos = rng.random((3, n)) * p.L
    mass = rng.uniform(0.5, 2.0, n)
    a = oracle_mod.accel(pos, mass, p)["acc"]
    sh = np.mod(pos + np.array([[3.3], [-7.1], [12.9]]), p.L)
    a_sh = oracle_mod.accel(sh, mass, p)["acc"]
    tol = 1e-9 * np.abs(a).max()
    assert np.abs(a_sh - a).max() < tol
    a_perm = oracle_mod.accel(pos[[2, 0, 1]], mass, p)["acc"]
    assert np.abs(a_perm - a[[2, 0, 1]]).max() < tol
    mir = pos.copy()
    mir[0] = np.mod(p.L - mir[0], p.L)
    a_mir = oracle_mod.accel(mir, mass, p)["acc"]
    assert np.abs(a_mir[0] + a[0]).max() < tol and np.abs(a_mir[1:] - a[1:]).max() < tol


def test_reduces_to_textbook_min_image_plummer_sum(oracle_mod):
    rng = np.random.default_rng(11)
    L = 10.0
    p = BoxParams(L=L, rs=1e12, rcut=0.4999 * L, eps=0.03, G=1.0)
    n = 400
    pos = rng.random((3, n)) * L
    mass = rng.uniform(0.5, 2.0, n)
    got = oracle_mod.accel(pos, mass, p)
    d = pos[:, None, :] - pos[:, :, None]          # d[:, i, j] = x_j - x_i
    d -= L * np.round(d / L)
    s2 = (d * d).sum(axis=0)
    keep = (s2 < p.rcut ** 2) & ~np.eye(n, dtype=bool)
    w = np.where(keep, mass[None, :] / np.where(keep, s2 + p.eps ** 2, 1.0) ** 1.5, 0.0)
    ref = (d * w[None]).sum(axis=2)
    assert np.allclose(got["acc"], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert (got["n_inter"] == keep.sum(axis=1)).all()


def test_targets_subset_matches_full(oracle_mod):
    rng = np.random.default_rng(5)
    p = P(L=12.0, rs=0.5)
    pos = rng.random((3, 900)) * p.L
    mass = np.ones(900)
    full = oracle_mod.accel(pos, mass, p)
    t = np.array([0, 17, 899, 450, 17])
    sub = oracle_mod.accel(pos, mass, p, targets=t)
    assert np.array_equal(sub["acc"], full["acc"][:, t])
    assert np.array_equal(sub["n_inter"], full["n_inter"][t])


def test_rejects_cut_beyond_half_box(oracle_mod):
    p = BoxParams(L=10.0, rs=1.0, rcut=5.0, eps=0.0)
    with pytest.raises(ValueError):
        oracle_mod.accel(np.zeros((3, 2)), np.ones(2), p)


def test_pair_magnitude_sum(oracle_mod):
    p = P()
    rng = np.random.default_rng(5)
    # two bodies: the sum over one pair is that pair's |a|
    pos = np.array([[3.0, 3.0 + 1.1], [4.0, 4.2], [5.0, 4.7]])
    mass = np.array([0.7, 1.9])
    r = oracle_mod.accel(pos, mass, p, pair_abs=True)
    for k in range(2):
        ref = two_body_ref(pos[:, 1 - k] - pos[:, k], mass[1 - k], p)
        assert r["pair_abs"][k] == pytest.approx(np.linalg.norm(ref), rel=1e-13)
    # a target midway between two equal masses: no force, twice one pair
    pos = np.array([[4.0, 5.0, 6.0], [5.0, 5.0, 5.0], [5.0, 5.0, 5.0]])
    r = oracle_mod.accel(pos, np.ones(3), p, pair_abs=True)
    one = np.linalg.norm(two_body_ref(np.array([1.0, 0.0, 0.0]), 1.0, p))
    assert np.abs(r["acc"][:, 1]).max() <= 1e-15 * one
    assert r["pair_abs"][1] == pytest.approx(2 * one, rel=1e-13)
    # triangle inequality on a random box; zero without neighbours
    pos = rng.uniform(0, p.L, (3, 300))
    pos[:, 0] = [0.5 * p.L] * 3
    pos[:, 1:] = np.where(np.linalg.norm(pos[:, 1:] - pos[:, :1], axis=0) < 1.05 * p.rcut,
                          np.mod(pos[:, 1:] + 0.5 * p.L, p.L), pos[:, 1:])
    r = oracle_mod.accel(pos, rng.uniform(0.5, 2.0, 300), p, pair_abs=True)
    assert np.all(r["pair_abs"] >= np.linalg.norm(r["acc"], axis=0) * (1 - 1e-14))
    assert np.all((r["pair_abs"] > 0) == (r["n_inter"] > 0))


def test_neighbours_brute_force_over_images(oracle_mod):
    """oracle.neighbours against a brute force over all 27 periodic images:
    j is a neighbour of i with shift s exactly when |x_j + s L - x_i| < r_cut
    for that image (at most one image can be, since r_cut < L / 2), and the
    counts agree with oracle.accel's."""
    from workloads import BoxParams
    rng = np.random.default_rng(21)
    L = 10.0
    pos = rng.random((3, 300)) * L
    pos[:, :20] = pos[:, :20] * 0.05 + L - 0.3          # a clump across the corner
    p = BoxParams(L=L, rs=1.0, rcut=4.5, eps=0.01)
    rp, nbr, code = oracle_mod.neighbours(pos, p)
    ref = oracle_mod.accel(pos, np.ones(300), p)
    assert np.array_equal(np.diff(rp), ref["n_inter"])
    w = pos - L * np.floor(pos / L)
    sh = np.array([(c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1) for c in range(27)], dtype=np.float64)
    for i in range(300):
        d = w[:, None, :] + L * sh.T[:, :, None] - w[:, i][:, None, None]     # [3, 27, n]
        s2 = (d * d).sum(axis=0)                                               # [27, n]
        s2[:, i] = np.inf
        c, j = np.nonzero(s2 < p.rcut ** 2)
        order = np.argsort(j)
        assert np.array_equal(nbr[rp[i]:rp[i + 1]], j[order]), i
        assert np.array_equal(code[rp[i]:rp[i + 1]], c[order]), i
    sub = np.array([3, 17, 250])
    rps, nbs, cds = oracle_mod.neighbours(pos, p, targets=sub)
    for t, i in enumerate(sub):
        assert np.array_equal(nbs[rps[t]:rps[t + 1]], nbr[rp[i]:rp[i + 1]])
        assert np.array_equal(cds[rps[t]:rps[t + 1]], code[rp[i]:rp[i + 1]])
