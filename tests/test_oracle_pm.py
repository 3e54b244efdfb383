"""Pins of the FP64 PM oracle (oracle/pm.py) to what the mathematics fixes.

Independent checks only: the real-space 7-point Laplacian of the unfiltered
mesh potential, the continuum solution of a single density mode with the
Gaussian filter, the analytic derivative of a cosine, exact interpolation
at mesh points, conservation laws, the force-free lattice, and the split
identity end to end: PM plus the short-range sum reproduces the periodic
Newtonian force computed by a separate Ewald summation in this file.
"""
import numpy as np
import pytest
from scipy.special import erfc

from oracle import pm
from workloads import BoxParams


def test_cic_conserves_mass_and_hits_mesh_points():
    rng = np.random.default_rng(1)
    L, n = 10.0, 16
    pos = rng.random((3, 500)) * L
    m = rng.uniform(0.5, 2.0, 500)
    rho = pm.cic_deposit(pos, m, L, n)
    assert rho.sum() * (L / n) ** 3 == pytest.approx(m.sum(), rel=1e-13)
    # a particle exactly on a mesh point puts all its mass there
    one = pm.cic_deposit(np.array([[3 * L / n], [5 * L / n], [0.0]]), np.array([2.0]), L, n)
    assert one[3, 5, 0] * (L / n) ** 3 == pytest.approx(2.0, rel=1e-14)
    assert np.count_nonzero(one) == 1
    # positions outside [0, L) wrap
    w = pm.cic_deposit(pos + L * np.array([[1.0], [-2.0], [3.0]]), m, L, n)
    assert np.allclose(w, rho, rtol=1e-9, atol=1e-12)


def test_unfiltered_potential_inverts_the_discrete_laplacian():
    """nabla_h^2 phi = 4 pi G (rho - mean rho) with the 7-point Laplacian in
    real space (np.roll), independent of the Fourier-space Green function."""
    rng = np.random.default_rng(2)
    L, n, G = 7.0, 24, 1.7
    rho = rng.random((n, n, n))
    phi = pm.pm_potential(rho, L, G, None)
    d = L / n
    lap = sum(np.roll(phi, 1, a) + np.roll(phi, -1, a) for a in range(3)) - 6 * phi
    lap /= d * d
    want = 4 * np.pi * G * (rho - rho.mean())
    assert np.abs(lap - want).max() <= 1e-10 * np.abs(want).max()
    assert abs(phi.mean()) <= 1e-12 * np.abs(phi).max()


@pytest.mark.parametrize("mode,rs_frac", [(1, 0.0), (4, 0.05), (3, 0.08)])
def test_filtered_mode_matches_the_continuum(mode, rs_frac):
    """rho = A cos(k x): the continuum long-range potential is
    -4 pi G A exp(-k^2 r_s^2) cos(k x) / k^2; the mesh agrees to its
    discretisation error (k Delta)^2 / 12."""
    L, n, G, A = 50.0, 128, 1.0, 0.3
    d = L / n
    x = np.arange(n) * d
    k = 2 * np.pi * mode / L
    rho = np.broadcast_to(A * np.cos(k * x)[:, None, None], (n, n, n)).copy()
    rs = rs_frac * L if rs_frac > 0 else None
    phi = pm.pm_potential(rho, L, G, rs)
    filt = np.exp(-(k * rs) ** 2) if rs else 1.0
    want = -4 * np.pi * G * A * filt * np.cos(k * x) / k ** 2
    tol = 2 * (k * d) ** 2 / 12 + 1e-12
    assert np.abs(phi[:, 5, 7] - want).max() <= tol * np.abs(want).max()
    if rs:
        assert filt < 0.7       # the filter is doing something here


def test_gradient_of_a_cosine():
    L, n = 30.0, 96
    d = L / n
    x = np.arange(n) * d
    k = 2 * np.pi * 3 / L
    phi = np.broadcast_to(np.cos(k * x)[None, :, None], (n, n, n)).copy()     # varies along y
    g = pm.mesh_accel(phi, L)
    want = k * np.sin(k * x)                                                  # -d/dy cos(k y)
    assert np.abs(g[1][4, :, 9] - want).max() <= 1e-4 * k
    assert np.abs(g[0]).max() < 1e-12 and np.abs(g[2]).max() < 1e-12


def test_interpolation_exact_at_mesh_points_and_smooth_between():
    rng = np.random.default_rng(3)
    L, n = 12.0, 32
    d = L / n
    field = rng.random((3, n, n, n))
    idx = rng.integers(0, n, (3, 50))
    vals = pm.cic_interp(field, idx * d, L)
    for ax in range(3):
        assert np.allclose(vals[ax], field[ax][idx[0], idx[1], idx[2]], rtol=0, atol=1e-14)
    # a smooth mode between mesh points: error of linear interpolation
    k = 2 * np.pi * 2 / L
    x = np.arange(n) * d
    f = np.broadcast_to(np.sin(k * x)[None, None, :], (n, n, n))
    f3 = np.stack([f, f, f])
    pts = rng.random((3, 200)) * L
    got = pm.cic_interp(f3, pts, L)[0]
    assert np.abs(got - np.sin(k * pts[2])).max() <= (k * d) ** 2 / 8 + 1e-12


def test_momentum_and_lattice():
    rng = np.random.default_rng(4)
    p = BoxParams(L=20.0, rs=0.8, rcut=3.6, eps=0.01)
    pos = rng.random((3, 3000)) * p.L
    m = rng.uniform(0.5, 1.5, 3000)
    a = pm.pm_accel(pos, m, p, 32)
    net = np.linalg.norm((a * m).sum(1))
    assert net <= 1e-12 * (np.linalg.norm(a, axis=0) * m).sum()
    # particles on the mesh points of a uniform lattice feel no force
    n = 16
    g = (np.arange(n) + 0.0) * p.L / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    lat = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    a0 = pm.pm_accel(lat, np.ones(lat.shape[1]), p, n)
    assert np.abs(a0).max() <= 1e-12


def ewald_pair(ri, rj, L, G, m, alpha, nreal=3, kmax=12, real=True):
    """Acceleration of a particle at ri from a unit-cell image lattice of
    mass m at rj plus a uniform neutralising background (Ewald); real=False
    keeps only the reciprocal (long-range) part."""
    r0 = ri - rj
    a = np.zeros(3)
    if real:
        for nx in range(-nreal, nreal + 1):
            for ny in range(-nreal, nreal + 1):
                for nz in range(-nreal, nreal + 1):
                    r = r0 + L * np.array([nx, ny, nz])
                    s = np.linalg.norm(r)
                    a -= G * m * r / s ** 3 * (erfc(alpha * s) + 2 * alpha * s / np.sqrt(np.pi)
                                               * np.exp(-(alpha * s) ** 2))
    V = L ** 3
    for lx in range(-kmax, kmax + 1):
        for ly in range(-kmax, kmax + 1):
            for lz in range(-kmax, kmax + 1):
                if lx == ly == lz == 0:
                    continue
                kv = 2 * np.pi / L * np.array([lx, ly, lz])
                k2 = kv @ kv
                a -= G * m * 4 * np.pi / V * kv / k2 * np.exp(-k2 / (4 * alpha ** 2)) * np.sin(kv @ r0)
    return a


# Plain CIC assignment and interpolation (no window deconvolution) smooth
# the mesh force: a few per cent at 2-5 mesh cells, about 1 % beyond 7.
SPLIT_TOL = {2.0: 0.06, 3.5: 0.06, 5.0: 0.04, 7.0: 0.015, 9.0: 0.015}


def test_split_identity_pm_plus_pp_is_newtonian():
    """Two particles at separations of 2-9 mesh cells: the PM force plus the
    short-range pair sum (r_cut = 4.5 r_s) equals the periodic Newtonian
    force of an Ewald sum to the PM's discretisation error, and the PM part
    alone follows the reciprocal Ewald part with alpha = 1 / (2 r_s).  A
    wrong sign, factor or filter width would miss by tens of per cent."""
    import oracle
    L, n = 32.0, 32
    p = BoxParams(L=L, rs=1.25, rcut=4.5 * 1.25, eps=0.0)
    rng = np.random.default_rng(5)
    alpha = 1.0 / (2 * p.rs)
    for sep, tol in SPLIT_TOL.items():
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = rng.random(3) * L
        pos = np.stack([c, c + sep * u], axis=1) % L
        m = np.array([1.0, 1.0])
        a_pm = pm.pm_accel(pos, m, p, n)[:, 0]
        a_pp = oracle.accel(pos, m, p)["acc"][:, 0]
        a_ew = ewald_pair(pos[:, 0], pos[:, 1], L, 1.0, 1.0, alpha)
        a_lr = ewald_pair(pos[:, 0], pos[:, 1], L, 1.0, 1.0, alpha, real=False)
        err = np.linalg.norm(a_pm + a_pp - a_ew) / np.linalg.norm(a_ew)
        assert err < tol, (sep, err)
        err_lr = np.linalg.norm(a_pm - a_lr) / np.linalg.norm(a_lr)
        assert err_lr < 2 * tol, (sep, err_lr)
        # the short range carries most of the force at 2 cells, none past r_cut
        if sep == 2.0:
            assert np.linalg.norm(a_pp) > 0.5 * np.linalg.norm(a_ew)
        if sep * (L / n) >= p.rcut:
            assert np.all(a_pp == 0.0)
