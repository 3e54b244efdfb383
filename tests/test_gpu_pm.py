"""GPU parity of the long-range PM force (pp_pm_accel) against the FP64
numpy oracle (oracle/pm.py): the same CIC assignment, Green function,
filter, gradient stencil and interpolation; the GPU keeps FP64 meshes and
rounds the result to FP32, so the two agree to FP32 rounding."""
import numpy as np
import pytest

import workloads as W
from workloads import BoxParams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09824_amd as m
    return m


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel_errors(acc, ref):
    """|a - a_ref| / |a_ref| with a floor of 1e-6 of the RMS force (where the
    long-range force nearly cancels the relative error means nothing)."""
    mag = np.linalg.norm(ref, axis=0)
    floor = 1e-6 * np.sqrt(np.mean(mag ** 2)) + 1e-300
    return np.linalg.norm(acc.astype(np.float64) - ref, axis=0) / np.maximum(mag, floor)


def check(pp, pos, mass, p, n_mesh, med=1e-6, mx=1e-4):
    from oracle import pm as opm
    ref = opm.pm_accel(pos, mass.astype(np.float64), p, n_mesh)
    plan = pp.PMPlan(p, n_mesh)
    acc = plan.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    e = rel_errors(acc, ref)
    assert np.median(e) <= med and e.max() <= mx, (np.median(e), e.max())
    return acc, ref


def test_pm_cfg1(pp):
    b = W.make_config(1)
    check(pp, b.pos, b.mass, b.params, 32)


def test_pm_clustered_and_unequal_masses(pp):
    rng = np.random.default_rng(7)
    L = 60.0
    pos = W.mixture(rng, 50000, L, 0.6, 40)
    mass = rng.uniform(0.2, 3.0, pos.shape[1]).astype(np.float32)
    check(pp, pos, mass, BoxParams.from_mesh(L, 48), 48)


@pytest.mark.parametrize("n_mesh", [4, 5, 16, 27, 64])
def test_pm_mesh_sizes_and_edges(pp, n_mesh):
    rng = np.random.default_rng(n_mesh)
    L = 25.0
    pos = rng.random((3, 3000)) * L
    # particles on the box faces, exactly on mesh points, and unwrapped
    pos[:, :5] = 0.0
    pos[0, 5:10] = L * (1 - 1e-16)
    pos[:, 10:20] = np.round(pos[:, 10:20] / (L / n_mesh)) * (L / n_mesh)
    pos[:, 20:40] += rng.integers(-3, 4, (3, 20)) * L
    mass = rng.uniform(0.5, 1.5, pos.shape[1]).astype(np.float32)
    rs = 1.25 * L / n_mesh
    check(pp, pos, mass, BoxParams(L=L, rs=rs, rcut=min(4.5 * rs, 0.45 * L), eps=0.0), n_mesh)


def test_pm_single_particle_and_empty(pp):
    p = BoxParams(L=10.0, rs=0.5, rcut=2.25, eps=0.0)
    plan = pp.PMPlan(p, 16)
    one = plan.accel(dev(np.array([[3.3], [7.1], [0.2]]), torch.float64), dev(np.ones(1), torch.float32))
    assert np.abs(one.cpu().numpy()).max() < 1e-12     # no self-force
    empty = plan.accel(torch.empty((3, 0), dtype=torch.float64, device="cuda"),
                       torch.empty(0, dtype=torch.float32, device="cuda"))
    assert empty.shape == (3, 0)


def test_pm_cfg2_full(pp):
    """2,097,152 particles on the 128^3 mesh of the benchmark box."""
    b = W.make_config(2)
    acc, ref = check(pp, b.pos, b.mass, b.params, 128)
    m = b.mass.astype(np.float64)
    net = np.linalg.norm((acc.astype(np.float64) * m).sum(1)) / (np.linalg.norm(acc, axis=0) * m).sum()
    assert net < 1e-5


def test_pm_plus_pp_is_newtonian_on_gpu(pp):
    """The two GPU halves of the split together: a pair at 2-9 mesh cells
    against the periodic Newtonian (Ewald) force, as the oracle pin does."""
    from tests.test_oracle_pm import ewald_pair, SPLIT_TOL
    L, n = 32.0, 32
    p = BoxParams(L=L, rs=1.25, rcut=4.5 * 1.25, eps=0.0)
    rng = np.random.default_rng(5)
    pm_plan = pp.PMPlan(p, n)
    for sep, tol in SPLIT_TOL.items():
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = rng.random(3) * L
        pos = np.stack([c, c + sep * u], axis=1) % L
        m = np.ones(2, dtype=np.float32)
        a_pm = pm_plan.accel(dev(pos, torch.float64), dev(m, torch.float32)).cpu().numpy()[:, 0]
        a_pp = pp.Plan(p, 2).accel(dev(pos, torch.float64), dev(m, torch.float32)).cpu().numpy()[:, 0]
        a_ew = ewald_pair(pos[:, 0], pos[:, 1], L, 1.0, 1.0, 1.0 / (2 * p.rs))
        err = np.linalg.norm(a_pm + a_pp - a_ew) / np.linalg.norm(a_ew)
        assert err < tol, (sep, err)


def test_pm_is_deterministic_and_reuses_plan_across_sizes(pp):
    """The assignment has no atomics: repeated calls give identical bits;
    a plan serves calls of different particle counts (its sort buffers
    grow), each matching the oracle."""
    rng = np.random.default_rng(8)
    L, nm = 50.0, 32
    p = BoxParams.from_mesh(L, nm)
    plan = pp.PMPlan(p, nm)
    for n in (5000, 300, 20000):
        pos = W.mixture(rng, n, L, 0.7, 5)
        mass = rng.uniform(0.5, 1.5, n).astype(np.float32) / n
        P, M = dev(pos, torch.float64), dev(mass, torch.float32)
        a1 = plan.accel(P, M).cpu().numpy()
        a2 = plan.accel(P, M).cpu().numpy()
        assert np.array_equal(a1, a2), n
        from oracle import pm as opm
        e = rel_errors(a1, opm.pm_accel(pos, mass.astype(np.float64), p, nm))
        assert np.median(e) <= 1e-6 and e.max() <= 1e-4, (n, np.median(e), e.max())
