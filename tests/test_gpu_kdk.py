"""GPU tests of the adaptive KDK driver (pp_kdk_*) against the FP64 oracle
integration (oracle/kdk.py with the oracle's PP and PM forces).

The step levels are a decision taken from the FP32 forces on the GPU and
from FP64 forces in the oracle; the oracle run is therefore handed the
GPU's levels, and the level rule itself is checked separately on the GPU's
own accelerations."""
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


@pytest.mark.parametrize("skin", [0.0, 0.4])
def test_kdk_matches_oracle_integration(pp, skin):
    """With a skin the substeps reuse the short-range lists; the trajectory
    must meet the same bars (the pair test is exact either way)."""
    import oracle
    from oracle import kdk as okdk, pm as opm
    rng = np.random.default_rng(11)
    L, nm = 40.0, 32
    p = BoxParams.from_mesh(L, nm)
    n = 3000
    pos0 = W.mixture(rng, n, L, 0.5, 6)
    vel0 = rng.normal(scale=0.05, size=(3, n))
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    eta, dt, kmax = 0.02, 4.0, 4
    m64 = mass.astype(np.float64)

    def force(x):
        return oracle.accel(x, m64, p)["acc"] + opm.pm_accel(x, m64, p, nm)

    K = pp.KDK(p, n, n_mesh=nm, eta=eta, max_level=kmax)
    K.set_skin(skin)
    P, V, M = dev(pos0, torch.float64), dev(vel0, torch.float64), dev(mass, torch.float32)
    K.init(P, M)
    po, vo = pos0.copy(), vel0.copy()
    ao = force(po)
    evals = 1
    targets = n                                    # pp_kdk_init evaluates every target
    for step in range(2):
        a_gpu = K.accel().cpu().numpy().astype(np.float64)
        a_tot = a_gpu[:3] + a_gpu[3:]
        K.step(P, V, M, dt)
        lev = K.levels().cpu().numpy().astype(np.int64)
        # the level rule on the GPU's own accelerations
        want = okdk.step_levels(a_tot, eta, p.eps, dt, kmax)
        assert np.mean(lev == want) > 0.999, np.mean(lev == want)
        po, vo, ao, ev = okdk.kdk_top_step(po, vo, ao, force, dt, lev, L)
        evals += ev
        info = K.info()
        assert info["deepest_level"] == lev.max() and info["force_evaluations"] == evals
        assert sum(info["level_count"]) == n
        # short-range forces only for the particles whose step ends: particle
        # i gets 2^level_i of them per top step
        targets += int((2 ** lev).sum())
        assert info["short_range_targets"] == targets < n * evals
    assert len(set(lev.tolist())) >= 2              # the test exercises several levels
    info = K.info()
    if skin > 0:
        assert 1 <= info["list_builds"] < info["force_evaluations"] / 2, info
    else:
        assert info["list_builds"] == info["force_evaluations"]
    pg, vg = P.cpu().numpy(), V.cpu().numpy()
    dp = pg - po
    dp -= L * np.round(dp / L)
    disp = np.linalg.norm(((po - pos0 + L / 2) % L) - L / 2, axis=0)
    assert np.median(np.linalg.norm(dp, axis=0)) <= 1e-5 * np.median(disp) + 1e-12
    assert np.linalg.norm(dp, axis=0).max() <= 1e-3 * disp.max()
    dv = np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), 1e-12)
    assert np.median(dv) <= 1e-5


def test_kdk_three_body_stays_bound(pp):
    """The sec. 3.4 setting on the GPU: a close binary orbiting a massive
    body under PM + PP stays bound over 20 binary periods."""
    L, nm = 64.0, 32
    p = BoxParams(L=L, rs=1.5, rcut=4.5 * 1.5, eps=0.02)
    M, m, R, sep = 100.0, 1.0, 12.0, 0.3
    c = np.array([L / 2] * 3)
    vc, vb = np.sqrt(M / R), np.sqrt(2 * m / sep) / 2
    pos0 = np.stack([c, c + [R, sep / 2, 0], c + [R, -sep / 2, 0]], axis=1)
    vel0 = np.stack([[0, 0, 0], [-vb, vc, 0], [vb, vc, 0]], axis=1).astype(float)
    vel0[:, 0] = -(vel0[:, 1] + vel0[:, 2]) * m / M
    mass = np.array([M, m, m], dtype=np.float32)
    K = pp.KDK(p, 3, n_mesh=nm, eta=1e6, max_level=0)       # one shared step
    P, V, Ms = dev(pos0, torch.float64), dev(vel0, torch.float64), dev(mass, torch.float32)
    K.init(P, Ms)
    seps = []
    for _ in range(300):
        K.step(P, V, Ms, 0.05)
        x = P.cpu().numpy()
        seps.append(np.linalg.norm(x[:, 1] - x[:, 2]))
    assert 0.25 < min(seps) and max(seps) < 0.4, (min(seps), max(seps))


def test_kdk_argument_checks(pp):
    p = BoxParams(L=10.0, rs=0.5, rcut=2.25, eps=0.01)
    for kw in (dict(eta=0.0), dict(max_level=16), dict(n_mesh=3)):
        with pytest.raises(pp.PPError):
            pp.KDK(p, 10, **kw)
    with pytest.raises(pp.PPError):
        pp.KDK(BoxParams(L=10.0, rs=0.5, rcut=2.25, eps=0.0), 10)
    K = pp.KDK(p, 10)
    x = torch.rand((3, 10), dtype=torch.float64, device="cuda") * 10
    with pytest.raises(pp.PPError):            # init first
        K.step(x, torch.zeros_like(x), torch.ones(10, dtype=torch.float32, device="cuda"), 0.1)
    for bad in (-0.1, float("nan"), 5.0 - 2.25):   # negative, non-finite, rcut + skin = L/2
        with pytest.raises(pp.PPError):
            K.set_skin(bad)


def test_kdk_short_range_only_matches_oracle(pp):
    """n_mesh = 0: the driver integrates the short-range force alone; the
    sub-steps evaluate it for the particles whose step ends only."""
    import oracle
    from oracle import kdk as okdk
    rng = np.random.default_rng(21)
    L = 30.0
    p = BoxParams.from_mesh(L, 24)
    n = 2000
    pos0 = W.mixture(rng, n, L, 0.6, 5)
    vel0 = rng.normal(scale=0.05, size=(3, n))
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    eta, dt, kmax = 0.02, 3.0, 3
    m64 = mass.astype(np.float64)

    def force(x):
        return oracle.accel(x, m64, p)["acc"]

    K = pp.KDK(p, n, n_mesh=0, eta=eta, max_level=kmax)
    P, V, M = dev(pos0, torch.float64), dev(vel0, torch.float64), dev(mass, torch.float32)
    K.init(P, M)
    K.step(P, V, M, dt)
    lev = K.levels().cpu().numpy().astype(np.int64)
    assert len(set(lev.tolist())) >= 2
    po, vo, _, ev = okdk.kdk_top_step(pos0, vel0, force(pos0), force, dt, lev, L)
    info = K.info()
    assert info["force_evaluations"] == 1 + ev
    assert info["short_range_targets"] == n + int((2 ** lev).sum())
    pg, vg = P.cpu().numpy(), V.cpu().numpy()
    dp = pg - po
    dp -= L * np.round(dp / L)
    disp = np.linalg.norm(((po - pos0 + L / 2) % L) - L / 2, axis=0)
    assert np.median(np.linalg.norm(dp, axis=0)) <= 1e-5 * np.median(disp) + 1e-12
    dv = np.linalg.norm(vg - vo, axis=0) / np.maximum(np.linalg.norm(vo, axis=0), 1e-12)
    assert np.median(dv) <= 1e-5
