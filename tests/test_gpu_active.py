"""GPU tests of pp_accel_active: the short-range force for a subset of the
targets (the force evaluation of the block time steps of sec. 3.4).  The
active targets must get pp_accel's values bit for bit (same lists, items and
summation order) and the other outputs must stay untouched."""
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


def boxes():
    rng = np.random.default_rng(31)
    L = 60.0
    p = BoxParams.from_mesh(L, 32, leaf_max=8)
    n = 20000
    pos = W.mixture(rng, n, L, 0.6, 8)
    return {
        "equal": (pos, W.equal_masses(n), p),
        "unequal": (pos, rng.uniform(0.5, 1.5, n).astype(np.float32) / n, p),
    }


def masks(n, rng):
    dense = (rng.random(n) < 0.3).astype(np.uint8)
    sparse = np.zeros(n, dtype=np.uint8)
    sparse[rng.choice(n, 40, replace=False)] = 1
    return {"30%": dense, "40 targets": sparse, "none": np.zeros(n, dtype=np.uint8),
            "all": np.ones(n, dtype=np.uint8)}


@pytest.mark.parametrize("masses", ["equal", "unequal"])
@pytest.mark.parametrize("graph", [False, True])
def test_active_subset_is_bit_identical(pp, masses, graph):
    pos, mass, p = boxes()[masses]
    n = pos.shape[1]
    plan = pp.Plan(p, n)
    if graph:
        plan.set_tuning(persistent=1, use_graph=1)
    P, M = dev(pos, torch.float64), dev(mass, torch.float32)
    full = plan.accel(P, M).cpu().numpy()
    rng = np.random.default_rng(5)
    sentinel = 12345.0
    for name, m in masks(n, rng).items():
        out = torch.full((3, n), sentinel, dtype=torch.float32, device="cuda")
        plan.accel_active(P, M, dev(m, torch.uint8), out)
        a = out.cpu().numpy()
        on = m.astype(bool)
        assert np.array_equal(a[:, on], full[:, on]), name
        assert np.all(a[:, ~on] == sentinel), name
        # the full call afterwards still covers every target
        again = plan.accel(P, M).cpu().numpy()
        assert np.array_equal(again, full), name


def test_active_subset_with_monopoles_and_counts(pp):
    # the box of the monopole tests (it has accepted nodes at theta = 0.5)
    rng = np.random.default_rng(3)
    n, L = 16000, 60.0
    pos = W.mixture(rng, n, L, 0.7, 6)
    b = BoxParams.from_mesh(L, 32)
    p = BoxParams(L=b.L, rs=b.rs, rcut=b.rcut, eps=b.eps, leaf_max=4)
    mass = rng.uniform(0.5, 1.5, n).astype(np.float32) / n
    plan = pp.Plan(p, n)
    P, M = dev(pos, torch.float64), dev(mass, torch.float32)
    m = (np.random.default_rng(6).random(n) < 0.2).astype(np.uint8)
    out = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    plan.accel_active(P, M, dev(m, torch.uint8), out)
    with pytest.raises(pp.PPError):                 # the lists cover a subset
        plan.count_interactions()
    plan.set_monopole(0.5)
    full = plan.accel(P, M).cpu().numpy()
    assert plan.stats()["monopoles"] > 0
    out = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    plan.accel_active(P, M, dev(m, torch.uint8), out)
    a = out.cpu().numpy()
    on = m.astype(bool)
    assert np.array_equal(a[:, on], full[:, on])
    assert np.all(a[:, ~on] == 0)


def test_active_argument_checks(pp):
    pos, mass, p = boxes()["equal"]
    n = pos.shape[1]
    plan = pp.Plan(p, n)
    P, M = dev(pos, torch.float64), dev(mass, torch.float32)
    out = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        plan.accel_active(P, M, torch.ones(n, dtype=torch.int32, device="cuda"), out)
    import ctypes as C
    with pytest.raises(pp.PPError):
        pp._check(pp._lib.pp_accel_active(plan._h, C.c_void_p(P.data_ptr()), C.c_void_p(M.data_ptr()),
                                          n, None, C.c_void_p(out.data_ptr()), None), "pp_accel_active")
