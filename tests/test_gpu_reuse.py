"""GPU tests of list reuse (pp_plan_set_skin): lists built with the cut
widened by a skin serve later calls while every particle stays within half
the skin of where it was at the build.

Every case is checked against the FP64 oracle at the positions of the call
(the pair test keeps the exact cut, so reuse must not change which pairs
count); the plan's counters show whether the call reused or rebuilt."""
import numpy as np
import pytest

import workloads as W
from workloads import BoxParams
from tests import parity

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


L = 60.0
P_ = BoxParams.from_mesh(L, 48)          # rcut = 7.03
SKIN = 0.6


@pytest.fixture(scope="module")
def box():
    rng = np.random.default_rng(8)
    n = 12000
    pos = W.mixture(rng, n, L, 0.6, 6)
    mass = rng.uniform(0.5, 1.5, n).astype(np.float32) / n
    return pos, mass


def moved(pos, rng, dmax, frac=1.0):
    """Every particle (or a fraction) moved by a random displacement of
    length below dmax, wrapped into [0, L)."""
    n = pos.shape[1]
    d = rng.normal(size=(3, n))
    d *= (rng.uniform(0, dmax, n) / np.linalg.norm(d, axis=0))[None]
    if frac < 1.0:
        d[:, rng.random(n) > frac] = 0.0
    x = pos + d
    return x - L * np.floor(x / L)


def check(acc, pos, mass, oracle_mod):
    ref = oracle_mod.accel(pos, mass.astype(np.float64), P_)
    s = parity.summary(acc, ref)
    assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, s


def test_reuse_within_half_skin(pp, box, oracle_mod):
    pos, mass = box
    rng = np.random.default_rng(1)
    plan = pp.Plan(P_, pos.shape[1])
    plan.set_skin(SKIN)
    M = dev(mass, torch.float32)
    check(plan.accel(dev(pos, torch.float64), M).cpu().numpy(), pos, mass, oracle_mod)
    assert (plan.stats()["list_builds"], plan.stats()["list_reuses"]) == (1, 0)
    x = pos
    for k in range(3):                        # drifts that stay within skin / 2 of the build
        x = moved(pos, rng, 0.45 * SKIN)
        a = plan.accel(dev(x, torch.float64), M).cpu().numpy()
        st = plan.stats()
        assert (st["list_builds"], st["list_reuses"]) == (1, k + 1), st
        check(a, x, mass, oracle_mod)
    # a fresh plan at the same positions agrees to FP32 rounding
    fresh = pp.Plan(P_, pos.shape[1]).accel(dev(x, torch.float64), M).cpu().numpy()
    e = np.linalg.norm(a - fresh, axis=0) / np.maximum(np.linalg.norm(fresh, axis=0), 1e-30)
    assert np.median(e) <= 1e-6 and e.max() <= 1e-4


def test_reuse_across_the_boundary(pp, oracle_mod):
    """Particles within a skin of the box faces cross them while the lists
    are reused (the caller's positions are wrapped into [0, L))."""
    rng = np.random.default_rng(2)
    n = 4000
    pos = rng.random((3, n)) * L
    pos[0, : n // 2] = rng.uniform(-0.2, 0.2, n // 2) % L
    mass = np.full(n, 1.0 / n, dtype=np.float32)
    plan = pp.Plan(P_, n)
    plan.set_skin(SKIN)
    M = dev(mass, torch.float32)
    plan.accel(dev(pos, torch.float64), M)
    x = pos.copy()
    x[0, : n // 2] += np.where(pos[0, : n // 2] < L / 2, -0.25, 0.25)   # across x = 0
    x = x - L * np.floor(x / L)
    crossed = np.abs(x[0, : n // 2] - pos[0, : n // 2]) > L / 2
    assert crossed.sum() > n // 4
    a = plan.accel(dev(x, torch.float64), M).cpu().numpy()
    assert plan.stats()["list_reuses"] == 1
    check(a, x, mass, oracle_mod)


def test_moving_too_far_rebuilds(pp, box, oracle_mod):
    pos, mass = box
    rng = np.random.default_rng(3)
    plan = pp.Plan(P_, pos.shape[1])
    plan.set_skin(SKIN)
    M = dev(mass, torch.float32)
    plan.accel(dev(pos, torch.float64), M)
    x = moved(pos, rng, 0.4 * SKIN)
    x[:, 17] = (x[:, 17] + [0.6 * SKIN, 0, 0]) % L      # one particle past skin / 2
    a = plan.accel(dev(x, torch.float64), M).cpu().numpy()
    st = plan.stats()
    assert (st["list_builds"], st["list_reuses"]) == (2, 0), st
    check(a, x, mass, oracle_mod)
    # the rebuild made x the reference: small moves from x reuse again
    y = moved(x, rng, 0.4 * SKIN)
    a = plan.accel(dev(y, torch.float64), M).cpu().numpy()
    assert plan.stats()["list_reuses"] == 1
    check(a, y, mass, oracle_mod)


def test_reuse_with_active_targets(pp, box, oracle_mod):
    pos, mass = box
    rng = np.random.default_rng(4)
    n = pos.shape[1]
    plan = pp.Plan(P_, n)
    plan.set_skin(SKIN)
    M = dev(mass, torch.float32)
    plan.accel(dev(pos, torch.float64), M)
    x = moved(pos, rng, 0.45 * SKIN)
    act = rng.random(n) < 0.2
    out = torch.full((3, n), 7.0, dtype=torch.float32, device="cuda")
    plan.accel_active(dev(x, torch.float64), M, dev(act.astype(np.uint8), torch.uint8), out=out)
    assert plan.stats()["list_reuses"] == 1
    a = out.cpu().numpy()
    ref = oracle_mod.accel(x, mass.astype(np.float64), P_)["acc"]
    e = np.linalg.norm(a[:, act] - ref[:, act], axis=0) / np.linalg.norm(ref[:, act], axis=0)
    assert np.median(e) <= 1e-6 and np.percentile(e, 99.9) <= 1e-4
    assert np.all(a[:, ~act] == 7.0)           # inactive targets untouched


def test_counts_refused_after_reuse(pp, box, oracle_mod):
    pos, mass = box
    rng = np.random.default_rng(5)
    plan = pp.Plan(P_, pos.shape[1])
    plan.set_skin(SKIN)
    M = dev(mass, torch.float32)
    plan.accel(dev(pos, torch.float64), M)
    plan.count_interactions()                  # lists as built: counts allowed
    x = moved(pos, rng, 0.4 * SKIN)
    plan.accel(dev(x, torch.float64), M)
    with pytest.raises(pp.PPError):
        plan.count_interactions()
    plan.accel_f64(dev(x, torch.float64), dev(mass.astype(np.float64), torch.float64))
    ref = oracle_mod.accel(x, mass.astype(np.float64), P_)
    assert plan.count_interactions() == int(ref["n_inter"].sum())


def test_no_reuse_with_monopoles_or_box_pruning(pp, box, oracle_mod):
    pos, mass = box
    rng = np.random.default_rng(6)
    M = dev(mass, torch.float32)
    x = moved(pos, rng, 0.4 * SKIN)
    # a variant that prunes against the block boxes of the build (an
    # ablation in absolute FP32 coordinates, less precise than the default:
    # compared with a fresh plan of the same variant, which it must equal)
    plan = pp.Plan(P_, pos.shape[1])
    plan.set_skin(SKIN)
    plan.set_tuning(variant=4, waves_per_block=1)
    plan.accel(dev(pos, torch.float64), M)
    a = plan.accel(dev(x, torch.float64), M).cpu().numpy()
    assert (plan.stats()["list_builds"], plan.stats()["list_reuses"]) == (2, 0)
    fresh = pp.Plan(P_, pos.shape[1])
    fresh.set_skin(SKIN)
    fresh.set_tuning(variant=4, waves_per_block=1)
    assert np.array_equal(a, fresh.accel(dev(x, torch.float64), M).cpu().numpy())
    # monopole acceptance
    plan = pp.Plan(P_, pos.shape[1])
    plan.set_skin(SKIN)
    plan.set_monopole(0.3)
    plan.accel(dev(pos, torch.float64), M)
    plan.accel(dev(x, torch.float64), M)
    assert (plan.stats()["list_builds"], plan.stats()["list_reuses"]) == (2, 0)


def test_skin_argument_checks(pp):
    plan = pp.Plan(P_, 100)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(pp.PPError) as e:
            plan.set_skin(bad)
        assert e.value.code == pp.PP_EINVAL
    with pytest.raises(pp.PPError) as e:
        plan.set_skin(L / 2 - P_.rcut)
    assert e.value.code == pp.PP_ERANGE
    plan.set_skin(0.0)


def test_reuse_survives_changing_active_sets(pp, box, oracle_mod):
    """A time integrator's substeps alternate small and large active sets:
    a call that needs more work items than the last one grows them and
    still reuses the lists (64-position chunks make the item counts large
    enough to overflow)."""
    pos, mass = box
    rng = np.random.default_rng(7)
    n = pos.shape[1]
    plan = pp.Plan(P_, n)
    plan.set_skin(SKIN)
    plan.set_tuning(chunk=64, waves_per_block=1)
    M = dev(mass, torch.float32)
    out = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    x = pos
    items = []
    for k, frac in enumerate((0.02, 1.0, 0.1, 1.0, 0.02, 0.5)):
        if k:
            x = moved(pos, rng, 0.45 * SKIN)
        act = x[0] < frac * L                 # a slab: few target blocks when thin
        plan.accel_active(dev(x, torch.float64), M, dev(act.astype(np.uint8), torch.uint8), out=out)
        st = plan.stats()
        assert (st["list_builds"], st["list_reuses"]) == (1, k), (k, st)
        items.append(st["nitem"])
        a = out.cpu().numpy()
        ref = oracle_mod.accel(x, mass.astype(np.float64), P_)["acc"]
        e = np.linalg.norm(a[:, act] - ref[:, act], axis=0) / np.linalg.norm(ref[:, act], axis=0)
        assert np.median(e) <= 1e-6 and np.percentile(e, 99.9) <= 1e-4, (k, np.median(e))
    assert items[1] > items[0] + items[0] // 4 + 1024     # the full call outgrew the first one's items
