"""GPU test of the allocation-free entry point pp_accel_scratch: called
through the C ABI twice in a row (the second call with a smaller input),
its accelerations must equal those of pp_accel on a plan with the default
tuning, bit for bit, and meet the oracle's tolerances."""
import ctypes as C

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


def scratch_call(pp, params, pos, mass):
    """pp_accel_scratch through the raw C ABI."""
    n = pos.shape[1]
    out = torch.full((3, n), float("nan"), dtype=torch.float32, device="cuda")
    prm = pp.make_params(params)
    rc = pp._lib.pp_accel_scratch(C.byref(prm), C.c_void_p(pos.data_ptr()), C.c_void_p(mass.data_ptr()),
                                  n, C.c_void_p(out.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, pp._lib.pp_last_error().decode()
    return out.cpu().numpy()


def test_no_alloc_matches_pp_accel_twice(pp, oracle_mod):
    big = W.make_config(1)                                     # 32768 uniform, L = 100
    rng = np.random.Generator(np.random.PCG64(77))
    small_pos = W.mixture(rng, 9001, 40.0, 0.6, 5)
    small = W.Box(pos=small_pos, mass=rng.uniform(0.5, 1.5, 9001).astype(np.float32),
                  params=BoxParams.from_mesh(40.0, 20), name="small-clustered")
    for b in (big, small):
        pos, mass = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
        got = scratch_call(pp, b.params, pos, mass)
        ref_plan = pp.Plan(b.params, b.n)
        want = ref_plan.accel(pos, mass).cpu().numpy()
        assert np.array_equal(got, want), b.name
        ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params)
        s = parity.summary(got, ref)
        assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, (b.name, s)


def test_no_alloc_rejects_too_many_particles(pp):
    p = BoxParams(L=10.0, rs=1.0, rcut=4.5, eps=0.01)
    n = 65537
    pos = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    mass = torch.ones(n, dtype=torch.float32, device="cuda")
    with pytest.raises(pp.PPError) as e:
        pp.pp_accel_scratch(p, pos, mass)
    assert e.value.code == pp.PP_EINVAL
