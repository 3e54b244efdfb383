"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact: Hilbert keys, the key sort, the leaf table and the canonical
near-pair CSR.  Floating point: FP32 accelerations within median relative
error 1e-6 and 99.9th percentile 1e-4 of the FP64 oracle (band-tolerant at
the cut, see tests/parity.py); the FP64 kernel within 1e-12 median; pair
counts exact.  Inputs are the seeded workloads and hand-made edge cases.
"""
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


def small_clustered(n, L, frac, n_sph, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return W.mixture(rng, n, L, frac, n_sph)


def edge_positions(L, rng, n=600):
    pos = rng.random((3, n)) * L
    pos[:, 0] = 0.0
    pos[:, 1] = L - 1e-12
    pos[:, 2] = -1e-300
    pos[:, 3] = L
    pos[:, 4] = 3.5 * L
    pos[:, 5] = -0.75 * L
    pos[:, 6] = L / 2
    return pos


@pytest.mark.parametrize("case", ["cfg1", "edges", "clustered"])
@pytest.mark.parametrize("bits", [21, 5, 1])
def test_keys_bit_exact(pp, oracle_mod, case, bits):
    rng = np.random.default_rng(bits)
    if case == "cfg1":
        b = W.make_config(1)
        pos, L = b.pos, b.params.L
    elif case == "edges":
        L = 37.5
        pos = edge_positions(L, rng)
    else:
        L = 80.0
        pos = small_clustered(20000, L, 0.8, 20, 7)
    keys = pp.pp_hilbert_keys(dev(pos, torch.float64), L, bits).cpu().numpy().view(np.uint64)
    ref = oracle_mod.hilbert_keys(pos, L, bits)
    assert np.array_equal(keys, ref)


def test_sort_bit_exact(pp, oracle_mod):
    pos = small_clustered(30001, 50.0, 0.7, 10, 3)
    pos[:, 100:200] = pos[:, 100:101]          # duplicate keys: order must follow the index
    keys = oracle_mod.hilbert_keys(pos, 50.0, 21)
    perm, sk = pp.pp_sort_by_key(dev(keys.view(np.int64), torch.int64))
    ref = oracle_mod.sort_order(keys)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), ref)
    assert np.array_equal(sk.cpu().numpy().view(np.uint64), keys[ref])


def leaves_case(name):
    if name == "cfg1":
        b = W.make_config(1)
        return b.pos, b.params
    if name == "clustered-lm8":
        return small_clustered(20000, 80.0, 0.8, 15, 11), BoxParams(L=80.0, rs=1.0, rcut=4.5, eps=0.02, leaf_max=8)
    if name == "duplicates":
        rng = np.random.default_rng(5)
        pos = np.concatenate([np.full((3, 300), 12.25), rng.random((3, 3000)) * 40.0], axis=1)
        return pos, BoxParams(L=40.0, rs=1.0, rcut=4.5, eps=0.0, leaf_max=16)
    if name == "tiny":
        rng = np.random.default_rng(9)
        return rng.random((3, 7)) * 10.0, BoxParams(L=10.0, rs=1.0, rcut=4.5, eps=0.0, leaf_max=32)
    if name == "coarse-bits":
        return small_clustered(5000, 30.0, 0.5, 5, 2), BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.01, leaf_max=4, key_bits=6)
    if name == "edge-wrap":
        # coordinates that wrap to exactly L (clamped into the last cell), to 0,
        # and from several periods away: keys, leaf boxes and blocks must agree
        return edge_positions(37.5, np.random.default_rng(12)), BoxParams(L=37.5, rs=1.0, rcut=4.5, eps=0.01, leaf_max=8)
    raise KeyError(name)


LEAF_CASES = ["cfg1", "clustered-lm8", "duplicates", "tiny", "coarse-bits", "edge-wrap"]


@pytest.mark.parametrize("case", LEAF_CASES)
def test_leaves_bit_exact(pp, oracle_mod, case):
    pos, p = leaves_case(case)
    st = oracle_mod.structure(pos, p)
    ps = pos[:, st["perm"]]
    lv = pp.pp_build_leaves(dev(st["sorted_keys"].view(np.int64), torch.int64), dev(ps, torch.float64), p)
    got = lv.export()
    ref = st["leaves"]
    assert got["begin"].size == ref["begin"].size
    for k in ("begin", "count", "level", "prefix"):
        assert np.array_equal(got[k].astype(np.int64), ref[k].astype(np.int64)), k
    assert np.array_equal(got["lo"].astype(np.int64), st["lo"])
    assert np.array_equal(got["hi"].astype(np.int64), st["hi"])


@pytest.mark.parametrize("case", ["clustered-lm8", "duplicates", "tiny", "coarse-bits", "cfg1", "edge-wrap"])
def test_near_pairs_bit_exact(pp, oracle_mod, case):
    pos, p = leaves_case(case)
    st = oracle_mod.structure(pos, p)
    ps = pos[:, st["perm"]]
    lv = pp.pp_build_leaves(dev(st["sorted_keys"].view(np.int64), torch.int64), dev(ps, torch.float64), p)
    rp, src, code = pp.pp_near_pairs(lv, p).export()
    m = st["lo"].shape[1]
    rows = np.arange(m) if m <= 1500 else np.random.default_rng(0).choice(m, 400, replace=False)
    rrp, rsrc, rcode = oracle_mod.near_pairs(st["lo"], st["hi"], p.L, p.rcut, p.key_bits, rows=rows)
    for t, a in enumerate(rows):
        assert np.array_equal(src[rp[a]:rp[a + 1]], rsrc[rrp[t]:rrp[t + 1]]), a
        assert np.array_equal(code[rp[a]:rp[a + 1]], rcode[rrp[t]:rrp[t + 1]]), a


@pytest.fixture(scope="module")
def cfg1_ref(oracle_mod):
    b = W.make_config(1)
    return b, oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, pair_abs=True)


def test_accel_f32_cfg1_full(pp, cfg1_ref):
    b, ref = cfg1_ref
    plan = pp.Plan(b.params, b.n)
    acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()
    s = parity.summary(acc, ref)
    print("cfg1 f32", s, plan.stats())
    assert s["zero_ok"]
    assert s["median"] <= 1e-6
    assert s["p999"] <= 1e-4
    assert s["robust_max"] <= parity.ROBUST_MAX


def test_accel_f64_cfg1_full(pp, cfg1_ref):
    b, ref = cfg1_ref
    plan = pp.Plan(b.params, b.n)
    acc = plan.accel_f64(dev(b.pos, torch.float64), dev(b.mass, torch.float64)).cpu().numpy()
    s = parity.summary(acc, ref)
    print("cfg1 f64", s)
    assert s["median"] <= 1e-12
    assert s["max"] <= 1e-9


def test_count_interactions_cfg1_exact(pp, cfg1_ref):
    b, ref = cfg1_ref
    plan = pp.Plan(b.params, b.n)
    plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32))
    tot, counts = plan.count_interactions(per_target=True)
    assert np.array_equal(counts.cpu().numpy(), ref["n_inter"])
    assert tot == int(ref["n_inter"].sum())


def test_deterministic_repeat(pp):
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    pos, mass = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    a1 = plan.accel(pos, mass).cpu().numpy()
    a2 = plan.accel(pos, mass).cpu().numpy()
    assert np.array_equal(a1, a2)


EDGE_CASES = {
    "n1": lambda: (np.array([[1.0], [2.0], [3.0]]), BoxParams(L=10.0, rs=1.0, rcut=4.5, eps=0.01)),
    "n2-across-boundary": lambda: (np.array([[0.1, 9.8], [5.0, 5.0], [5.0, 5.0]]), BoxParams(L=10.0, rs=1.0, rcut=4.5, eps=0.01)),
    "n63": lambda: (np.random.default_rng(63).random((3, 63)) * 20, BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01)),
    "n64": lambda: (np.random.default_rng(64).random((3, 64)) * 20, BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01)),
    "n65": lambda: (np.random.default_rng(65).random((3, 65)) * 20, BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01)),
    "ragged-3000": lambda: (small_clustered(3001, 30.0, 0.6, 4, 1), BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.02)),
    "coincident-eps0": lambda: (np.concatenate([np.full((3, 5), 2.5), np.random.default_rng(1).random((3, 200)) * 10], axis=1), BoxParams(L=10.0, rs=0.5, rcut=2.25, eps=0.0)),
    "wide-cut": lambda: (np.random.default_rng(2).random((3, 2000)) * 10, BoxParams(L=10.0, rs=1.1, rcut=4.95, eps=0.01)),
    "unwrapped": lambda: (np.random.default_rng(3).random((3, 1500)) * 60 - 20, BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01)),
    "edge-wrap": lambda: (edge_positions(37.5, np.random.default_rng(12)), BoxParams(L=37.5, rs=1.0, rcut=4.5, eps=0.01)),
    "lattice": lambda: (W.lattice(8, 8.0), BoxParams(L=8.0, rs=0.6, rcut=2.7, eps=0.02)),
    "leaf1": lambda: (np.random.default_rng(4).random((3, 1000)) * 20, BoxParams(L=20.0, rs=1.0, rcut=4.5, eps=0.01, leaf_max=1)),
    "leaf1024": lambda: (small_clustered(5000, 30.0, 0.6, 4, 8), BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.01, leaf_max=1024)),
    # a 16^3 key grid: clustered cells hold more than leaf_max particles, so
    # leaves at the finest level exceed leaf_max
    "bits4": lambda: (small_clustered(3000, 30.0, 0.7, 3, 9), BoxParams(L=30.0, rs=1.0, rcut=4.5, eps=0.01, key_bits=4)),
    # a cut well inside the split scale (the polynomial's variable stays near 0)
    "short-cut": lambda: (np.random.default_rng(5).random((3, 3000)) * 20, BoxParams(L=20.0, rs=1.0, rcut=1.5, eps=0.01)),
    # lengths and G far from 1: the kernel's length unit follows r_s
    "large-units": lambda: (np.random.default_rng(6).random((3, 2000)) * 2e4, BoxParams(L=2e4, rs=1e3, rcut=4.5e3, eps=10.0, G=6.674e-11)),
    "small-units": lambda: (small_clustered(2500, 2e-3, 0.5, 3, 10), BoxParams(L=2e-3, rs=1e-4, rcut=4.5e-4, eps=2e-6, G=3.0e4)),
}


@pytest.mark.parametrize("case", sorted(EDGE_CASES))
def test_accel_edge_cases(pp, oracle_mod, case):
    pos, p = EDGE_CASES[case]()
    n = pos.shape[1]
    mass = np.random.default_rng(n).uniform(0.5, 1.5, n).astype(np.float32)
    if case == "lattice":
        mass[:] = 1.0                      # a lattice is force-free only with equal masses
    ref = oracle_mod.accel(pos, mass.astype(np.float64), p, pair_abs=True)
    plan = pp.Plan(p, n + 10)
    acc = plan.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    if case == "lattice":
        unit = 1.0 / (p.L / 8) ** 2
        assert np.abs(acc).max() < 1e-5 * unit
        # the forces cancel exactly: only the condition-robust error is defined
        assert parity.robust_errors(acc, ref).max() <= parity.ROBUST_MAX
        return
    s = parity.summary(acc, ref)
    assert s["zero_ok"], case
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4, (case, s)
    assert s["robust_max"] <= parity.ROBUST_MAX, (case, s)
    a64 = plan.accel_f64(dev(pos, torch.float64), dev(mass.astype(np.float64), torch.float64)).cpu().numpy()
    s64 = parity.summary(a64, ref)
    assert s64["max"] <= 1e-10, (case, s64)


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("case", ["leaf1", "ragged-3000", "edge-wrap", "bits4", "n65"])
def test_edge_cases_several_waves_per_block(pp, oracle_mod, case, k):
    """K waves per block with two windows of 64 list positions per wave and
    item: each wave's windows lie (K - 1) x 64 positions apart, so its range
    cursor skips ranges between windows (single-particle leaves make them
    short) and every window is mapped afresh; results must meet the same
    bars as the default tiles."""
    pos, p = EDGE_CASES[case]()
    n = pos.shape[1]
    mass = np.random.default_rng(n + k).uniform(0.5, 1.5, n).astype(np.float32)
    ref = oracle_mod.accel(pos, mass.astype(np.float64), p, pair_abs=True)
    plan = pp.Plan(p, n + 10)
    plan.set_tuning(waves_per_block=k, chunk=128 * k, persistent=1, waves_per_cu=24, use_graph=0)
    acc = plan.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    s = parity.summary(acc, ref)
    assert s["zero_ok"], case
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4, (case, k, s)
    assert s["robust_max"] <= parity.ROBUST_MAX, (case, k, s)


@pytest.mark.parametrize("k,variant", [(1, 0), (2, 0), (4, 0), (4, 8)])
def test_grid_launch_forms_agree_on_small_box(pp, oracle_mod, k, variant):
    """One workgroup per item on the 32 k uniform box.  A fresh plan's first
    call knows no item count yet and launches the form built for many
    resident waves; the next call sees few enough items (at most two waves
    per SIMD of the 256-CU MI355X) and launches the form built for two.  Both
    run the same arithmetic in the same order: the results must be
    bit-identical and meet the oracle bars."""
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    plan.set_tuning(chunk=2048 * k, waves_per_block=k, persistent=0, waves_per_cu=20, use_graph=0,
                    variant=variant)
    pos, mass = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    first = plan.accel(pos, mass).cpu().numpy()
    assert plan.stats()["nitem"] * k <= 2 * 4 * 256
    later = plan.accel(pos, mass).cpu().numpy()
    assert np.array_equal(first.view(np.uint32), later.view(np.uint32))
    t = np.sort(np.random.default_rng(5).choice(b.n, 512, replace=False))
    ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, targets=t, pair_abs=True)
    s = parity.summary(later[:, t], ref)
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4, s


def test_rejects_nonfinite(pp):
    p = BoxParams(L=10.0, rs=1.0, rcut=4.5, eps=0.01)
    pos = np.random.default_rng(0).random((3, 100)) * 10
    pos[1, 17] = np.nan
    plan = pp.Plan(p, 100)
    with pytest.raises(pp.PPError) as e:
        plan.accel(dev(pos, torch.float64), dev(np.ones(100), torch.float32))
    assert e.value.code == pp.PP_EINVAL


@pytest.fixture(scope="module")
def cfg2_sample(oracle_mod):
    b = W.make_config(2)
    rng = np.random.default_rng(2024)
    targets = np.sort(rng.choice(b.n, 1536, replace=False))
    ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, targets=targets, pair_abs=True)
    return b, targets, ref


def test_accel_f32_cfg2_sampled(pp, cfg2_sample):
    b, targets, ref = cfg2_sample
    plan = pp.Plan(b.params, b.n)
    acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()[:, targets]
    s = parity.summary(acc, ref)
    print("cfg2 f32 sampled", s, plan.stats())
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4
    assert s["robust_max"] <= parity.ROBUST_MAX
    tot, counts = plan.count_interactions(per_target=True)
    assert np.array_equal(counts.cpu().numpy()[targets], ref["n_inter"])


def test_fp32_momentum_and_translation(pp, oracle_mod):
    """Pairwise antisymmetry gives sum_i m_i a_i = 0; the FP32 kernel keeps it
    to FP32 rounding.  Shifting every position by a constant (mod L) moves
    keys, leaves and blocks but not the forces."""
    b = W.make_config(1)
    m = b.mass.astype(np.float64)
    plan = pp.Plan(b.params, b.n)
    acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy().astype(np.float64)
    net = np.linalg.norm((acc * m).sum(axis=1))
    scale = (np.linalg.norm(acc, axis=0) * m).sum()
    print("FP32 |sum m a| / sum m |a| =", net / scale)
    assert net / scale <= 1e-5
    shifted = np.mod(b.pos + np.array([[13.7], [-41.25], [77.03125]]), b.params.L)
    acc2 = plan.accel(dev(shifted, torch.float64), dev(b.mass, torch.float32)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.accel(b.pos, m, b.params)
    s1 = parity.summary(acc.astype(np.float32), ref)
    s2 = parity.summary(acc2.astype(np.float32), ref)
    assert s2["median"] <= 1e-6 and s2["p999"] <= 1e-4, s2
    rel = np.linalg.norm(acc2 - acc, axis=0) / np.maximum(np.linalg.norm(ref["acc"], axis=0), 1e-300)
    assert np.median(rel) <= 2e-6, (np.median(rel), s1, s2)


TABLE_CASES = ["n1", "n2-across-boundary", "n65", "ragged-3000", "coincident-eps0", "wide-cut",
               "edge-wrap", "leaf1024"]


@pytest.mark.parametrize("case", [c for c in TABLE_CASES if c in EDGE_CASES])
@pytest.mark.parametrize("equal", [False, True])
def test_split_table_variant_edge_cases(pp, oracle_mod, case, equal):
    """Variant 8 takes the split factor from the interpolated LDS table (the
    form of sec. 3.1) instead of the polynomial; same tolerance."""
    pos, p = EDGE_CASES[case]()
    n = pos.shape[1]
    mass = np.random.default_rng(n).uniform(0.5, 1.5, n).astype(np.float32)
    if equal:
        mass[:] = np.float32(1.0 / n)
    ref = oracle_mod.accel(pos, mass.astype(np.float64), p)
    plan = pp.Plan(p, n + 10)
    plan.set_tuning(variant=8)
    acc = plan.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    s = parity.summary(acc, ref)
    assert s["zero_ok"], case
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4, (case, s)


def test_split_table_variant_cfg2_sampled(pp, cfg2_sample):
    b, targets, ref = cfg2_sample
    plan = pp.Plan(b.params, b.n)
    plan.set_tuning(variant=8)
    acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()[:, targets]
    s = parity.summary(acc, ref)
    print("cfg2 split-table variant sampled", s)
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4
