"""GPU tests of the batched form (many boxes, one persistent work-stealing
launch replayed from a hipGraph) and of the launch-shape options.

The batched path must give, box by box, bit-identical accelerations to one
plain pp_accel per box (same lists, same work items, fixed-order
reductions), must match the FP64 oracle to the same tolerances, and graph
replays must repeat the eager result exactly, with other GPU work between
the replays.
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


def small_batch(nbox=7, seed=5):
    rng = np.random.default_rng(seed)
    boxes = []
    for b in range(nbox):
        n = int(rng.integers(1, 6000)) if b != 3 else 1
        L = float(rng.uniform(20.0, 80.0))
        frac = float(rng.uniform(0.0, 0.8))
        n_mesh = max(12, int(round(n ** (1 / 3))))
        pos = W.mixture(rng, n, L, frac, max(1, n // 500))
        boxes.append(W.Box(pos=pos, mass=rng.uniform(0.5, 1.5, n).astype(np.float32),
                           params=BoxParams.from_mesh(L, n_mesh), name=f"b{b}"))
    return boxes


def concat(boxes):
    pos = np.concatenate([b.pos for b in boxes], axis=1)
    mass = np.concatenate([b.mass for b in boxes])
    return pos, mass


def test_batch_bit_identical_to_per_box(pp):
    boxes = small_batch()
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    acc = bp.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    off = 0
    for b in boxes:
        plan = pp.Plan(b.params, b.n)
        a1 = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()
        assert np.array_equal(acc[:, off:off + b.n], a1), b.name
        off += b.n


def test_batch_vs_oracle(pp, oracle_mod):
    boxes = small_batch(5, seed=11)
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    acc = bp.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    tot, counts = bp.count_interactions(per_target=True)
    off = 0
    n_inter = 0
    for b in boxes:
        ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params)
        s = parity.summary(acc[:, off:off + b.n], ref)
        assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, (b.name, s)
        assert np.array_equal(counts.cpu().numpy()[off:off + b.n], ref["n_inter"]), b.name
        n_inter += int(ref["n_inter"].sum())
        off += b.n
    assert tot == n_inter


def test_graph_replays_repeat_eager(pp):
    boxes = small_batch(6, seed=3)
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    p, m = dev(pos, torch.float64), dev(mass, torch.float32)
    bp.set_tuning(use_graph=0)
    eager = bp.accel(p, m).cpu().numpy()
    bp.set_tuning(use_graph=1)
    out = torch.empty((3, bp.N), dtype=torch.float32, device="cuda")
    for r in range(4):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()      # unrelated eager work between replays
        bp.accel(p, m, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), r
        assert torch.isfinite(junk)


def test_graph_recaptured_after_chunk_change(pp):
    """The chunk the work items are cut with is a kernel argument baked into
    the captured graph: after set_tuning(chunk=...) the replay must give what
    the same chunk gives without a graph, bit for bit."""
    boxes = small_batch(6, seed=31)
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    p, m = dev(pos, torch.float64), dev(mass, torch.float32)
    assert bp.get_tuning()["use_graph"] == 1
    bp.accel(p, m)
    bp.accel(p, m)                                   # a replay at the default chunk
    bp.set_tuning(chunk=128)
    got = bp.accel(p, m).cpu().numpy()
    got2 = bp.accel(p, m).cpu().numpy()
    bp.set_tuning(use_graph=0)
    ref = bp.accel(p, m).cpu().numpy()
    assert bp.stats()["nitem"] > bp.stats()["nblock"]   # the small chunk splits lists
    assert np.array_equal(got, ref) and np.array_equal(got2, ref)


def test_graph_recaptured_after_smaller_n(pp):
    """The particle count (the row stride of the SoA arrays) is a kernel
    argument too: a plan replaying its graph at n and then at n/2 must give
    the non-graph results, and write nothing past 3 (n/2) floats."""
    b = W.make_config(1)
    n2 = b.n // 2
    plan = pp.Plan(b.params, b.n)
    plan.set_tuning(persistent=1, use_graph=1)
    ref_plan = pp.Plan(b.params, b.n)
    p, m = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    full = plan.accel(p, m).cpu().numpy()
    assert np.array_equal(full, ref_plan.accel(p, m).cpu().numpy())
    p2, m2 = p[:, :n2].contiguous(), m[:n2].contiguous()
    buf = torch.full((3 * b.n,), 7.0, dtype=torch.float32, device="cuda")
    out = buf[:3 * n2].view(3, n2)
    plan.accel(p2, m2, out=out)
    half = out.cpu().numpy()
    assert np.array_equal(half, ref_plan.accel(p2, m2).cpu().numpy())
    assert torch.all(buf[3 * n2:] == 7.0)
    again = plan.accel(p, m).cpu().numpy()
    assert np.array_equal(again, full)


@pytest.mark.parametrize("tuning", [dict(persistent=1, waves_per_cu=4), dict(chunk=256),
                                    dict(chunk=64, persistent=1, waves_per_cu=1),
                                    dict(persistent=1, use_graph=1, waves_per_cu=32),
                                    dict(waves_per_block=2), dict(waves_per_block=4, chunk=8192),
                                    dict(waves_per_block=4, chunk=256, persistent=0),
                                    dict(waves_per_block=2, persistent=1, use_graph=1, waves_per_cu=7),
                                    dict(waves_per_block=4, variant=8),
                                    dict(waves_per_block=8, chunk=8192),
                                    dict(waves_per_block=8, chunk=512, persistent=0),
                                    dict(waves_per_block=8, persistent=1, use_graph=1, waves_per_cu=24)])
def test_launch_shapes_agree(pp, tuning):
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    p, m = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    base = plan.accel(p, m).cpu().numpy()
    plan.set_tuning(**tuning)
    got = plan.accel(p, m).cpu().numpy()
    again = plan.accel(p, m).cpu().numpy()
    assert np.array_equal(got, again)                # reproducible for a given tuning
    if "chunk" in tuning or "waves_per_block" in tuning or "variant" in tuning:
        # a different chunk or split among waves changes the summation order
        assert np.allclose(got, base, rtol=1e-5, atol=1e-6 * np.abs(base).max())
    else:
        assert np.array_equal(got, base)


def test_kernel_counters_agree_across_launch_shapes(pp):
    """Every work item runs exactly once in every launch shape: the
    kernel's counters of evaluated pairs and lane-pairs (sums over the
    sources each item stages) do not depend on the chunk, the waves per
    block or the launch form, and bound the interaction count from above."""
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    p, m = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    plan.accel(p, m)
    inter = plan.count_interactions()
    seen = set()
    for t in [dict(chunk=2048, waves_per_block=1, persistent=0), dict(chunk=256, waves_per_block=1, persistent=0),
              dict(chunk=256, waves_per_block=1, persistent=1, waves_per_cu=12),
              dict(chunk=1024, waves_per_block=2, persistent=1, waves_per_cu=20),
              dict(chunk=4096, waves_per_block=4, persistent=0),
              dict(chunk=4096, waves_per_block=4, persistent=1, waves_per_cu=32),
              dict(chunk=8192, waves_per_block=8, persistent=1, waves_per_cu=24)]:
        plan.set_tuning(use_graph=0, **t)
        plan.accel(p, m)
        torch.cuda.synchronize()
        st = plan.stats()
        seen.add((st["evaluated"], st["lane_pairs"]))
        assert inter <= st["evaluated"] <= st["lane_pairs"], t
    assert len(seen) == 1, seen


@pytest.mark.parametrize("k,persistent", [(2, 1), (4, 1), (4, 0), (8, 1)])
def test_waves_per_block_vs_oracle(pp, oracle_mod, k, persistent):
    """K waves sharing a target block: the oracle's tolerances on the 32k
    box and on a ragged clustered box with lists spanning several items."""
    for b in (W.make_config(1),
              W.Box(pos=W.mixture(np.random.default_rng(41), 9001, 40.0, 0.8, 6),
                    mass=np.random.default_rng(42).uniform(0.5, 1.5, 9001).astype(np.float32),
                    params=BoxParams.from_mesh(40.0, 20), name="ragged")):
        plan = pp.Plan(b.params, b.n)
        plan.set_tuning(waves_per_block=k, persistent=persistent, chunk=256 * min(k, 4))
        acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()
        assert plan.stats()["nitem"] > plan.stats()["nblock"]
        ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, pair_abs=True)
        s = parity.summary(acc, ref)
        assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, (b.name, s)
        assert s["robust_max"] <= parity.ROBUST_MAX, (b.name, s)


def test_batch_bit_identical_with_waves_per_block(pp):
    boxes = small_batch(5, seed=17)
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    bp.set_tuning(waves_per_block=4, chunk=1024)
    acc = bp.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    off = 0
    for b in boxes:
        plan = pp.Plan(b.params, b.n)
        plan.set_tuning(waves_per_block=4, chunk=1024)
        a1 = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()
        assert np.array_equal(acc[:, off:off + b.n], a1), b.name
        off += b.n


def test_tuning_validation(pp):
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    for bad in [dict(chunk=100), dict(chunk=0), dict(waves_per_cu=0), dict(use_graph=1, persistent=0),
                dict(waves_per_block=3), dict(waves_per_block=0), dict(waves_per_block=16),
                dict(waves_per_block=2, variant=1), dict(waves_per_block=8, variant=4)]:
        with pytest.raises(pp.PPError):
            plan.set_tuning(**{**dict(chunk=4096, persistent=0, waves_per_cu=16, use_graph=0), **bad})


def test_autotune_and_cache(pp, tmp_path):
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    p, m = dev(b.pos, torch.float64), dev(b.mass, torch.float32)
    base = plan.accel(p, m).cpu().numpy()
    cache = str(tmp_path / "tune.txt")
    t = plan.autotune(p, m, cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1] == str(t["chunk"])
    plan2 = pp.Plan(b.params, b.n)
    t2 = plan2.autotune(p, m, cache)           # served from the cache
    assert t2 == t
    got = plan2.accel(p, m).cpu().numpy()
    assert np.allclose(got, base, rtol=1e-5, atol=1e-6 * np.abs(base).max())


@pytest.mark.parametrize("variant", [1, 2, 4, 6])
def test_variants_run_and_stay_close(pp, oracle_mod, variant):
    b = W.make_config(1)
    plan = pp.Plan(b.params, b.n)
    plan.set_tuning(variant=variant)
    acc = plan.accel(dev(b.pos, torch.float64), dev(b.mass, torch.float32)).cpu().numpy()
    ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params)
    s = parity.summary(acc, ref)
    assert s["zero_ok"] and s["p999"] <= 1e-3, (variant, s)
    if variant in (1, 2):
        assert s["median"] <= 1e-6, (variant, s)


def test_equal_mass_boxes_mixed_with_unequal(pp, oracle_mod):
    """Boxes whose masses are all equal take the shorter pair loop (the mass
    joins the final scale); boxes with unequal masses in the same batch keep
    the general loop.  Both kinds must match the oracle, and nudging one mass
    by one ulp (which switches that box to the general loop) may move the
    result only by rounding."""
    boxes = small_batch(6, seed=23)
    for k in (0, 2, 4):
        boxes[k].mass[:] = np.float32(1.0 / max(1, boxes[k].n))
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    acc = bp.accel(dev(pos, torch.float64), dev(mass, torch.float32)).cpu().numpy()
    off = 0
    for b in boxes:
        ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params)
        s = parity.summary(acc[:, off:off + b.n], ref)
        assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, (b.name, s)
        off += b.n
    nudged = mass.copy()
    nudged[boxes[0].n // 2] = np.nextafter(nudged[boxes[0].n // 2], np.float32(1))
    acc2 = bp.accel(dev(pos, torch.float64), dev(nudged, torch.float32)).cpu().numpy()
    a, c = acc[:, :boxes[0].n], acc2[:, :boxes[0].n]
    mag = np.linalg.norm(a, axis=0)
    rel = np.linalg.norm(a - c, axis=0) / np.where(mag > 0, mag, 1)
    assert np.median(rel) <= 1e-6 and rel.max() <= 1e-4
    assert np.array_equal(acc[:, boxes[0].n:], acc2[:, boxes[0].n:])


def test_full_64_box_batch_sampled(pp, oracle_mod):
    """The benchmark's batch (64 boxes, about 32 M particles) in the launch
    configuration it is timed in (persistent kernel replayed from a graph),
    on 256 seeded targets of every 8th box against the FP64 oracle."""
    boxes = W.make_batch()
    pos, mass = concat(boxes)
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    assert bp.get_tuning()["use_graph"] == 1 and bp.get_tuning()["persistent"] == 1
    P, M = dev(pos, torch.float64), dev(mass, torch.float32)
    bp.accel(P, M)
    acc = bp.accel(P, M).cpu().numpy()                 # a graph replay
    rng = np.random.default_rng(1803)
    off = np.cumsum([0] + [b.n for b in boxes])
    for k in range(0, len(boxes), 8):
        b = boxes[k]
        t = np.sort(rng.choice(b.n, min(b.n, 256), replace=False))
        ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, targets=t, pair_abs=True)
        s = parity.summary(acc[:, off[k] + t], ref)
        assert s["zero_ok"] and s["median"] <= 1e-6 and s["p999"] <= 1e-4, (b.name, s)
        assert s["robust_max"] <= parity.ROBUST_MAX, (b.name, s)
