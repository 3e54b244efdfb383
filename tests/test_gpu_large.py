"""GPU runs at the workloads' full sizes, checked on sampled targets.

* precision study, 16.8 M clustered particles: the FP32 kernel (FP64 block
  origins, FP32 pairs, Kahan sums) against the FP64 GPU kernel for every
  particle, both against the FP64 oracle on sampled targets, and the
  arithmetic ablations (Newton step on, Kahan off, box-origin offsets);
* the large 134 M-particle box, sampled against the oracle.

Each prints one JSON summary line (``PRECISION ...``, ``LARGE ...``).
"""
import json
import math
import time

import numpy as np
import pytest

import workloads as W
from tests import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09824_amd as m
    return m


def rel_err(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nrm = np.linalg.norm(ref, axis=0)
    ok = nrm > 0
    return np.linalg.norm(a[:, ok] - ref[:, ok], axis=0) / nrm[ok]


def pct(e):
    return {"median": parity.nearest_rank(e, 50), "p999": parity.nearest_rank(e, 99.9),
            "max": float(np.max(e)) if e.size else 0.0}


def test_precision_study_16M(pp, oracle_mod):
    t0 = time.time()
    b = W.make_config(3)
    print(f"generated {b.n} particles in {time.time() - t0:.1f} s", flush=True)
    pos = torch.tensor(b.pos, device="cuda")
    mass = torch.tensor(b.mass, device="cuda")
    plan = pp.Plan(b.params, b.n)
    plan.set_timing(True)
    acc32 = plan.accel(pos, mass)
    st = plan.stats()
    t32 = st["pp_kernel_ms"]
    inter = plan.count_interactions()
    a32 = acc32.cpu().numpy()
    print(f"fp32 kernel {t32:.1f} ms, {inter} interactions", flush=True)
    acc64 = plan.accel_f64(pos, mass.double())
    t64 = plan.stats()["pp_kernel_ms"]
    a64 = acc64.cpu().numpy()
    print(f"fp64 kernel {t64:.1f} ms", flush=True)
    rng = np.random.default_rng(3)
    targets = np.sort(rng.choice(b.n, 192, replace=False))
    ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, targets=targets)
    s64 = parity.summary(a64[:, targets], ref)
    s32 = parity.summary(a32[:, targets], ref)
    e32_64 = rel_err(a32, a64)
    out = {"n": b.n, "interactions": inter,
           "fp32": {"kernel_ms": t32, "interactions_per_s": inter / (t32 * 1e-3),
                    "vs_fp64_gpu_all": pct(e32_64), "vs_oracle_sample": s32},
           "fp64": {"kernel_ms": t64, "interactions_per_s": inter / (t64 * 1e-3),
                    "vs_oracle_sample": s64}}
    ablations = {}
    for var, name in [(1, "newton"), (2, "no_kahan"), (4, "box_origin"), (6, "no_kahan_box_origin")]:
        plan.set_tuning(variant=var)
        a = plan.accel(pos, mass).cpu().numpy()
        ablations[name] = {"vs_fp64_gpu_all": pct(rel_err(a, a64)), "kernel_ms": plan.stats()["pp_kernel_ms"]}
        print(name, ablations[name], flush=True)
    plan.set_tuning(variant=0)
    out["ablations"] = ablations
    print("PRECISION " + json.dumps(out), flush=True)
    assert s64["median"] <= 1e-12
    assert s32["median"] <= 1e-6 and s32["p999"] <= 1e-4
    assert out["fp32"]["vs_fp64_gpu_all"]["median"] <= 1e-6
    assert out["fp32"]["vs_fp64_gpu_all"]["p999"] <= 1e-4
    # the FP64 block origins are what keep the close pairs precise
    assert ablations["box_origin"]["vs_fp64_gpu_all"]["median"] > out["fp32"]["vs_fp64_gpu_all"]["median"]


def test_large_134M_sampled(pp, oracle_mod):
    t0 = time.time()
    b = W.make_config(5)
    print(f"generated {b.n} particles in {time.time() - t0:.1f} s", flush=True)
    pos = torch.tensor(b.pos, device="cuda")
    mass = torch.tensor(b.mass, device="cuda")
    plan = pp.Plan(b.params, b.n)
    plan.set_timing(True)
    t1 = time.time()
    acc = plan.accel(pos, mass)
    torch.cuda.synchronize()
    wall = time.time() - t1
    st = plan.stats()
    print(f"accel {wall:.1f} s, kernel {st['pp_kernel_ms']:.0f} ms, lists {st}", flush=True)
    a = acc.cpu().numpy()
    del acc
    rng = np.random.default_rng(5)
    targets = np.sort(rng.choice(b.n, 64, replace=False))
    t2 = time.time()
    ref = oracle_mod.accel(b.pos, b.mass.astype(np.float64), b.params, targets=targets)
    print(f"oracle sample {time.time() - t2:.1f} s", flush=True)
    s = parity.summary(a[:, targets], ref)
    inter_sample = int(ref["n_inter"].sum())
    est_total = inter_sample / targets.size * b.n
    out = {"n": b.n, "step_s": wall, "pp_kernel_ms": st["pp_kernel_ms"],
           "estimated_interactions": est_total,
           "estimated_interactions_per_s_kernel": est_total / (st["pp_kernel_ms"] * 1e-3),
           "vs_oracle_sample": s, "lists": {k: st[k] for k in ("nleaf", "nblock", "nrange", "nitem")}}
    print("LARGE " + json.dumps(out), flush=True)
    assert s["zero_ok"]
    assert s["median"] <= 1e-6 and s["p999"] <= 1e-4
