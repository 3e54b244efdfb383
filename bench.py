#!/usr/bin/env python3
"""Benchmark of the short-range PP gravity path on one MI355X.

One step = the whole path on one box resident in HBM: Peano-Hilbert keys,
key sort and gather, octree leaves, near lists, the FP32 PP kernel and the
scatter back to input order (pp_accel).  The workload is the plain-kernel
headline set: 128^3 = 2,097,152 equal-mass particles in a periodic box of
200 Mpc/h, half uniform and half in 2000 Plummer spheres (dN/dM ~ M^-1.9),
PM mesh 128^3, r_s = 1.25 cells, r_cut = 4.5 r_s, eps = 0.02 cells.

Prints one JSON line.  value = interactions (ordered pairs with s < r_cut)
per second of whole steps.  roofline: the PP kernel's FP32 flop rate (its
stated per-interaction count x interactions / kernel time from HIP events
on the launch stream) against the FP32 vector peak.  cpu_baseline: the FP64
CPU oracle timed on this host on a bounded sample of targets.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PP pair-interactions/s and % FP32 VALU peak; batched vs plain at fixed error"
# FP32 operations the PP kernel performs per evaluated pair (an FMA counts 2):
# 3 sub (d), 3 FMA (s^2 + eps^2), 1 rsqrt, 1 sub (polynomial variable t),
# 9 FMA (degree-9 polynomial), 1 mul + 1 FMA (y^3 - H), 3 FMA (sum) = 38;
# boxes whose masses differ add 1 mul (the source mass) = 39.  Compares and
# selects are not counted; the compensated sum is amortised over 64-pair
# tiles.  The hardware FP32 flop counter, per evaluated lane-pair, is the
# cross-check (it also sees the FP32 work of staging the sources).
FLOPS_EQUAL_MASS = 38
FLOPS_GENERAL = 39
PAPER_FLOPS_PER_INTERACTION = 22      # convention of sec. 5 (Newtonian pair count)
FP32_VECTOR_PEAK = 157.3e12           # MI355X, 256 CU x 2.4 GHz x 256 flop/clk
# HBM bytes per PP-kernel launch on the headline workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE passes (KiB per dispatch) scaled by what the same
# counters read for a plain 1 GiB copy (factors below), one pair of passes
# per launch shape the autotuner is likely to pick.  Valid only for the
# kernel sources they were taken on (SHA-1 over the files listed) and for a
# measured launch shape; otherwise the roofline reports null.  The SHA-1 is
# moved forward only over edits that leave the machine code and metadata of
# every kernel already built identical (compared function by function in the
# gfx950 code objects built before and after).
TRAFFIC = {
    "sources": ["paper_1802_09824_amd/csrc/pp_kernels.hip",
                "paper_1802_09824_amd/csrc/pp_internal.h",
                "paper_1802_09824_amd/csrc/tree.hip"],
    "sha1": "720ab4d49720f40a153c28a79d3c85e7edaf4e64",
    "fetch_scale": 1.99996,       # 1 GiB copy: 1048576 KiB / 524299.5 KiB of FETCH_SIZE
    "write_scale": 1.00000,       # 1 GiB copy: 1048576 KiB / 1048576.0 KiB of WRITE_SIZE
    # (chunk, waves per block, waves per CU (0: one workgroup per item), persistent):
    # (FETCH_SIZE KiB, WRITE_SIZE KiB) of the timed step's PP dispatch
    "kib": {
        (1024, 1, 0, 0): (98508.5, 183744.5),
        (1024, 1, 12, 1): (125898.2, 177636.7),
        (1024, 1, 20, 1): (146260.6, 178276.7),
        (1024, 1, 24, 1): (164353.3, 178596.7),
        (1024, 1, 32, 1): (162324.5, 179108.7),
        (2048, 1, 0, 0): (105528.3, 108829.9),
        (2048, 1, 12, 1): (140234.6, 106034.8),
        (2048, 1, 20, 1): (186092.7, 106656.2),
        (2048, 1, 24, 1): (211390.6, 106965.2),
        (2048, 1, 32, 1): (211354.8, 107477.7),
        (2048, 2, 20, 1): (139695.2, 106031.5),
        (2048, 2, 24, 1): (139916.9, 106156.1),
        (2048, 2, 32, 1): (137368.6, 106416.7),
        (4096, 1, 20, 1): (310858.3, 137882.4),
        (4096, 1, 32, 1): (365708.2, 138533.8),
        (4096, 2, 20, 1): (201871.1, 137840.6),
        (4096, 2, 24, 1): (199949.9, 137962.2),
        (4096, 2, 32, 1): (202702.9, 138224.7),
        (4096, 4, 0, 0): (107140.8, 152063.1),
        (4096, 4, 12, 1): (141256.6, 137574.5),
        (4096, 4, 20, 1): (152858.9, 137806.2),
        (4096, 4, 24, 1): (152999.6, 137875.5),
        (4096, 4, 32, 1): (153520.7, 137999.6),
        (8192, 2, 32, 1): (264249.4, 180883.7),
        (8192, 4, 0, 0): (117253.4, 190447.5),
        (8192, 4, 12, 1): (153192.7, 180898.8),
        (8192, 4, 20, 1): (186151.2, 180916.6),
        (8192, 4, 24, 1): (186111.5, 180942.6),
        (8192, 4, 32, 1): (186622.2, 181113.0),
        (8192, 8, 20, 1): (154129.4, 180899.1),
        (8192, 8, 32, 1): (151935.3, 180978.5),
        (16384, 4, 20, 1): (195679.2, 195550.9),
        (16384, 4, 24, 1): (198638.8, 195604.2),
        (16384, 4, 32, 1): (198745.4, 195723.9),
        (16384, 8, 20, 1): (160202.6, 195599.1),
        (16384, 8, 32, 1): (160010.7, 195668.2),
    },
}


def sources_sha1(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tuning):
    """HBM bytes per launch of the PP kernel at this launch shape, or None if
    the shape was not measured or the kernel sources changed since."""
    t = TRAFFIC
    if t["sha1"] is None or t["fetch_scale"] is None:
        return None
    key = (tuning["chunk"], tuning["waves_per_block"], tuning["waves_per_cu"] if tuning["persistent"] else 0,
           tuning["persistent"])
    if key not in t["kib"]:
        return None
    try:
        if sources_sha1(t["sources"]) != t["sha1"]:
            return None
    except OSError:
        return None
    fetch, write = t["kib"][key]
    return 1024.0 * (fetch * t["fetch_scale"] + write * t["write_scale"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-box batched-vs-per-box comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the monopole and adaptive-KDK legs (for profiling runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 64-box batched-vs-per-box comparison (for profiling)")
    ap.add_argument("--only-small-box", action="store_true",
                    help="run only the 32k uniform box's whole-step leg (for profiling)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 16.8M precision and 134M large-box legs")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tiles instead of running the autotuner first")
    ap.add_argument("--tuning", default=None, metavar="CHUNK,WAVES_PER_BLOCK,WAVES_PER_CU[,PERSISTENT]",
                    help="run the headline box with this launch shape instead of autotuning (for "
                         "profiling runs of a known launch shape); PERSISTENT 0 is one workgroup "
                         "per item, default 1")
    ap.add_argument("--print-sources-sha1", action="store_true",
                    help="print the SHA-1 of the PP kernel sources the traffic figure is tied to")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (reference kernel "
                         "for scaling the HBM byte counters of a profiler run)")
    return ap.parse_args()


_T0 = time.perf_counter()


def progress(leg):
    """One line on stderr when a leg ends (the JSON line stays on stdout)."""
    print(f"bench: {leg} done at {time.perf_counter() - _T0:.0f} s", file=sys.stderr, flush=True)


def nearest_rank(x, q):
    import numpy as np
    x = np.sort(np.asarray(x))
    if x.size == 0:
        return 0.0
    return float(x[max(1, int(math.ceil(q / 100.0 * x.size))) - 1])


def host_cores():
    """Cores this process may run on (what `nproc` prints)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_baseline(box, acc_gpu, budget_s):
    """Time the FP64 oracle on a seeded sample of targets; compare the GPU
    accelerations of the same targets."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(1802)
    mass64 = box.mass.astype(np.float64)
    probe = np.sort(rng.choice(box.n, 512, replace=False))
    t0 = time.perf_counter()
    oracle.accel(box.pos, mass64, box.params, targets=probe)
    dt = max(time.perf_counter() - t0, 1e-3)
    k = int(min(box.n, max(512, 512 * budget_s / dt)))
    targets = np.sort(rng.choice(box.n, k, replace=False))
    t0 = time.perf_counter()
    ref = oracle.accel(box.pos, mass64, box.params, targets=targets)
    sec = time.perf_counter() - t0
    inter = int(ref["n_inter"].sum())
    checks = k * (box.n - 1)
    base = {"value": inter / sec, "unit": "interactions/s", "cores": host_cores(),
            "threads": oracle.num_threads(), "kind": "oracle",
            "pair_checks_per_s": checks / sec,
            "sample": f"{k} seeded random targets of the same box against all {box.n} sources "
                      f"(FP64 direct sum over every source: {checks} pair distance checks, "
                      f"{inter} of them within the cut, {sec:.1f} s)"}
    errs = sample_errors(acc_gpu, targets, ref)
    # condition-robust error |a - a*| / sum_j |a_ij| on every 8th sampled
    # target (a second, untimed oracle call that also sums the pair magnitudes)
    sub = targets[::8]
    rs = oracle.accel(box.pos, mass64, box.params, targets=sub, pair_abs=True)
    a = acc_gpu[:, sub].astype(np.float64)
    r = rs["acc"]
    cands = [r, r - rs["band_in"] + rs["band_out"], r - rs["band_in"], r + rs["band_out"]]
    d = np.min([np.linalg.norm(a - c, axis=0) for c in cands], axis=0)
    has = rs["n_inter"] > 0
    e = d[has] / rs["pair_abs"][has]
    errs["robust"] = {"targets": int(has.sum()), "p999": nearest_rank(e, 99.9),
                      "max": float(e.max()) if e.size else 0.0}
    return base, errs, targets, ref


def sample_errors(acc_gpu, targets, ref):
    """Band-tolerant relative errors of GPU accelerations on oracle targets."""
    import numpy as np
    a = acc_gpu[:, targets].astype(np.float64)
    r = ref["acc"]
    cands = [r, r - ref["band_in"] + ref["band_out"], r - ref["band_in"], r + ref["band_out"]]
    err = np.min([np.linalg.norm(a - c, axis=0) for c in cands], axis=0)
    norm = np.linalg.norm(r, axis=0)
    has = ref["n_inter"] > 0
    e = err[has] / norm[has]
    return {"targets": int(has.sum()), "median": nearest_rank(e, 50), "p999": nearest_rank(e, 99.9),
            "max": float(e.max()) if e.size else 0.0,
            "zero_neighbour_exact": bool(np.all(a[:, ~has] == 0))}


def batched_error(boxes, acc_batched, per_box_targets=256, every=8):
    """Errors of the batched result against the FP64 oracle on a seeded
    sample of targets of every 8th box (the same tolerance as the plain path)."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(1803)
    off = np.cumsum([0] + [b.n for b in boxes])
    es = []
    for k in range(0, len(boxes), every):
        b = boxes[k]
        t = np.sort(rng.choice(b.n, min(b.n, per_box_targets), replace=False))
        ref = oracle.accel(b.pos, b.mass.astype(np.float64), b.params, targets=t)
        a = acc_batched[:, off[k] + t].astype(np.float64)
        r = ref["acc"]
        cands = [r, r - ref["band_in"] + ref["band_out"], r - ref["band_in"], r + ref["band_out"]]
        err = np.min([np.linalg.norm(a - c, axis=0) for c in cands], axis=0)
        norm = np.linalg.norm(r, axis=0)
        has = ref["n_inter"] > 0
        es.append(err[has] / norm[has])
    e = np.concatenate(es) if es else np.zeros(0)
    return {"boxes": len(range(0, len(boxes), every)), "targets": int(e.size),
            "median": nearest_rank(e, 50), "p999": nearest_rank(e, 99.9),
            "max": float(e.max()) if e.size else 0.0}


def drifted(pos_t, params, seed):
    """Positions one small step later: every particle moved by 0.02 r_s per
    axis (Gaussian), wrapped.  The step before them gives the reference
    accelerations of the relative opening test, as in a simulation."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    step = torch.randn(pos_t.shape, generator=g, device="cuda", dtype=torch.float64) * (0.02 * params.rs)
    return torch.remainder(pos_t + step, params.L).contiguous()


def bench_monopoles(plan, box, pos, mass, theta=0.3, alpha=0.005, steps=3):
    """Monopole acceptance (sec. 3.3 dual walk, Gadget-2's relative test of
    sec. 3.1) one step after the reference accelerations were taken: the
    exact FP32 accelerations at the current positions serve as a_ref, the
    particles drift by a small step, and the monopole result at the new
    positions is compared with the exact one there (all targets), and timed
    against the exact path."""
    import numpy as np
    import torch
    acc_ref = plan.accel(pos, mass)                          # previous step's forces
    pos1 = drifted(pos, box.params, 1234)
    exact = plan.accel(pos1, mass)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.accel(pos1, mass, out=exact)
    torch.cuda.synchronize()
    exact_ms = 1e3 * (time.perf_counter() - t0) / steps
    plan.set_monopole(theta)
    plan.set_monopole_relative(alpha, acc_ref)
    acc = plan.accel(pos1, mass)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.accel(pos1, mass, out=acc)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = plan.stats()
    mag = torch.linalg.vector_norm(exact.double(), dim=0)
    err = torch.linalg.vector_norm(acc.double() - exact.double(), dim=0)
    keep = mag > 0
    e = (err[keep] / mag[keep]).cpu().numpy()
    plan.set_monopole(0.0)
    plan.set_monopole_relative(0.0)
    del acc_ref, pos1, exact, acc
    return {"theta": theta, "alpha": alpha, "a_ref": "exact FP32 forces one drift step earlier "
            "(0.02 r_s Gaussian per axis)", "ms_per_step": ms, "exact_ms_per_step": exact_ms,
            "speedup": exact_ms / ms, "monopole_pairs": int(st["monopoles"]),
            "lane_pairs": int(st["lane_pairs"]) if st["lane_pairs"] >= 0 else None,
            "error_vs_exact": {"particles": int(e.size), "median": nearest_rank(e, 50),
                               "p999": nearest_rank(e, 99.9), "max": float(e.max())}}


def bench_kdk(box, pos, mass, acc_exact, n_mesh=128, eta=0.025, max_level=6, steps=2, skin=0.0):
    """Adaptive block-step KDK over the whole force (PP + PM) on the same box:
    the top step is twice the median particle's step criterion, so the
    particles spread over several levels; sub-steps evaluate the short-range
    force for the particles whose step ends only.  skin > 0: the sub-steps
    reuse the short-range lists (built with the cut widened by skin) while
    no particle has moved skin / 2."""
    import numpy as np
    import torch
    import paper_1802_09824_amd as pp
    amag = np.linalg.norm(acc_exact.cpu().numpy().astype(np.float64), axis=0)
    dt = 2.0 * math.sqrt(2.0 * eta * box.params.eps / float(np.median(amag)))
    P = pos.clone()
    rng = np.random.default_rng(3)
    V = torch.tensor(rng.normal(scale=1e-3, size=(3, box.n)), device="cuda")
    K = pp.KDK(box.params, box.n, n_mesh=n_mesh, eta=eta, max_level=max_level)
    K.set_skin(skin)
    K.init(P, mass)
    K.step(P, V, mass, dt)
    torch.cuda.synchronize()
    i0 = K.info()
    t0 = time.perf_counter()
    for _ in range(steps):
        K.step(P, V, mass, dt)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    i1 = K.info()
    evals = (i1["force_evaluations"] - i0["force_evaluations"]) / steps
    targets = (i1["short_range_targets"] - i0["short_range_targets"]) / steps
    builds = (i1["list_builds"] - i0["list_builds"]) / steps
    del K
    return {"n_mesh": n_mesh, "eta": eta, "dt": dt, "skin": skin, "ms_per_top_step": 1e3 * sec,
            "force_evaluations_per_top_step": evals, "list_builds_per_top_step": builds,
            "short_range_targets_per_top_step": targets,
            "fraction_of_full_short_range": targets / (evals * box.n),
            "level_count": i1["level_count"][:max_level + 1]}


def bench_small_box(steps=20, tune=True):
    """The 32,768-particle uniform box (L = 100), one whole pp_accel step
    per call: few work items, so the tiles are autotuned for it like the
    headline box's (default tiles reported beside)."""
    import torch
    import workloads
    import paper_1802_09824_amd as pp
    b = workloads.make_config(1)
    pos = torch.tensor(b.pos, device="cuda")
    mass = torch.tensor(b.mass, device="cuda")
    plan = pp.Plan(b.params, b.n)
    acc = plan.accel(pos, mass)
    inter = plan.count_interactions()

    def timed():
        for _ in range(3):
            plan.accel(pos, mass, out=acc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.accel(pos, mass, out=acc)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    sec_default = timed()
    tuning = plan.autotune(pos, mass) if tune else plan.get_tuning()
    sec = timed()
    del plan
    return {"workload": b.name, "n": b.n, "interactions_per_step": inter, "ms_per_step": 1e3 * sec,
            "interactions_per_s": inter / sec, "tuning": tuning, "ms_per_step_default_tiles": 1e3 * sec_default}


def bench_pm(box, pos, mass, n_mesh, steps, with_error=True):
    """The long-range PM force of the same box (pp_pm_accel): CIC, FFTs,
    Green function with the Gaussian filter, gradient, interpolation.
    Timed with events on the stream the library launches on."""
    import numpy as np
    import torch
    import paper_1802_09824_amd as pp
    plan = pp.PMPlan(box.params, n_mesh)
    acc = torch.empty((3, box.n), dtype=torch.float32, device="cuda")
    for _ in range(2):
        plan.accel(pos, mass, out=acc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plan.accel(pos, mass, out=acc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"n_mesh": n_mesh, "ms_per_call": ms, "particles_per_s": box.n / (ms * 1e-3)}
    if with_error:
        from oracle import pm as opm
        ref = opm.pm_accel(box.pos, box.mass.astype(np.float64), box.params, n_mesh)
        a = acc.cpu().numpy().astype(np.float64)
        mag = np.linalg.norm(ref, axis=0)
        floor = 1e-6 * np.sqrt(np.mean(mag ** 2))
        e = np.linalg.norm(a - ref, axis=0) / np.maximum(mag, floor)
        res["error_vs_oracle"] = {"particles": int(box.n), "median": nearest_rank(e, 50),
                                  "p999": nearest_rank(e, 99.9), "max": float(e.max())}
    del plan
    return res


def gpu_rel_errors(a, ref):
    """Nearest-rank median, 99.9th percentile and max of |a - ref| / |ref|
    over targets with ref != 0, computed on the device."""
    import torch
    mag = torch.linalg.vector_norm(ref.double(), dim=0)
    err = torch.linalg.vector_norm(a.double() - ref.double(), dim=0)
    keep = mag > 0
    e = torch.sort(err[keep] / mag[keep]).values
    n = e.numel()
    def rank(q):
        return float(e[max(1, math.ceil(q / 100.0 * n)) - 1]) if n else 0.0
    return {"targets": int(n), "median": rank(50), "p999": rank(99.9), "max": float(e[-1]) if n else 0.0}


def bench_precision(steps=3):
    """The 16.8M-particle clustered box (L = 400, 8000 spheres): the FP32
    kernel (FP64 block origins, FP32 pairs, compensated sums) against the
    FP64 kernel on the same lists: rates, and the FP32 error over all targets
    taking the FP64 result as the reference."""
    import torch
    import workloads
    import paper_1802_09824_amd as pp
    box = workloads.make_config(3)
    n = box.n
    pos = torch.tensor(box.pos, device="cuda")
    mass = torch.tensor(box.mass, device="cuda")
    mass64 = mass.double()
    box.pos = None                       # the host copy is not needed any more
    plan = pp.Plan(box.params, n)
    acc = plan.accel(pos, mass)
    inter = plan.count_interactions()
    plan.set_timing(True)
    k32, t0 = [], time.perf_counter()
    for _ in range(steps):
        plan.accel(pos, mass, out=acc)
        k32.append(plan.stats()["pp_kernel_ms"])
    torch.cuda.synchronize()
    step32 = 1e3 * (time.perf_counter() - t0) / steps
    a64 = plan.accel_f64(pos, mass64)
    k64 = plan.stats()["pp_kernel_ms"]
    err = gpu_rel_errors(acc, a64)
    del plan, pos, mass, mass64, acc, a64
    torch.cuda.empty_cache()
    k32m = sum(k32) / len(k32)
    return {"workload": workloads.CONFIGS[3]["name"], "n": n, "interactions_per_step": inter,
            "f32": {"ms_per_step": step32, "kernel_ms": k32m, "interactions_per_s_kernel": inter / (k32m * 1e-3),
                    "interactions_per_s_step": inter / (step32 * 1e-3)},
            "f64_yardstick": {"kernel_ms": k64, "interactions_per_s_kernel": inter / (k64 * 1e-3)},
            "f32_error_vs_f64_all_targets": err}


def bench_large(steps=2, sample_targets=64):
    """The largest single-GPU machine: 134M particles in L = 1000, 60 % in 50000
    Plummer spheres.  Whole-step time, the PP kernel's rate and FP32 peak
    fraction, the error on a seeded sample of targets against the FP64 CPU
    oracle, and monopole acceptance (theta = 0.3, alpha = 0.005) one drift
    step after the reference forces, against the exact path."""
    import numpy as np
    import torch
    import oracle
    import workloads
    import paper_1802_09824_amd as pp
    box = workloads.make_config(5)
    n = box.n
    pos = torch.tensor(box.pos, device="cuda")
    mass = torch.tensor(box.mass, device="cuda")
    plan = pp.Plan(box.params, n)
    acc = plan.accel(pos, mass)
    inter = plan.count_interactions()
    plan.set_timing(True)
    kms, t0 = [], time.perf_counter()
    for _ in range(steps):
        plan.accel(pos, mass, out=acc)
        kms.append(plan.stats()["pp_kernel_ms"])
    torch.cuda.synchronize()
    step = 1e3 * (time.perf_counter() - t0) / steps
    k = sum(kms) / len(kms)
    rng = np.random.default_rng(1805)
    t = np.sort(rng.choice(n, sample_targets, replace=False))
    ref = oracle.accel(box.pos, box.mass.astype(np.float64), box.params, targets=t)
    errs = sample_errors(acc[:, torch.as_tensor(t, device="cuda")].cpu().numpy(),
                         np.arange(t.size), ref)
    box.pos = None                       # the host copy is not needed any more
    mono = bench_monopoles(plan, box, pos, mass, steps=1)
    del plan, pos, mass, acc
    torch.cuda.empty_cache()
    achieved = inter * FLOPS_EQUAL_MASS / (k * 1e-3)
    return {"workload": workloads.CONFIGS[5]["name"], "n": n, "interactions_per_step": inter,
            "ms_per_step": step, "interactions_per_s": inter / (step * 1e-3),
            "kernel_ms": k, "interactions_per_s_kernel": inter / (k * 1e-3),
            "fp32_peak_frac": achieved / FP32_VECTOR_PEAK,
            "error_vs_oracle_sample": errs, "monopoles": mono}


def bench_batched(steps, warmup, with_error=True, tune=True):
    """64 independent boxes (N uniform in 16^3..96^3, L in 50-300 Mpc/h,
    clustered fraction 0-0.8): one batched pp_batch_accel per step (all
    stages over all boxes, one persistent work-stealing PP launch replayed
    from a hipGraph) against 64 separate pp_accel calls per step.  Both
    sides run tiles chosen by the autotuner: the batch its own, every
    per-box plan its own.  Bit identity with per-box runs is checked at equal
    tiles (the batch's)."""
    import numpy as np
    import torch
    import workloads
    import paper_1802_09824_amd as pp

    boxes = workloads.make_batch()
    pos = torch.tensor(np.concatenate([b.pos for b in boxes], axis=1), device="cuda")
    mass = torch.tensor(np.concatenate([b.mass for b in boxes]), device="cuda")
    N = pos.shape[1]
    acc = torch.empty((3, N), dtype=torch.float32, device="cuda")
    bp = pp.BatchPlan([b.params for b in boxes], [b.n for b in boxes])
    batch_tuning = bp.autotune(pos, mass) if tune else bp.get_tuning()
    bp.accel(pos, mass, out=acc)
    interactions = bp.count_interactions()
    for _ in range(warmup):
        bp.accel(pos, mass, out=acc)
    bp.set_timing(True)
    stage_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bp.accel(pos, mass, out=acc)
        stage_ms.append(bp.stats()["pp_stage_ms"])
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / steps
    acc_batched = acc.cpu().numpy()
    err = batched_error(boxes, acc_batched) if with_error else None

    # per box: separate inputs, plans (each tuned on its own box) and launches
    per = []
    tunings = {}
    for b in boxes:
        pb = torch.tensor(b.pos, device="cuda")
        mb = torch.tensor(b.mass, device="cuda")
        ab = torch.empty((3, b.n), dtype=torch.float32, device="cuda")
        plan = pp.Plan(b.params, b.n)
        if tune:
            t = plan.autotune(pb, mb)
            key = (t["chunk"], t["waves_per_block"], t["persistent"], t["waves_per_cu"])
            tunings[key] = tunings.get(key, 0) + 1
        per.append((plan, pb, mb, ab))
    for plan, pb, mb, ab in per:
        plan.accel(pb, mb, out=ab)
        plan.set_timing(True)
    per_stage_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for plan, pb, mb, ab in per:
            plan.accel(pb, mb, out=ab)
            per_stage_ms += plan.stats()["pp_stage_ms"]
    torch.cuda.synchronize()
    t_per = (time.perf_counter() - t0) / steps
    # bit identity at equal tiles
    same = True
    offs = np.cumsum([0] + [x.n for x in boxes])
    for (plan, pb, mb, ab), b, o in zip(per, boxes, offs):
        plan.set_tuning(**{**batch_tuning, "use_graph": 0})
        plan.accel(pb, mb, out=ab)
        same = same and np.array_equal(ab.cpu().numpy(), acc_batched[:, o:o + b.n])
    return {
        "workload": "batch-64-boxes-N16^3..96^3-L50-300",
        "boxes": len(boxes), "particles": int(N), "interactions_per_step": interactions,
        "batched": {"ms_per_step": 1e3 * t_batched, "value": interactions / t_batched,
                    "pp_stage_ms": float(np.mean(stage_ms)), "tuning": batch_tuning},
        "per_box": {"ms_per_step": 1e3 * t_per, "value": interactions / t_per,
                    "pp_stage_ms_sum": per_stage_ms / steps,
                    "tunings": {f"chunk {k[0]} waves/block {k[1]} persistent {k[2]} waves/CU {k[3]}": v
                                for k, v in sorted(tunings.items())}},
        "speedup_whole_step": t_per / t_batched,
        "speedup_pp_stage": (per_stage_ms / steps) / float(np.mean(stage_ms)),
        "bit_identical_to_per_box_at_equal_tiles": bool(same),
        "error_vs_oracle": err,
        "unit": "interactions/s",
    }


def main():
    args = parse()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "repeats": 3}), flush=True)
        return
    if args.print_sources_sha1:
        print(sources_sha1(TRAFFIC["sources"]))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is a single-GPU "
              "kernel library and has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_1802_09824_amd as pp

    if args.only_batched:
        print(json.dumps({"batched_vs_per_box": bench_batched(max(1, min(args.steps, 5)), 1,
                                                              with_error=False,
                                                              tune=not args.no_tune)}), flush=True)
        return
    if args.only_small_box:
        print(json.dumps({"small_box": bench_small_box(steps=max(1, args.steps), tune=not args.no_tune)}),
              flush=True)
        return
    box = workloads.make_config(2)
    p = box.params
    pos = torch.tensor(box.pos, device="cuda")
    mass = torch.tensor(box.mass, device="cuda")
    acc = torch.empty((3, box.n), dtype=torch.float32, device="cuda")
    plan = pp.Plan(p, box.n)
    if args.tuning:
        v = [int(x) for x in args.tuning.split(",")]
        chunk, wpb, wpc = v[:3]
        plan.set_tuning(chunk=chunk, persistent=v[3] if len(v) > 3 else 1, waves_per_cu=wpc, use_graph=0,
                        variant=0, waves_per_block=wpb)
        tuning = plan.get_tuning()
    else:
        tuning = plan.get_tuning() if args.no_tune else plan.autotune(pos, mass)   # untimed, one-off
    plan.accel(pos, mass, out=acc)
    interactions = plan.count_interactions()
    for _ in range(args.warmup):
        plan.accel(pos, mass, out=acc)
    plan.set_timing(True)
    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.accel(pos, mass, out=acc)
        kernel_ms.append(plan.stats()["pp_kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = plan.stats()
    ms_step = 1e3 * elapsed / args.steps
    value = interactions * args.steps / elapsed
    k_ms = float(np.mean(kernel_ms))
    if tuning["persistent"]:
        kname = "pp_f32_persistent"
    else:
        # the one-workgroup-per-item launch takes its two-wave build when the
        # items give at most two waves per SIMD
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        few = tuning["variant"] in (0, 8) and int(st["nitem"]) * tuning["waves_per_block"] <= 2 * 4 * cus
        kname = "pp_f32_kernel_few" if few else "pp_f32_kernel"
    kname += f"<{tuning['variant']}, {tuning['waves_per_block']}>"
    equal_mass = bool(np.all(box.mass == box.mass[0]))
    flops = FLOPS_EQUAL_MASS if equal_mass else FLOPS_GENERAL
    achieved = interactions * flops / (k_ms * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": box.name, "n": box.n, "L": p.L, "n_mesh": 128, "rs": p.rs,
                   "rcut": p.rcut, "eps": p.eps, "G": p.G, "leaf_max": p.leaf_max,
                   "clustered_fraction": 0.5, "spheres": 2000, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
                     "traffic": measured_traffic(tuning), "traffic_unit": "bytes/launch",
                     "kernel": kname, "kernel_ms": k_ms,
                     "flops_per_interaction": flops},
        "tuning": tuning,
        "interactions_per_step": interactions,
        "candidates_per_step": int(st["candidates"]),
        "evaluated_pairs_per_step": int(st["evaluated"]),
        "pp_kernel_evaluated_pairs_per_s": int(st["evaluated"]) / (k_ms * 1e-3),
        "useful_fraction": interactions / max(int(st["evaluated"]), 1),
        "pp_kernel_interactions_per_s": interactions / (k_ms * 1e-3),
        "pct_fp32_peak_paper_22flop": 100.0 * interactions * PAPER_FLOPS_PER_INTERACTION
        / (k_ms * 1e-3) / FP32_VECTOR_PEAK,
        "lists": {k: int(st[k]) for k in ("nleaf", "nblock", "nrange", "nitem")},
    }
    progress("headline")
    if not args.no_cpu_baseline:
        base, errs, targets, ref = cpu_baseline(box, acc.cpu().numpy(), args.cpu_seconds)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = errs
        # the split factor from the interpolated LDS table (variant 8)
        # instead of the polynomial: same lists, same steps
        plan.set_tuning(variant=8)
        for _ in range(2):
            plan.accel(pos, mass, out=acc)
        tab_ms = []
        for _ in range(max(3, min(args.steps, 10))):
            plan.accel(pos, mass, out=acc)
            tab_ms.append(plan.stats()["pp_kernel_ms"])
        t_ms = float(np.mean(tab_ms))
        out["split_table_variant"] = {
            "kernel_ms": t_ms, "pp_kernel_interactions_per_s": interactions / (t_ms * 1e-3),
            "vs_polynomial_kernel": k_ms / t_ms,
            "error_vs_oracle": sample_errors(acc.cpu().numpy(), targets, ref)}
        plan.set_tuning(variant=0)
        progress("cpu baseline and split table")
    out["pm_long_range"] = bench_pm(box, pos, mass, 128, max(3, min(args.steps, 10)),
                                    with_error=not args.no_cpu_baseline)
    progress("PM")
    if not args.no_extras:
        out["monopoles"] = bench_monopoles(plan, box, pos, mass)
        progress("monopoles")
        kdk = bench_kdk(box, pos, mass, acc)
        reuse = bench_kdk(box, pos, mass, acc, skin=0.2 * box.params.rcut)
        kdk["list_reuse"] = {k: reuse[k] for k in ("skin", "ms_per_top_step", "list_builds_per_top_step",
                                                   "force_evaluations_per_top_step")}
        kdk["list_reuse"]["speedup"] = kdk["ms_per_top_step"] / reuse["ms_per_top_step"]
        out["kdk_adaptive"] = kdk
        progress("adaptive KDK")
        out["small_box"] = bench_small_box()
        progress("small box")
    del plan, pos, mass, acc
    torch.cuda.empty_cache()
    if not args.no_large:
        out["precision_16.8M"] = bench_precision()
        progress("16.8M precision")
        out["large_134M"] = bench_large()
        progress("134M")
    if not args.no_batched:
        out["batched_vs_per_box"] = bench_batched(max(1, min(args.steps, 5)), 1,
                                                  tune=not args.no_tune)
        progress("batched")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
