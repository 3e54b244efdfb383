"""Comparison helpers for the parity tests (no method arithmetic here).

Relative error per target, e_i = |a_i - a*_i| / |a*_i|, over targets with at
least one neighbour inside the cut; a target whose oracle sum contains pairs
within the 2^-20 relative band around r_cut^2 is also compared against the
sums with those pairs flipped (an FP32 cut test may decide them either
way), and the smallest error is taken.  Targets with no neighbour must be
exactly zero.  Percentiles use the nearest-rank rule.
"""
import math

import numpy as np


def rel_errors(acc, ref):
    a = np.asarray(acc, dtype=np.float64)
    r = ref["acc"]
    has = ref["n_inter"] > 0
    norm = np.linalg.norm(r, axis=0)
    cands = [r, r - ref["band_in"] + ref["band_out"], r - ref["band_in"], r + ref["band_out"]]
    errs = np.min([np.linalg.norm(a - c, axis=0) for c in cands], axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(norm > 0, errs / norm, np.where(errs == 0, 0.0, np.inf))
    return e[has], a[:, ~has]


def nearest_rank(x, q):
    x = np.sort(np.asarray(x))
    if x.size == 0:
        return 0.0
    k = max(1, int(math.ceil(q / 100.0 * x.size)))
    return float(x[k - 1])


def summary(acc, ref):
    e, zero_part = rel_errors(acc, ref)
    return {"median": nearest_rank(e, 50), "p999": nearest_rank(e, 99.9),
            "max": float(e.max()) if e.size else 0.0,
            "zero_ok": bool(np.all(zero_part == 0)), "n": int(e.size)}
