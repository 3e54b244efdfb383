"""Comparison helpers for the parity tests (no method arithmetic here).

Relative error per target, e_i = |a_i - a*_i| / |a*_i|, over targets with at
least one neighbour inside the cut; a target whose oracle sum contains pairs
within the 2^-20 relative band around r_cut^2 is also compared against the
sums with those pairs flipped (an FP32 cut test may decide them either
way), and the smallest error is taken.  Targets with no neighbour must be
exactly zero.  Percentiles use the nearest-rank rule.

Where the oracle also returned the pair-magnitude sums S_i = sum_j |a_ij|,
the condition-robust error e'_i = |a_i - a*_i| / S_i is reported as well:
it stays small on targets whose force nearly cancels, where e_i cannot.
"""
import math

import numpy as np

# Bound on the condition-robust error e'_i of the FP32 path, from its
# arithmetic: each pair's factor y^3 g carries the polynomial's error of g
# (at most 1.1e-7, degree 9) plus the FP32 rounding of the Horner sum and of
# y^3, against g(x_max) >= 0.0168 at the cut, so no pair is off by more than
# about 7e-5 of its magnitude (1.8e-5 for the largest case found by a
# simulation of the FP32 sequence); the compensated sums add a few ulps.
ROBUST_MAX = 1e-4


def abs_errors(acc, ref):
    a = np.asarray(acc, dtype=np.float64)
    r = ref["acc"]
    cands = [r, r - ref["band_in"] + ref["band_out"], r - ref["band_in"], r + ref["band_out"]]
    return np.min([np.linalg.norm(a - c, axis=0) for c in cands], axis=0)


def _ratio(num, den):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, num / den, np.where(num == 0, 0.0, np.inf))


def rel_errors(acc, ref):
    a = np.asarray(acc, dtype=np.float64)
    has = ref["n_inter"] > 0
    e = _ratio(abs_errors(a, ref), np.linalg.norm(ref["acc"], axis=0))
    return e[has], a[:, ~has]


def robust_errors(acc, ref):
    """e'_i over targets with at least one neighbour (needs ref['pair_abs'])."""
    has = ref["n_inter"] > 0
    return _ratio(abs_errors(acc, ref), ref["pair_abs"])[has]


def nearest_rank(x, q):
    x = np.sort(np.asarray(x))
    if x.size == 0:
        return 0.0
    k = max(1, int(math.ceil(q / 100.0 * x.size)))
    return float(x[k - 1])


def summary(acc, ref):
    e, zero_part = rel_errors(acc, ref)
    out = {"median": nearest_rank(e, 50), "p999": nearest_rank(e, 99.9),
           "max": float(e.max()) if e.size else 0.0,
           "zero_ok": bool(np.all(zero_part == 0)), "n": int(e.size)}
    if "pair_abs" in ref:
        r = robust_errors(acc, ref)
        out["robust_p999"] = nearest_rank(r, 99.9)
        out["robust_max"] = float(r.max()) if r.size else 0.0
    return out
