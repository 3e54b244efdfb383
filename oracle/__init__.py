"""FP64 CPU oracle for the short-range PP gravity path.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library (paper_1802_09824_amd) and never imports it.

The arithmetic lives in pp_oracle.c (plain C, FP64); this module only
marshals numpy arrays.  Function-by-function citations are in that file:
split factor (sec. 3.1, Eq. equ:split), direct short-range sum (sec. 3.1
r_cut = 4.5 r_s; sec. 3.3 N-to-M PP), Peano-Hilbert keys (sec. 4.1),
octree leaves (sec. 3.2-3.3), near leaf pairs (sec. 3.3).  The long-range
PM force (sec. 3.1) is plain numpy in pm.py.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SHIFT_CODES = [(c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1) for c in range(27)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    i64, dbl, i32 = C.c_int64, C.c_double, C.c_int
    lib.oracle_split_factor.restype = dbl
    lib.oracle_split_factor.argtypes = [dbl]
    lib.oracle_num_threads.restype = i32
    lib.oracle_accel.restype = i32
    lib.oracle_accel.argtypes = [P, P, i64, dbl, dbl, dbl, dbl, dbl, P, i64, P, P, P, P, P, P]
    lib.oracle_hilbert_keys.restype = i32
    lib.oracle_hilbert_keys.argtypes = [P, i64, dbl, i32, P]
    lib.oracle_hilbert_decode.restype = None
    lib.oracle_hilbert_decode.argtypes = [P, i64, i32, P]
    lib.oracle_quantise.restype = None
    lib.oracle_quantise.argtypes = [P, i64, dbl, i32, P]
    lib.oracle_leaves.restype = i64
    lib.oracle_leaves.argtypes = [P, i64, i32, i32, i64, P, P, P, P]
    lib.oracle_leaf_boxes.restype = None
    lib.oracle_leaf_boxes.argtypes = [P, i64, P, P, i64, P, P]
    lib.oracle_neighbours.restype = i64
    lib.oracle_neighbours.argtypes = [P, i64, dbl, dbl, P, i64, i64, P, P, P]
    lib.oracle_near_pairs.restype = i64
    lib.oracle_near_pairs.argtypes = [P, P, i64, dbl, dbl, i32, P, i64, i64, P, P, P]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def split_factor(x) -> np.ndarray:
    """g(x) = erfc(x) + 2x/sqrt(pi) exp(-x^2), x = s / (2 r_s) (Eq. equ:split)."""
    lib = _load()
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([lib.oracle_split_factor(float(v)) for v in xs])


def accel(pos, mass, params, targets=None, pair_abs=False):
    """Direct FP64 short-range sum.

    pos: float64 [3, n]; mass: [n]; params: object with L, rs, rcut, eps, G.
    targets: optional int64 indices.  Returns dict with 'acc' [3, nt],
    'band_in', 'band_out' [3, nt], 'n_inter' [nt], 'n_band' [nt], and with
    pair_abs, 'pair_abs' [nt]: the sum over the kept pairs of the pair
    accelerations' magnitudes (the scale of the condition-robust error).
    """
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = pos.shape[1]
    if targets is None:
        tp, nt = None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tp, nt = _p(targets), targets.size
    acc = np.zeros((3, nt))
    bi = np.zeros((3, nt))
    bo = np.zeros((3, nt))
    ni = np.zeros(nt, dtype=np.int64)
    nb = np.zeros(nt, dtype=np.int64)
    pa = np.zeros(nt) if pair_abs else None
    rc = lib.oracle_accel(_p(pos), _p(mass), n, params.L, params.rs, params.rcut, params.eps,
                          params.G, tp, nt, _p(acc), _p(bi), _p(bo), _p(ni), _p(nb),
                          _p(pa) if pair_abs else None)
    if rc != 0:
        raise ValueError(f"oracle_accel failed ({rc})")
    out = {"acc": acc, "band_in": bi, "band_out": bo, "n_inter": ni, "n_band": nb}
    if pair_abs:
        out["pair_abs"] = pa
    return out


def quantise(pos, L, bits=21) -> np.ndarray:
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.zeros(pos.shape, dtype=np.uint32)
    lib.oracle_quantise(_p(pos), pos.shape[1], float(L), int(bits), _p(q))
    return q


def hilbert_keys(pos, L, bits=21) -> np.ndarray:
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    keys = np.zeros(pos.shape[1], dtype=np.uint64)
    rc = lib.oracle_hilbert_keys(_p(pos), pos.shape[1], float(L), int(bits), _p(keys))
    if rc != 0:
        raise ValueError(f"oracle_hilbert_keys failed ({rc})")
    return keys


def hilbert_decode(keys, bits=21) -> np.ndarray:
    lib = _load()
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    q = np.zeros((3, keys.size), dtype=np.uint32)
    lib.oracle_hilbert_decode(_p(keys), keys.size, int(bits), _p(q))
    return q


def sort_order(keys) -> np.ndarray:
    """Ascending (key, original index) order."""
    return np.argsort(np.asarray(keys, dtype=np.uint64), kind="stable").astype(np.int64)


def leaves(sorted_keys, bits=21, leaf_max=32):
    """Maximal octree nodes with <= leaf_max particles: dict of begin, count,
    level, prefix arrays (one row per leaf, in key order)."""
    lib = _load()
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = sk.size
    cap = max(1, n)
    begin = np.zeros(cap, dtype=np.int64)
    cnt = np.zeros(cap, dtype=np.int32)
    lev = np.zeros(cap, dtype=np.int32)
    pre = np.zeros(cap, dtype=np.uint64)
    m = lib.oracle_leaves(_p(sk), n, int(bits), int(leaf_max), cap, _p(begin), _p(cnt), _p(lev), _p(pre))
    if m < 0:
        raise ValueError(f"oracle_leaves failed ({m})")
    return {"begin": begin[:m].copy(), "count": cnt[:m].copy(), "level": lev[:m].copy(),
            "prefix": pre[:m].copy()}


def leaf_boxes(q_sorted, lv):
    """Integer AABBs [lo, hi) per leaf, int64 [3, nleaf] each."""
    lib = _load()
    q_sorted = np.ascontiguousarray(q_sorted, dtype=np.uint32)
    n = q_sorted.shape[1]
    m = lv["begin"].size
    lo = np.zeros((3, max(m, 1)), dtype=np.int64)
    hi = np.zeros((3, max(m, 1)), dtype=np.int64)
    begin = np.ascontiguousarray(lv["begin"], dtype=np.int64)
    cnt = np.ascontiguousarray(lv["count"], dtype=np.int32)
    lib.oracle_leaf_boxes(_p(q_sorted), n, _p(begin), _p(cnt), m, _p(lo), _p(hi))
    return lo[:, :m].copy(), hi[:, :m].copy()


def near_pairs(lo, hi, L, rcut, bits=21, rows=None):
    """Brute-force near-leaf-pair CSR: (row_ptr, src, code) for target rows
    (all leaves by default)."""
    lib = _load()
    lo = np.ascontiguousarray(lo, dtype=np.int64)
    hi = np.ascontiguousarray(hi, dtype=np.int64)
    m = lo.shape[1]
    if rows is None:
        rp, nt = None, m
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        rp, nt = _p(rows), rows.size
    row_ptr = np.zeros(nt + 1, dtype=np.int64)
    cap = 1 << 16
    while True:
        src = np.zeros(cap, dtype=np.int32)
        code = np.zeros(cap, dtype=np.uint8)
        tot = lib.oracle_near_pairs(_p(lo), _p(hi), m, float(L), float(rcut), int(bits), rp, nt,
                                    cap, _p(row_ptr), _p(src), _p(code))
        if tot < 0:
            raise ValueError(f"oracle_near_pairs failed ({tot})")
        if tot <= cap:
            return row_ptr, src[:tot].copy(), code[:tot].copy()
        cap = int(tot)


def neighbours(pos, params, targets=None):
    """In-cut neighbours (FP64 s < r_cut, minimum image, j != i) of the
    targets (all particles by default): (row_ptr, nbr, code) with the
    neighbours of target t in nbr[row_ptr[t]:row_ptr[t + 1]] (ascending) and
    code the image's shift code 9 (s_x + 1) + 3 (s_y + 1) + (s_z + 1)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[1]
    if targets is None:
        tp, nt = None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tp, nt = _p(targets), targets.size
    row_ptr = np.zeros(nt + 1, dtype=np.int64)
    cap = 1 << 20
    while True:
        nbr = np.zeros(cap, dtype=np.int64)
        code = np.zeros(cap, dtype=np.uint8)
        tot = lib.oracle_neighbours(_p(pos), n, float(params.L), float(params.rcut), tp, nt, cap,
                                    _p(row_ptr), _p(nbr), _p(code))
        if tot < 0:
            raise ValueError(f"oracle_neighbours failed ({tot})")
        if tot <= cap:
            return row_ptr, nbr[:tot].copy(), code[:tot].copy()
        cap = int(tot)


def structure(pos, params):
    """Keys, sort order, leaves and boxes of one box (oracle side)."""
    bits = params.key_bits
    keys = hilbert_keys(pos, params.L, bits)
    perm = sort_order(keys)
    sk = keys[perm]
    lv = leaves(sk, bits, params.leaf_max)
    q = quantise(pos, params.L, bits)[:, perm]
    lo, hi = leaf_boxes(q, lv)
    return {"keys": keys, "perm": perm, "sorted_keys": sk, "leaves": lv, "q_sorted": q,
            "lo": lo, "hi": hi}
