"""photon_pp: short-range PP gravity on one MI355X GPU (Python binding).

A thin ctypes layer over libphoton_pp.so (C ABI in include/photon_pp.h).
It only marshals arguments: every stage of the path runs in the library's
HIP kernels.  Torch is used for device memory and the current stream.
If the library has not been built the import fails loudly; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphoton_pp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1802_09824_amd/build.py` "
                      "(hipcc, gfx950); there is no CPU fallback")
_lib = C.CDLL(LIB_PATH)

PP_OK, PP_EINVAL, PP_ENOMEM, PP_EDEVICE, PP_ERANGE, PP_EOVERFLOW = 0, -1, -2, -3, -4, -5


class PPError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.pp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.pp_strerror(code).decode()} ({code}): {msg}")
        self.code = code


class pp_box_params(C.Structure):
    _fields_ = [("L", C.c_double), ("rs", C.c_double), ("rcut", C.c_double), ("eps", C.c_double),
                ("G", C.c_double), ("leaf_max", C.c_int32), ("key_bits", C.c_int32)]


class pp_tuning(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("persistent", C.c_int32), ("waves_per_cu", C.c_int32),
                ("use_graph", C.c_int32), ("variant", C.c_int32), ("waves_per_block", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class pp_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nleaf", C.c_int64), ("nblock", C.c_int64),
                ("nrange", C.c_int64), ("nitem", C.c_int64), ("candidates", C.c_int64),
                ("evaluated", C.c_int64), ("lane_pairs", C.c_int64),
                ("interactions", C.c_int64), ("pp_kernel_ms", C.c_double),
                ("monopoles", C.c_int64), ("pp_stage_ms", C.c_double),
                ("list_builds", C.c_int64), ("list_reuses", C.c_int64)]


_P, _i64, _i32, _dbl, _sz = C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_size_t
_SIGS = {
    "pp_strerror": (C.c_char_p, [_i32]),
    "pp_last_error": (C.c_char_p, []),
    "pp_hilbert_keys": (_i32, [_P, _i64, _dbl, _i32, _P, _P]),
    "pp_sort_workspace_size": (_i32, [_i64, C.POINTER(_sz)]),
    "pp_sort_by_key": (_i32, [_P, _i64, _P, _P, _P, _sz, _P]),
    "pp_build_leaves": (_i32, [_P, _P, _i64, C.POINTER(pp_box_params), C.POINTER(_P), _P]),
    "pp_leaves_count": (_i32, [_P, C.POINTER(_i64)]),
    "pp_leaves_export": (_i32, [_P, _P, _P, _P, _P, _P, _P]),
    "pp_leaves_free": (None, [_P]),
    "pp_near_pairs": (_i32, [_P, C.POINTER(pp_box_params), C.POINTER(_P), _P]),
    "pp_pairs_count": (_i32, [_P, C.POINTER(_i64), C.POINTER(_i64)]),
    "pp_pairs_export": (_i32, [_P, _P, _P, _P]),
    "pp_pairs_free": (None, [_P]),
    "pp_plan_create": (_i32, [C.POINTER(pp_box_params), _i64, C.POINTER(_P)]),
    "pp_plan_destroy": (None, [_P]),
    "pp_accel": (_i32, [_P, _P, _P, _i64, _P, _P]),
    "pp_accel_f64": (_i32, [_P, _P, _P, _i64, _P, _P]),
    "pp_accel_scratch": (_i32, [C.POINTER(pp_box_params), _P, _P, _i64, _P, _P]),
    "pp_plan_stats": (_i32, [_P, C.POINTER(pp_stats)]),
    "pp_plan_set_monopole": (_i32, [_P, C.c_double]),
    "pp_plan_set_skin": (_i32, [_P, C.c_double]),
    "pp_kdk_set_skin": (_i32, [_P, C.c_double]),
    "pp_accel_active": (_i32, [_P, _P, _P, _i64, _P, _P, _P]),
    "pp_plan_set_monopole_relative": (_i32, [_P, C.c_double, _P, _i64, _P]),
    "pp_count_interactions": (_i32, [_P, _P, C.POINTER(_i64), _P]),
    "pp_plan_lists_size": (_i32, [_P, C.POINTER(_i64), C.POINTER(_i64)]),
    "pp_plan_lists_export": (_i32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pp_plan_set_timing": (_i32, [_P, _i32]),
    "pp_plan_get_tuning": (_i32, [_P, C.POINTER(pp_tuning)]),
    "pp_plan_set_tuning": (_i32, [_P, C.POINTER(pp_tuning)]),
    "pp_batch_plan_create": (_i32, [_i32, _P, _P, C.POINTER(_P)]),
    "pp_batch_plan_destroy": (None, [_P]),
    "pp_batch_accel": (_i32, [_P, _P, _P, _P, _P]),
    "pp_batch_count_interactions": (_i32, [_P, _P, C.POINTER(_i64), _P]),
    "pp_batch_stats": (_i32, [_P, C.POINTER(pp_stats)]),
    "pp_batch_set_timing": (_i32, [_P, _i32]),
    "pp_batch_get_tuning": (_i32, [_P, C.POINTER(pp_tuning)]),
    "pp_batch_set_tuning": (_i32, [_P, C.POINTER(pp_tuning)]),
    "pp_autotune": (_i32, [_P, _P, _P, _i64, C.c_char_p, _P]),
    "pp_batch_autotune": (_i32, [_P, _P, _P, C.c_char_p, _P]),
    "pp_pm_plan_create": (_i32, [C.POINTER(pp_box_params), _i32, C.POINTER(_P)]),
    "pp_pm_accel": (_i32, [_P, _P, _P, _i64, _P, _P]),
    "pp_pm_plan_destroy": (None, [_P]),
    "pp_kdk_create": (_i32, [C.POINTER(pp_box_params), _i32, _i64, C.c_double, _i32, C.POINTER(_P)]),
    "pp_kdk_init": (_i32, [_P, _P, _P, _P]),
    "pp_kdk_step": (_i32, [_P, _P, _P, _P, C.c_double, _P]),
    "pp_kdk_get_info": (_i32, [_P, _P]),
    "pp_kdk_levels": (_i32, [_P, _P, _P]),
    "pp_kdk_accel": (_i32, [_P, _P, _P]),
    "pp_kdk_destroy": (None, [_P]),
}
EXPORTED = tuple(_SIGS)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc: int, where: str):
    if rc != PP_OK:
        raise PPError(rc, where)


def make_params(p) -> pp_box_params:
    """pp_box_params from any object with L, rs, rcut, eps, G, leaf_max, key_bits."""
    return pp_box_params(float(p.L), float(p.rs), float(p.rcut), float(p.eps), float(p.G),
                         int(getattr(p, "leaf_max", 32)), int(getattr(p, "key_bits", 21)))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def pp_hilbert_keys(pos: torch.Tensor, L: float, key_bits: int = 21, stream=None) -> torch.Tensor:
    n = pos.shape[1]
    keys = torch.empty(n, dtype=torch.int64, device=pos.device)   # bit pattern of uint64
    _check(_lib.pp_hilbert_keys(_dev(pos, torch.float64, (3, n), "pos"), n, float(L), int(key_bits),
                                C.c_void_p(keys.data_ptr()), _stream(stream)), "pp_hilbert_keys")
    return keys


def pp_sort_by_key(keys: torch.Tensor, stream=None):
    """Returns (perm int32, sorted_keys) for keys given as the int64 bit pattern."""
    n = keys.numel()
    need = _sz(0)
    _check(_lib.pp_sort_workspace_size(n, C.byref(need)), "pp_sort_workspace_size")
    ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=keys.device)
    perm = torch.empty(n, dtype=torch.int32, device=keys.device)
    sk = torch.empty(n, dtype=torch.int64, device=keys.device)
    _check(_lib.pp_sort_by_key(_dev(keys, torch.int64, name="keys"), n, C.c_void_p(perm.data_ptr()),
                               C.c_void_p(sk.data_ptr()), C.c_void_p(ws.data_ptr()), need.value,
                               _stream(stream)), "pp_sort_by_key")
    torch.cuda.current_stream().synchronize()
    return perm, sk


class Leaves:
    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    def __del__(self):
        # (at interpreter exit the module's _lib may already be gone)
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.pp_leaves_free(self._h)
            self._h = C.c_void_p(None)

    @property
    def count(self) -> int:
        m = _i64(0)
        _check(_lib.pp_leaves_count(self._h, C.byref(m)), "pp_leaves_count")
        return int(m.value)

    def export(self) -> dict:
        import numpy as np
        m = self.count
        out = {"begin": np.zeros(m, np.int64), "count": np.zeros(m, np.int32),
               "level": np.zeros(m, np.int32), "prefix": np.zeros(m, np.uint64),
               "lo": np.zeros((3, m), np.int32), "hi": np.zeros((3, m), np.int32)}
        _check(_lib.pp_leaves_export(self._h, *(a.ctypes.data_as(_P) for a in out.values())),
               "pp_leaves_export")
        return out


def pp_build_leaves(sorted_keys: torch.Tensor, pos_sorted: torch.Tensor, params, stream=None) -> Leaves:
    n = sorted_keys.numel()
    h = _P(None)
    prm = make_params(params)
    _check(_lib.pp_build_leaves(_dev(sorted_keys, torch.int64, name="sorted_keys"),
                                _dev(pos_sorted, torch.float64, (3, n), "pos_sorted"), n,
                                C.byref(prm), C.byref(h), _stream(stream)), "pp_build_leaves")
    return Leaves(h.value)


class Pairs:
    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    def __del__(self):
        # (at interpreter exit the module's _lib may already be gone)
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.pp_pairs_free(self._h)
            self._h = C.c_void_p(None)

    def export(self):
        import numpy as np
        nr, ne = _i64(0), _i64(0)
        _check(_lib.pp_pairs_count(self._h, C.byref(nr), C.byref(ne)), "pp_pairs_count")
        rp = np.zeros(nr.value + 1, np.int64)
        src = np.zeros(max(ne.value, 1), np.int32)
        code = np.zeros(max(ne.value, 1), np.uint8)
        _check(_lib.pp_pairs_export(self._h, rp.ctypes.data_as(_P), src.ctypes.data_as(_P),
                                    code.ctypes.data_as(_P)), "pp_pairs_export")
        return rp, src[:ne.value], code[:ne.value]


def pp_near_pairs(leaves: Leaves, params, stream=None) -> Pairs:
    h = _P(None)
    prm = make_params(params)
    _check(_lib.pp_near_pairs(leaves._h, C.byref(prm), C.byref(h), _stream(stream)), "pp_near_pairs")
    return Pairs(h.value)


class Plan:
    """pp_plan: parameters, scratch memory for up to n_max particles."""

    def __init__(self, params, n_max: int):
        self.params = params
        self.n_max = int(n_max)
        h = _P(None)
        prm = make_params(params)
        _check(_lib.pp_plan_create(C.byref(prm), self.n_max, C.byref(h)), "pp_plan_create")
        self._h = h

    def __del__(self):
        # (at interpreter exit the module's _lib may already be gone)
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.pp_plan_destroy(self._h)
            self._h = C.c_void_p(None)

    def accel(self, pos: torch.Tensor, mass: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        n = pos.shape[1]
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
        _check(_lib.pp_accel(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                             _dev(mass, torch.float32, (n,), "mass"), n,
                             _dev(out, torch.float32, (3, n), "acc"), _stream(stream)), "pp_accel")
        return out

    def accel_active(self, pos: torch.Tensor, mass: torch.Tensor, active: torch.Tensor,
                     out: torch.Tensor, stream=None) -> torch.Tensor:
        """accel for the targets with active[i] != 0 (uint8 [n]); the other
        columns of out are left as they were."""
        n = pos.shape[1]
        _check(_lib.pp_accel_active(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                    _dev(mass, torch.float32, (n,), "mass"), n,
                                    _dev(active, torch.uint8, (n,), "active"),
                                    _dev(out, torch.float32, (3, n), "acc"), _stream(stream)),
               "pp_accel_active")
        return out

    def accel_f64(self, pos: torch.Tensor, mass: torch.Tensor, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
        n = pos.shape[1]
        if out is None:
            out = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        _check(_lib.pp_accel_f64(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                 _dev(mass, torch.float64, (n,), "mass"), n,
                                 _dev(out, torch.float64, (3, n), "acc"), _stream(stream)),
               "pp_accel_f64")
        return out

    def stats(self) -> dict:
        st = pp_stats()
        _check(_lib.pp_plan_stats(self._h, C.byref(st)), "pp_plan_stats")
        return {k: getattr(st, k) for k, _ in pp_stats._fields_}

    def set_timing(self, on: bool = True):
        _check(_lib.pp_plan_set_timing(self._h, 1 if on else 0), "pp_plan_set_timing")

    def set_monopole(self, theta: float):
        """Monopole acceptance for accel (0 = exact pair sums)."""
        _check(_lib.pp_plan_set_monopole(self._h, float(theta)), "pp_plan_set_monopole")

    def set_skin(self, skin: float):
        """Lists built with the cut widened by skin are reused by later accel
        calls while every particle stays within skin / 2 (0 = build every call)."""
        _check(_lib.pp_plan_set_skin(self._h, float(skin)), "pp_plan_set_skin")

    def set_monopole_relative(self, alpha: float, acc_ref: torch.Tensor | None = None, stream=None):
        """Gadget-2's relative opening test for accel against reference
        accelerations acc_ref [3][n] (FP32, device); alpha = 0 turns it off."""
        if alpha > 0:
            if acc_ref is None:
                raise ValueError("alpha > 0 needs the reference accelerations acc_ref")
            n = acc_ref.shape[1]
            ptr = _dev(acc_ref, torch.float32, (3, n), "acc_ref")
        else:
            n, ptr = 0, C.c_void_p(None)
        _check(_lib.pp_plan_set_monopole_relative(self._h, float(alpha), ptr, n, _stream(stream)),
               "pp_plan_set_monopole_relative")

    def get_tuning(self) -> dict:
        t = pp_tuning()
        _check(_lib.pp_plan_get_tuning(self._h, C.byref(t)), "pp_plan_get_tuning")
        return t.as_dict()

    def set_tuning(self, **kw):
        t = pp_tuning(**{**self.get_tuning(), **kw})
        _check(_lib.pp_plan_set_tuning(self._h, C.byref(t)), "pp_plan_set_tuning")

    def autotune(self, pos: torch.Tensor, mass: torch.Tensor, cache_path: str | None = None,
                 stream=None) -> dict:
        n = pos.shape[1]
        _check(_lib.pp_autotune(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                _dev(mass, torch.float32, (n,), "mass"), n,
                                cache_path.encode() if cache_path else None, _stream(stream)),
               "pp_autotune")
        return self.get_tuning()

    def export_lists(self) -> dict:
        """The per-block source lists of the last accel call (host arrays)."""
        import numpy as np
        nb, nr = _i64(0), _i64(0)
        _check(_lib.pp_plan_lists_size(self._h, C.byref(nb), C.byref(nr)), "pp_plan_lists_size")
        nb, nr = int(nb.value), int(nr.value)
        n = self.stats()["n"]
        out = {"perm": np.zeros(max(n, 1), np.int32), "bstart": np.zeros(max(nb, 1), np.int32),
               "bcount": np.zeros(max(nb, 1), np.int32), "blo": np.zeros((3, max(nb, 1)), np.int32),
               "bhi": np.zeros((3, max(nb, 1)), np.int32), "roff": np.zeros(nb + 1, np.int64),
               "slen": np.zeros(max(nb, 1), np.int32), "rbeg": np.zeros(max(nr, 1), np.int32),
               "rpre": np.zeros(max(nr, 1), np.int32), "rcode": np.zeros(max(nr, 1), np.uint8)}
        _check(_lib.pp_plan_lists_export(self._h, *(a.ctypes.data_as(_P) for a in out.values())),
               "pp_plan_lists_export")
        for k in ("bstart", "bcount", "slen"):
            out[k] = out[k][:nb]
        out["blo"], out["bhi"] = out["blo"][:, :nb], out["bhi"][:, :nb]
        for k in ("rbeg", "rpre", "rcode"):
            out[k] = out[k][:nr]
        out["perm"] = out["perm"][:n]
        return out

    def count_interactions(self, per_target: bool = False, stream=None):
        tot = _i64(0)
        counts = None
        ptr = C.c_void_p(None)
        if per_target:
            n = self.stats()["n"]
            counts = torch.zeros(n, dtype=torch.int64, device="cuda")
            ptr = C.c_void_p(counts.data_ptr())
        _check(_lib.pp_count_interactions(self._h, ptr, C.byref(tot), _stream(stream)),
               "pp_count_interactions")
        return (int(tot.value), counts) if per_target else int(tot.value)


def pp_accel_scratch(params, pos: torch.Tensor, mass: torch.Tensor, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """pp_accel without allocation: one box of at most 65536 particles, every
    buffer in the library's static device scratch."""
    n = pos.shape[1]
    if out is None:
        out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
    prm = make_params(params)
    _check(_lib.pp_accel_scratch(C.byref(prm), _dev(pos, torch.float64, (3, n), "pos"),
                                 _dev(mass, torch.float32, (n,), "mass"), n,
                                 _dev(out, torch.float32, (3, n), "acc"), _stream(stream)),
           "pp_accel_scratch")
    return out


def pp_plan_create(params, n_max: int) -> Plan:
    return Plan(params, n_max)


class BatchPlan:
    """pp_batch_plan: many independent boxes, one persistent launch."""

    def __init__(self, params_list, ns):
        import numpy as np
        self.nbox = len(params_list)
        arr = (pp_box_params * self.nbox)(*[make_params(p) for p in params_list])
        self._keep = arr
        self.ns = np.ascontiguousarray(ns, dtype=np.int64)
        self.N = int(self.ns.sum())
        h = _P(None)
        _check(_lib.pp_batch_plan_create(self.nbox, C.cast(arr, _P), self.ns.ctypes.data_as(_P),
                                         C.byref(h)), "pp_batch_plan_create")
        self._h = h

    def __del__(self):
        # (at interpreter exit the module's _lib may already be gone)
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.pp_batch_plan_destroy(self._h)
            self._h = C.c_void_p(None)

    def accel(self, pos: torch.Tensor, mass: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        n = self.N
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
        _check(_lib.pp_batch_accel(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                   _dev(mass, torch.float32, (n,), "mass"),
                                   _dev(out, torch.float32, (3, n), "acc"), _stream(stream)),
               "pp_batch_accel")
        return out

    def count_interactions(self, per_target: bool = False, stream=None):
        tot = _i64(0)
        counts = None
        ptr = C.c_void_p(None)
        if per_target:
            counts = torch.zeros(self.N, dtype=torch.int64, device="cuda")
            ptr = C.c_void_p(counts.data_ptr())
        _check(_lib.pp_batch_count_interactions(self._h, ptr, C.byref(tot), _stream(stream)),
               "pp_batch_count_interactions")
        return (int(tot.value), counts) if per_target else int(tot.value)

    def stats(self) -> dict:
        st = pp_stats()
        _check(_lib.pp_batch_stats(self._h, C.byref(st)), "pp_batch_stats")
        return {k: getattr(st, k) for k, _ in pp_stats._fields_}

    def set_timing(self, on: bool = True):
        _check(_lib.pp_batch_set_timing(self._h, 1 if on else 0), "pp_batch_set_timing")

    def get_tuning(self) -> dict:
        t = pp_tuning()
        _check(_lib.pp_batch_get_tuning(self._h, C.byref(t)), "pp_batch_get_tuning")
        return t.as_dict()

    def set_tuning(self, **kw):
        t = pp_tuning(**{**self.get_tuning(), **kw})
        _check(_lib.pp_batch_set_tuning(self._h, C.byref(t)), "pp_batch_set_tuning")

    def autotune(self, pos: torch.Tensor, mass: torch.Tensor, cache_path: str | None = None,
                 stream=None) -> dict:
        n = self.N
        _check(_lib.pp_batch_autotune(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                      _dev(mass, torch.float32, (n,), "mass"),
                                      cache_path.encode() if cache_path else None, _stream(stream)),
               "pp_batch_autotune")
        return self.get_tuning()


def pp_batch_plan_create(params_list, ns) -> BatchPlan:
    return BatchPlan(params_list, ns)


class PMPlan:
    """Long-range particle-mesh force of one periodic box (pp_pm_*)."""

    def __init__(self, params, n_mesh: int):
        self.params = params
        self.n_mesh = int(n_mesh)
        h = C.c_void_p()
        bp = make_params(params)
        _check(_lib.pp_pm_plan_create(C.byref(bp), self.n_mesh, C.byref(h)), "pp_pm_plan_create")
        self._h = h

    def accel(self, pos: torch.Tensor, mass: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        n = pos.shape[1]
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device=pos.device)
        _check(_lib.pp_pm_accel(self._h, _dev(pos, torch.float64, (3, n), "pos"),
                                _dev(mass, torch.float32, (n,), "mass"), n,
                                _dev(out, torch.float32, (3, n), "out"), _stream(stream)),
               "pp_pm_accel")
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pp_pm_plan_destroy(h)
            self._h = None


def pp_pm_plan_create(params, n_mesh: int) -> PMPlan:
    return PMPlan(params, n_mesh)


class pp_kdk_info(C.Structure):
    _fields_ = [("deepest_level", C.c_int32), ("pad", C.c_int32), ("top_steps", C.c_int64),
                ("force_evaluations", C.c_int64), ("level_count", C.c_int64 * 16),
                ("short_range_targets", C.c_int64), ("list_builds", C.c_int64)]


class KDK:
    """Adaptive KDK integration over pp_accel + pp_pm_accel (pp_kdk_*).
    pos and vel are FP64 [3][n] device tensors updated in place."""

    def __init__(self, params, n: int, n_mesh: int = 0, eta: float = 0.025, max_level: int = 8):
        self.n = int(n)
        self.pm = int(n_mesh) > 0
        h = C.c_void_p()
        bp = make_params(params)
        _check(_lib.pp_kdk_create(C.byref(bp), int(n_mesh), self.n, float(eta), int(max_level), C.byref(h)),
               "pp_kdk_create")
        self._h = h

    def init(self, pos: torch.Tensor, mass: torch.Tensor, stream=None):
        _check(_lib.pp_kdk_init(self._h, _dev(pos, torch.float64, (3, self.n), "pos"),
                                _dev(mass, torch.float32, (self.n,), "mass"), _stream(stream)), "pp_kdk_init")

    def step(self, pos: torch.Tensor, vel: torch.Tensor, mass: torch.Tensor, dt: float, stream=None):
        _check(_lib.pp_kdk_step(self._h, _dev(pos, torch.float64, (3, self.n), "pos"),
                                _dev(vel, torch.float64, (3, self.n), "vel"),
                                _dev(mass, torch.float32, (self.n,), "mass"), float(dt), _stream(stream)),
               "pp_kdk_step")

    def info(self) -> dict:
        i = pp_kdk_info()
        _check(_lib.pp_kdk_get_info(self._h, C.byref(i)), "pp_kdk_get_info")
        return {"deepest_level": i.deepest_level, "top_steps": i.top_steps,
                "force_evaluations": i.force_evaluations, "level_count": list(i.level_count),
                "short_range_targets": i.short_range_targets, "list_builds": i.list_builds}

    def set_skin(self, skin: float):
        """Reuse the short-range lists across substeps (pp_kdk_set_skin)."""
        _check(_lib.pp_kdk_set_skin(self._h, float(skin)), "pp_kdk_set_skin")

    def levels(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.int8, device="cuda")
        _check(_lib.pp_kdk_levels(self._h, C.c_void_p(out.data_ptr()), _stream(stream)), "pp_kdk_levels")
        return out

    def accel(self, stream=None) -> torch.Tensor:
        """Current forces: [3][n] short range, and [3][n] long range with PM."""
        out = torch.empty((6 if self.pm else 3, self.n), dtype=torch.float32, device="cuda")
        _check(_lib.pp_kdk_accel(self._h, C.c_void_p(out.data_ptr()), _stream(stream)), "pp_kdk_accel")
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pp_kdk_destroy(h)
            self._h = None
