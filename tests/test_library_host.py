"""Host-side checks of the HIP library that need no GPU: it loads, it
exports every symbol include/photon_pp.h declares, and argument validation
rejects bad input with the documented codes before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1802_09824_amd", "libphoton_pp.so")
HDR = os.path.join(ROOT, "include", "photon_pp.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1802_09824_amd import build  # noqa: F401  (import fails without the .so)
    return C.CDLL(LIB)


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_abi():
    import paper_1802_09824_amd as pp
    assert set(declared_functions()) <= set(pp.EXPORTED)


class Params(C.Structure):
    _fields_ = [("L", C.c_double), ("rs", C.c_double), ("rcut", C.c_double), ("eps", C.c_double),
                ("G", C.c_double), ("leaf_max", C.c_int32), ("key_bits", C.c_int32)]


@pytest.mark.parametrize("kw,code", [
    (dict(rcut=50.0), -4),                     # rcut >= L/2
    (dict(rcut=60.0), -4),
    (dict(L=-1.0), -1),
    (dict(rs=0.0), -1),
    (dict(eps=-0.1), -1),
    (dict(eps=float("nan")), -1),
    (dict(leaf_max=0), -1),
    (dict(leaf_max=2000), -1),
    (dict(key_bits=22), -1),
    (dict(rs=1.0, rcut=10.0), -4),             # beyond the split polynomial's range
])
def test_plan_create_validation(lib, kw, code):
    base = dict(L=100.0, rs=3.90625, rcut=17.578125, eps=0.0625, G=1.0, leaf_max=32, key_bits=21)
    base.update(kw)
    p = Params(**base)
    h = C.c_void_p()
    lib.pp_plan_create.argtypes = [C.POINTER(Params), C.c_int64, C.POINTER(C.c_void_p)]
    rc = lib.pp_plan_create(C.byref(p), 1000, C.byref(h))
    assert rc == code
    lib.pp_last_error.restype = C.c_char_p
    assert len(lib.pp_last_error()) > 0
    assert not h.value


def test_plan_create_without_device_or_bad_n(lib):
    p = Params(L=100.0, rs=3.90625, rcut=17.578125, eps=0.0625, G=1.0, leaf_max=32, key_bits=21)
    h = C.c_void_p()
    lib.pp_plan_create.argtypes = [C.POINTER(Params), C.c_int64, C.POINTER(C.c_void_p)]
    assert lib.pp_plan_create(C.byref(p), -5, C.byref(h)) == -1
    rc = lib.pp_plan_create(C.byref(p), 100, C.byref(h))
    import torch
    if not torch.cuda.is_available():
        assert rc == -3            # PP_EDEVICE: no GPU here
    elif rc == 0:
        lib.pp_plan_destroy.argtypes = [C.c_void_p]
        lib.pp_plan_destroy(h)


def test_strerror(lib):
    lib.pp_strerror.restype = C.c_char_p
    assert lib.pp_strerror(0) == b"ok"
    assert lib.pp_strerror(-4).startswith(b"parameter")


def test_keys_argument_checks(lib):
    lib.pp_hilbert_keys.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_void_p, C.c_void_p]
    assert lib.pp_hilbert_keys(None, -1, 1.0, 21, None, None) == -1
    assert lib.pp_hilbert_keys(None, 10, 1.0, 21, None, None) == -1
    assert lib.pp_hilbert_keys(None, 0, 1.0, 0, None, None) == -1
    assert lib.pp_hilbert_keys(None, 0, 1.0, 21, None, None) == 0


def test_pm_plan_create_validation(lib):
    p = Params(L=100.0, rs=3.90625, rcut=17.578125, eps=0.0625, G=1.0, leaf_max=32, key_bits=21)
    h = C.c_void_p()
    lib.pp_pm_plan_create.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(C.c_void_p)]
    for bad in (3, 0, -8, 4096):
        assert lib.pp_pm_plan_create(C.byref(p), bad, C.byref(h)) == -1
        assert not h.value
    q = Params(L=100.0, rs=3.90625, rcut=60.0, eps=0.0625, G=1.0, leaf_max=32, key_bits=21)
    assert lib.pp_pm_plan_create(C.byref(q), 32, C.byref(h)) == -4
    rc = lib.pp_pm_plan_create(C.byref(p), 32, C.byref(h))
    import torch
    if not torch.cuda.is_available():
        assert rc == -3            # PP_EDEVICE: no GPU here
    elif rc == 0:
        lib.pp_pm_plan_destroy.argtypes = [C.c_void_p]
        lib.pp_pm_plan_destroy(h)
    lib.pp_pm_accel.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    assert lib.pp_pm_accel(None, None, None, 0, None, None) == -1
