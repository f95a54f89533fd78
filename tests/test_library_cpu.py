"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every
symbol include/ddi.h declares, and rejects invalid plans before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddi.h")
LIB = os.path.join(ROOT, "paper_1504_02897_amd", "libddi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:ddi_status|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libddi.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["ddi_plan", "ddi_apply", "ddi_apply_adjoint", "gpe_energy_grad", "ddi_destroy", "ddi_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_matches_header():
    # the Python binding names the same entry points (parsed, not imported: importing needs torch + the lib)
    src = open(os.path.join(ROOT, "paper_1504_02897_amd", "ddi.py")).read()
    m = re.search(r"EXPORTED = \[(.*?)\]", src, flags=re.S)
    exported = re.findall(r'"(\w+)"', m.group(1))
    assert sorted(exported) == sorted(declared_functions())


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("L", ctypes.c_double * 3),
                ("dip_n", ctypes.c_double * 3), ("dip_m", ctypes.c_double * 3),
                ("n_rad", ctypes.c_int64), ("n_pol", ctypes.c_int64), ("n_azi", ctypes.c_int64),
                ("kmax", ctypes.c_double), ("nyquist_mask", ctypes.c_int32), ("tol", ctypes.c_double),
                ("prec", ctypes.c_int32), ("kernel_width", ctypes.c_int32),
                ("split", ctypes.c_int32), ("split_s", ctypes.c_double), ("stretch", ctypes.c_double * 3)]


def _params(**kw):
    p = Params()
    p.dim = kw.get("dim", 3)
    for i, v in enumerate(kw.get("n", (32, 32, 32))):
        p.n[i] = v
    for i, v in enumerate(kw.get("L", (8.0, 8.0, 8.0))):
        p.L[i] = v
    for i, v in enumerate(kw.get("dip_n", (0.0, 0.0, 1.0))):
        p.dip_n[i] = v
    p.n_rad, p.n_pol, p.n_azi = kw.get("quad", (8, 4, 8))
    p.nyquist_mask = 1
    p.tol = kw.get("tol", 1e-13)
    p.prec = kw.get("prec", 0)
    p.kernel_width = kw.get("kernel_width", 0)
    p.split = kw.get("split", 0)
    p.split_s = kw.get("split_s", 0.0)
    for i, v in enumerate(kw.get("stretch", (1.0, 1.0, 1.0))):
        p.stretch[i] = v
    return p


@pytest.mark.parametrize("bad,code", [
    (dict(dim=4), 1),
    (dict(n=(30, 32, 32)), 1),              # not a power of two
    (dict(n=(1024, 32, 32)), 4),            # above the supported size
    (dict(n=(4, 32, 32)), 4),               # below the supported size
    (dict(L=(0.0, 8.0, 8.0)), 1),
    (dict(dip_n=(0.0, 0.0, 0.0)), 1),
    (dict(quad=(0, 4, 8)), 1),
    (dict(tol=0.0), 1),
    (dict(kernel_width=17), 1),
    (dict(prec=7), 1),
    (dict(split=2), 1),
    (dict(split=1, split_s=float("inf")), 1),
    (dict(stretch=(1.0, float("nan"), 1.0)), 1),
])
def test_invalid_plans_are_rejected_before_device_use(lib, bad, code):
    lib.ddi_plan.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.ddi_plan.restype = ctypes.c_int
    lib.ddi_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p(123)
    st = lib.ddi_plan(ctypes.byref(_params(**bad)), None, ctypes.byref(h))
    assert st == code
    assert h.value is None
    assert len(lib.ddi_last_error()) > 0


def test_null_arguments(lib):
    lib.ddi_apply.argtypes = [ctypes.c_void_p] * 4
    lib.ddi_apply.restype = ctypes.c_int
    assert lib.ddi_apply(None, None, None, None) == 1
    lib.ddi_plan.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.ddi_plan.restype = ctypes.c_int
    assert lib.ddi_plan(None, None, None) == 1
    lib.ddi_destroy.argtypes = [ctypes.c_void_p]
    lib.ddi_destroy(None)
