"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point that include/gnp.h declares, and rejects malformed CSR
input with GNP_EINVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = "\n".join(l for l in txt.splitlines() if not l.lstrip().startswith("#"))
        for m in re.finditer(r"GNP_API\s+[^;(]*?\**\s*(\w+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2406_00809_amd import _lib
    L = _lib.load()
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    # the binding's signature table covers the header exactly
    assert declared == set(_lib.SIGNATURES), declared ^ set(_lib.SIGNATURES)
    assert L.gnp_version().startswith(b"libgnp")


def _create(n, rp, ci, val):
    from paper_2406_00809_amd import _lib
    L = _lib.load()
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    h = C.c_void_p()
    st = L.gnp_system_create(n, ci.size, rp.ctypes.data_as(C.c_void_p),
                             ci.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p), 1,
                             None, C.byref(h))
    return st, L.gnp_last_error().decode()


@pytest.mark.parametrize("case,rp,ci,val,msg", [
    ("n<1", [0], [], [], "n must be"),
    ("rowptr0", [1, 2, 3], [0, 1], [1.0, 1.0], "rowptr[0]"),
    ("rowptr-n", [0, 1, 1], [0, 1], [1.0, 1.0], "rowptr[n]"),
    ("decreasing", [0, 2, 1, 2], [0, 1], [1.0, 1.0], "non-decreasing"),
    ("col-range", [0, 1, 2], [0, 2], [1.0, 1.0], "out of range"),
    ("col-negative", [0, 1, 2], [0, -1], [1.0, 1.0], "out of range"),
    ("unsorted", [0, 2, 3], [1, 0, 1], [1.0, 1.0, 1.0], "strictly increasing"),
    ("duplicate", [0, 2, 3], [0, 0, 1], [1.0, 1.0, 1.0], "strictly increasing"),
    ("nan", [0, 1, 2], [0, 1], [1.0, np.nan], "non-finite"),
    ("inf", [0, 1, 2], [0, 1], [np.inf, 1.0], "non-finite"),
])
def test_system_create_rejects_malformed_csr(case, rp, ci, val, msg):
    n = len(rp) - 1
    if case == "n<1":
        n = 0
    st, err = _create(n, rp, ci if ci else [0], val if val else [1.0])
    assert st == 1, (case, st, err)  # GNP_EINVAL
    assert msg in err, err


def test_null_arguments_rejected():
    from paper_2406_00809_amd import _lib
    L = _lib.load()
    h = C.c_void_p()
    assert L.gnp_system_create(4, 4, None, None, None, 1, None, C.byref(h)) == 1
    assert L.gnp_model_create(None, 2, 16, 32, None, 0, C.byref(h)) == 1
    assert L.fgmres_solve(None, None, None, None, 10, 1e-8, 10, 1, None, None, None) == 1
    assert L.gnp_apply(None, None, None, 1, 1, None) == 1
