"""C ABI: the library loads, exports every symbol include/qslater.h declares,
and host-side validation rejects bad descriptors before touching the GPU."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qslater.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qsl_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("qsl_system_create", "qsl_forward", "qsl_backward", "qsl_set_mo", "qsl_workspace_size"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1209_6630_amd import _lib
    L = _lib.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines()}
    for name in _declared():
        assert name in exported, name
        assert hasattr(L, name)
    assert set(_lib.SIGNATURES) == set(_declared())


def test_status_strings():
    from paper_1209_6630_amd import _lib
    L = _lib.lib()
    assert L.qsl_status_string(0) == b"ok"
    assert L.qsl_status_string(4) == b"workspace too small"


def _desc(**over):
    from paper_1209_6630_amd._lib import SystemDesc
    xyz = np.zeros((1, 3))
    sa = np.zeros(1, np.int32)
    sl = np.array([over.pop("l", 0)], np.int32)
    sn = np.array([over.pop("nprim", 1)], np.int32)
    ex = np.full(max(1, int(sn[0])), over.pop("exp", 1.0))
    co = np.ones_like(ex)
    keep = [xyz, sa, sl, sn, ex, co]
    dp, ip = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32)
    d = SystemDesc(1, xyz.ctypes.data_as(dp), 1, sa.ctypes.data_as(ip), sl.ctypes.data_as(ip),
                   sn.ctypes.data_as(ip), ex.ctypes.data_as(dp), co.ctypes.data_as(dp),
                   over.pop("n_up", 1), over.pop("n_dn", 0), 30.0, over.pop("flags", 0))
    return d, keep


@pytest.mark.parametrize("kw,code", [
    (dict(l=3), 2),            # UNSUPPORTED: f shell
    (dict(nprim=9), 2),        # UNSUPPORTED: too many primitives
    (dict(exp=-1.0), 1),       # INVALID_ARG: non-positive exponent
    (dict(n_up=0, n_dn=1), 1),  # INVALID_ARG: n_up < n_dn
    (dict(flags=1), 1),        # INVALID_ARG: reserved flags
])
def test_create_validation_errors(kw, code):
    from paper_1209_6630_amd._lib import lib
    d, keep = _desc(**kw)
    h = ct.c_void_p()
    assert lib().qsl_system_create(ct.byref(d), ct.byref(h)) == code
    assert h.value is None
    assert len(lib().qsl_last_error()) > 0


def test_nonfinite_atom_coordinate_rejected():
    """A NaN or infinite atom coordinate is an INVALID_ARG before any device
    work."""
    import math
    from paper_1209_6630_amd._lib import lib
    for bad in (math.nan, math.inf):
        d, keep = _desc()
        keep[0][0, 1] = bad
        h = ct.c_void_p()
        assert lib().qsl_system_create(ct.byref(d), ct.byref(h)) == 1
        assert h.value is None
        assert b"non-finite" in lib().qsl_last_error()


def test_workspace_size_argument_checks():
    from paper_1209_6630_amd._lib import lib
    n = ct.c_size_t()
    assert lib().qsl_workspace_size(None, 4, 0, 3, ct.byref(n)) == 1


def test_null_arguments():
    from paper_1209_6630_amd._lib import lib
    h = ct.c_void_p()
    assert lib().qsl_system_create(None, ct.byref(h)) == 1
    assert lib().qsl_forward(None, None, None) == 1
    assert lib().qsl_backward(None, None, None) == 1
    assert lib().qsl_n_basis(None) == -1
    assert lib().qsl_system_destroy(None) == 0


def test_plan_argument_checks():
    """Plan entry points reject NULL / out-of-range arguments on the host."""
    from paper_1209_6630_amd._lib import Tuning, lib
    L = lib()
    h = ct.c_void_p()
    W = (ct.c_int64 * 1)(4)
    assert L.qsl_plan_create(0, None, W, 0, 0, ct.byref(h)) == 1
    assert L.qsl_plan_create(1, None, W, 0, 0, ct.byref(h)) == 1
    assert L.qsl_plan_launch(None, None) == 1
    assert L.qsl_plan_bind(None, 0, None, None) == 1
    t = Tuning(1, 0, 0, 0, 0, 0)
    assert L.qsl_plan_set_tuning(None, ct.byref(t)) == 1
    assert L.qsl_plan_get_tuning(None, ct.byref(t)) == 1
    assert L.qsl_autotune(None, None, None, None) == 1
    assert L.qsl_plan_destroy(None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1209_6630_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()
