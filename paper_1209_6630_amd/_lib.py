"""ctypes declarations of the C ABI in include/qslater.h.

Loads the in-tree libqslater.so built for gfx950.  There is no fallback: if
the library is missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqslater.so")

QSL_OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "shape mismatch",
                4: "workspace too small", 5: "HIP runtime error", 6: "out of device memory"}
MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2}
STATUS_SINGULAR, STATUS_NEAR_TIE, STATUS_NONFINITE = 1, 2, 4

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int32)


class SystemDesc(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int32), ("atom_xyz", _dp), ("n_shells", ct.c_int32),
                ("shell_atom", _ip), ("shell_l", _ip), ("shell_nprim", _ip),
                ("prim_exp", _dp), ("prim_coef", _dp), ("n_up", ct.c_int32), ("n_dn", ct.c_int32),
                ("screen_T", ct.c_double), ("flags", ct.c_uint32)]


class FwdArgs(ct.Structure):
    _fields_ = [("W", ct.c_int64), ("R", ct.c_void_p), ("mode", ct.c_int32),
                ("C", ct.c_void_p * 2), ("logdet", ct.c_void_p), ("sign", ct.c_void_p),
                ("Dinv", ct.c_void_p * 2), ("drift", ct.c_void_p), ("lap", ct.c_void_p),
                ("status", ct.c_void_p), ("ws", ct.c_void_p), ("ws_bytes", ct.c_size_t)]


class BwdArgs(ct.Structure):
    _fields_ = [("W", ct.c_int64), ("R", ct.c_void_p), ("mode", ct.c_int32),
                ("Dinv", ct.c_void_p * 2), ("g_logdet", ct.c_void_p), ("dR", ct.c_void_p),
                ("dA", ct.c_void_p * 2), ("accumulate_dA", ct.c_int32), ("ws", ct.c_void_p),
                ("ws_bytes", ct.c_size_t), ("drift", ct.c_void_p)]


class Tuning(ct.Structure):
    _fields_ = [("batched", ct.c_int32), ("adj_group", ct.c_int32), ("gj_bias", ct.c_int32),
                ("contract_tile", ct.c_int32), ("persistent", ct.c_int32), ("det_dA", ct.c_int32)]


TUNING_FIELDS = ("batched", "adj_group", "gj_bias", "contract_tile", "persistent", "det_dA")
# what a field left out of a tuning dict takes (the library's defaults)
TUNING_DEFAULTS = {"batched": 1, "adj_group": 0, "gj_bias": 0, "contract_tile": 2, "persistent": 0, "det_dA": 0}


class LocalArgs(ct.Structure):
    _fields_ = [("W", ct.c_int64), ("R", ct.c_void_p), ("drift_det", ct.c_void_p), ("lap_det", ct.c_void_p),
                ("logdet", ct.c_void_p), ("sign", ct.c_void_p), ("EL", ct.c_void_p), ("drift", ct.c_void_p),
                ("logpsi", ct.c_void_p), ("psisign", ct.c_void_p), ("J", ct.c_void_p), ("V", ct.c_void_p)]


class DmcArgs(ct.Structure):
    _fields_ = [("sys_index", ct.c_int32), ("W", ct.c_int64), ("tau", ct.c_double), ("E_T", ct.c_double),
                ("R", ct.c_void_p), ("EL", ct.c_void_p), ("drift", ct.c_void_p), ("psisign", ct.c_void_p),
                ("logpsi", ct.c_void_p), ("eta", ct.c_void_p), ("u", ct.c_void_p), ("idx", ct.c_void_p),
                ("wsum", ct.c_void_p), ("ws", ct.c_void_p), ("ws_bytes", ct.c_size_t)]


class MultidetArgs(ct.Structure):
    _fields_ = [("W", ct.c_int64), ("R", ct.c_void_p), ("mode", ct.c_int32), ("n_det", ct.c_int32),
                ("occ", ct.POINTER(ct.c_int32)), ("coef", ct.POINTER(ct.c_double)), ("logpsi", ct.c_void_p),
                ("sign", ct.c_void_p), ("drift", ct.c_void_p), ("lap", ct.c_void_p), ("status", ct.c_void_p),
                ("det_logdet", ct.c_void_p), ("det_sign", ct.c_void_p), ("ws", ct.c_void_p), ("ws_bytes", ct.c_size_t)]


PLAN_GRAPH = 1
WS_FORWARD, WS_BACKWARD, WS_BOTH = 1, 2, 3
NOALLOC_SCRATCH_BYTES = 64 << 20


class KernelTime(ct.Structure):
    _fields_ = [("name", ct.c_char * 48), ("launches", ct.c_int64), ("total_ms", ct.c_double)]


# name -> (restype, argtypes); every symbol declared in include/qslater.h
SIGNATURES = {
    "qsl_system_create": (ct.c_int, [ct.POINTER(SystemDesc), ct.POINTER(ct.c_void_p)]),
    "qsl_system_destroy": (ct.c_int, [ct.c_void_p]),
    "qsl_n_basis": (ct.c_int64, [ct.c_void_p]),
    "qsl_ao_info": (ct.c_int, [ct.c_void_p, _ip, _ip, ct.POINTER(ct.c_int8)]),
    "qsl_set_mo": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p]),
    "qsl_workspace_size": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_size_t)]),
    "qsl_forward": (ct.c_int, [ct.c_void_p, ct.POINTER(FwdArgs), ct.c_void_p]),
    "qsl_forward_noalloc": (ct.c_int, [ct.c_void_p, ct.POINTER(FwdArgs), ct.c_void_p]),
    "qsl_backward": (ct.c_int, [ct.c_void_p, ct.POINTER(BwdArgs), ct.c_void_p]),
    "qsl_plan_create": (ct.c_int, [ct.c_int32, ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_int64), ct.c_int32,
                                   ct.c_uint32, ct.POINTER(ct.c_void_p)]),
    "qsl_plan_bind": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.POINTER(FwdArgs), ct.POINTER(BwdArgs)]),
    "qsl_plan_set_tuning": (ct.c_int, [ct.c_void_p, ct.POINTER(Tuning)]),
    "qsl_plan_get_tuning": (ct.c_int, [ct.c_void_p, ct.POINTER(Tuning)]),
    "qsl_plan_launch": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "qsl_plan_destroy": (ct.c_int, [ct.c_void_p]),
    "qsl_autotune": (ct.c_int, [ct.c_void_p, ct.c_char_p, ct.c_void_p, ct.POINTER(Tuning)]),
    "qsl_profile_enable": (ct.c_int, [ct.c_int32]),
    "qsl_profile_read": (ct.c_int, [ct.POINTER(KernelTime), ct.c_int32, ct.POINTER(ct.c_int32), ct.c_int32]),
    "qsl_set_orbitals": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_int32,
                                    ct.c_void_p]),
    "qsl_multidet_workspace_size": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32,
                                               ct.POINTER(ct.c_size_t)]),
    "qsl_multidet_forward": (ct.c_int, [ct.c_void_p, ct.POINTER(MultidetArgs), ct.c_void_p]),
    "qsl_set_jastrow": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double), ct.c_double, ct.c_double, ct.c_double,
                                   ct.c_double]),
    "qsl_local_energy": (ct.c_int, [ct.c_void_p, ct.POINTER(LocalArgs), ct.c_void_p]),
    "qsl_drift_diffuse": (ct.c_int, [ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_double, ct.c_void_p,
                                     ct.c_void_p]),
    "qsl_branch_weights": (ct.c_int, [ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_double,
                                      ct.c_double, ct.c_void_p, ct.c_void_p]),
    "qsl_reconfigure": (ct.c_int, [ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                   ct.c_void_p]),
    "qsl_gather_walkers": (ct.c_int, [ct.c_int64, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "qsl_dmc_workspace_size": (ct.c_int, [ct.c_int64, ct.c_int32, ct.POINTER(ct.c_size_t)]),
    "qsl_dmc_init": (ct.c_int, [ct.c_void_p, ct.POINTER(DmcArgs), ct.c_void_p]),
    "qsl_dmc_step": (ct.c_int, [ct.c_void_p, ct.POINTER(DmcArgs), ct.c_void_p]),
    "qsl_status_string": (ct.c_char_p, [ct.c_int]),
    "qsl_last_error": (ct.c_char_p, []),
}

_lib = None


class QslError(RuntimeError):
    def __init__(self, code, detail=""):
        self.code = code
        super().__init__(f"qslater: {STATUS_NAMES.get(code, code)}" + (f" ({detail})" if detail else ""))


def lib():
    """The loaded library (raises if libqslater.so was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1209_6630_amd/build.py "
                              "(there is no CPU fallback)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != QSL_OK:
        raise QslError(code, lib().qsl_last_error().decode())


def profile_enable(on=True):
    check(lib().qsl_profile_enable(1 if on else 0))


def profile_read(reset=True):
    """{kernel name: (launches, total ms)} of the launches timed so far."""
    n = ct.c_int32()
    check(lib().qsl_profile_read(None, 0, ct.byref(n), 0))
    buf = (KernelTime * max(1, n.value))()
    check(lib().qsl_profile_read(buf, n.value, ct.byref(n), 1 if reset else 0))
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}
