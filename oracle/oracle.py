"""ctypes wrapper around the plain C FP64 oracle (test infrastructure only).

Every function here marshals numpy arrays into the C routines of
qsl_oracle.c; no arithmetic of the method is done in Python.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsl_oracle.c")
_LIB = os.path.join(_HERE, "libqsl_oracle.so")
_lib = None

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int32)


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
           "-fPIC", "-std=c99", "-D_DEFAULT_SOURCE", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Sys(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int32), ("atom_xyz", _dp),
                ("n_shells", ct.c_int32), ("shell_atom", _ip), ("shell_l", _ip),
                ("shell_nprim", _ip), ("prim_exp", _dp), ("prim_coef", _dp),
                ("n_up", ct.c_int32), ("n_dn", ct.c_int32), ("screen_T", ct.c_double)]


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ct.CDLL(_LIB)
        S = ct.POINTER(_Sys)
        lib.orc_n_basis.argtypes = [S]
        lib.orc_n_basis.restype = ct.c_int
        lib.orc_normalize.argtypes = [S, _dp]
        lib.orc_cart_factor.argtypes = [ct.c_int] * 4
        lib.orc_cart_factor.restype = ct.c_double
        lib.orc_ao_eval.argtypes = [S, _dp, _ip, _dp, ct.c_int, _ip]
        lib.orc_ao_eval.restype = ct.c_int
        lib.orc_lu_inverse.argtypes = [_dp, ct.c_int, _dp, _dp, _ip]
        lib.orc_lu_inverse.restype = ct.c_int
        lib.orc_forward.argtypes = [S, _dp, _dp, ct.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                    ct.POINTER(ct.c_int8), _dp, _dp, _dp, _dp,
                                    ct.POINTER(ct.c_uint32), ct.c_int32]
        lib.orc_backward.argtypes = [S, _dp, _dp, ct.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                     _dp, _dp, _dp, _dp, ct.c_int32]
        lib.orc_max_threads.restype = ct.c_int
        lib.orc_jastrow_potential.argtypes = [S, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                              ct.c_int32, _dp, _dp, _dp, _dp, _dp, ct.c_int32]
        lib.orc_local_energy.argtypes = [ct.c_int32, ct.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_drift_diffuse.argtypes = [ct.c_int64, _dp, _dp, _dp, ct.c_double, _dp]
        lib.orc_branch_weights.argtypes = [ct.c_int64, _dp, _dp, ct.POINTER(ct.c_int8), ct.POINTER(ct.c_int8),
                                           ct.c_double, ct.c_double, _dp]
        lib.orc_reconfigure.argtypes = [ct.c_int64, _dp, _dp, ct.POINTER(ct.c_int64), _dp]
        lib.orc_multidet.argtypes = [S, _dp, _dp, ct.c_int32, _ip, _dp, ct.c_int32, _dp, _dp,
                                     ct.POINTER(ct.c_int8), _dp, _dp, _dp, ct.POINTER(ct.c_int8), ct.c_int32]
        _lib = lib
    return _lib


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class OracleSystem:
    """Holds contiguous copies of a system description for the C oracle."""

    def __init__(self, sys):
        self.xyz = np.ascontiguousarray(sys.atom_xyz, np.float64)
        self.sa = np.ascontiguousarray(sys.shell_atom, np.int32)
        self.sl = np.ascontiguousarray(sys.shell_l, np.int32)
        self.sn = np.ascontiguousarray(sys.shell_nprim, np.int32)
        self.ex = np.ascontiguousarray(sys.prim_exp, np.float64)
        self.co = np.ascontiguousarray(sys.prim_coef, np.float64)
        self.n_up, self.n_dn = int(sys.n_up), int(sys.n_dn)
        self.T = float(sys.screen_T)
        self.c = _Sys(self.xyz.shape[0], _p(self.xyz), self.sl.shape[0], _p(self.sa, _ip),
                      _p(self.sl, _ip), _p(self.sn, _ip), _p(self.ex), _p(self.co),
                      self.n_up, self.n_dn, self.T)

    @property
    def ref(self):
        return ct.byref(self.c)


def _osys(sys):
    return sys if isinstance(sys, OracleSystem) else OracleSystem(sys)


def n_basis(sys) -> int:
    o = _osys(sys)
    return load().orc_n_basis(o.ref)


def normalize(sys) -> np.ndarray:
    o = _osys(sys)
    out = np.zeros_like(o.co)
    load().orc_normalize(o.ref, _p(out))
    return out


def cart_factor(l, a, b, c) -> float:
    return load().orc_cart_factor(l, a, b, c)


def ao_eval(sys, r):
    """Screened AOs at one point: (idx[s], B[5, s], near_tie)."""
    o = _osys(sys)
    nb = n_basis(o)
    idx = np.zeros(nb + 1, np.int32)
    B = np.zeros((5, nb + 1))
    nt = np.zeros(1, np.int32)
    r = np.ascontiguousarray(r, np.float64)
    n = load().orc_ao_eval(o.ref, _p(r), _p(idx, _ip), _p(B), nb + 1, _p(nt, _ip))
    return idx[:n].copy(), B[:, :n].copy(), bool(nt[0])


def lu_inverse(m):
    m = np.ascontiguousarray(m, np.float64)
    n = m.shape[0]
    inv = np.zeros_like(m)
    ld = np.zeros(1)
    sg = np.zeros(1, np.int32)
    ok = load().orc_lu_inverse(_p(m), n, _p(inv), _p(ld), _p(sg, _ip))
    return bool(ok), float(ld[0]), int(sg[0]), inv


def forward(sys, A_up, A_dn, R, want_abs=False, nthreads=0):
    """Full FP64 forward.  Returns a dict of numpy arrays."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, np.float64)
    W, N = R.shape[0], R.shape[1]
    nu, nd = o.n_up, o.n_dn
    A_up = np.ascontiguousarray(A_up, np.float64)
    A_dn = np.ascontiguousarray(A_dn, np.float64)
    out = dict(
        C_up=np.zeros((W, 5, nu, nu)), C_dn=np.zeros((W, 5, nd, nd)),
        logdet=np.zeros((W, 2)), sign=np.zeros((W, 2), np.int8),
        Dinv_up=np.zeros((W, nu, nu)), Dinv_dn=np.zeros((W, nd, nd)),
        drift=np.zeros((W, N, 3)), lap=np.zeros((W, N)), status=np.zeros(W, np.uint32))
    if want_abs:
        out["Cabs_up"] = np.zeros((W, 5, nu, nu))
        out["Cabs_dn"] = np.zeros((W, 5, nd, nd))
    load().orc_forward(o.ref, _p(A_up), _p(A_dn), W, _p(R), _p(out["C_up"]), _p(out["C_dn"]),
                       _p(out.get("Cabs_up")), _p(out.get("Cabs_dn")), _p(out["logdet"]),
                       _p(out["sign"], ct.POINTER(ct.c_int8)), _p(out["Dinv_up"]),
                       _p(out["Dinv_dn"]), _p(out["drift"]), _p(out["lap"]),
                       _p(out["status"], ct.POINTER(ct.c_uint32)), int(nthreads))
    return out


def backward(sys, A_up, A_dn, R, Dinv_up, Dinv_dn, g, nthreads=0, want_abs=False):
    """Adjoint of log|det|: returns (dR[W,N,3], dA_up, dA_dn); with want_abs
    also (dR_abs, dA_abs_up, dA_abs_dn), the same sums over the absolute
    values of every term."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, np.float64)
    W, N = R.shape[0], R.shape[1]
    A_up = np.ascontiguousarray(A_up, np.float64)
    A_dn = np.ascontiguousarray(A_dn, np.float64)
    Dinv_up = np.ascontiguousarray(Dinv_up, np.float64)
    Dinv_dn = np.ascontiguousarray(Dinv_dn, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    dR = np.zeros((W, N, 3))
    dA_up = np.zeros_like(A_up)
    dA_dn = np.zeros_like(A_dn)
    ab = (np.zeros((W, N, 3)), np.zeros_like(A_up), np.zeros_like(A_dn)) if want_abs else (None, None, None)
    load().orc_backward(o.ref, _p(A_up), _p(A_dn), W, _p(R), _p(Dinv_up), _p(Dinv_dn), _p(g),
                        _p(dR), _p(dA_up), _p(dA_dn), _p(ab[0]), _p(ab[1]), _p(ab[2]), int(nthreads))
    if want_abs:
        return dR, dA_up, dA_dn, ab
    return dR, dA_up, dA_dn


def max_threads() -> int:
    return int(load().orc_max_threads())


# ------------------------------------------------------------- QMC step

def jastrow_potential(sys, Z, R, c_ee=1.0, b_ee=1.0, c_en=1.0, b_en=1.0, nthreads=0):
    """Jastrow exponent J[W], its gradient gJ[W,N,3] and Laplacian lJ[W,N]
    per electron, and the Coulomb potential V[W]."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, np.float64)
    W, N = R.shape[0], R.shape[1]
    Z = np.ascontiguousarray(Z, np.float64)
    J, gJ, lJ, V = np.zeros(W), np.zeros((W, N, 3)), np.zeros((W, N)), np.zeros(W)
    load().orc_jastrow_potential(o.ref, _p(Z), float(c_ee), float(b_ee), float(c_en), float(b_en), W, _p(R), _p(J),
                                 _p(gJ), _p(lJ), _p(V), int(nthreads))
    return J, gJ, lJ, V


def local_energy(drift_det, lap_det, gJ, lJ, V):
    """E_L[W] and the full drift b[W,N,3] of Psi = e^J Det_up Det_dn."""
    bd = np.ascontiguousarray(drift_det, np.float64)
    ld = np.ascontiguousarray(lap_det, np.float64)
    gJ = np.ascontiguousarray(gJ, np.float64)
    lJ = np.ascontiguousarray(lJ, np.float64)
    V = np.ascontiguousarray(V, np.float64)
    W, N = ld.shape
    EL, b = np.zeros(W), np.zeros((W, N, 3))
    load().orc_local_energy(W, N, _p(bd), _p(ld), _p(gJ), _p(lJ), _p(V), _p(EL), _p(b))
    return EL, b


def drift_diffuse(R, b, eta, tau):
    R = np.ascontiguousarray(R, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    eta = np.ascontiguousarray(eta, np.float64)
    out = np.zeros_like(R)
    load().orc_drift_diffuse(R.size, _p(R), _p(b), _p(eta), float(tau), _p(out))
    return out


def branch_weights(EL_new, EL_old, sign_new, sign_old, E_T, tau):
    EL_new = np.ascontiguousarray(EL_new, np.float64)
    EL_old = np.ascontiguousarray(EL_old, np.float64)
    sn = np.ascontiguousarray(sign_new, np.int8)
    so = np.ascontiguousarray(sign_old, np.int8)
    w = np.zeros(EL_new.shape[0])
    i8 = ct.POINTER(ct.c_int8)
    load().orc_branch_weights(w.size, _p(EL_new), _p(EL_old), _p(sn, i8), _p(so, i8), float(E_T), float(tau),
                              _p(w))
    return w


def reconfigure(w, u):
    """Parent index of each new walker and the total weight."""
    w = np.ascontiguousarray(w, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    idx = np.zeros(w.size, np.int64)
    s = np.zeros(1)
    load().orc_reconfigure(w.size, _p(w), _p(u), _p(idx, ct.POINTER(ct.c_int64)), _p(s))
    return idx, float(s[0])


def multidet(sys, A_up_orb, A_dn_orb, occ, coef, R, nthreads=0):
    """Psi_det = sum_K coef[K] Det_K_up Det_K_dn: log|Psi|[W], sign[W],
    drift[W,N,3], lap[W,N], and per determinant logdet, sign [n_det,W,2]."""
    o = _osys(sys)
    R = np.ascontiguousarray(R, np.float64)
    W, N = R.shape[0], R.shape[1]
    Au = np.ascontiguousarray(A_up_orb, np.float64)
    Ad = np.ascontiguousarray(A_dn_orb, np.float64)
    occ = np.ascontiguousarray(occ, np.int32)
    coef = np.ascontiguousarray(coef, np.float64)
    nd = occ.shape[0]
    out = dict(logpsi=np.zeros(W), sign=np.zeros(W, np.int8), drift=np.zeros((W, N, 3)), lap=np.zeros((W, N)),
               det_logdet=np.zeros((nd, W, 2)), det_sign=np.zeros((nd, W, 2), np.int8))
    i8 = ct.POINTER(ct.c_int8)
    load().orc_multidet(o.ref, _p(Au), _p(Ad), nd, _p(occ, _ip), _p(coef), W, _p(R), _p(out["logpsi"]),
                        _p(out["sign"], i8), _p(out["drift"]), _p(out["lap"]), _p(out["det_logdet"]),
                        _p(out["det_sign"], i8), int(nthreads))
    return out
