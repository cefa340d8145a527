"""Python binding of the Slater-matrix builder: argument marshalling only.

Torch supplies device memory and the current HIP stream; every step of the
computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _lib
from ._lib import (BwdArgs, DmcArgs, FwdArgs, LocalArgs, MODES, MultidetArgs, PLAN_GRAPH, SystemDesc, Tuning, check,
                   lib)


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def mode_id(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


class System:
    """A molecular system (atoms, contracted Cartesian Gaussian shells) and the
    MO coefficients of both spins, resident on the current GPU."""

    def __init__(self, atom_xyz, shell_atom, shell_l, shell_nprim, prim_exp, prim_coef,
                 n_up, n_dn, screen_T=30.0):
        self._keep = [np.ascontiguousarray(atom_xyz, np.float64),
                      np.ascontiguousarray(shell_atom, np.int32),
                      np.ascontiguousarray(shell_l, np.int32),
                      np.ascontiguousarray(shell_nprim, np.int32),
                      np.ascontiguousarray(prim_exp, np.float64),
                      np.ascontiguousarray(prim_coef, np.float64)]
        xyz, sa, sl, sn, ex, co = self._keep
        dp, ip = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32)
        desc = SystemDesc(xyz.shape[0], xyz.ctypes.data_as(dp), sl.shape[0], sa.ctypes.data_as(ip),
                          sl.ctypes.data_as(ip), sn.ctypes.data_as(ip), ex.ctypes.data_as(dp),
                          co.ctypes.data_as(dp), int(n_up), int(n_dn), float(screen_T), 0)
        h = ct.c_void_p()
        check(lib().qsl_system_create(ct.byref(desc), ct.byref(h)))
        self._h = h
        self.n_up, self.n_dn = int(n_up), int(n_dn)
        self.n_basis = int(lib().qsl_n_basis(h))
        self._ws = {}

    @classmethod
    def from_synth(cls, s):
        return cls(s.atom_xyz, s.shell_atom, s.shell_l, s.shell_nprim, s.prim_exp, s.prim_coef,
                   s.n_up, s.n_dn, s.screen_T)

    def close(self):
        if getattr(self, "_h", None):
            lib().qsl_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_elec(self):
        return self.n_up + self.n_dn

    def n_spin(self, spin):
        return self.n_dn if spin else self.n_up

    def ao_info(self):
        nb = self.n_basis
        at = np.zeros(nb, np.int32)
        sh = np.zeros(nb, np.int32)
        nxyz = np.zeros(3 * nb, np.int8)
        check(lib().qsl_ao_info(self._h, at.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                sh.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                nxyz.ctypes.data_as(ct.POINTER(ct.c_int8))))
        return at, sh, nxyz.reshape(nb, 3)

    def set_mo(self, spin, A):
        """A: [n_spin, N_basis] float64, a CUDA tensor or a host array."""
        if isinstance(A, torch.Tensor) and A.is_cuda:
            A = A.to(torch.float64).contiguous()
            check(lib().qsl_set_mo(self._h, spin, _ptr(A), A.shape[1], 1, _stream()))
            torch.cuda.current_stream().synchronize()
        else:
            a = np.ascontiguousarray(np.asarray(A, np.float64))
            check(lib().qsl_set_mo(self._h, spin, ct.c_void_p(a.ctypes.data), a.shape[1], 0, _stream()))

    def set_orbitals(self, spin, A):
        """Orbital set of a spin for several determinants: A [n_orb, N_basis]
        float64 host array, n_orb >= the spin's electrons."""
        a = np.ascontiguousarray(np.asarray(A, np.float64))
        check(lib().qsl_set_orbitals(self._h, spin, ct.c_void_p(a.ctypes.data), a.shape[0], a.shape[1], 0,
                                     _stream()))

    def multidet_forward(self, R, occ, coef, mode="fp64"):
        """Psi_det = sum_K coef[K] Det_K_up Det_K_dn with occ [n_det, n_up +
        n_dn] orbital indices (up then down).  Returns a dict of CUDA
        tensors: logpsi, sign, drift, lap, status, det_logdet, det_sign."""
        occ = np.ascontiguousarray(occ, np.int32)
        coef = np.ascontiguousarray(coef, np.float64)
        W, N, nd = R.shape[0], self.n_elec, occ.shape[0]
        dev = R.device
        out = dict(logpsi=torch.empty(W, dtype=torch.float64, device=dev),
                   sign=torch.empty(W, dtype=torch.int8, device=dev),
                   drift=torch.empty((W, N, 3), dtype=torch.float64, device=dev),
                   lap=torch.empty((W, N), dtype=torch.float64, device=dev),
                   status=torch.empty(W, dtype=torch.int32, device=dev),
                   det_logdet=torch.empty((nd, W, 2), dtype=torch.float64, device=dev),
                   det_sign=torch.empty((nd, W, 2), dtype=torch.int8, device=dev))
        n = ct.c_size_t()
        check(lib().qsl_multidet_workspace_size(self._h, W, mode_id(mode), nd, ct.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        a = MultidetArgs(W, R.data_ptr(), mode_id(mode), nd, occ.ctypes.data_as(ct.POINTER(ct.c_int32)),
                         coef.ctypes.data_as(ct.POINTER(ct.c_double)), out["logpsi"].data_ptr(),
                         out["sign"].data_ptr(), out["drift"].data_ptr(), out["lap"].data_ptr(),
                         out["status"].data_ptr(), out["det_logdet"].data_ptr(), out["det_sign"].data_ptr(),
                         ws.data_ptr(), ws.numel())
        check(lib().qsl_multidet_forward(self._h, ct.byref(a), _stream()))
        out["_ws"] = ws
        return out

    def set_jastrow(self, Z, c_ee=1.0, b_ee=1.0, c_en=1.0, b_en=1.0):
        """Nuclear charges Z[n_atoms] and the Jastrow parameters (see
        qsl_set_jastrow)."""
        z = np.ascontiguousarray(Z, np.float64)
        self._Z = z
        check(lib().qsl_set_jastrow(self._h, z.ctypes.data_as(ct.POINTER(ct.c_double)), float(c_ee), float(b_ee),
                                    float(c_en), float(b_en)))

    def local_energy(self, R, out):
        """E_L, the full drift, log|Psi| and sign of Psi at R from the forward
        outputs `out` at R.  Returns a dict of CUDA tensors."""
        W, N = R.shape[0], self.n_elec
        dev = R.device
        res = dict(EL=torch.empty(W, dtype=torch.float64, device=dev),
                   drift=torch.empty((W, N, 3), dtype=torch.float64, device=dev),
                   logpsi=torch.empty(W, dtype=torch.float64, device=dev),
                   psisign=torch.empty(W, dtype=torch.int8, device=dev),
                   J=torch.empty(W, dtype=torch.float64, device=dev),
                   V=torch.empty(W, dtype=torch.float64, device=dev))
        a = LocalArgs(W, R.data_ptr(), out["drift"].data_ptr(), out["lap"].data_ptr(), out["logdet"].data_ptr(),
                      out["sign"].data_ptr(), res["EL"].data_ptr(), res["drift"].data_ptr(),
                      res["logpsi"].data_ptr(), res["psisign"].data_ptr(), res["J"].data_ptr(), res["V"].data_ptr())
        check(lib().qsl_local_energy(self._h, ct.byref(a), _stream()))
        return res

    def workspace(self, W, mode, backward=True):
        """A device workspace for W walkers (grown on demand and kept): the
        forward's regions only, or (backward) everything."""
        n = ct.c_size_t()
        what = _lib.WS_BOTH if backward else _lib.WS_FORWARD
        check(lib().qsl_workspace_size(self._h, int(W), mode_id(mode), what, ct.byref(n)))
        key = torch.cuda.current_device()
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n.value:
            ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
            self._ws[key] = ws
        return ws

    def alloc_outputs(self, W, mode, drift=True):
        dev = "cuda"
        cdt = torch.float64 if mode_id(mode) == 0 else torch.float32
        nu, nd, N = self.n_up, self.n_dn, self.n_elec
        out = dict(
            C_up=torch.empty((W, 5, nu, nu), dtype=cdt, device=dev),
            C_dn=torch.empty((W, 5, nd, nd), dtype=cdt, device=dev),
            logdet=torch.empty((W, 2), dtype=torch.float64, device=dev),
            sign=torch.empty((W, 2), dtype=torch.int8, device=dev),
            Dinv_up=torch.empty((W, nu, nu), dtype=torch.float64, device=dev),
            Dinv_dn=torch.empty((W, nd, nd), dtype=torch.float64, device=dev),
            status=torch.empty((W,), dtype=torch.int32, device=dev),
        )
        if drift:
            out["drift"] = torch.empty((W, N, 3), dtype=torch.float64, device=dev)
            out["lap"] = torch.empty((W, N), dtype=torch.float64, device=dev)
        return out

    def forward(self, R, mode="fp64", out=None, drift=True):
        """R: CUDA float64 [W, N, 3].  Returns a dict of CUDA tensors."""
        assert R.is_cuda and R.dtype == torch.float64 and R.is_contiguous()
        W = R.shape[0]
        assert R.shape[1:] == (self.n_elec, 3), "R must be [W, n_up+n_dn, 3]"
        if out is None:
            out = self.alloc_outputs(W, mode, drift)
        ws = self.workspace(W, mode, backward=False)
        a = _fwd_args(self, R, mode, out)
        a.ws = ws.data_ptr()
        a.ws_bytes = ws.numel()
        check(lib().qsl_forward(self._h, ct.byref(a), _stream()))
        return out

    def backward(self, R, Dinv_up, Dinv_dn, g, mode="fp64", dR=None, dA=None, accumulate=False,
                 want_dR=True, want_dA=True, drift=None):
        """Adjoint of sum g[w,s] logdet[w,s].  Returns (dR, dA_up, dA_dn).
        drift: the forward's drift on the same R (then dR = g drift);
        None recomputes the AO gradients for dR."""
        W = R.shape[0]
        dev = "cuda"
        if want_dR and dR is None:
            dR = torch.empty((W, self.n_elec, 3), dtype=torch.float64, device=dev)
        if want_dA and dA is None:
            dA = (torch.zeros((self.n_up, self.n_basis), dtype=torch.float64, device=dev),
                  torch.zeros((self.n_dn, self.n_basis), dtype=torch.float64, device=dev))
        g = g.to(torch.float64).contiguous()
        ws = self.workspace(W, mode)
        a = BwdArgs()
        a.W = W
        a.R = R.data_ptr()
        a.mode = mode_id(mode)
        a.Dinv[0] = Dinv_up.data_ptr()
        a.Dinv[1] = Dinv_dn.data_ptr()
        a.g_logdet = g.data_ptr()
        a.dR = dR.data_ptr() if want_dR else None
        a.dA[0] = dA[0].data_ptr() if want_dA else None
        a.dA[1] = dA[1].data_ptr() if want_dA else None
        a.accumulate_dA = 1 if accumulate else 0
        a.ws = ws.data_ptr()
        a.ws_bytes = ws.numel()
        a.drift = drift.data_ptr() if drift is not None else None
        check(lib().qsl_backward(self._h, ct.byref(a), _stream()))
        return dR, (dA[0] if want_dA else None), (dA[1] if want_dA else None)


def _fwd_args(system, R, mode, out):
    a = FwdArgs()
    a.W = R.shape[0]
    a.R = R.data_ptr()
    a.mode = mode_id(mode)
    a.C[0] = out["C_up"].data_ptr()
    a.C[1] = out["C_dn"].data_ptr()
    a.logdet = out["logdet"].data_ptr()
    a.sign = out["sign"].data_ptr()
    a.Dinv[0] = out["Dinv_up"].data_ptr()
    a.Dinv[1] = out["Dinv_dn"].data_ptr()
    a.drift = out["drift"].data_ptr() if "drift" in out else None
    a.lap = out["lap"].data_ptr() if "lap" in out else None
    a.status = out["status"].data_ptr()
    return a


class Plan:
    """An uneven batch: the forward (and optionally the adjoint) of several
    systems, one batched launch per kernel phase, optionally replayed from a
    HIP graph.  Buffers are bound once and must stay allocated."""

    def __init__(self, systems, walkers, mode="fp32", graph=True):
        self.systems = list(systems)
        self.W = [int(w) for w in walkers]
        self.mode = mode
        n = len(self.systems)
        hs = (ct.c_void_p * n)(*[s._h.value for s in self.systems])
        ws = (ct.c_int64 * n)(*self.W)
        h = ct.c_void_p()
        check(lib().qsl_plan_create(n, hs, ws, mode_id(mode), PLAN_GRAPH if graph else 0, ct.byref(h)))
        self._h = h
        self._keep = {}

    def bind(self, i, R, out, g=None, dR=None, dA=None, accumulate=False):
        """Bind system i: coordinates R, forward outputs `out` (from
        System.alloc_outputs) and, with g, the adjoint buffers dR / dA."""
        S = self.systems[i]
        f = _fwd_args(S, R, self.mode, out)
        b = None
        if g is not None:
            b = BwdArgs()
            b.W = R.shape[0]
            b.R = R.data_ptr()
            b.mode = mode_id(self.mode)
            b.Dinv[0] = out["Dinv_up"].data_ptr()
            b.Dinv[1] = out["Dinv_dn"].data_ptr()
            b.g_logdet = g.data_ptr()
            b.dR = dR.data_ptr() if dR is not None else None
            b.dA[0] = dA[0].data_ptr() if dA is not None else None
            b.dA[1] = dA[1].data_ptr() if dA is not None else None
            b.accumulate_dA = 1 if accumulate else 0
        check(lib().qsl_plan_bind(self._h, i, ct.byref(f), ct.byref(b) if b is not None else None))
        self._keep[i] = (R, out, g, dR, dA)  # keep the bound tensors alive

    def launch(self):
        check(lib().qsl_plan_launch(self._h, _stream()))

    @property
    def tuning(self):
        t = Tuning()
        check(lib().qsl_plan_get_tuning(self._h, ct.byref(t)))
        return {k: getattr(t, k) for k in _lib.TUNING_FIELDS}

    @tuning.setter
    def tuning(self, d):
        t = Tuning(*[int(d.get(k, _lib.TUNING_DEFAULTS[k])) for k in _lib.TUNING_FIELDS])
        check(lib().qsl_plan_set_tuning(self._h, ct.byref(t)))

    def autotune(self, cache_path=None):
        t = Tuning()
        check(lib().qsl_autotune(self._h, cache_path.encode() if cache_path else None, _stream(), ct.byref(t)))
        return {k: getattr(t, k) for k in _lib.TUNING_FIELDS}

    def close(self):
        if getattr(self, "_h", None):
            lib().qsl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SlaterLogDet(torch.autograd.Function):
    """logdet[W, 2] of the up/down Slater matrices; differentiable in R, A_up
    and A_dn through the library's hand-written adjoint kernel."""

    @staticmethod
    def forward(ctx, R, A_up, A_dn, system, mode="fp64"):
        system.set_mo(0, A_up.detach())
        system.set_mo(1, A_dn.detach())
        out = system.forward(R.detach().contiguous(), mode)
        ctx.system, ctx.mode = system, mode
        ctx.save_for_backward(R.detach(), out["Dinv_up"], out["Dinv_dn"], out["drift"], out["status"])
        ctx.mark_non_differentiable(out["sign"])
        return out["logdet"], out["sign"]

    @staticmethod
    def backward(ctx, g_logdet, _g_sign):
        R, Di_up, Di_dn, drift, status = ctx.saved_tensors
        # a walker with a singular spin has log|det| = -inf and an undefined
        # inverse: it gets no gradient (the kernels require g = 0 there)
        singular = (status & 1).bool()
        g = torch.where(singular[:, None], torch.zeros_like(g_logdet), g_logdet)
        dR, dA_up, dA_dn = ctx.system.backward(R, Di_up, Di_dn, g, ctx.mode, drift=drift)
        return dR, dA_up, dA_dn, None, None


def slater_logdet(R, A_up, A_dn, system, mode="fp64"):
    return SlaterLogDet.apply(R, A_up, A_dn, system, mode)


# ------------------------------------------------------------- QMC step

def drift_diffuse(R, drift, eta, tau):
    out = torch.empty_like(R)
    check(lib().qsl_drift_diffuse(R.numel(), _ptr(R), _ptr(drift), _ptr(eta), float(tau), _ptr(out), _stream()))
    return out


def branch_weights(EL_new, EL_old, sign_new, sign_old, E_T, tau):
    w = torch.empty_like(EL_new)
    check(lib().qsl_branch_weights(EL_new.numel(), _ptr(EL_new), _ptr(EL_old), _ptr(sign_new), _ptr(sign_old),
                                   float(E_T), float(tau), _ptr(w), _stream()))
    return w


def reconfigure(w, u):
    """Parent indices (int64) and the total weight (a 1-element tensor)."""
    W = w.numel()
    idx = torch.empty(W, dtype=torch.int64, device=w.device)
    wsum = torch.empty(1, dtype=torch.float64, device=w.device)
    cum = torch.empty(max(W, 1), dtype=torch.float64, device=w.device)
    check(lib().qsl_reconfigure(W, _ptr(w), _ptr(u), _ptr(idx), _ptr(wsum), _ptr(cum), _stream()))
    return idx, wsum


def gather_walkers(idx, src):
    dst = torch.empty_like(src)
    W = idx.numel()
    width = src.numel() // max(W, 1) * src.element_size()
    check(lib().qsl_gather_walkers(W, width, _ptr(idx), _ptr(src), _ptr(dst), _stream()))
    return dst


class DMC:
    """Fixed-node DMC with reconfiguration for one system: the population R
    (kept on the GPU) and its state; each step() moves, rebuilds the Slater
    part through a forward-only plan (graph-replayed), evaluates the local
    energy, weights and reconfigures.  eta and u are the caller's random
    deviates of the step (CUDA float64 tensors)."""

    def __init__(self, system, R, mode="fp32", tau=0.01, E_T=0.0, graph=True):
        W, N = R.shape[0], system.n_elec
        self.S, self.W, self.N, self.mode = system, W, N, mode
        self.tau, self.E_T = float(tau), float(E_T)
        dev = R.device
        self.R = R.clone().contiguous()
        self.Rp = torch.empty_like(self.R)
        self.out = system.alloc_outputs(W, mode)
        self.plan = Plan([system], [W], mode, graph=graph)
        self.plan.bind(0, self.Rp, self.out)
        self.EL = torch.empty(W, dtype=torch.float64, device=dev)
        self.drift = torch.empty((W, N, 3), dtype=torch.float64, device=dev)
        self.psisign = torch.empty(W, dtype=torch.int8, device=dev)
        self.logpsi = torch.empty(W, dtype=torch.float64, device=dev)
        self.idx = torch.empty(W, dtype=torch.int64, device=dev)
        self.wsum = torch.empty(1, dtype=torch.float64, device=dev)
        n = ct.c_size_t()
        check(lib().qsl_dmc_workspace_size(W, N, ct.byref(n)))
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        self._eta = self._u = None
        check(lib().qsl_dmc_init(self.plan._h, ct.byref(self._args()), _stream()))

    def _args(self):
        return DmcArgs(0, self.W, self.tau, self.E_T, self.R.data_ptr(), self.EL.data_ptr(), self.drift.data_ptr(),
                       self.psisign.data_ptr(), self.logpsi.data_ptr(),
                       self._eta.data_ptr() if self._eta is not None else None,
                       self._u.data_ptr() if self._u is not None else None,
                       self.idx.data_ptr(), self.wsum.data_ptr(), self.ws.data_ptr(), self.ws.numel())

    def step(self, eta, u):
        self._eta, self._u = eta, u
        check(lib().qsl_dmc_step(self.plan._h, ct.byref(self._args()), _stream()))

    def close(self):
        self.plan.close()
