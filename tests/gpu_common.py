"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs, and the error bounds of each
precision mode, derived from the arithmetic.

Bounds (u32 = 2^-24, the FP32 unit roundoff; S = sum_k |a_ik| |B_n(k,e)| is
the oracle's absolute sum for C_n[e][i]; nnz = survivors per electron):
  FP64    |dC| <= 1e-12 S  (FP64 sums of <= ~10^3 terms and 1-ulp exp)
  FP32    |dC| <= (64 + 2 nnz) u32 S   (AO values with a few roundings and a
          1-ulp expf, a sum of nnz products)
  BF16X3  |dC| <= (3 * 2^-16 + (64 + 2 nnz) u32) S   (bf16 keeps 8 significant
          bits, so |x - hi| <= 2^-8 |x|: the dropped lo*lo term and the bf16
          rounding of each lo part are each <= 2^-16 |a||b|)
  log|det|: first order, |d logdet| <= 2 sum_ei |Dinv[e][i]| tol S_1[e][i]
  Dinv:     |dDinv| <= 2 |Dinv| (tol S_1)^T |Dinv| + 1e-12 |Dinv|-scale
"""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24


def tol_C(mode, nnz_max):
    if mode == "fp64":
        return 1e-12
    base = (64 + 2 * nnz_max) * U32
    return base if mode == "fp32" else base + 3 * 2.0 ** -16


def default_dA_group(mode, W, det=False):
    """Walkers per dA walker group when the tuning leaves adj_group at 0:
    1024 for the FP32 dA by electron index, 128 for the dA by 32-electron
    range (FP64, split BF16, and FP32 with the deterministic reduction)."""
    return min(W, 1024 if mode == "fp32" and not det else 128)


def dA_tol(mode, W, n, gw=None, det=False):
    """Worst-case bound on |dA_gpu - dA| / bA (bA: the oracle's sum of
    absolute values of the terms), FP32 and split-BF16 modes: 64 u32 for
    the FP32 AO value, 1 u32 for the FP32 rounding of G = g D^-1, and the
    longest chain m of FP32 additions into one dA element:
      by electron (FP32): the gw walkers of a group in one MFMA
        accumulator, then one atomic add per (electron, walker group):
        m = gw + ceil(W / gw) n;
      by 32-electron range: gw walkers of 32 electrons with up to three
        split products per term, then one atomic add per (walker group,
        electron range): m = 3 gw 32 + ceil(W / gw) ceil(n / 32);
    plus 3 2^-16 for the split-BF16 products."""
    gw = gw or default_dA_group(mode, W, det)
    if mode == "fp32" and not det:
        m = gw + -(-W // gw) * n
    else:
        m = 3 * gw * 32 + -(-W // gw) * -(-n // 32)
    return (64 + 1 + m) * U32 + (3 * 2.0 ** -16 if mode == "bf16x3" else 0.0)


def max_survivors(sysm, R):
    return max(oracle.ao_eval(sysm, r)[0].size for r in R.reshape(-1, 3))


def run_gpu_forward(S, R_np, mode):
    import torch
    R = torch.from_numpy(np.ascontiguousarray(R_np)).cuda()
    out = S.forward(R, mode)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def make_gpu_system(sysm, A_up, A_dn):
    from paper_1209_6630_amd.api import System
    S = System.from_synth(sysm)
    S.set_mo(0, A_up)
    S.set_mo(1, A_dn)
    return S


def compare_forward(sysm, A_up, A_dn, R, gpu, mode, ref=None, walkers=None, check_status=True):
    """Element-wise comparison of every forward output against the oracle."""
    if ref is None:
        ref = oracle.forward(sysm, A_up, A_dn, R, want_abs=True)
    W = R.shape[0]
    walkers = range(W) if walkers is None else walkers
    nnz = max_survivors(sysm, R[list(walkers)[:4]]) if mode != "fp64" else 0
    tol = tol_C(mode, nnz)
    report = {}
    for s, (Ck, Dk, Ak) in enumerate([("C_up", "Dinv_up", "Cabs_up"), ("C_dn", "Dinv_dn", "Cabs_dn")]):
        n = sysm.n_dn if s else sysm.n_up
        if n == 0:
            assert np.all(gpu["logdet"][:, s] == 0.0) and np.all(gpu["sign"][:, s] == 1)
            continue
        for gi, w in enumerate(walkers):
            Cg = gpu[Ck][gi].astype(np.float64)
            Cr = ref[Ck][w]
            S_ = ref[Ak][w]
            err = np.abs(Cg - Cr)
            bound = tol * S_ + 1e-300
            bad = err > bound
            assert not bad.any(), (Ck, w, float((err / np.maximum(S_, 1e-300)).max()), tol)
            report.setdefault("C_relS", []).append(float((err / np.maximum(S_, 1e-300)).max()))
            if ref["sign"][w, s] == 0:  # this spin's matrix is singular
                assert gpu["sign"][gi, s] == 0 and np.isneginf(gpu["logdet"][gi, s])
                assert gpu["status"][gi] & 1
                continue
            assert gpu["sign"][gi, s] == ref["sign"][w, s], (w, s)
            Di = ref[Dk][w]
            if mode == "fp64":
                assert abs(gpu["logdet"][gi, s] - ref["logdet"][w, s]) <= 1e-10 * max(1.0, abs(ref["logdet"][w, s]))
                cond = np.linalg.cond(Cr[0].T)
                if cond < 1e8:
                    rel = np.linalg.norm(gpu[Dk][gi] - Di) / np.linalg.norm(Di)
                    assert rel <= 1e-10, (w, s, rel, cond)
                    report.setdefault("Dinv_rel", []).append(rel)
            else:
                dS1 = tol * S_[0].T          # bound on |dD| (D[i][e] = C_1[e][i])
                b_ld = 2.0 * np.sum(np.abs(Di) * dS1.T)
                assert abs(gpu["logdet"][gi, s] - ref["logdet"][w, s]) <= b_ld + 1e-12, (w, s, b_ld)
                b_Di = 2.0 * np.abs(Di) @ dS1 @ np.abs(Di)
                errD = np.abs(gpu[Dk][gi] - Di)
                assert np.all(errD <= b_Di + 1e-12 * np.abs(Di).max()), (w, s, float((errD / (b_Di + 1e-300)).max()))
                report.setdefault("logdet_abs", []).append(abs(gpu["logdet"][gi, s] - ref["logdet"][w, s]))
        # drift / Laplacian rows of this spin
        e0 = sysm.n_up if s else 0
        for gi, w in enumerate(walkers):
            if ref["status"][w] & 1:
                continue  # drift/Laplacian of a walker with a singular spin are undefined
            dg = gpu["drift"][gi, e0:e0 + n]
            dr = ref["drift"][w, e0:e0 + n]
            lg = gpu["lap"][gi, e0:e0 + n]
            lr = ref["lap"][w, e0:e0 + n]
            if mode == "fp64":
                for l in range(3):
                    sc = np.abs(ref[Dk][w] * ref[Ck][w][1 + l]).sum(1)
                    assert np.all(np.abs(dg[:, l] - dr[:, l]) <= 1e-10 * sc + 1e-300)
                sc = np.abs(ref[Dk][w] * ref[Ck][w][4]).sum(1)
                assert np.all(np.abs(lg - lr) <= 1e-10 * sc + 1e-300)
            else:
                Di = ref[Dk][w]
                dS1 = tol * ref[Ak][w][0].T
                b_Di = 2.0 * np.abs(Di) @ dS1 @ np.abs(Di)
                for l in range(4):
                    Cn = ref[Ck][w][1 + l]
                    bnd = (b_Di * np.abs(Cn)).sum(1) + 2.0 * (np.abs(Di) * tol * ref[Ak][w][1 + l]).sum(1)
                    got = dg[:, l] if l < 3 else lg
                    want = dr[:, l] if l < 3 else lr
                    assert np.all(np.abs(got - want) <= bnd + 1e-12), (w, s, l)
    if check_status:
        for gi, w in enumerate(walkers):
            assert (gpu["status"][gi] & 1) == (ref["status"][w] & 1)
    return report
