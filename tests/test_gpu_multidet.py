"""Several determinants on the GPU (one product over the orbital set per spin,
each determinant's columns gathered and inverted in FP64, combined per
walker) against the FP64 oracle.

Bounds: FP64, 1e-10 relative on log|Psi| and each determinant's log|det|;
drift and Laplacian ratio 1e-8 of their scale.  FP32 and split BF16: each
determinant's log|det| within the first-order bound of the forward tests,
2 sum |D^-1| tol_C S_1 (tests/gpu_common.py); log|Psi| within
sum_K |w_K| times those bounds (w_K = c_K Det_K / Psi, its first-order
sensitivity to each log|det_K|)."""
import numpy as np
import pytest

import oracle
import qsl_synth as q
from tests.gpu_common import make_gpu_system, max_survivors, tol_C

pytestmark = pytest.mark.gpu


def _orbital_system(name, W, extra, seed=3):
    sysm, A_up, A_dn, R = q.make_config(name, W=W)
    rng = np.random.default_rng(seed)
    nb = sysm.n_basis
    Au = np.concatenate([A_up, rng.normal(size=(extra, nb)) / np.sqrt(nb)])
    Ad = np.concatenate([A_dn, rng.normal(size=(extra, nb)) / np.sqrt(nb)])
    if q.CONFIGS[name]["a_fp32"]:
        Au, Ad = Au.astype(np.float32).astype(np.float64), Ad.astype(np.float32).astype(np.float64)
    return sysm, Au, Ad, R


def _occupations(sysm, extra, n_det, seed=4):
    """Ground state and single / double excitations into the extra orbitals."""
    rng = np.random.default_rng(seed)
    nu, nd = sysm.n_up, sysm.n_dn
    occ = [np.concatenate([np.arange(nu), np.arange(nd)])]
    while len(occ) < n_det:
        o = occ[0].copy()
        for _ in range(rng.integers(1, 3)):
            s = rng.integers(0, 2)
            if s == 0:
                o[rng.integers(0, nu)] = nu + rng.integers(0, extra)
            else:
                o[nu + rng.integers(0, nd)] = nd + rng.integers(0, extra)
        if len(set(o[:nu])) == nu and len(set(o[nu:])) == nd:
            occ.append(o)
    coef = np.concatenate([[1.0], rng.normal(scale=0.2, size=n_det - 1)])
    return np.array(occ, np.int32), coef


def _run(sysm, Au, Ad, R, occ, coef, mode):
    import torch
    S = make_gpu_system(sysm, Au[:sysm.n_up], Ad[:sysm.n_dn])
    S.set_orbitals(0, Au)
    S.set_orbitals(1, Ad)
    out = S.multidet_forward(torch.from_numpy(np.ascontiguousarray(R)).cuda(), occ, coef, mode)
    torch.cuda.synchronize()
    return S, {k: v.cpu().numpy() for k, v in out.items() if not k.startswith("_")}


@pytest.mark.parametrize("name,W,extra,n_det", [("44e", 16, 6, 5), ("158e", 4, 8, 4), ("44e", 8, 130, 3)])
def test_multidet_fp64(name, W, extra, n_det):
    print(f"[case] multidet fp64 {name} W={W} dets={n_det}", flush=True)
    sysm, Au, Ad, R = _orbital_system(name, W, extra)
    occ, coef = _occupations(sysm, extra, n_det)
    S, got = _run(sysm, Au, Ad, R, occ, coef, "fp64")
    ref = oracle.multidet(sysm, Au, Ad, occ, coef, R)
    np.testing.assert_array_equal(got["sign"], ref["sign"])
    np.testing.assert_array_equal(got["det_sign"], ref["det_sign"])
    np.testing.assert_allclose(got["logpsi"], ref["logpsi"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(got["det_logdet"], ref["det_logdet"], rtol=1e-10, atol=1e-10)
    for k in ("drift", "lap"):
        sc = np.abs(ref[k]).max()
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-8, atol=1e-8 * sc)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_multidet_reduced_precision_434e(mode):
    """434 electrons, 8 walkers, 4 determinants from 6 extra orbitals per
    spin, products in FP32 or split BF16."""
    print(f"[case] multidet 434e {mode}", flush=True)
    W, extra = 8, 6
    sysm, Au, Ad, R = _orbital_system("434e", W, extra)
    occ, coef = _occupations(sysm, extra, 4)
    S, got = _run(sysm, Au, Ad, R, occ, coef, mode)
    ref = oracle.multidet(sysm, Au, Ad, occ, coef, R)
    np.testing.assert_array_equal(got["det_sign"], ref["det_sign"])
    tol = tol_C(mode, max_survivors(sysm, R[:2]))
    nu, nd = sysm.n_up, sysm.n_dn
    bound = np.zeros((occ.shape[0], W, 2))
    for K in range(occ.shape[0]):
        f = oracle.forward(sysm, Au[occ[K, :nu]], Ad[occ[K, nu:]], R, want_abs=True)
        for s, (Dk, Ak) in enumerate([("Dinv_up", "Cabs_up"), ("Dinv_dn", "Cabs_dn")]):
            for w in range(W):
                bound[K, w, s] = 2.0 * np.sum(np.abs(f[Dk][w]) * tol * f[Ak][w][0])
    err = np.abs(got["det_logdet"] - ref["det_logdet"])
    assert np.all(err <= bound + 1e-12), float((err / (bound + 1e-300)).max())
    L = ref["det_logdet"].sum(2) + np.log(np.abs(coef))[:, None]
    wK = np.exp(L - ref["logpsi"][None, :])        # |c_K Det_K / Psi|
    b_psi = (wK * bound.sum(2)).sum(0)
    np.testing.assert_array_equal(got["sign"], ref["sign"])
    assert np.all(np.abs(got["logpsi"] - ref["logpsi"]) <= b_psi + 1e-12)


def test_single_determinant_forward_needs_square_orbitals():
    """With an orbital set larger than the electrons the one-determinant
    forward reports SHAPE; qsl_set_mo restores it."""
    print("[case] orbital set shape checks", flush=True)
    import torch
    from paper_1209_6630_amd import QslError
    sysm, Au, Ad, R = _orbital_system("44e", 4, 3)
    S = make_gpu_system(sysm, Au[:sysm.n_up], Ad[:sysm.n_dn])
    S.set_orbitals(0, Au)
    Rt = torch.from_numpy(R).cuda()
    with pytest.raises(QslError) as ei:
        S.forward(Rt, "fp64")
    assert ei.value.code == 3
    S.set_mo(0, Au[:sysm.n_up])
    out = S.forward(Rt, "fp64")
    torch.cuda.synchronize()
    ref = oracle.forward(sysm, Au[:sysm.n_up], Ad[:sysm.n_dn], R)
    np.testing.assert_allclose(out["logdet"].cpu().numpy(), ref["logdet"], rtol=1e-10)
