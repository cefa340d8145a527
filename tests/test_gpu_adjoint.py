"""GPU adjoint (d log|det| / dA and / dR) against the FP64 oracle, the
Jacobi drift and the identity dA A^T = (sum_w g_w) I."""
import numpy as np
import pytest

import oracle
import qsl_synth as q
from tests.gpu_common import U32, dA_tol, make_gpu_system, max_survivors
from tests.systems import random_tiny, walkers_near

pytestmark = pytest.mark.gpu


def _abs_bounds(sysm, A_up, A_dn, R, ref, g):
    """sum_{w,e} |G[e][i]| |chi_j(r_e)| (for dA) and
    sum_j (|G| |A|)_j |grad chi_j| (for dR), from the oracle's AOs."""
    W, N = R.shape[:2]
    nb = sysm.n_basis
    bA = [np.zeros((sysm.n_up, nb)), np.zeros((sysm.n_dn, nb))]
    bR = np.zeros((W, N, 3))
    for w in range(W):
        for e in range(N):
            s = 0 if e < sysm.n_up else 1
            el = e if s == 0 else e - sysm.n_up
            Di = ref["Dinv_up" if s == 0 else "Dinv_dn"][w]
            A = A_up if s == 0 else A_dn
            G = np.abs(g[w, s] * Di[el])
            idx, B, _ = oracle.ao_eval(sysm, R[w, e])
            bA[s][:, idx] += np.outer(G, np.abs(B[0]))
            H = G @ np.abs(A[:, idx])
            bR[w, e] = np.abs(B[1:4]) @ H
    return bA, bR


def _run(sysm, A_up, A_dn, R, mode, seed=0, use_drift=False):
    import torch
    S = make_gpu_system(sysm, A_up, A_dn)
    Rt = torch.from_numpy(R).cuda()
    out = S.forward(Rt, mode)
    g = np.random.default_rng(seed).normal(size=(R.shape[0], 2))
    gt = torch.from_numpy(g).cuda()
    dR, dAu, dAd = S.backward(Rt, out["Dinv_up"], out["Dinv_dn"], gt, mode,
                              drift=out["drift"] if use_drift else None)
    torch.cuda.synchronize()
    return g, dR.cpu().numpy(), dAu.cpu().numpy(), dAd.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("name,W,use_drift", [("44e", 8, False), ("158e", 4, False), ("434e", 2, False),
                                              ("1731e", 1, False), ("44e", 8, True), ("158e", 4, True),
                                              ("434e", 2, True)])
@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_backward_configs(name, W, use_drift, mode):
    """dR from recomputed AO gradients, or from the forward's drift: both
    within the same bound (the drift's C_2..C_4 carry the forward's
    product error, which that bound covers)."""
    print(f"[case] backward {name} W={W} mode={mode} drift={use_drift}", flush=True)
    sysm, A_up, A_dn, R = q.make_config(name, W=W)
    g, dR, dAu, dAd, out = _run(sysm, A_up, A_dn, R, mode, use_drift=use_drift)
    # the adjoint arithmetic: the oracle adjoint from the GPU's own inverse
    # (same G; the forward tests bound the inverse itself)
    ref = {"Dinv_up": out["Dinv_up"], "Dinv_dn": out["Dinv_dn"]}
    if mode == "fp64":
        tol = 1e-10
    else:
        # G rounded to FP32, AO values in FP32 (64 u32), FP32 sums of 32
        # electrons (dA) or of MOs (dR) and of nnz AOs
        nnz = max_survivors(sysm, R[:1])
        tol = (64 + 64 + 2 * nnz) * U32 + (3 * 2.0 ** -16 if mode == "bf16x3" else 0.0)
    rdR, rdAu, rdAd = oracle.backward(sysm, A_up, A_dn, R, ref["Dinv_up"], ref["Dinv_dn"], g)
    bA, bR = _abs_bounds(sysm, A_up, A_dn, R, ref, g)
    tu, td = tol, tol
    if mode != "fp64":  # the dA sums' own chain (tests/gpu_common.py dA_tol)
        tu, td = max(tol, dA_tol(mode, W, sysm.n_up)), max(tol, dA_tol(mode, W, sysm.n_dn))
    assert np.all(np.abs(dAu - rdAu) <= tu * bA[0] + 1e-300), float((np.abs(dAu - rdAu) / (bA[0] + 1e-300)).max())
    assert np.all(np.abs(dAd - rdAd) <= td * bA[1] + 1e-300)
    assert np.all(np.abs(dR - rdR) <= tol * bR + 1e-300), float((np.abs(dR - rdR) / (bR + 1e-300)).max())
    if mode == "fp64":
        # identities of the exact adjoint
        np.testing.assert_allclose(dAu @ A_up.T, g[:, 0].sum() * np.eye(sysm.n_up), atol=1e-8)
        gg = np.concatenate([np.repeat(g[:, :1], sysm.n_up, 1), np.repeat(g[:, 1:], sysm.n_dn, 1)], 1)
        np.testing.assert_allclose(dR, gg[:, :, None] * out["drift"], rtol=1e-8, atol=1e-10 * np.abs(dR).max())


@pytest.mark.parametrize("n_atoms,n_up,n_dn,W", [(2, 3, 2, 3), (5, 12, 11, 5), (12, 40, 39, 3)])
@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_backward_few_windows(n_atoms, n_up, n_dn, W, mode):
    """Systems with fewer windows than one dA block of 32: waves that own
    no window, partly filled slot blocks, a single walker iteration or a
    few; against the oracle adjoint within the bound of the full-size
    configurations."""
    print(f"[case] backward few windows atoms={n_atoms} n={n_up}/{n_dn} W={W} mode={mode}", flush=True)
    sysm, A_up, A_dn = random_tiny(n_atoms=n_atoms, n_up=n_up, n_dn=n_dn, seed=21 + n_atoms)
    R = walkers_near(sysm, W, seed=3 + n_atoms)
    for use_drift in (False, True):
        g, dR, dAu, dAd, out = _run(sysm, A_up, A_dn, R, mode, use_drift=use_drift)
        ref = {"Dinv_up": out["Dinv_up"], "Dinv_dn": out["Dinv_dn"]}
        nnz = max_survivors(sysm, R[:1])
        tol = (64 + 64 + 2 * nnz) * U32 + (3 * 2.0 ** -16 if mode == "bf16x3" else 0.0)
        rdR, rdAu, rdAd = oracle.backward(sysm, A_up, A_dn, R, ref["Dinv_up"], ref["Dinv_dn"], g)
        bA, bR = _abs_bounds(sysm, A_up, A_dn, R, ref, g)
        tu, td = max(tol, dA_tol(mode, W, n_up)), max(tol, dA_tol(mode, W, n_dn))
        assert np.all(np.abs(dAu - rdAu) <= tu * bA[0] + 1e-300)
        assert np.all(np.abs(dAd - rdAd) <= td * bA[1] + 1e-300)
        assert np.all(np.abs(dR - rdR) <= tol * bR + 1e-300)


def test_autograd_function_matches_oracle():
    print("[case] autograd", flush=True)
    import torch
    from paper_1209_6630_amd.api import System, slater_logdet
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=5, n_dn=4, seed=9)
    R = walkers_near(sysm, 3, seed=4)
    S = System.from_synth(sysm)
    Rt = torch.from_numpy(R).cuda().requires_grad_(True)
    Au = torch.from_numpy(A_up).cuda().requires_grad_(True)
    Ad = torch.from_numpy(A_dn).cuda().requires_grad_(True)
    ld, sg = slater_logdet(Rt, Au, Ad, S, "fp64")
    w = torch.tensor([[1.0, -0.5], [0.3, 2.0], [-1.2, 0.7]], dtype=torch.float64, device="cuda")
    (ld * w).sum().backward()
    ref = oracle.forward(sysm, A_up, A_dn, R)
    rdR, rdAu, rdAd = oracle.backward(sysm, A_up, A_dn, R, ref["Dinv_up"], ref["Dinv_dn"], w.cpu().numpy())
    np.testing.assert_allclose(ld.detach().cpu().numpy(), ref["logdet"], rtol=1e-12)
    np.testing.assert_allclose(Rt.grad.cpu().numpy(), rdR, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Au.grad.cpu().numpy(), rdAu, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Ad.grad.cpu().numpy(), rdAd, rtol=1e-9, atol=1e-12)


def test_backward_accumulate_and_finite_difference():
    print("[case] accumulate + FD", flush=True)
    import torch
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=13)
    sysm.screen_T = 1e300
    R = walkers_near(sysm, 2, seed=5)
    S = make_gpu_system(sysm, A_up, A_dn)
    Rt = torch.from_numpy(R).cuda()
    out = S.forward(Rt, "fp64")
    g = torch.ones((2, 2), dtype=torch.float64, device="cuda")
    dR, dAu, dAd = S.backward(Rt, out["Dinv_up"], out["Dinv_dn"], g, "fp64")
    dR2, dAu2, dAd2 = S.backward(Rt, out["Dinv_up"], out["Dinv_dn"], g, "fp64", dA=(dAu.clone(), dAd.clone()),
                                 accumulate=True)
    np.testing.assert_allclose(dAu2.cpu().numpy(), 2 * dAu.cpu().numpy(), rtol=1e-14)

    def L(Au):
        S.set_mo(0, Au)
        o = S.forward(Rt, "fp64")
        return float(o["logdet"].sum())
    h = 1e-6
    for (i, j) in [(0, 0), (2, 7)]:
        Ap = A_up.copy(); Ap[i, j] += h
        Am = A_up.copy(); Am[i, j] -= h
        fd = (L(Ap) - L(Am)) / (2 * h)
        assert dAu.cpu().numpy()[i, j] == pytest.approx(fd, rel=1e-5, abs=1e-7)


@pytest.mark.parametrize("use_drift", [False, True])
def test_singular_walker_zero_weight_gives_zero_dR(use_drift):
    """A singular walker (NaN inverse and drift) with g = 0 contributes
    exactly nothing: its dR rows are 0 and dA stays finite, on both dR paths;
    the other walkers' dR equal g times their drift."""
    print(f"[case] singular walker adjoint drift={use_drift}", flush=True)
    import torch
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=5)
    R = walkers_near(sysm, 3, seed=2)
    R[1, 2] = [400.0, -300.0, 250.0]   # beyond every atomic radius
    S = make_gpu_system(sysm, A_up, A_dn)
    Rt = torch.from_numpy(R).cuda()
    out = S.forward(Rt, "fp64")
    assert int(out["status"][1].item()) & 1
    g = np.array([[0.7, -1.1], [0.0, 0.0], [1.3, 0.4]])
    dR, dAu, dAd = S.backward(Rt, out["Dinv_up"], out["Dinv_dn"], torch.from_numpy(g).cuda(), "fp64",
                              drift=out["drift"] if use_drift else None)
    dR = dR.cpu().numpy()
    assert np.all(dR[1] == 0.0)
    assert np.all(np.isfinite(dAu.cpu().numpy())) and np.all(np.isfinite(dAd.cpu().numpy()))
    drift = out["drift"].cpu().numpy()
    for w in (0, 2):
        gg = np.concatenate([np.full(sysm.n_up, g[w, 0]), np.full(sysm.n_dn, g[w, 1])])
        np.testing.assert_allclose(dR[w], gg[:, None] * drift[w], rtol=1e-9, atol=1e-12)


def test_autograd_singular_walker_gets_no_gradient():
    """slater_logdet(...).sum().backward() with a singular walker (log|det|
    = -inf): that walker contributes no gradient, every gradient stays
    finite, and the rest equals the oracle adjoint with its weight zeroed."""
    print("[case] autograd singular walker", flush=True)
    import torch
    from paper_1209_6630_amd.api import System, slater_logdet
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=5)
    R = walkers_near(sysm, 3, seed=2)
    R[1, 2] = [400.0, -300.0, 250.0]   # beyond every atomic radius: spin up singular
    S = System.from_synth(sysm)
    Rt = torch.from_numpy(R).cuda().requires_grad_(True)
    Au = torch.from_numpy(A_up).cuda().requires_grad_(True)
    Ad = torch.from_numpy(A_dn).cuda().requires_grad_(True)
    ld, _ = slater_logdet(Rt, Au, Ad, S, "fp64")
    assert torch.isneginf(ld[1, 0])
    ld.sum().backward()
    for t in (Rt.grad, Au.grad, Ad.grad):
        assert torch.isfinite(t).all()
    ref = oracle.forward(sysm, A_up, A_dn, R)
    g = np.ones((3, 2))
    g[1] = 0.0
    Du, Dd = np.nan_to_num(ref["Dinv_up"]), np.nan_to_num(ref["Dinv_dn"])
    rdR, rdAu, rdAd = oracle.backward(sysm, A_up, A_dn, R, Du, Dd, g)
    np.testing.assert_allclose(Au.grad.cpu().numpy(), rdAu, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Ad.grad.cpu().numpy(), rdAd, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Rt.grad.cpu().numpy(), rdR, rtol=1e-9, atol=1e-12)
