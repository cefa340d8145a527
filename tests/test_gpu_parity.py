"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (element by element, bounds in tests/gpu_common.py)."""
import numpy as np
import pytest

import oracle
import qsl_synth as q
from tests.gpu_common import compare_forward, make_gpu_system, max_survivors, run_gpu_forward, tol_C
from tests.systems import make_tiny, random_tiny, walkers_near

pytestmark = pytest.mark.gpu


def _cfg(name, W):
    sysm, A_up, A_dn, R = q.make_config(name, W=W)
    return sysm, A_up, A_dn, R


@pytest.mark.parametrize("name,W", [("44e", 16), ("158e", 6), ("434e", 3), ("1731e", 2)])
@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_forward_configs(name, W, mode):
    print(f"[case] forward {name} W={W} mode={mode}", flush=True)
    sysm, A_up, A_dn, R = _cfg(name, W)
    S = make_gpu_system(sysm, A_up, A_dn)
    gpu = run_gpu_forward(S, R, mode)
    compare_forward(sysm, A_up, A_dn, R, gpu, mode)


@pytest.mark.parametrize("n_up,n_dn", [(1, 0), (1, 1), (3, 2), (32, 31), (33, 33), (64, 63), (65, 64),
                                       (128, 127), (129, 100), (224, 223), (225, 224), (257, 256),
                                       (480, 479), (545, 511), (1024, 1000)])
def test_forward_tile_and_inversion_boundaries(n_up, n_dn):
    """Electron counts at the 32-electron tile and at every inversion
    variant boundary (32, 64, 128, 224 register-resident, then blocked up to
    the 1024 maximum), with s, p and d shells.  The blocked sizes end their
    last pass of two 32-column panels in every way: with the second panel 1
    (225, 545), 31 (511) or 8 (1000) columns wide, with the first panel
    alone, whole (480) or not (479, 257), and on a whole pass (256, 1024)."""
    print(f"[case] boundaries n_up={n_up} n_dn={n_dn}", flush=True)
    nat = max(2, (n_up + n_dn) // 6 + 1)
    sysm, A_up, A_dn = random_tiny(n_atoms=nat, n_up=n_up, n_dn=n_dn, seed=n_up * 7 + n_dn)
    # enough AOs for a non-singular square Slater matrix
    if sysm.n_basis < n_up:
        pytest.skip("basis smaller than the electron count")
    R = walkers_near(sysm, 3, seed=n_up)
    S = make_gpu_system(sysm, A_up, A_dn)
    for mode in ("fp64", "fp32"):
        gpu = run_gpu_forward(S, R, mode)
        compare_forward(sysm, A_up, A_dn, R, gpu, mode)


def test_more_electrons_than_supported_is_an_error():
    print("[case] n above the inversion maximum", flush=True)
    from paper_1209_6630_amd import QslError
    sysm, A_up, A_dn = random_tiny(n_atoms=180, n_up=1025, n_dn=2, seed=3)
    R = walkers_near(sysm, 1, seed=1)
    S = make_gpu_system(sysm, A_up, A_dn)
    with pytest.raises(QslError) as ei:
        run_gpu_forward(S, R, "fp32")
    assert ei.value.code == 2  # QSL_ERR_UNSUPPORTED


@pytest.mark.parametrize("n_up", [40, 300])
def test_singular_walker_blocked_and_register(n_up):
    """A walker whose electron lies beyond every atomic radius has a zero
    column: log|det| = -inf, sign 0, status bit, in both inversion forms."""
    print(f"[case] singular n_up={n_up}", flush=True)
    nat = max(3, (2 * n_up) // 6 + 1)
    sysm, A_up, A_dn = random_tiny(n_atoms=nat, n_up=n_up, n_dn=n_up - 1, seed=11)
    R = walkers_near(sysm, 2, seed=5)
    R[0, n_up - 1] = [900.0, -700.0, 650.0]
    S = make_gpu_system(sysm, A_up, A_dn)
    gpu = run_gpu_forward(S, R, "fp64")
    assert gpu["sign"][0, 0] == 0 and np.isneginf(gpu["logdet"][0, 0]) and gpu["status"][0] & 1
    assert gpu["sign"][1, 0] != 0 and not (gpu["status"][1] & 1)
    compare_forward(sysm, A_up, A_dn, R, gpu, "fp64")


def test_singular_walker():
    print("[case] singular walker", flush=True)
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=5)
    R = walkers_near(sysm, 3, seed=2)
    R[1, 2] = [400.0, -300.0, 250.0]   # beyond every atomic radius
    S = make_gpu_system(sysm, A_up, A_dn)
    gpu = run_gpu_forward(S, R, "fp64")
    assert gpu["sign"][1, 0] == 0 and np.isneginf(gpu["logdet"][1, 0])
    assert gpu["status"][1] & 1 and gpu["status"][0] == 0
    assert np.all(gpu["C_up"][1, :, 2, :] == 0.0)
    compare_forward(sysm, A_up, A_dn, R, gpu, "fp64")


def test_contraction_identity_is_scatter():
    """A = I: C_n is the dense scatter of the screened AO block."""
    print("[case] identity A", flush=True)
    sysm = make_tiny([(0, 0, [0.8, 2.0], [0.6, 0.3]), (0, 1, [0.9], [1.0]), (1, 0, [0.5], [1.0])],
                     [[0, 0, 0], [1.4, 0.3, -0.2]], 5, 5)
    I = np.eye(5)
    R = walkers_near(sysm, 4, seed=3)
    S = make_gpu_system(sysm, I, I)
    gpu = run_gpu_forward(S, R, "fp64")
    for w in range(4):
        for e in range(10):
            idx, B, _ = oracle.ao_eval(sysm, R[w, e])
            dense = np.zeros((5, 5))
            dense[:, idx] = B
            C = gpu["C_up"] if e < 5 else gpu["C_dn"]
            np.testing.assert_allclose(C[w, :, e % 5, :], dense, rtol=1e-13, atol=1e-300)


def test_walker_permutation_and_electron_swap():
    """Same walkers in another order give the same rows; swapping two
    same-spin electrons flips the GPU sign and keeps log|det|."""
    print("[case] permutation", flush=True)
    sysm, A_up, A_dn, R = _cfg("158e", 4)
    S = make_gpu_system(sysm, A_up, A_dn)
    g1 = run_gpu_forward(S, R, "fp64")
    g2 = run_gpu_forward(S, R[::-1].copy(), "fp64")
    np.testing.assert_array_equal(g1["logdet"], g2["logdet"][::-1])
    np.testing.assert_array_equal(g1["C_up"], g2["C_up"][::-1])
    R3 = R.copy()
    R3[:, [3, 40]] = R3[:, [40, 3]]
    g3 = run_gpu_forward(S, R3, "fp64")
    np.testing.assert_array_equal(g3["sign"][:, 0], -g1["sign"][:, 0])
    np.testing.assert_allclose(g3["logdet"], g1["logdet"], rtol=1e-12)


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_full_size_sampled_434e(mode):
    """The 434-electron workload at its full batch of 4096 walkers (the
    benchmark's launch shapes): sampled walkers against the oracle."""
    print(f"[case] full-size 434e mode={mode}", flush=True)
    import torch
    sysm, A_up, A_dn, R = _cfg("434e", 4096)
    S = make_gpu_system(sysm, A_up, A_dn)
    Rt = torch.from_numpy(R).cuda()
    out = S.forward(Rt, mode)
    torch.cuda.synchronize()
    sample = [0, 1, 2047, 4095]
    gpu = {k: v[sample].cpu().numpy() for k, v in out.items()}
    del out
    ref = oracle.forward(sysm, A_up, A_dn, R[sample], want_abs=True)
    compare_forward(sysm, A_up, A_dn, R[sample], gpu, mode, ref=ref)


def test_status_near_tie_is_flagged():
    """An electron placed exactly at gamma r^2 = T for one primitive."""
    print("[case] near tie", flush=True)
    g = 0.75
    sysm = make_tiny([(0, 0, [g, 3.0], [0.5, 0.5]), (1, 0, [0.4], [1.0])],
                     [[0, 0, 0], [1.0, 0.0, 0.0]], 1, 1)
    r = np.sqrt(30.0 / g)
    R = np.array([[[r, 0.0, 0.0], [1.2, 0.1, 0.0]]])
    S = make_gpu_system(sysm, np.array([[1.0, 0.5]]), np.array([[0.3, 1.0]]))
    gpu = run_gpu_forward(S, R, "fp64")
    assert gpu["status"][0] & 2


def test_workspace_too_small_is_an_error():
    """A missing or short workspace is QSL_ERR_WORKSPACE; the forward needs
    only its own regions, the adjoint everything."""
    print("[case] workspace errors", flush=True)
    import ctypes as ct
    import torch
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import _fwd_args
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=8)
    R = walkers_near(sysm, 4, seed=3)
    S = make_gpu_system(sysm, A_up, A_dn)
    L = _lib.lib()
    nf, nb = ct.c_size_t(), ct.c_size_t()
    _lib.check(L.qsl_workspace_size(S._h, 4, 1, _lib.WS_FORWARD, ct.byref(nf)))
    _lib.check(L.qsl_workspace_size(S._h, 4, 1, _lib.WS_BOTH, ct.byref(nb)))
    assert 0 < nf.value < nb.value
    assert L.qsl_workspace_size(S._h, 4, 1, 7, ct.byref(nf)) == 1
    Rt = torch.from_numpy(R).cuda()
    out = S.alloc_outputs(4, "fp32")
    a = _fwd_args(S, Rt, "fp32", out)
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    a.ws, a.ws_bytes = None, 0
    assert L.qsl_forward(S._h, ct.byref(a), None) == 4
    a.ws, a.ws_bytes = ws.data_ptr(), nf.value - 1
    assert L.qsl_forward(S._h, ct.byref(a), None) == 4
    a.ws_bytes = nf.value
    _lib.check(L.qsl_forward(S._h, ct.byref(a), None))
    b = _lib.BwdArgs()
    b.W, b.R, b.mode = 4, Rt.data_ptr(), 1
    b.Dinv[0], b.Dinv[1] = out["Dinv_up"].data_ptr(), out["Dinv_dn"].data_ptr()
    g = torch.ones((4, 2), dtype=torch.float64, device="cuda")
    dA = torch.zeros((4, sysm.n_basis), dtype=torch.float64, device="cuda")
    b.g_logdet, b.dA[0] = g.data_ptr(), dA.data_ptr()
    b.ws, b.ws_bytes = ws.data_ptr(), nf.value
    assert L.qsl_backward(S._h, ct.byref(b), None) == 4
    b.ws_bytes = nb.value
    _lib.check(L.qsl_backward(S._h, ct.byref(b), None))
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,W,radius", [("434e", 3, 10.0), ("1731e", 2, 12.0), ("158e", 4, 6.0)])
@pytest.mark.parametrize("mode", ["fp32", "fp64", "bf16x3"])
def test_forward_localized_mos(name, W, radius, mode):
    """Block-sparse MO coefficients (localised stand-ins): the FP32 products
    skip the MFMAs of MO blocks with no non-zero coefficient on a group's
    slots; every mode against the oracle on the same sparse A."""
    print(f"[case] localised MOs {name} W={W} radius={radius} mode={mode}", flush=True)
    sysm, A_up, A_dn, R = _cfg(name, W)
    A_up, A_dn = q.localize_mos(sysm, A_up, A_dn, radius)
    S = make_gpu_system(sysm, A_up, A_dn)
    gpu = run_gpu_forward(S, R, mode)
    compare_forward(sysm, A_up, A_dn, R, gpu, mode)
