"""Pins of the oracle's several-determinant wavefunction (CPU only): a
single determinant reproduces the one-determinant forward, equal
determinants add their coefficients, opposite ones cancel, a numpy brute
force (dense AO values, numpy determinants) gives Psi, finite differences of
that brute force give the drift and the Laplacian ratio, and exchanging two
electrons of one spin flips the sign."""
import numpy as np
import pytest

import oracle
from tests import bruteforce as bf
from tests.systems import random_tiny, walkers_near


def _setup(seed=5, n_up=3, n_dn=2, extra=3, W=3):
    sysm, _, _ = random_tiny(n_atoms=3, n_up=n_up, n_dn=n_dn, seed=seed)
    sysm.screen_T = 1e300
    rng = np.random.default_rng(seed)
    nb = sysm.n_basis
    Au = rng.normal(size=(n_up + extra, nb)) / np.sqrt(nb)
    Ad = rng.normal(size=(n_dn + extra, nb)) / np.sqrt(nb)
    R = walkers_near(sysm, W, seed=seed + 1)
    return sysm, Au, Ad, R


OCC = np.array([[0, 1, 2, 0, 1],      # ground state
                [0, 1, 3, 0, 1],      # single up excitation
                [0, 1, 2, 2, 4],      # single down excitation (orbital 1 -> 4, reordered)
                [4, 1, 3, 0, 3]])     # double excitation
COEF = np.array([0.9, -0.3, 0.25, 0.1])


def _brute_psi(sysm, Au, Ad, occ, coef, R):
    """sum_K c_K det(phi_i(r_e)) det(...) from dense AO values (numpy)."""
    nu, nd = sysm.n_up, sysm.n_dn
    out = np.zeros(R.shape[0])
    for w in range(R.shape[0]):
        B, _ = bf.ao_dense(sysm, R[w], screen=False)
        phi_u = B[0][:nu] @ Au.T   # [e][orbital]
        phi_d = B[0][nu:] @ Ad.T
        for K in range(occ.shape[0]):
            Du = phi_u[:, occ[K, :nu]] if nu else np.ones((0, 0))
            Dd = phi_d[:, occ[K, nu:]] if nd else np.ones((0, 0))
            out[w] += coef[K] * np.linalg.det(Du) * np.linalg.det(Dd)
    return out


def test_single_determinant_is_the_forward():
    sysm, Au, Ad, R = _setup()
    md = oracle.multidet(sysm, Au, Ad, OCC[:1], [1.0], R)
    ref = oracle.forward(sysm, Au[[0, 1, 2]], Ad[[0, 1]], R)
    np.testing.assert_allclose(md["logpsi"], ref["logdet"].sum(1), rtol=1e-13)
    np.testing.assert_array_equal(md["sign"], ref["sign"].prod(1))
    np.testing.assert_allclose(md["drift"], ref["drift"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(md["lap"], ref["lap"], rtol=1e-12, atol=1e-13)


def test_equal_determinants_add_and_opposite_ones_cancel():
    sysm, Au, Ad, R = _setup()
    one = oracle.multidet(sysm, Au, Ad, OCC[:1], [1.0], R)
    two = oracle.multidet(sysm, Au, Ad, np.repeat(OCC[:1], 2, 0), [0.3, 0.5], R)
    np.testing.assert_allclose(two["logpsi"], one["logpsi"] + np.log(0.8), rtol=1e-13)
    np.testing.assert_allclose(two["drift"], one["drift"], rtol=1e-12, atol=1e-13)
    zero = oracle.multidet(sysm, Au, Ad, np.repeat(OCC[:1], 2, 0), [1.0, -1.0], R)
    assert np.all(zero["sign"] == 0) and np.all(np.isneginf(zero["logpsi"]))


def test_against_numpy_brute_force_and_finite_differences():
    sysm, Au, Ad, R = _setup(W=2)
    md = oracle.multidet(sysm, Au, Ad, OCC, COEF, R)
    psi = _brute_psi(sysm, Au, Ad, OCC, COEF, R)
    np.testing.assert_allclose(md["logpsi"], np.log(np.abs(psi)), rtol=1e-11)
    np.testing.assert_array_equal(md["sign"], np.sign(psi).astype(np.int8))
    h = 1e-4
    for w in range(R.shape[0]):
        l0 = np.log(abs(psi[w]))
        for e in range(R.shape[1]):
            lap = 0.0
            g2 = 0.0
            for ax in range(3):
                Rp = R[w:w + 1].copy(); Rp[0, e, ax] += h
                Rm = R[w:w + 1].copy(); Rm[0, e, ax] -= h
                lp = np.log(abs(_brute_psi(sysm, Au, Ad, OCC, COEF, Rp)[0]))
                lm = np.log(abs(_brute_psi(sysm, Au, Ad, OCC, COEF, Rm)[0]))
                gr = (lp - lm) / (2 * h)
                assert md["drift"][w, e, ax] == pytest.approx(gr, rel=1e-6, abs=1e-7)
                lap += (lp - 2 * l0 + lm) / (h * h)
                g2 += gr * gr
            assert md["lap"][w, e] == pytest.approx(lap + g2, rel=1e-4, abs=1e-4)


def test_exchange_of_two_electrons_flips_the_sign():
    sysm, Au, Ad, R = _setup()
    md = oracle.multidet(sysm, Au, Ad, OCC, COEF, R)
    Rs = R.copy()
    Rs[:, [0, 2]] = Rs[:, [2, 0]]
    sw = oracle.multidet(sysm, Au, Ad, OCC, COEF, Rs)
    np.testing.assert_allclose(sw["logpsi"], md["logpsi"], rtol=1e-12)
    np.testing.assert_array_equal(sw["sign"], -md["sign"])
