"""Pins of the oracle's Monte Carlo step (CPU only): the Jastrow factor, the
local energy, the drift-diffusion move, the branching weight and the
reconfiguration, each against something other than itself: closed forms
derived by hand for one- and two-electron atoms, finite differences of
log|Psi|, the cusp conditions, and properties of the selection.
"""
import math

import numpy as np
import pytest

import oracle
from tests.systems import make_tiny, random_tiny, walkers_near


def _one_center(n_up, n_dn, gamma):
    """One nucleus at the origin, one s primitive of exponent gamma; every MO
    is that AO (screening off)."""
    sysm = make_tiny([(0, 0, [gamma], [1.0])], [[0.0, 0.0, 0.0]], n_up, n_dn, T=1e300)
    return sysm, np.ones((n_up, 1)), np.ones((n_dn, 1))


def _EL(sysm, A_up, A_dn, R, Z, **jp):
    out = oracle.forward(sysm, A_up, A_dn, R)
    J, gJ, lJ, V = oracle.jastrow_potential(sysm, Z, R, **jp)
    EL, b = oracle.local_energy(out["drift"], out["lap"], gJ, lJ, V)
    return EL, b, out, J, V


def test_hydrogen_like_closed_form():
    """Psi = e^{-r} e^{-gamma r^2} for one electron and a unit charge
    (electron-nucleus Jastrow u = -r, b = 0):
    E_L = 3 gamma - 1/2 - 2 gamma r - 2 gamma^2 r^2 (the 1/r terms cancel);
    without the Jastrow, E_L = 3 gamma - 2 gamma^2 r^2 - 1/r."""
    g = 0.37
    sysm, Au, Ad = _one_center(1, 0, g)
    R = np.array([[[0.3, -0.7, 0.45]], [[1.9, 0.2, -0.6]], [[-0.05, 0.02, 0.11]]])
    r = np.linalg.norm(R[:, 0], axis=1)
    EL, b, _, _, _ = _EL(sysm, Au, Ad, R, [1.0], c_ee=0.0, c_en=1.0, b_en=0.0)
    np.testing.assert_allclose(EL, 3 * g - 0.5 - 2 * g * r - 2 * g * g * r * r, rtol=1e-12, atol=1e-12)
    # drift: grad ln Psi = -(1 + 2 gamma r) r_hat
    np.testing.assert_allclose(b[:, 0], -(1 + 2 * g * r)[:, None] * R[:, 0] / r[:, None], rtol=1e-12, atol=1e-13)
    EL0, _, _, _, _ = _EL(sysm, Au, Ad, R, [1.0], c_ee=0.0, c_en=0.0)
    np.testing.assert_allclose(EL0, 3 * g - 2 * g * g * r * r - 1 / r, rtol=1e-12, atol=1e-12)


def test_helium_like_closed_form_with_electron_repulsion():
    """Two electrons of opposite spin on a nucleus of charge Z, each in the
    same Gaussian, electron-nucleus Jastrow u = -Z r (b = 0), no
    electron-electron Jastrow:
    E_L = sum_i (3 gamma - Z^2/2 - 2 Z gamma r_i - 2 gamma^2 r_i^2) + 1/r_12."""
    g, Z = 0.8, 2.0
    sysm, Au, Ad = _one_center(1, 1, g)
    rng = np.random.default_rng(3)
    R = rng.normal(scale=0.7, size=(5, 2, 3))
    r = np.linalg.norm(R, axis=2)
    r12 = np.linalg.norm(R[:, 0] - R[:, 1], axis=1)
    EL, _, _, _, V = _EL(sysm, Au, Ad, R, [Z], c_ee=0.0, c_en=1.0, b_en=0.0)
    want = (3 * g - Z * Z / 2 - 2 * Z * g * r - 2 * g * g * r * r).sum(1) + 1 / r12
    np.testing.assert_allclose(EL, want, rtol=1e-12, atol=1e-12)


def _log_psi(sysm, A_up, A_dn, R, Z, **jp):
    out = oracle.forward(sysm, A_up, A_dn, R)
    J, _, _, _ = oracle.jastrow_potential(sysm, Z, R, **jp)
    return J + out["logdet"].sum(1)


def test_local_energy_against_finite_differences_of_log_psi():
    """On a random system with every term switched on: the drift equals the
    central-difference gradient of log|Psi| and E_L equals
    -1/2 (lap log|Psi| + |grad log|Psi||^2) + V by central differences."""
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=17)
    sysm.screen_T = 1e300
    Z = np.array([2.0, 3.0])
    jp = dict(c_ee=1.0, b_ee=0.8, c_en=1.0, b_en=1.3)
    R = walkers_near(sysm, 2, seed=4)
    EL, b, _, _, V = _EL(sysm, A_up, A_dn, R, Z, **jp)
    h = 1e-4
    for w in range(R.shape[0]):
        lap = 0.0
        grad2 = 0.0
        l0 = _log_psi(sysm, A_up, A_dn, R[w:w + 1], Z, **jp)[0]
        for e in range(R.shape[1]):
            for ax in range(3):
                Rp = R[w:w + 1].copy(); Rp[0, e, ax] += h
                Rm = R[w:w + 1].copy(); Rm[0, e, ax] -= h
                lp = _log_psi(sysm, A_up, A_dn, Rp, Z, **jp)[0]
                lm = _log_psi(sysm, A_up, A_dn, Rm, Z, **jp)[0]
                gr = (lp - lm) / (2 * h)
                assert b[w, e, ax] == pytest.approx(gr, rel=1e-6, abs=1e-7)
                lap += (lp - 2 * l0 + lm) / (h * h)
                grad2 += gr * gr
        assert EL[w] == pytest.approx(-0.5 * (lap + grad2) + V[w], rel=1e-5, abs=1e-5)


def test_jastrow_cusp_conditions():
    """du/dr at coalescence: 1/2 for opposite spins, 1/4 for the same spin,
    -Z at a nucleus (slopes of J by central differences at small r)."""
    h = 1e-7
    for n_up, n_dn, want in [(1, 1, 0.5), (2, 0, 0.25)]:
        sysm = make_tiny([(0, 0, [1.0], [1.0])], [[0.0, 0.0, 0.0]], n_up, n_dn, T=1e300)

        def J(r):
            R = np.array([[[5.0, 0.0, 0.0], [5.0 + r, 0.0, 0.0]]])
            return oracle.jastrow_potential(sysm, [0.0], R, c_ee=1.0, b_ee=1.2, c_en=0.0)[0][0]
        slope = (J(2e-6 + h) - J(2e-6 - h)) / (2 * h)
        assert slope == pytest.approx(want, rel=1e-4)
    sysm = make_tiny([(0, 0, [1.0], [1.0])], [[0.0, 0.0, 0.0]], 1, 0, T=1e300)

    def Jn(r):
        return oracle.jastrow_potential(sysm, [3.0], np.array([[[r, 0.0, 0.0]]]), c_en=1.0, b_en=0.9)[0][0]
    assert (Jn(2e-6 + h) - Jn(2e-6 - h)) / (2 * h) == pytest.approx(-3.0, rel=1e-4)


def test_jastrow_gradient_laplacian_finite_differences_and_invariance():
    sysm, _, _ = random_tiny(n_atoms=3, n_up=3, n_dn=3, seed=19)
    Z = np.array([1.0, 4.0, 2.0])
    jp = dict(c_ee=1.0, b_ee=0.6, c_en=1.0, b_en=1.1)
    R = walkers_near(sysm, 2, seed=9)
    J, gJ, lJ, V = oracle.jastrow_potential(sysm, Z, R, **jp)
    h = 1e-4
    for w in range(2):
        for e in range(6):
            lap = 0.0
            for ax in range(3):
                Rp = R.copy(); Rp[w, e, ax] += h
                Rm = R.copy(); Rm[w, e, ax] -= h
                jpv = oracle.jastrow_potential(sysm, Z, Rp, **jp)[0][w]
                jmv = oracle.jastrow_potential(sysm, Z, Rm, **jp)[0][w]
                assert gJ[w, e, ax] == pytest.approx((jpv - jmv) / (2 * h), rel=1e-6, abs=1e-8)
                lap += (jpv - 2 * J[w] + jmv) / (h * h)
            assert lJ[w, e] == pytest.approx(lap, rel=1e-4, abs=1e-5)
    # exchanging two electrons of one spin changes neither J nor V
    Rs = R.copy()
    Rs[:, [0, 2]] = Rs[:, [2, 0]]
    J2, _, _, V2 = oracle.jastrow_potential(sysm, Z, Rs, **jp)
    np.testing.assert_allclose(J2, J, rtol=1e-13)
    np.testing.assert_allclose(V2, V, rtol=1e-13)


def test_drift_diffusion_special_cases():
    rng = np.random.default_rng(1)
    R, b, eta = rng.normal(size=(3, 4, 3)), rng.normal(size=(3, 4, 3)), rng.normal(size=(3, 4, 3))
    tau = 0.0625  # sqrt(tau) = 1/4 exactly
    np.testing.assert_array_equal(oracle.drift_diffuse(R, b, np.zeros_like(eta), tau), R + tau * b)
    np.testing.assert_array_equal(oracle.drift_diffuse(R, np.zeros_like(b), eta, tau), R + 0.25 * eta)
    np.testing.assert_array_equal(oracle.drift_diffuse(R, b, eta, 0.0), R)


def test_branch_weight_values():
    EL_new, EL_old = np.array([1.0, -2.0, 0.5, 3.0, 0.0]), np.array([1.0, 3.0, 0.5, 3.0, 0.0])
    s_new = np.array([1, -1, 1, -1, 0], np.int8)
    s_old = np.array([1, -1, -1, -1, 1], np.int8)
    tau = 2 * math.log(2.0)
    w = oracle.branch_weights(EL_new, EL_old, s_new, s_old, E_T=0.5, tau=tau)
    # (1 - .5) + (1 - .5) = 1 -> 1/2; (-2.5) + 2.5 = 0 -> 1; node crossed -> 0;
    # (2.5 + 2.5) -> 2^-5; Psi vanishes -> 0
    np.testing.assert_allclose(w, [0.5, 1.0, 0.0, 2.0 ** -5, 0.0], rtol=1e-15)
    # a non-finite local energy, or a weight past the double range, drops the walker
    w = oracle.branch_weights(np.array([np.nan, np.inf, -1e6, 1.0]), np.array([1.0, 1.0, -1e6, 1.0]),
                              np.ones(4, np.int8), np.ones(4, np.int8), E_T=0.0, tau=1.0)
    np.testing.assert_array_equal(w, [0.0, 0.0, 0.0, math.exp(-1.0)])


def test_reconfiguration_properties():
    W = 64
    # equal weights and stratified uniforms: every walker drawn once
    idx, s = oracle.reconfigure(np.full(W, 0.25), (np.arange(W) + 0.5) / W)
    np.testing.assert_array_equal(idx, np.arange(W))
    assert s == pytest.approx(0.25 * W)
    # a single non-zero weight takes every draw; zero weights are never drawn
    w = np.zeros(W)
    w[17] = 3.0
    u = np.random.default_rng(2).random(W)
    np.testing.assert_array_equal(oracle.reconfigure(w, u)[0], np.full(W, 17))
    w = np.random.default_rng(3).random(W)
    w[::3] = 0.0
    idx, _ = oracle.reconfigure(w, np.random.default_rng(4).random(W))
    assert np.all(w[idx] > 0)
    # u just below 1 still selects the last walker with weight
    idx, _ = oracle.reconfigure(np.ones(4), np.array([1.0 - 2.0 ** -53] * 4))
    np.testing.assert_array_equal(idx, [3, 3, 3, 3])
    # a zero total keeps the population
    np.testing.assert_array_equal(oracle.reconfigure(np.zeros(5), np.full(5, 0.3))[0], np.arange(5))


def test_reconfiguration_draws_follow_the_weights():
    """Over many independent draws the counts follow p_k = w_k / sum w
    (chi-square, seeded; the 0.999 quantile for 7 degrees of freedom is
    24.3)."""
    w = np.array([1.0, 2.0, 0.5, 4.0, 0.0, 1.5, 3.0, 2.0, 1.0])
    p = w / w.sum()
    rng = np.random.default_rng(12)
    counts = np.zeros(w.size)
    for _ in range(4000):
        idx, _ = oracle.reconfigure(w, rng.random(w.size))
        counts += np.bincount(idx, minlength=w.size)
    n = counts.sum()
    keep = p > 0
    chi2 = (((counts - n * p) ** 2)[keep] / (n * p[keep])).sum()
    assert counts[4] == 0 and chi2 < 24.3
