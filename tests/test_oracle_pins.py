"""Pins of the FP64 oracle against mathematics (CPU only).

Each test checks the oracle against something other than itself: a
quadrature, a closed form, finite differences, LAPACK, an independent numpy
brute force, or an exact identity of determinants.
"""
import math

import numpy as np
import pytest

import oracle
from tests import bruteforce as bf
from tests.systems import make_tiny, random_tiny, walkers_near


# ---------------------------------------------------------------- AOs

def _ao_at(sysm, r):
    """Dense (5, N_b) screened AO block at one point from the oracle."""
    idx, B, _ = oracle.ao_eval(sysm, r)
    out = np.zeros((5, sysm.n_basis))
    out[:, idx] = B
    return out, idx


@pytest.mark.parametrize("l,comp", [(0, 0), (1, 0), (2, 0), (2, 1)])
def test_unit_norm_by_hermite_quadrature(l, comp):
    """<chi|chi> = 1 for one primitive, by tensor Gauss-Hermite quadrature
    (exact for the polynomial degree), screening disabled."""
    g = 0.7
    sysm = make_tiny([(0, l, [g], [0.4])], [[0.0, 0.0, 0.0]], 1, 0, T=1e300)
    t, w = np.polynomial.hermite.hermgauss(12)
    s = math.sqrt(2 * g)  # chi^2 ~ exp(-2 g r^2) = exp(-(s r)^2)
    total = 0.0
    for i in range(t.size):
        for j in range(t.size):
            for k in range(t.size):
                r = np.array([t[i], t[j], t[k]]) / s
                v, _ = _ao_at(sysm, r)
                total += w[i] * w[j] * w[k] * v[0, comp] ** 2 * math.exp(t[i] ** 2 + t[j] ** 2 + t[k] ** 2)
    assert abs(total / s ** 3 - 1.0) < 1e-12


@pytest.mark.parametrize("l", [0, 1, 2])
def test_contracted_norm_pairwise_quadrature(l):
    """Contracted shells: sum_km c_k c_m f^2 <P g_k|P g_m> = 1, each pair
    integrated by 1D Gauss-Hermite per axis with the oracle's weights."""
    ex = [0.3, 1.7, 9.0]
    sysm = make_tiny([(0, l, ex, [0.2, 0.5, 0.9])], [[0, 0, 0]], 1, 0)
    c = oracle.normalize(sysm)
    t, w = np.polynomial.hermite.hermgauss(10)
    for (a, b, cc) in bf.CART[l]:
        f = oracle.cart_factor(l, a, b, cc)
        tot = 0.0
        for k in range(3):
            for m in range(3):
                p = ex[k] + ex[m]
                ax = [np.sum(w * (t / math.sqrt(p)) ** (2 * n)) / math.sqrt(p) for n in (a, b, cc)]
                tot += c[k] * c[m] * f * f * ax[0] * ax[1] * ax[2]
        assert abs(tot - 1.0) < 1e-12


def test_s_primitive_closed_form():
    """One normalised s primitive: chi = (2g/pi)^(3/4) e^{-g r^2},
    grad chi = -2 g Delta chi, lap chi = (4 g^2 r^2 - 6 g) chi."""
    g = 1.3
    Q = np.array([0.2, -0.1, 0.5])
    sysm = make_tiny([(0, 0, [g], [0.37])], [Q], 1, 0)
    for r in ([0.1, 0.2, 0.3], [1.0, -0.5, 0.9], [0.2, -0.1, 0.5]):
        r = np.array(r)
        d = r - Q
        r2 = d @ d
        chi = (2 * g / math.pi) ** 0.75 * math.exp(-g * r2)
        v, _ = _ao_at(sysm, r)
        assert v[0, 0] == pytest.approx(chi, rel=1e-14)
        np.testing.assert_allclose(v[1:4, 0], -2 * g * d * chi, rtol=1e-13, atol=1e-300)
        assert v[4, 0] == pytest.approx((4 * g * g * r2 - 6 * g) * chi, rel=1e-13, abs=1e-14)


def test_golden_s_primitive_table():
    """Stored closed-form values (tests/golden/s_primitive_closed_form.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "s_primitive_closed_form.txt")
    rows = np.loadtxt(path)
    for g, x, y, z, chi, dx, lap in rows:
        sysm = make_tiny([(0, 0, [g], [1.0])], [[0, 0, 0]], 1, 0)
        v, _ = _ao_at(sysm, np.array([x, y, z]))
        assert v[0, 0] == pytest.approx(chi, rel=1e-13)
        assert v[1, 0] == pytest.approx(dx, rel=1e-12, abs=1e-300)
        assert v[4, 0] == pytest.approx(lap, rel=1e-12, abs=1e-14)


def test_ao_derivatives_finite_difference():
    sysm, _, _ = random_tiny(n_atoms=2, seed=3)
    sysm.screen_T = 1e300  # no screening jumps
    rng = np.random.default_rng(5)
    for _ in range(6):
        r = sysm.atom_xyz[rng.integers(0, 2)] + rng.normal(scale=0.7, size=3)
        v, _ = _ao_at(sysm, r)
        h = 1e-5
        for ax in range(3):
            dp = np.zeros(3); dp[ax] = h
            fd = (_ao_at(sysm, r + dp)[0][0] - _ao_at(sysm, r - dp)[0][0]) / (2 * h)
            np.testing.assert_allclose(v[1 + ax], fd, rtol=1e-6, atol=1e-8 * np.abs(v[0]).max())
        def lap_fd(h):
            acc = -6 * v[0]
            for ax in range(3):
                dp = np.zeros(3); dp[ax] = h
                acc = acc + _ao_at(sysm, r + dp)[0][0] + _ao_at(sysm, r - dp)[0][0]
            return acc / (h * h)
        lap = (4 * lap_fd(1e-3) - lap_fd(2e-3)) / 3  # Richardson
        np.testing.assert_allclose(v[4], lap, rtol=1e-6, atol=1e-7 * np.abs(v[4]).max())


def test_screening_matches_bruteforce():
    """Survivor set equals the brute-force rule over all shells and
    primitives; values agree with the independent numpy evaluation."""
    sysm, _, _ = random_tiny(n_atoms=3, seed=11)
    sysm.screen_T = 6.0  # make screening bite inside a small box
    rng = np.random.default_rng(2)
    pts = sysm.atom_xyz[rng.integers(0, 3, 40)] + rng.normal(scale=1.5, size=(40, 3))
    dense, alive = bf.ao_dense(sysm, pts, screen=True)
    for p in range(pts.shape[0]):
        v, idx = _ao_at(sysm, pts[p])
        assert np.array_equal(np.sort(idx), idx)
        assert np.array_equal(idx, np.nonzero(alive[p])[0])
        for n in range(5):
            np.testing.assert_allclose(v[n], dense[n, p], rtol=1e-12,
                                       atol=1e-14 * max(1.0, np.abs(dense[n, p]).max()))


def test_unscreened_difference_within_dropped_bound():
    sysm, A, _ = random_tiny(n_atoms=3, n_up=4, seed=4)
    sysm.screen_T = 4.0
    rng = np.random.default_rng(8)
    pts = sysm.atom_xyz[rng.integers(0, 3, 30)] + rng.normal(scale=1.2, size=(30, 3))
    full, _ = bf.ao_dense(sysm, pts, screen=False)
    bound = bf.dropped_bound(sysm, pts, A)
    for p in range(pts.shape[0]):
        v, _ = _ao_at(sysm, pts[p])
        for n in range(5):
            diff = np.abs(A @ v[n] - A @ full[n, p])
            assert np.all(diff <= bound[n, p] + 1e-13), (p, n, diff.max(), bound[n, p].max())


# --------------------------------------------------- products and MOs

def _two_s_system():
    """Two atoms with one s shell each: N_b = 2 = n_up = n_dn."""
    return make_tiny([(0, 0, [0.8, 2.0], [0.6, 0.3]), (1, 0, [0.5], [1.0])],
                     [[0, 0, 0], [1.4, 0.3, -0.2]], 2, 2)


def test_contraction_with_identity_is_scatter_of_B():
    sysm = _two_s_system()
    I = np.eye(2)
    R = walkers_near(sysm, 3, seed=2)
    out = oracle.forward(sysm, I, I, R)
    for w in range(3):
        for e in range(4):
            v, _ = _ao_at(sysm, R[w, e])
            C = out["C_up"] if e < 2 else out["C_dn"]
            np.testing.assert_array_equal(C[w, :, e % 2, :], v)


def test_permuting_the_basis_leaves_outputs_unchanged():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=3, seed=7)
    R = walkers_near(sysm, 4, seed=9)
    ref = oracle.forward(sysm, A_up, A_dn, R)
    # swap the atoms (atom-major AO order changes) and permute A's columns
    nsh = sysm.shell_l.shape[0] // 2
    order = list(range(nsh, 2 * nsh)) + list(range(nsh))
    off = np.concatenate([[0], np.cumsum(sysm.shell_nprim)])
    nao = (sysm.shell_l + 1) * (sysm.shell_l + 2) // 2
    aoff = np.concatenate([[0], np.cumsum(nao)])
    prim = np.concatenate([np.arange(off[s], off[s + 1]) for s in order])
    cols = np.concatenate([np.arange(aoff[s], aoff[s + 1]) for s in order])
    p = make_tiny([(1 - sysm.shell_atom[s], sysm.shell_l[s], sysm.prim_exp[off[s]:off[s + 1]],
                    sysm.prim_coef[off[s]:off[s + 1]]) for s in order],
                  sysm.atom_xyz[::-1], 3, 3)
    assert np.array_equal(p.prim_exp, sysm.prim_exp[prim])
    out = oracle.forward(p, A_up[:, cols], A_dn[:, cols], R)
    for k in ("C_up", "C_dn", "Dinv_up", "Dinv_dn", "logdet", "drift", "lap"):
        np.testing.assert_allclose(out[k], ref[k], rtol=1e-12, atol=1e-13 * np.abs(ref[k]).max())
    np.testing.assert_array_equal(out["sign"], ref["sign"])


def test_translation_invariance():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=12)
    R = walkers_near(sysm, 3, seed=1)
    ref = oracle.forward(sysm, A_up, A_dn, R)
    shift = np.array([3.25, -1.5, 0.75])
    sysm.atom_xyz = sysm.atom_xyz + shift
    out = oracle.forward(sysm, A_up, A_dn, R + shift)
    for k in ("C_up", "C_dn", "logdet", "drift", "lap"):
        np.testing.assert_allclose(out[k], ref[k], rtol=1e-9, atol=1e-11 * np.abs(ref[k]).max())


def test_mo_derivatives_finite_difference():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=21)
    sysm.screen_T = 1e300
    R = walkers_near(sysm, 1, seed=3)
    out = oracle.forward(sysm, A_up, A_dn, R)
    h = 1e-5
    for e in range(5):
        sp, el = ("C_up", e) if e < 3 else ("C_dn", e - 3)
        for ax in range(3):
            Rp = R.copy(); Rp[0, e, ax] += h
            Rm = R.copy(); Rm[0, e, ax] -= h
            fd = (oracle.forward(sysm, A_up, A_dn, Rp)[sp][0, 0, el] -
                  oracle.forward(sysm, A_up, A_dn, Rm)[sp][0, 0, el]) / (2 * h)
            np.testing.assert_allclose(out[sp][0, 1 + ax, el], fd, rtol=1e-6, atol=1e-9)
        def lap_fd(hh):
            acc = -6 * out[sp][0, 0, el]
            for ax in range(3):
                for sgn in (1, -1):
                    Rq = R.copy(); Rq[0, e, ax] += sgn * hh
                    acc = acc + oracle.forward(sysm, A_up, A_dn, Rq)[sp][0, 0, el]
            return acc / hh ** 2
        lap = (4 * lap_fd(1e-3) - lap_fd(2e-3)) / 3  # Richardson
        np.testing.assert_allclose(out[sp][0, 4, el], lap, rtol=1e-6, atol=1e-7)


# ------------------------------------------------ determinant and inverse

def test_logdet_inverse_vs_lapack():
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=5, n_dn=4, seed=31)
    R = walkers_near(sysm, 6, seed=4)
    out = oracle.forward(sysm, A_up, A_dn, R)
    for w in range(6):
        for s, (C, Di) in enumerate([("C_up", "Dinv_up"), ("C_dn", "Dinv_dn")]):
            D = out[C][w, 0].T
            sg, ld = np.linalg.slogdet(D)
            assert out["sign"][w, s] == int(sg)
            assert out["logdet"][w, s] == pytest.approx(ld, rel=1e-12, abs=1e-12)
            np.testing.assert_allclose(out[Di][w], np.linalg.inv(D), rtol=1e-9,
                                       atol=1e-11 * np.abs(np.linalg.inv(D)).max())
            np.testing.assert_allclose(out[Di][w] @ D, np.eye(D.shape[0]), atol=1e-10)


def test_lu_random_matrices_vs_lapack():
    rng = np.random.default_rng(0)
    for n in (1, 2, 7, 33):
        M = rng.normal(size=(n, n))
        ok, ld, sg, inv = oracle.lu_inverse(M)
        s2, l2 = np.linalg.slogdet(M)
        assert ok and sg == int(s2) and ld == pytest.approx(l2, rel=1e-12, abs=1e-12)
        np.testing.assert_allclose(inv, np.linalg.inv(M), rtol=1e-9, atol=1e-10)


def test_one_electron_per_spin():
    """1x1 Slater matrices: logdet = ln|phi_1(r)|, Dinv = 1/phi_1."""
    sysm, A_up, A_dn = random_tiny(n_atoms=1, n_up=1, n_dn=1, seed=5)
    R = walkers_near(sysm, 4, seed=6)
    out = oracle.forward(sysm, A_up, A_dn, R)
    for w in range(4):
        for s, A in enumerate((A_up, A_dn)):
            v, _ = _ao_at(sysm, R[w, s])
            phi = float(A[0] @ v[0])
            assert out["logdet"][w, s] == pytest.approx(math.log(abs(phi)), rel=1e-13)
            assert out["sign"][w, s] == (1 if phi > 0 else -1)
            Di = out["Dinv_up" if s == 0 else "Dinv_dn"][w, 0, 0]
            assert Di == pytest.approx(1.0 / phi, rel=1e-13)


def test_antisymmetry_and_row_scaling():
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=41)
    R = walkers_near(sysm, 2, seed=7)
    ref = oracle.forward(sysm, A_up, A_dn, R)
    # swap two up electrons
    R2 = R.copy(); R2[:, [0, 2]] = R2[:, [2, 0]]
    out = oracle.forward(sysm, A_up, A_dn, R2)
    np.testing.assert_array_equal(out["sign"][:, 0], -ref["sign"][:, 0])
    np.testing.assert_allclose(out["logdet"], ref["logdet"], rtol=1e-12)
    np.testing.assert_allclose(out["Dinv_up"][:, [2, 0]], ref["Dinv_up"][:, [0, 2]], rtol=1e-8, atol=1e-10)
    # swap two MO rows of A_dn
    A3 = A_dn.copy(); A3[[0, 1]] = A3[[1, 0]]
    out = oracle.forward(sysm, A_up, A3, R)
    np.testing.assert_array_equal(out["sign"][:, 1], -ref["sign"][:, 1])
    # scale one MO row
    A4 = A_up.copy(); A4[2] *= -2.5
    out = oracle.forward(sysm, A4, A_dn, R)
    np.testing.assert_allclose(out["logdet"][:, 0], ref["logdet"][:, 0] + math.log(2.5), rtol=1e-12)
    np.testing.assert_array_equal(out["sign"][:, 0], -ref["sign"][:, 0])


def test_electron_beyond_every_radius_is_singular():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=51)
    R = walkers_near(sysm, 2, seed=8)
    R[1, 1] = np.array([500.0, 500.0, 500.0])
    out = oracle.forward(sysm, A_up, A_dn, R)
    assert out["logdet"][1, 0] == -np.inf and out["sign"][1, 0] == 0
    assert out["status"][1] & 1
    assert np.all(out["C_up"][1, :, 1, :] == 0.0)
    assert np.isfinite(out["logdet"][0]).all() and out["status"][0] == 0


# ------------------------------------------------------- drift, Laplacian

def _logdet_spin(sysm, A_up, A_dn, R, s):
    return oracle.forward(sysm, A_up, A_dn, R)["logdet"][0, s]


def test_drift_and_laplacian_finite_difference():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=61)
    sysm.screen_T = 1e300
    R = walkers_near(sysm, 1, seed=9)
    out = oracle.forward(sysm, A_up, A_dn, R)
    for e in range(5):
        s = 0 if e < 3 else 1
        h = 1e-5
        grad = np.zeros(3)
        for ax in range(3):
            Rp = R.copy(); Rp[0, e, ax] += h
            Rm = R.copy(); Rm[0, e, ax] -= h
            grad[ax] = (_logdet_spin(sysm, A_up, A_dn, Rp, s) - _logdet_spin(sysm, A_up, A_dn, Rm, s)) / (2 * h)
        np.testing.assert_allclose(out["drift"][0, e], grad, rtol=1e-6, atol=1e-7)
        l0 = _logdet_spin(sysm, A_up, A_dn, R, s)

        def lap_fd(hh):
            acc = -6 * l0
            for ax in range(3):
                for sg in (1, -1):
                    Rq = R.copy(); Rq[0, e, ax] += sg * hh
                    acc += _logdet_spin(sysm, A_up, A_dn, Rq, s)
            return acc / (hh * hh)
        lap_log = (4 * lap_fd(1e-3) - lap_fd(2e-3)) / 3  # Richardson
        # lap Det / Det = lap log|Det| + |grad log|Det||^2
        assert out["lap"][0, e] == pytest.approx(lap_log + grad @ grad, rel=1e-5, abs=1e-5)


# ------------------------------------------------------------- adjoint

def test_adjoint_identities():
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=71)
    R = walkers_near(sysm, 5, seed=10)
    out = oracle.forward(sysm, A_up, A_dn, R)
    g = np.random.default_rng(1).normal(size=(5, 2))
    dR, dAu, dAd = oracle.backward(sysm, A_up, A_dn, R, out["Dinv_up"], out["Dinv_dn"], g)
    # dA A^T = (sum_w g_w) I
    np.testing.assert_allclose(dAu @ A_up.T, g[:, 0].sum() * np.eye(4), atol=1e-10)
    np.testing.assert_allclose(dAd @ A_dn.T, g[:, 1].sum() * np.eye(3), atol=1e-10)
    # dR through the adjoint route equals g times the Jacobi drift
    gg = np.concatenate([np.repeat(g[:, :1], 4, 1), np.repeat(g[:, 1:], 3, 1)], 1)
    np.testing.assert_allclose(dR, gg[:, :, None] * out["drift"], rtol=1e-9, atol=1e-11)


def test_adjoint_finite_difference():
    sysm, A_up, A_dn = random_tiny(n_atoms=2, n_up=3, n_dn=2, seed=81)
    sysm.screen_T = 1e300
    R = walkers_near(sysm, 3, seed=11)
    g = np.random.default_rng(2).normal(size=(3, 2))
    out = oracle.forward(sysm, A_up, A_dn, R)
    dR, dAu, dAd = oracle.backward(sysm, A_up, A_dn, R, out["Dinv_up"], out["Dinv_dn"], g)

    def L(Au, Ad, RR):
        return float((oracle.forward(sysm, Au, Ad, RR)["logdet"] * g).sum())

    h = 1e-6
    for (i, j) in [(0, 0), (1, 5), (2, 11)]:
        Ap = A_up.copy(); Ap[i, j] += h
        Am = A_up.copy(); Am[i, j] -= h
        assert dAu[i, j] == pytest.approx((L(Ap, A_dn, R) - L(Am, A_dn, R)) / (2 * h), rel=1e-5, abs=1e-7)
        Ap = A_dn.copy(); Ap[i % 2, j] += h
        Am = A_dn.copy(); Am[i % 2, j] -= h
        assert dAd[i % 2, j] == pytest.approx((L(A_up, Ap, R) - L(A_up, Am, R)) / (2 * h), rel=1e-5, abs=1e-7)
    for (w, e, ax) in [(0, 0, 0), (1, 3, 2), (2, 4, 1)]:
        Rp = R.copy(); Rp[w, e, ax] += h
        Rm = R.copy(); Rm[w, e, ax] -= h
        assert dR[w, e, ax] == pytest.approx((L(A_up, A_dn, Rp) - L(A_up, A_dn, Rm)) / (2 * h), rel=1e-5, abs=1e-7)


def test_adjoint_absolute_sums():
    """The absolute-value sums that scale the adjoint's error bounds: they
    dominate |dA| and |dR| term by term, scale with |g|, and equal dA exactly
    when every term is non-negative (s shells only, so chi > 0, with A >= 0,
    D^-1 >= 0 and g >= 0 passed in)."""
    sysm, A_up, A_dn = random_tiny(n_atoms=3, n_up=4, n_dn=3, seed=73)
    R = walkers_near(sysm, 4, seed=12)
    out = oracle.forward(sysm, A_up, A_dn, R)
    g = np.random.default_rng(5).normal(size=(4, 2))
    dR, dAu, dAd, (bR, bAu, bAd) = oracle.backward(sysm, A_up, A_dn, R, out["Dinv_up"], out["Dinv_dn"], g,
                                                    want_abs=True)
    assert np.all(bAu >= np.abs(dAu)) and np.all(bAd >= np.abs(dAd)) and np.all(bR >= np.abs(dR))
    assert bAu.max() > 0 and bR.max() > 0
    _, _, _, (bR2, bAu2, _) = oracle.backward(sysm, A_up, A_dn, R, out["Dinv_up"], out["Dinv_dn"], -2.0 * g,
                                              want_abs=True)
    np.testing.assert_allclose(bAu2, 2.0 * bAu, rtol=1e-14)
    np.testing.assert_allclose(bR2, 2.0 * bR, rtol=1e-14)
    # every term non-negative: the absolute sums are the sums themselves
    rng = np.random.default_rng(6)
    atoms = rng.normal(scale=1.0, size=(2, 3))
    shells = [(a, 0, np.exp(rng.uniform(np.log(0.3), np.log(3.0), 2)), rng.uniform(0.2, 1.0, 2))
              for a in range(2) for _ in range(3)]
    sp = make_tiny(shells, atoms, 3, 2)
    nb = sp.n_basis
    Au, Ad = rng.uniform(0.1, 1.0, size=(3, nb)), rng.uniform(0.1, 1.0, size=(2, nb))
    Rs = walkers_near(sp, 3, seed=13)
    Du, Dd = rng.uniform(0.1, 1.0, size=(3, 3, 3)), rng.uniform(0.1, 1.0, size=(3, 2, 2))
    gp = rng.uniform(0.5, 2.0, size=(3, 2))
    _, eAu, eAd, (_, fAu, fAd) = oracle.backward(sp, Au, Ad, Rs, Du, Dd, gp, want_abs=True)
    assert np.array_equal(eAu, fAu) and np.array_equal(eAd, fAd)


# ----------------------------------------------- synthetic workload shape

def test_synthetic_survivor_statistics_plausible():
    """Survivors per electron are ~10^2 and do not grow with system size,
    as the paper's Table 1 reports for real molecules (plausibility)."""
    import qsl_synth as q
    means = []
    for name in ("158e", "434e", "1731e"):
        sysm, _, _, R = q.make_config(name, W=1)
        sel = R[0][:: max(1, R.shape[1] // 150)]
        cnt = [oracle.ao_eval(sysm, r)[0].size for r in sel]
        means.append(np.mean(cnt))
    assert all(60 < m < 400 for m in means)
    assert max(means) < 2.0 * min(means)
