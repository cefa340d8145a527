"""Independent numpy brute force for tiny inputs (test helper).

Written separately from the C oracle and from the GPU library: the AO
derivatives use the plain product rule on P(r) g(r) (no homogeneity
shortcut), normalisation is done numerically from the primitive overlap
formula, and screening is optional.
"""
from __future__ import annotations

import math

import numpy as np

CART = {0: [(0, 0, 0)],
        1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
        2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]}


def _df(m):  # (2m-1)!!
    return float(np.prod(np.arange(2 * m - 1, 0, -2))) if m > 0 else 1.0


def _prim_norm_xyz(g, a, b, c):
    # 1 / sqrt( int x^2a y^2b z^2c exp(-2 g r^2) )
    l = a + b + c
    integ = _df(a) * _df(b) * _df(c) / (4 * g) ** l * (math.pi / (2 * g)) ** 1.5
    return 1.0 / math.sqrt(integ)


def basis_table(sys):
    """List of AOs: (atom, shell, (a,b,c), exps, normalised coefs)."""
    aos = []
    off = 0
    for sh in range(sys.shell_l.shape[0]):
        l = int(sys.shell_l[sh])
        npr = int(sys.shell_nprim[sh])
        ex = sys.prim_exp[off:off + npr]
        d = sys.prim_coef[off:off + npr]
        off += npr
        for (a, b, c) in CART[l]:
            # numerically normalised contracted function for this component
            nk = np.array([_prim_norm_xyz(g, a, b, c) for g in ex])
            S = 0.0
            for k in range(npr):
                for m in range(npr):
                    p = ex[k] + ex[m]
                    ov = _df(a) * _df(b) * _df(c) / (2 * p) ** (a + b + c) * (math.pi / p) ** 1.5
                    S += d[k] * d[m] * nk[k] * nk[m] * ov
            aos.append((int(sys.shell_atom[sh]), sh, (a, b, c), ex.copy(), d * nk / math.sqrt(S)))
    return aos


def _pw(x, n):
    return x ** n if n >= 0 else np.zeros_like(x)


def ao_dense(sys, pts, screen=True):
    """Dense AO values [5, n_pts, N_b] (value, dx, dy, dz, lap) and a mask of
    which AOs survive.  When screen is False every primitive is kept."""
    pts = np.atleast_2d(pts)
    aos = basis_table(sys)
    T = sys.screen_T
    out = np.zeros((5, pts.shape[0], len(aos)))
    alive = np.zeros((pts.shape[0], len(aos)), bool)
    for j, (at, sh, (a, b, c), ex, co) in enumerate(aos):
        d = pts - sys.atom_xyz[at][None, :]
        dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
        r2 = (dx * dx + dy * dy) + dz * dz
        g = np.zeros(pts.shape[0])
        gx = np.zeros(pts.shape[0]); gy = np.zeros_like(gx); gz = np.zeros_like(gx)
        gxx = np.zeros_like(gx); gyy = np.zeros_like(gx); gzz = np.zeros_like(gx)
        for k in range(ex.shape[0]):
            keep = (ex[k] * r2 <= T) if screen else np.ones_like(r2, bool)
            alive[:, j] |= keep
            e = np.where(keep, co[k] * np.exp(-ex[k] * r2), 0.0)
            g += e
            # partial derivatives of exp(-gamma r^2)
            gx += -2 * ex[k] * dx * e; gy += -2 * ex[k] * dy * e; gz += -2 * ex[k] * dz * e
            gxx += (4 * ex[k] ** 2 * dx * dx - 2 * ex[k]) * e
            gyy += (4 * ex[k] ** 2 * dy * dy - 2 * ex[k]) * e
            gzz += (4 * ex[k] ** 2 * dz * dz - 2 * ex[k]) * e
        P = _pw(dx, a) * _pw(dy, b) * _pw(dz, c)
        Px = a * _pw(dx, a - 1) * _pw(dy, b) * _pw(dz, c)
        Py = b * _pw(dx, a) * _pw(dy, b - 1) * _pw(dz, c)
        Pz = c * _pw(dx, a) * _pw(dy, b) * _pw(dz, c - 1)
        Pxx = a * (a - 1) * _pw(dx, a - 2) * _pw(dy, b) * _pw(dz, c)
        Pyy = b * (b - 1) * _pw(dx, a) * _pw(dy, b - 2) * _pw(dz, c)
        Pzz = c * (c - 1) * _pw(dx, a) * _pw(dy, b) * _pw(dz, c - 2)
        out[0, :, j] = P * g
        out[1, :, j] = Px * g + P * gx
        out[2, :, j] = Py * g + P * gy
        out[3, :, j] = Pz * g + P * gz
        out[4, :, j] = (Pxx + Pyy + Pzz) * g + 2 * (Px * gx + Py * gy + Pz * gz) + P * (gxx + gyy + gzz)
    return out, alive


def dropped_bound(sys, pts, A):
    """Upper bound on |C_unscreened - C_screened| per (point, MO, n): the sum
    over dropped primitives of |A| times a bound on |primitive term|."""
    pts = np.atleast_2d(pts)
    aos = basis_table(sys)
    T = sys.screen_T
    bnd = np.zeros((5, pts.shape[0], A.shape[0]))
    for j, (at, sh, (a, b, c), ex, co) in enumerate(aos):
        d = pts - sys.atom_xyz[at][None, :]
        r2 = (d[:, 0] ** 2 + d[:, 1] ** 2) + d[:, 2] ** 2
        r = np.sqrt(r2)
        l = a + b + c
        for k in range(ex.shape[0]):
            drop = ex[k] * r2 > T
            e = np.where(drop, abs(co[k]) * np.exp(-ex[k] * r2), 0.0)
            rl = np.maximum(r, 1.0) ** (l + 2)
            # |P| <= r^l, |dP| <= l r^(l-1), |lap P| <= l(l-1) r^(l-2); gamma factors
            fac = [rl, rl * (l + 2 * ex[k] * (1 + r2)),
                   rl * (l + 2 * ex[k] * (1 + r2)), rl * (l + 2 * ex[k] * (1 + r2)),
                   rl * (l * l + 4 * l * ex[k] * (1 + r2) + 4 * ex[k] ** 2 * (1 + r2) + 6 * ex[k])]
            for n in range(5):
                bnd[n] += np.abs(A[:, j])[None, :] * (e * fac[n])[:, None]
    return bnd
