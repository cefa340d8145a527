/*
 * qsl_oracle.c -- plain, slow FP64 CPU reference for the Slater-matrix build.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (Scemama, Caffarel, Oseret, Jalby, "Quantum Monte Carlo
 * for large chemical systems", arXiv:1209.6630):
 *   - contracted Cartesian Gaussian AOs chi(r) = (x-Qx)^nx (y-Qy)^ny (z-Qz)^nz g(r),
 *     g(r) = sum_k c_k exp(-gamma_k |r-Q|^2)   (section "The quantum Monte Carlo
 *     method", critical CPU part, equations for chi and g);
 *   - the values, gradients and Laplacians B_1..B_5 of the AOs that survive the
 *     screening, as a per-electron list of AO indices (section "Exploiting the
 *     highly localized character of atomic basis functions": threshold on the
 *     Gaussian part, atomic radius, the indices array);
 *   - the five products C_n = A B_n, n = 1..5 (equation (abc)), looping over
 *     electron i, then surviving AO k, then MO j, as that section's practical
 *     algorithm does;
 *   - log|det|, sign and inverse of the Slater matrix D_ij = phi_i(r_j) per
 *     spin (Slater determinant equation; inversion step);
 *   - the drift and Laplacian sums  sum_j D^(1)_{l,ij} D^-1_ji  and
 *     sum_j D^(2)_{l,ij} D^-1_ji (the two "vector products" equations);
 *   - the adjoint of log|det| with respect to the MO coefficients and the
 *     electron positions (not in the paper: the chain rule through the MO
 *     expansion equation (mo) and the Slater matrix definition).
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes of the repository):
 *   - screening: primitive k of a shell is kept iff gamma_k r^2 <= T (T = 30
 *     by default); a shell whose primitives are all dropped gives exactly 0.
 *     The test is done in FP64 with r^2 = (dx*dx + dy*dy) + dz*dz, no fused
 *     multiply-add.  An atom is skipped when min_k(gamma_k) r^2 > T, which is
 *     the same decision (atomic radius).
 *   - AO order: atom-major, shells in the order given, Cartesian components
 *     x,y,z for p and xx,xy,xz,yy,yz,zz for d.
 *   - normalisation: every Cartesian AO has unit norm.
 *   - survivors are listed in ascending AO index.
 *   - D[i][e] = C_1[e][i]; C and Dinv are stored [e][i] (MO index fastest),
 *     with sum_i Dinv[e][i] D[i][e'] = delta_ee'.
 *   - LU with partial pivoting on the rows of D, first maximal |a| on ties;
 *     log is natural; an exactly zero pivot gives logdet = -inf, sign = 0.
 *   - the first n_up electrons of a walker are spin up.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LMAX 2

/* Input description, mirrored by a ctypes Structure on the Python side. */
typedef struct {
    int32_t n_atoms;
    const double* atom_xyz;   /* [n_atoms][3] */
    int32_t n_shells;
    const int32_t* shell_atom; /* [n_shells], non-decreasing */
    const int32_t* shell_l;    /* [n_shells], 0..2 */
    const int32_t* shell_nprim;/* [n_shells] */
    const double* prim_exp;    /* [sum nprim] */
    const double* prim_coef;   /* [sum nprim], raw weights */
    int32_t n_up, n_dn;
    double screen_T;
} orc_system;

/* ------------------------------------------------------------------ */
/* Normalisation                                                       */
/* ------------------------------------------------------------------ */

/* (2m-1)!! with (-1)!! = 1 */
static double dfact_odd(int m) {
    double r = 1.0;
    for (int k = 2 * m - 1; k > 1; k -= 2) r *= (double)k;
    return r;
}

/* Cartesian components of shell l, in the fixed order. */
static int n_cart(int l) { return (l + 1) * (l + 2) / 2; }

static void cart_powers(int l, int c, int* a, int* b, int* d) {
    /* l=0: (0,0,0); l=1: x,y,z; l=2: xx,xy,xz,yy,yz,zz */
    static const int p1[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const int p2[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1},
                                 {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
    if (l == 0) { *a = *b = *d = 0; }
    else if (l == 1) { *a = p1[c][0]; *b = p1[c][1]; *d = p1[c][2]; }
    else { *a = p2[c][0]; *b = p2[c][1]; *d = p2[c][2]; }
}

int orc_n_basis(const orc_system* s) {
    int nb = 0;
    for (int i = 0; i < s->n_shells; ++i) nb += n_cart(s->shell_l[i]);
    return nb;
}

/*
 * Contraction weights c_k such that every Cartesian component of the shell,
 * multiplied by its factor f_abc, has unit norm.
 *   N_k = (2 g_k / pi)^(3/4) (4 g_k)^(l/2) / sqrt((2l-1)!!)
 *   S   = sum_km d_k d_m N_k N_m (pi/p)^(3/2) (2l-1)!! / (2p)^l,  p = g_k + g_m
 *   c_k = d_k N_k / sqrt(S)
 *   f_abc = sqrt((2l-1)!! / ((2a-1)!!(2b-1)!!(2c-1)!!))
 */
void orc_normalize(const orc_system* s, double* coef_out) {
    int off = 0;
    for (int sh = 0; sh < s->n_shells; ++sh) {
        int l = s->shell_l[sh], np = s->shell_nprim[sh];
        const double* g = s->prim_exp + off;
        const double* d = s->prim_coef + off;
        double dl = dfact_odd(l);
        double S = 0.0;
        for (int k = 0; k < np; ++k) {
            double Nk = pow(2.0 * g[k] / M_PI, 0.75) * pow(4.0 * g[k], 0.5 * l) / sqrt(dl);
            for (int m = 0; m < np; ++m) {
                double Nm = pow(2.0 * g[m] / M_PI, 0.75) * pow(4.0 * g[m], 0.5 * l) / sqrt(dl);
                double p = g[k] + g[m];
                S += d[k] * d[m] * Nk * Nm * pow(M_PI / p, 1.5) * dl / pow(2.0 * p, (double)l);
            }
        }
        for (int k = 0; k < np; ++k) {
            double Nk = pow(2.0 * g[k] / M_PI, 0.75) * pow(4.0 * g[k], 0.5 * l) / sqrt(dl);
            coef_out[off + k] = d[k] * Nk / sqrt(S);
        }
        off += np;
    }
}

double orc_cart_factor(int l, int a, int b, int c) {
    return sqrt(dfact_odd(l) / (dfact_odd(a) * dfact_odd(b) * dfact_odd(c)));
}

/* ------------------------------------------------------------------ */
/* Prepared system: normalised weights and per-shell offsets           */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_system* s;
    int n_basis;
    int* shell_off;   /* first primitive of each shell */
    int* shell_ao;    /* first AO of each shell */
    double* coef;     /* normalised c_k */
    double* atom_gmin;/* min exponent over all primitives of the atom */
} orc_prep;

static void prep_init(orc_prep* P, const orc_system* s) {
    P->s = s;
    P->n_basis = orc_n_basis(s);
    P->shell_off = (int*)malloc(sizeof(int) * (s->n_shells + 1));
    P->shell_ao = (int*)malloc(sizeof(int) * (s->n_shells + 1));
    int np = 0, na = 0;
    for (int i = 0; i < s->n_shells; ++i) {
        P->shell_off[i] = np; P->shell_ao[i] = na;
        np += s->shell_nprim[i]; na += n_cart(s->shell_l[i]);
    }
    P->shell_off[s->n_shells] = np; P->shell_ao[s->n_shells] = na;
    P->coef = (double*)malloc(sizeof(double) * (np > 0 ? np : 1));
    orc_normalize(s, P->coef);
    P->atom_gmin = (double*)malloc(sizeof(double) * (s->n_atoms > 0 ? s->n_atoms : 1));
    for (int a = 0; a < s->n_atoms; ++a) P->atom_gmin[a] = INFINITY;
    for (int i = 0; i < s->n_shells; ++i)
        for (int k = P->shell_off[i]; k < P->shell_off[i + 1]; ++k)
            if (s->prim_exp[k] < P->atom_gmin[s->shell_atom[i]])
                P->atom_gmin[s->shell_atom[i]] = s->prim_exp[k];
}

static void prep_free(orc_prep* P) {
    free(P->shell_off); free(P->shell_ao); free(P->coef); free(P->atom_gmin);
}

/* ------------------------------------------------------------------ */
/* AO evaluation at one electron                                        */
/* ------------------------------------------------------------------ */

static double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/*
 * Screened AOs at point r.  Writes the ascending list of surviving AO
 * indices to idx and B[n*ld + k] for n = 0..4 (value, d/dx, d/dy, d/dz,
 * Laplacian).  Returns the number of survivors.  *near_tie is set when some
 * gamma_k r^2 lies within 1e-12 T of T.
 */
static int ao_eval(const orc_prep* P, const double r[3], int* idx, double* B, int ld,
                   int* near_tie) {
    const orc_system* s = P->s;
    const double T = s->screen_T;
    int cnt = 0;
    for (int sh = 0; sh < s->n_shells; ++sh) {
        int at = s->shell_atom[sh];
        double dx = r[0] - s->atom_xyz[3 * at + 0];
        double dy = r[1] - s->atom_xyz[3 * at + 1];
        double dz = r[2] - s->atom_xyz[3 * at + 2];
        volatile double t0 = dx * dx;   /* volatile: keep the exact */
        volatile double t1 = t0 + dy * dy; /* FP64 evaluation order */
        double r2 = t1 + dz * dz;
        /* atomic radius: nothing on this atom survives */
        double ga = P->atom_gmin[at] * r2;
        if (ga > T) {
            if (fabs(ga - T) <= 1e-12 * T) *near_tie = 1;
            continue;
        }
        /* radial part and its derivatives, over the kept primitives */
        double g = 0.0, g1 = 0.0, g2 = 0.0;
        int kept = 0;
        for (int k = P->shell_off[sh]; k < P->shell_off[sh + 1]; ++k) {
            double gk = s->prim_exp[k];
            double t = gk * r2;
            if (fabs(t - T) <= 1e-12 * T) *near_tie = 1;
            if (t > T) continue;
            ++kept;
            double ek = P->coef[k] * exp(-t);
            g += ek;
            g1 += -2.0 * gk * ek;
            g2 += ek * (4.0 * gk * gk * r2 - 6.0 * gk);
        }
        if (!kept) continue;
        int l = s->shell_l[sh];
        double d[3] = {dx, dy, dz};
        for (int c = 0; c < n_cart(l); ++c) {
            int p[3];
            cart_powers(l, c, &p[0], &p[1], &p[2]);
            double f = orc_cart_factor(l, p[0], p[1], p[2]);
            double P0 = f * ipow(d[0], p[0]) * ipow(d[1], p[1]) * ipow(d[2], p[2]);
            double dP[3], lapP = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
                double rest = ipow(d[o1], p[o1]) * ipow(d[o2], p[o2]);
                dP[ax] = p[ax] ? f * p[ax] * ipow(d[ax], p[ax] - 1) * rest : 0.0;
                if (p[ax] >= 2) lapP += f * p[ax] * (p[ax] - 1) * ipow(d[ax], p[ax] - 2) * rest;
            }
            int ao = P->shell_ao[sh] + c;
            idx[cnt] = ao;
            B[0 * ld + cnt] = P0 * g;
            for (int ax = 0; ax < 3; ++ax) B[(1 + ax) * ld + cnt] = dP[ax] * g + P0 * g1 * d[ax];
            /* Delta . grad P = l P for a homogeneous polynomial of degree l */
            B[4 * ld + cnt] = lapP * g + 2.0 * l * g1 * P0 + P0 * g2;
            ++cnt;
        }
    }
    return cnt;
}

/* Public single-point AO evaluation, for the pins. */
int orc_ao_eval(const orc_system* s, const double* r, int32_t* idx, double* B, int ld,
                int32_t* near_tie) {
    orc_prep P;
    prep_init(&P, s);
    int* tmp = (int*)malloc(sizeof(int) * (P.n_basis > 0 ? P.n_basis : 1));
    int nt = 0;
    int n = ao_eval(&P, r, tmp, B, ld, &nt);
    for (int i = 0; i < n; ++i) idx[i] = tmp[i];
    if (near_tie) *near_tie = nt;
    free(tmp);
    prep_free(&P);
    return n;
}

/* ------------------------------------------------------------------ */
/* LU with partial pivoting, log|det|, sign, inverse                   */
/* ------------------------------------------------------------------ */

/*
 * a: n x n row-major, overwritten by L\U.  piv[k] = row swapped into k.
 * Returns 0 if singular (exact zero pivot), 1 otherwise.
 */
static int lu_factor(double* a, int n, int* piv, double* logdet, int* sign) {
    double ld = 0.0;
    int sg = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(a[i * n + k]);
            if (v > best) { best = v; p = i; }   /* first maximum wins ties */
        }
        piv[k] = p;
        if (best == 0.0) { *logdet = -INFINITY; *sign = 0; return 0; }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
            sg = -sg;
        }
        double ukk = a[k * n + k];
        if (ukk < 0) sg = -sg;
        ld += log(fabs(ukk));
        for (int i = k + 1; i < n; ++i) {
            double lik = a[i * n + k] / ukk;
            a[i * n + k] = lik;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= lik * a[k * n + j];
        }
    }
    *logdet = ld;
    *sign = sg;
    return 1;
}

/* Column c of the inverse: solve D x = e_c with the factors. */
static void lu_solve_unit(const double* lu, int n, const int* piv, int c, double* x) {
    for (int i = 0; i < n; ++i) x[i] = (i == c) ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) {             /* apply the row swaps */
        int p = piv[k];
        if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
    }
    for (int i = 0; i < n; ++i) {             /* L y = b, unit diagonal */
        double v = x[i];
        for (int j = 0; j < i; ++j) v -= lu[i * n + j] * x[j];
        x[i] = v;
    }
    for (int i = n - 1; i >= 0; --i) {        /* U x = y */
        double v = x[i];
        for (int j = i + 1; j < n; ++j) v -= lu[i * n + j] * x[j];
        x[i] = v / lu[i * n + i];
    }
}

/* Public: slogdet + inverse of a row-major n x n matrix (for the pins). */
int orc_lu_inverse(const double* m, int n, double* inv, double* logdet, int32_t* sign) {
    double* a = (double*)malloc(sizeof(double) * (size_t)n * n + 8);
    int* piv = (int*)malloc(sizeof(int) * (n + 1));
    double* x = (double*)malloc(sizeof(double) * (n + 1));
    memcpy(a, m, sizeof(double) * (size_t)n * n);
    int sg;
    int ok = lu_factor(a, n, piv, logdet, &sg);
    *sign = sg;
    if (ok && inv) {
        for (int c = 0; c < n; ++c) {
            lu_solve_unit(a, n, piv, c, x);
            for (int r = 0; r < n; ++r) inv[r * n + c] = x[r];
        }
    }
    free(a); free(piv); free(x);
    return ok;
}

/* ------------------------------------------------------------------ */
/* Forward                                                              */
/* ------------------------------------------------------------------ */

#define ORC_ST_SINGULAR 1u
#define ORC_ST_NEAR_TIE 2u
#define ORC_ST_NONFINITE 4u

/*
 * For every walker w:
 *   C^s[w][n][e][i] = sum_k A^s[i][idx(k,e)] B_n(k,e)   (n = 0..4, e in spin s)
 *   Cabs^s (optional) = sum_k |A^s[i][idx(k,e)]| |B_n(k,e)|
 *   logdet[w][s], sign[w][s], Dinv^s[w][e][i], drift[w][e][3], lap[w][e]
 * A^s is n_s x N_b row-major.  Outputs that are NULL are skipped (C is always
 * computed internally).
 */
void orc_forward(const orc_system* s, const double* A_up, const double* A_dn,
                 int32_t W, const double* R,
                 double* C_up, double* C_dn, double* Cabs_up, double* Cabs_dn,
                 double* logdet, int8_t* sign, double* Dinv_up, double* Dinv_dn,
                 double* drift, double* lap, uint32_t* status, int32_t nthreads) {
    orc_prep P;
    prep_init(&P, s);
    const int N = s->n_up + s->n_dn, nb = P.n_basis;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int* idx = (int*)malloc(sizeof(int) * (nb + 1));
        double* B = (double*)malloc(sizeof(double) * 5 * (nb + 1));
        int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
        size_t nn = (size_t)nmax * nmax + 1;
        double* Cw = (double*)malloc(sizeof(double) * 5 * nn);
        double* Aw = (double*)malloc(sizeof(double) * 5 * nn);
        double* Dm = (double*)malloc(sizeof(double) * nn);
        double* Iv = (double*)malloc(sizeof(double) * nn);
        int* piv = (int*)malloc(sizeof(int) * (nmax + 1));
        double* x = (double*)malloc(sizeof(double) * (nmax + 1));
#pragma omp for schedule(static)
        for (int w = 0; w < W; ++w) {
            uint32_t st = 0;
            for (int sp = 0; sp < 2; ++sp) {
                int n = sp ? s->n_dn : s->n_up;
                int e0 = sp ? s->n_up : 0;
                const double* A = sp ? A_dn : A_up;
                if (n == 0) {
                    if (logdet) logdet[2 * w + sp] = 0.0;
                    if (sign) sign[2 * w + sp] = 1;
                    continue;
                }
                memset(Cw, 0, sizeof(double) * 5 * (size_t)n * n);
                memset(Aw, 0, sizeof(double) * 5 * (size_t)n * n);
                /* products, loop order: electron, surviving AO, MO */
                for (int e = 0; e < n; ++e) {
                    const double* r = R + ((size_t)w * N + e0 + e) * 3;
                    int nt = 0;
                    int cnt = ao_eval(&P, r, idx, B, nb + 1, &nt);
                    if (nt) st |= ORC_ST_NEAR_TIE;
                    for (int k = 0; k < cnt; ++k) {
                        int j = idx[k];
                        for (int i = 0; i < n; ++i) {
                            double a = A[(size_t)i * nb + j];
                            for (int c = 0; c < 5; ++c) {
                                double b = B[c * (nb + 1) + k];
                                Cw[((size_t)c * n + e) * n + i] += a * b;
                                Aw[((size_t)c * n + e) * n + i] += fabs(a) * fabs(b);
                            }
                        }
                    }
                }
                double* Cout = sp ? C_dn : C_up;
                double* Cab = sp ? Cabs_dn : Cabs_up;
                size_t wsz = 5 * (size_t)n * n;
                if (Cout) memcpy(Cout + (size_t)w * wsz, Cw, sizeof(double) * wsz);
                if (Cab) memcpy(Cab + (size_t)w * wsz, Aw, sizeof(double) * wsz);
                /* Slater matrix D[i][e] = C_1[e][i] */
                for (int i = 0; i < n; ++i)
                    for (int e = 0; e < n; ++e) Dm[i * n + e] = Cw[(size_t)e * n + i];
                double ld;
                int sg;
                int ok = lu_factor(Dm, n, piv, &ld, &sg);
                if (!ok) st |= ORC_ST_SINGULAR;
                if (logdet) logdet[2 * w + sp] = ld;
                if (sign) sign[2 * w + sp] = (int8_t)sg;
                if (ok) {
                    /* Dinv[e][i]: column i of D^-1 is the solution of D x = e_i */
                    for (int i = 0; i < n; ++i) {
                        lu_solve_unit(Dm, n, piv, i, x);
                        for (int e = 0; e < n; ++e) Iv[(size_t)e * n + i] = x[e];
                    }
                } else {
                    for (size_t q = 0; q < (size_t)n * n; ++q) Iv[q] = NAN;
                }
                double* Dout = sp ? Dinv_dn : Dinv_up;
                if (Dout) memcpy(Dout + (size_t)w * n * n, Iv, sizeof(double) * (size_t)n * n);
                /* drift and Laplacian of the determinant (Jacobi) */
                for (int e = 0; e < n; ++e) {
                    double acc[4] = {0, 0, 0, 0};
                    for (int i = 0; i < n; ++i) {
                        double di = Iv[(size_t)e * n + i];
                        for (int c = 0; c < 4; ++c) acc[c] += di * Cw[((size_t)(c + 1) * n + e) * n + i];
                    }
                    size_t ge = (size_t)w * N + e0 + e;
                    if (drift) for (int c = 0; c < 3; ++c) drift[ge * 3 + c] = acc[c];
                    if (lap) lap[ge] = acc[3];
                    for (int c = 0; c < 4; ++c) if (!isfinite(acc[c])) st |= ok ? ORC_ST_NONFINITE : 0u;
                }
                if (!isfinite(ld) && ok) st |= ORC_ST_NONFINITE;
            }
            if (status) status[w] = st;
        }
        free(idx); free(B); free(Cw); free(Aw); free(Dm); free(Iv); free(piv); free(x);
    }
    prep_free(&P);
}

/* ------------------------------------------------------------------ */
/* Adjoint of log|det|                                                   */
/* ------------------------------------------------------------------ */

/*
 * g[w][s] = dL/dlogdet[w][s].  With G[e][i] = g Dinv[e][i] (the gradient of
 * log|det D| with respect to C_1[e][i]):
 *   dA^s[i][j] = sum_w sum_{e in s, j survivor of e} G[e][i] chi_j(r_e)
 *   dR[w][e]   = sum_k (sum_i A^s[i][idx(k,e)] G[e][i]) grad chi_idx(k,e)(r_e)
 * The survivor sets are held fixed (derivative of the screened function).
 * dR is overwritten; dA is overwritten with the sum over walkers.
 * Optional (NULL to skip): the same sums over absolute values of every term,
 *   dA_abs^s[i][j] = sum_w sum_e |G[e][i]| |chi_j(r_e)|
 *   dR_abs[w][e]   = sum_k (sum_i |A^s[i][idx(k,e)]| |G[e][i]|) |grad chi_idx(k,e)(r_e)|
 * (componentwise), the scale against which rounding errors are bounded.
 */
void orc_backward(const orc_system* s, const double* A_up, const double* A_dn,
                  int32_t W, const double* R, const double* Dinv_up, const double* Dinv_dn,
                  const double* g, double* dR, double* dA_up, double* dA_dn,
                  double* dR_abs, double* dAabs_up, double* dAabs_dn, int32_t nthreads) {
    orc_prep P;
    prep_init(&P, s);
    const int N = s->n_up + s->n_dn, nb = P.n_basis;
    int nthr = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    nthr = omp_get_max_threads();
#endif
    size_t szu = (size_t)s->n_up * nb, szd = (size_t)s->n_dn * nb;
    const int want_abs = dR_abs || dAabs_up || dAabs_dn;
    const size_t per = (szu + szd) * (want_abs ? 2 : 1);
    double* part = (double*)calloc((size_t)nthr * per + 1, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* my_up = part + (size_t)tid * per;
        double* my_dn = my_up + szu;
        double* myabs_up = want_abs ? my_dn + szd : NULL;
        double* myabs_dn = want_abs ? myabs_up + szu : NULL;
        int* idx = (int*)malloc(sizeof(int) * (nb + 1));
        double* B = (double*)malloc(sizeof(double) * 5 * (nb + 1));
#pragma omp for schedule(static)
        for (int w = 0; w < W; ++w) {
            for (int sp = 0; sp < 2; ++sp) {
                int n = sp ? s->n_dn : s->n_up;
                int e0 = sp ? s->n_up : 0;
                const double* A = sp ? A_dn : A_up;
                const double* Di = (sp ? Dinv_dn : Dinv_up) + (size_t)w * n * n;
                double* dA = sp ? my_dn : my_up;
                double* dAa = sp ? myabs_dn : myabs_up;
                double gw = g[2 * w + sp];
                for (int e = 0; e < n; ++e) {
                    size_t ge = (size_t)w * N + e0 + e;
                    const double* r = R + ge * 3;
                    int nt = 0;
                    int cnt = ao_eval(&P, r, idx, B, nb + 1, &nt);
                    double dr[3] = {0, 0, 0}, dra[3] = {0, 0, 0};
                    for (int k = 0; k < cnt; ++k) {
                        int j = idx[k];
                        double h = 0.0, ha = 0.0;
                        for (int i = 0; i < n; ++i) {
                            double Gi = gw * Di[(size_t)e * n + i];
                            h += A[(size_t)i * nb + j] * Gi;
                            dA[(size_t)i * nb + j] += Gi * B[k];
                            if (dAa) {
                                ha += fabs(A[(size_t)i * nb + j]) * fabs(Gi);
                                dAa[(size_t)i * nb + j] += fabs(Gi) * fabs(B[k]);
                            }
                        }
                        for (int c = 0; c < 3; ++c) dr[c] += h * B[(1 + c) * (nb + 1) + k];
                        if (dAa)
                            for (int c = 0; c < 3; ++c) dra[c] += ha * fabs(B[(1 + c) * (nb + 1) + k]);
                    }
                    for (int c = 0; c < 3; ++c) dR[ge * 3 + c] = dr[c];
                    if (dR_abs)
                        for (int c = 0; c < 3; ++c) dR_abs[ge * 3 + c] = dra[c];
                }
            }
        }
        free(idx); free(B);
    }
    if (dA_up) memset(dA_up, 0, sizeof(double) * szu);
    if (dA_dn) memset(dA_dn, 0, sizeof(double) * szd);
    if (dAabs_up) memset(dAabs_up, 0, sizeof(double) * szu);
    if (dAabs_dn) memset(dAabs_dn, 0, sizeof(double) * szd);
    for (int t = 0; t < nthr; ++t) {
        const double* pu = part + (size_t)t * per;
        if (dA_up) for (size_t q = 0; q < szu; ++q) dA_up[q] += pu[q];
        if (dA_dn) for (size_t q = 0; q < szd; ++q) dA_dn[q] += pu[szu + q];
        if (dAabs_up) for (size_t q = 0; q < szu; ++q) dAabs_up[q] += pu[szu + szd + q];
        if (dAabs_dn) for (size_t q = 0; q < szd; ++q) dAabs_dn[q] += pu[2 * szu + szd + q];
    }
    free(part);
    prep_free(&P);
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* One Monte Carlo step around the Slater part (section "The quantum    */
/* Monte Carlo method": drift-diffusion move, drift, branching weight,  */
/* local energy, reconfiguration with a constant number of walkers;    */
/* the trial wavefunction with a Jastrow factor of its "Critical CPU   */
/* part" subsection).                                                   */
/* ------------------------------------------------------------------ */

/*
 * Pair function of the Jastrow factor, u(r) = a r / (1 + b r), with its
 * first and second derivatives in r.  The electron-electron term takes
 * a = c_ee / 2 (opposite spins) or c_ee / 4 (same spin), the
 * electron-nucleus term a = -c_en Z; b >= 0 sets the range.  u'(0) = a:
 * with c = 1 these are the cusp conditions.  (The paper leaves the U
 * functions open; this is the reading taken.)
 */
static void pair_u(double a, double b, double r, double* u, double* du, double* d2u) {
    double q = 1.0 + b * r;
    *u = a * r / q;
    *du = a / (q * q);
    *d2u = -2.0 * a * b / (q * q * q);
}

/*
 * For every walker: the Jastrow exponent
 *   J = sum_{i<j} u_ee(r_ij) + sum_{i,alpha} u_en(r_i alpha),
 * its gradient gJ[w][i][3] and Laplacian lJ[w][i] with respect to each
 * electron, and the Coulomb potential
 *   V = sum_{i<j} 1/r_ij - sum_{i,alpha} Z_alpha / r_i alpha
 *       + sum_{alpha<beta} Z_alpha Z_beta / |Q_alpha - Q_beta|.
 * The first n_up electrons are spin up.  Any output may be NULL.
 */
void orc_jastrow_potential(const orc_system* s, const double* Z, double c_ee, double b_ee, double c_en,
                           double b_en, int32_t W, const double* R, double* J, double* gJ, double* lJ, double* V,
                           int32_t nthreads) {
    const int N = s->n_up + s->n_dn, na = s->n_atoms;
    double vnn = 0.0;
    for (int a = 0; a < na; ++a)
        for (int b = a + 1; b < na; ++b) {
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = s->atom_xyz[3 * a + k] - s->atom_xyz[3 * b + k];
            vnn += Z[a] * Z[b] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int w = 0; w < W; ++w) {
        const double* Rw = R + (size_t)w * N * 3;
        double jw = 0.0, vw = vnn;
        for (int i = 0; i < N; ++i) {
            double g[3] = {0, 0, 0}, l = 0.0;
            const int si = i < s->n_up;
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = Rw[3 * i + k] - Rw[3 * j + k];
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double a = c_ee * ((si == (j < s->n_up)) ? 0.25 : 0.5);
                double u, du, d2u;
                pair_u(a, b_ee, r, &u, &du, &d2u);
                for (int k = 0; k < 3; ++k) g[k] += du * d[k] / r;
                l += d2u + 2.0 * du / r;
                if (j > i) {
                    jw += u;
                    vw += 1.0 / r;
                }
            }
            for (int al = 0; al < na; ++al) {
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = Rw[3 * i + k] - s->atom_xyz[3 * al + k];
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double u, du, d2u;
                pair_u(-c_en * Z[al], b_en, r, &u, &du, &d2u);
                for (int k = 0; k < 3; ++k) g[k] += du * d[k] / r;
                l += d2u + 2.0 * du / r;
                jw += u;
                vw -= Z[al] / r;
            }
            if (gJ) for (int k = 0; k < 3; ++k) gJ[((size_t)w * N + i) * 3 + k] = g[k];
            if (lJ) lJ[(size_t)w * N + i] = l;
        }
        if (J) J[w] = jw;
        if (V) V[w] = vw;
    }
}

/*
 * Local energy E_L = H Psi / Psi of Psi = e^J Det_up Det_dn, and the drift
 * b = grad Psi / Psi, from the determinant's drift bd and Laplacian ratio ld
 * (per electron, the forward's drift and lap) and the Jastrow derivatives:
 *   grad_i Psi / Psi = gJ_i + bd_i,
 *   lap_i Psi / Psi  = lJ_i + |gJ_i|^2 + 2 gJ_i . bd_i + ld_i,
 *   E_L = -1/2 sum_i lap_i Psi / Psi + V.
 */
void orc_local_energy(int32_t W, int32_t N, const double* bd, const double* ld, const double* gJ,
                      const double* lJ, const double* V, double* EL, double* drift) {
    for (int w = 0; w < W; ++w) {
        double t = 0.0;
        for (int i = 0; i < N; ++i) {
            size_t q = (size_t)w * N + i;
            double gg = 0.0, gb = 0.0;
            for (int k = 0; k < 3; ++k) {
                gg += gJ[3 * q + k] * gJ[3 * q + k];
                gb += gJ[3 * q + k] * bd[3 * q + k];
                if (drift) drift[3 * q + k] = gJ[3 * q + k] + bd[3 * q + k];
            }
            t += lJ[q] + gg + 2.0 * gb + ld[q];
        }
        EL[w] = -0.5 * t + V[w];
    }
}

/* Drift-diffusion move R' = R + tau b(R) + sqrt(tau) eta, per coordinate. */
void orc_drift_diffuse(int64_t count, const double* R, const double* b, const double* eta, double tau,
                       double* Rout) {
    const double st = sqrt(tau);
    for (int64_t q = 0; q < count; ++q) {
        double m = tau * b[q];
        double d = st * eta[q];
        Rout[q] = (R[q] + m) + d;
    }
}

/*
 * Branching weight w = exp(-tau/2 [(E_L(R') - E_T) + (E_L(R) - E_T)]) of
 * each walker.  A move that changes the sign of Psi crossed a node of the
 * trial wavefunction, which the fixed-node walkers cannot: weight 0; so is
 * a walker whose Psi vanishes.
 */
void orc_branch_weights(int64_t W, const double* EL_new, const double* EL_old, const int8_t* sign_new,
                        const int8_t* sign_old, double E_T, double tau, double* w) {
    for (int64_t k = 0; k < W; ++k) {
        if (sign_new[k] == 0 || sign_new[k] != sign_old[k]) {
            w[k] = 0.0;
            continue;
        }
        double e = (EL_new[k] - E_T) + (EL_old[k] - E_T);
        double v = exp(-0.5 * tau * e);
        /* a walker whose weight is not a finite number (a non-finite local
           energy, or an overflow) is dropped */
        w[k] = isfinite(v) ? v : 0.0;
    }
}

/*
 * Reconfiguration: M = W new walkers drawn among the W walkers with
 * probabilities p_k = w_k / sum_i w_i.  Draw m takes the uniform u[m] in
 * [0, 1) and selects the first k whose cumulative weight (summed in walker
 * order) exceeds u[m] times the total.  idx[m] = k; *wsum = the total
 * (the population weight of this step is wsum / W).  With a zero total the
 * population is kept (idx[m] = m).
 */
void orc_reconfigure(int64_t W, const double* w, const double* u, int64_t* idx, double* wsum) {
    double* cum = (double*)malloc(sizeof(double) * (W > 0 ? W : 1));
    double c = 0.0;
    for (int64_t k = 0; k < W; ++k) {
        c += w[k];
        cum[k] = c;
    }
    *wsum = c;
    for (int64_t m = 0; m < W; ++m) {
        if (!(c > 0.0)) {
            idx[m] = m;
            continue;
        }
        double x = u[m] * c;
        int64_t k = 0;
        while (k < W - 1 && !(x < cum[k])) ++k;
        idx[m] = k;
    }
    free(cum);
}

/* ------------------------------------------------------------------ */
/* Several determinants (the trial wavefunction equation of section    */
/* "The quantum Monte Carlo method")                                    */
/* ------------------------------------------------------------------ */

/*
 * Psi_det = sum_K c_K Det_K_up Det_K_dn.  Determinant K takes the rows
 * occ[K][0..n_up) of the spin-up orbital set A_up_orb (n_orb_up x N_b) and
 * the rows occ[K][n_up..N) of the spin-down one; each is evaluated by the
 * single-determinant forward above.  Then per walker, with L_K = log|Det_K_up|
 * + log|Det_K_dn| + log|c_K| and s_K the sign of c_K Det_K_up Det_K_dn:
 *   m = max_K L_K over the non-zero terms, S = sum_K s_K e^(L_K - m),
 *   log|Psi_det| = m + log|S|, sign = sign(S),
 *   drift_e = sum_K w_K drift_K(e), lap_e = sum_K w_K lap_K(e),
 *   w_K = s_K e^(L_K - m) / S
 * (grad_e and lap_e of a product of an up and a down determinant act on
 * the one of electron e's spin).  Outputs det_logdet [n_det][W][2] and
 * det_sign [n_det][W][2] may be NULL.
 */
void orc_multidet(const orc_system* s, const double* A_up_orb, const double* A_dn_orb, int32_t n_det,
                  const int32_t* occ, const double* coef, int32_t W, const double* R, double* logpsi,
                  int8_t* sign, double* drift, double* lap, double* det_logdet, int8_t* det_sign,
                  int32_t nthreads) {
    const int N = s->n_up + s->n_dn, nb = orc_n_basis(s);
    const int nu = s->n_up, nd = s->n_dn;
    double* Au = (double*)malloc(sizeof(double) * ((size_t)nu * nb + 1));
    double* Ad = (double*)malloc(sizeof(double) * ((size_t)nd * nb + 1));
    double* L = (double*)malloc(sizeof(double) * (size_t)n_det * W * 2);
    int8_t* sg = (int8_t*)malloc((size_t)n_det * W * 2);
    double* dr = (double*)malloc(sizeof(double) * (size_t)n_det * W * N * 3);
    double* lp = (double*)malloc(sizeof(double) * (size_t)n_det * W * N);
    double* Cu = (double*)malloc(sizeof(double) * ((size_t)W * 5 * nu * nu + 1));
    double* Cd = (double*)malloc(sizeof(double) * ((size_t)W * 5 * nd * nd + 1));
    double* Iu = (double*)malloc(sizeof(double) * ((size_t)W * nu * nu + 1));
    double* Id = (double*)malloc(sizeof(double) * ((size_t)W * nd * nd + 1));
    uint32_t* st = (uint32_t*)malloc(sizeof(uint32_t) * (W > 0 ? W : 1));
    for (int K = 0; K < n_det; ++K) {
        for (int i = 0; i < nu; ++i)
            memcpy(Au + (size_t)i * nb, A_up_orb + (size_t)occ[(size_t)K * N + i] * nb, sizeof(double) * nb);
        for (int i = 0; i < nd; ++i)
            memcpy(Ad + (size_t)i * nb, A_dn_orb + (size_t)occ[(size_t)K * N + nu + i] * nb, sizeof(double) * nb);
        orc_forward(s, Au, Ad, W, R, Cu, Cd, NULL, NULL, L + (size_t)K * W * 2, sg + (size_t)K * W * 2, Iu, Id,
                    dr + (size_t)K * W * N * 3, lp + (size_t)K * W * N, st, nthreads);
    }
    for (int w = 0; w < W; ++w) {
        double m = -INFINITY;
        for (int K = 0; K < n_det; ++K) {
            int sK = sg[((size_t)K * W + w) * 2] * sg[((size_t)K * W + w) * 2 + 1];
            if (sK == 0 || coef[K] == 0.0) continue;
            double LK = L[((size_t)K * W + w) * 2] + L[((size_t)K * W + w) * 2 + 1] + log(fabs(coef[K]));
            if (LK > m) m = LK;
        }
        double S = 0.0;
        for (int K = 0; K < n_det; ++K) {
            int sK = sg[((size_t)K * W + w) * 2] * sg[((size_t)K * W + w) * 2 + 1];
            if (sK == 0 || coef[K] == 0.0) continue;
            if (coef[K] < 0) sK = -sK;
            double LK = L[((size_t)K * W + w) * 2] + L[((size_t)K * W + w) * 2 + 1] + log(fabs(coef[K]));
            S += sK * exp(LK - m);
        }
        logpsi[w] = S != 0.0 ? m + log(fabs(S)) : -INFINITY;
        sign[w] = S > 0 ? 1 : (S < 0 ? -1 : 0);
        for (int e = 0; e < N; ++e) {
            double g[3] = {0, 0, 0}, l = 0.0;
            for (int K = 0; K < n_det && S != 0.0; ++K) {
                int sK = sg[((size_t)K * W + w) * 2] * sg[((size_t)K * W + w) * 2 + 1];
                if (sK == 0 || coef[K] == 0.0) continue;
                if (coef[K] < 0) sK = -sK;
                double LK = L[((size_t)K * W + w) * 2] + L[((size_t)K * W + w) * 2 + 1] + log(fabs(coef[K]));
                double wK = sK * exp(LK - m) / S;
                size_t r = ((size_t)K * W + w) * N + e;
                for (int k = 0; k < 3; ++k) g[k] += wK * dr[3 * r + k];
                l += wK * lp[r];
            }
            if (S == 0.0) g[0] = g[1] = g[2] = l = NAN;
            if (drift) for (int k = 0; k < 3; ++k) drift[((size_t)w * N + e) * 3 + k] = g[k];
            if (lap) lap[(size_t)w * N + e] = l;
        }
    }
    if (det_logdet) memcpy(det_logdet, L, sizeof(double) * (size_t)n_det * W * 2);
    if (det_sign) memcpy(det_sign, sg, (size_t)n_det * W * 2);
    free(Au); free(Ad); free(L); free(sg); free(dr); free(lp); free(Cu); free(Cd); free(Iu); free(Id); free(st);
}
