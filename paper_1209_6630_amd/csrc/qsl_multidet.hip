// Several determinants: Psi_det = sum_K c_K Det_K_up Det_K_dn (the Psi_T
// equation of section "The quantum Monte Carlo method"), each determinant
// built from n_s orbitals (columns) of one orbital set of n_orb >= n_s MOs
// per spin.  The products C_n = A B_n run once for the whole orbital set
// (equation (abc)); each determinant gathers its columns of C, is inverted
// in FP64 (log|det|, sign, D^-1) and gives its drift and Laplacian ratio;
// the determinants are then combined per walker:
//   log|Psi_det| = m + log|S|,  S = sum_K s_K |c_K| e^(L_K - m),
//   L_K = log|Det_K_up| + log|Det_K_dn|,  m = max_K (L_K + log|c_K|) - log|c_K| shift,
//   drift_e = sum_K w_K drift_K(e),  lap_e = sum_K w_K lap_K(e),
//   w_K = c_K Det_K_up Det_K_dn / Psi_det,
// since grad_e and lap_e act on the one determinant of electron e's spin.
#include <math.h>

#include <algorithm>
#include <vector>

#include "qsl_internal.h"

namespace qsl {

// C_K[w][d][e][i] = C_orb[w][d][e][occ[i]], i, e < n (columns of one
// determinant out of the orbital set).
template <typename T>
__global__ void gather_det_kernel(int64_t W, int n, int nmo, const int* __restrict__ occ, const T* __restrict__ Corb,
                                  T* __restrict__ CK) {
    const int64_t total = W * 5 * (int64_t)n * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % n);
        const int64_t row = q / n;  // (w, d, e)
        CK[q] = Corb[row * nmo + occ[i]];
    }
}

struct MDComb {
    int64_t W;
    int N, n_up, n_det;
    const double* coef;       // [n_det]
    const double* logdet;     // [n_det][W][2]
    const int8_t* sign;       // [n_det][W][2]
    const double* drift;      // [n_det][W][N][3]
    const double* lap;        // [n_det][W][N]
    const uint32_t* dstatus;  // [n_det][W]
    const uint32_t* st0;      // [W] near ties of the products
    double* out_logpsi;       // [W]
    int8_t* out_sign;         // [W]
    double* out_drift;        // [W][N][3]
    double* out_lap;          // [W][N]
    uint32_t* out_status;     // [W]
};

// One thread per (walker, electron): the determinants' weights from their
// log|det| (max-shifted), then the weighted drift and Laplacian ratio.
__global__ void combine_kernel(MDComb c) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= c.W * c.N) return;
    const int64_t w = q / c.N;
    const int e = (int)(q % c.N);
    double m = -INFINITY;
    for (int K = 0; K < c.n_det; ++K) {
        const int8_t s = c.sign[(K * c.W + w) * 2] * c.sign[(K * c.W + w) * 2 + 1];
        if (s == 0 || c.coef[K] == 0.0) continue;
        const double L = c.logdet[(K * c.W + w) * 2] + c.logdet[(K * c.W + w) * 2 + 1] + log(fabs(c.coef[K]));
        m = fmax(m, L);
    }
    double S = 0.0;
    for (int K = 0; K < c.n_det; ++K) {
        const int8_t s = c.sign[(K * c.W + w) * 2] * c.sign[(K * c.W + w) * 2 + 1];
        if (s == 0 || c.coef[K] == 0.0) continue;
        const double L = c.logdet[(K * c.W + w) * 2] + c.logdet[(K * c.W + w) * 2 + 1] + log(fabs(c.coef[K]));
        S += (c.coef[K] > 0 ? s : -s) * exp(L - m);
    }
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0;
    if (S != 0.0) {
        for (int K = 0; K < c.n_det; ++K) {
            const int8_t s = c.sign[(K * c.W + w) * 2] * c.sign[(K * c.W + w) * 2 + 1];
            if (s == 0 || c.coef[K] == 0.0) continue;
            const double L = c.logdet[(K * c.W + w) * 2] + c.logdet[(K * c.W + w) * 2 + 1] + log(fabs(c.coef[K]));
            const double wk = (c.coef[K] > 0 ? s : -s) * exp(L - m) / S;
            const size_t r = ((size_t)K * c.W + w) * c.N + e;
            g0 += wk * c.drift[3 * r];
            g1 += wk * c.drift[3 * r + 1];
            g2 += wk * c.drift[3 * r + 2];
            l += wk * c.lap[r];
        }
    } else {
        g0 = g1 = g2 = l = NAN;
    }
    const size_t o = (size_t)w * c.N + e;
    if (c.out_drift) {
        c.out_drift[3 * o] = g0;
        c.out_drift[3 * o + 1] = g1;
        c.out_drift[3 * o + 2] = g2;
    }
    if (c.out_lap) c.out_lap[o] = l;
    if (e == 0) {
        if (c.out_logpsi) c.out_logpsi[w] = S != 0.0 ? m + log(fabs(S)) : -INFINITY;
        if (c.out_sign) c.out_sign[w] = S > 0 ? 1 : (S < 0 ? -1 : 0);
        if (c.out_status) {
            uint32_t st = c.st0[w] | (S == 0.0 ? QSL_STATUS_SINGULAR : 0u);
            for (int K = 0; K < c.n_det; ++K) st |= c.dstatus[K * c.W + w] & (QSL_STATUS_NEAR_TIE | QSL_STATUS_NONFINITE);
            c.out_status[w] = st;
        }
    }
}

struct MDLayout {
    WsLayout base;
    size_t corb[2], ck[2], dinv[2], logdet, sign, drift, lap, dstatus, st0, occ, coef, total;
};

static MDLayout md_layout(const DevSys& d, const DevMO mo[2], int64_t W, int mode, int n_det) {
    MDLayout L{};
    L.base = ws_layout(d, W, 1, mode, false);  // the forward's part
    size_t off = L.base.fwd_total;
    const size_t cb = mode == QSL_FP64 ? 8 : 4;
    const int N = d.n_up + d.n_dn;
    for (int s = 0; s < 2; ++s) {
        const size_t n = (size_t)n_spin(d, s);
        L.corb[s] = off;
        off = round_up(off + (size_t)W * 5 * n * mo[s].n * cb, 256);
        L.ck[s] = off;
        off = round_up(off + (size_t)W * 5 * n * n * cb, 256);
        L.dinv[s] = off;
        off = round_up(off + (size_t)W * n * n * 8, 256);
    }
    L.logdet = off;
    off = round_up(off + (size_t)n_det * W * 2 * 8, 256);
    L.sign = off;
    off = round_up(off + (size_t)n_det * W * 2, 256);
    L.drift = off;
    off = round_up(off + (size_t)n_det * W * N * 3 * 8, 256);
    L.lap = off;
    off = round_up(off + (size_t)n_det * W * N * 8, 256);
    L.dstatus = off;
    off = round_up(off + (size_t)n_det * W * 4, 256);
    L.st0 = off;
    off = round_up(off + (size_t)W * 4, 256);
    L.occ = off;
    off = round_up(off + (size_t)n_det * N * 4, 256);
    L.coef = off;
    off = round_up(off + (size_t)n_det * 8, 256);
    L.total = off;
    return L;
}

static int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

}  // namespace qsl

using namespace qsl;

extern "C" {

qsl_status qsl_multidet_workspace_size(const qsl_system* sys, int64_t W, int32_t mode, int32_t n_det, size_t* bytes) {
    if (!sys || !bytes || W < 0 || n_det < 1) return bad(QSL_ERR_INVALID_ARG, "NULL argument, W < 0 or n_det < 1");
    if (mode < QSL_FP64 || mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "bad mode");
    *bytes = md_layout(sys->d, sys->mo, W, mode, n_det).total;
    return QSL_OK;
}

qsl_status qsl_multidet_forward(qsl_system* sys, const qsl_multidet_args* a, void* stream) {
    if (!sys || !a) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (a->W < 0 || a->n_det < 1) return bad(QSL_ERR_INVALID_ARG, "W < 0 or n_det < 1");
    if (a->mode < QSL_FP64 || a->mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "bad mode");
    if (!a->occ || !a->coef) return bad(QSL_ERR_INVALID_ARG, "NULL occupations or coefficients");
    const DevSys& d = sys->d;
    const int N = d.n_up + d.n_dn;
    for (int s = 0; s < 2; ++s) {
        const int n = n_spin(d, s);
        if (!n) continue;
        if (!sys->mo[s].set) return bad(QSL_ERR_INVALID_ARG, "orbitals of a spin were never set");
        if (n > GJ_NMAX) return bad(QSL_ERR_UNSUPPORTED, "more electrons of one spin than the inversion supports");
    }
    for (int K = 0; K < a->n_det; ++K) {
        if (!std::isfinite(a->coef[K])) return bad(QSL_ERR_INVALID_ARG, "non-finite determinant coefficient");
        for (int e = 0; e < N; ++e) {
            const int s = e < d.n_up ? 0 : 1;
            const int o = a->occ[(size_t)K * N + e];
            if (o < 0 || o >= sys->mo[s].n) return bad(QSL_ERR_INVALID_ARG, "orbital index out of range");
        }
    }
    if (a->W == 0) return QSL_OK;
    if (!a->R) return bad(QSL_ERR_INVALID_ARG, "NULL R");
    const MDLayout L = md_layout(d, sys->mo, a->W, a->mode, a->n_det);
    if (!a->ws || a->ws_bytes < L.total) return bad(QSL_ERR_WORKSPACE, "workspace missing or too small");
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)a->ws;
    const int64_t W = a->W;
    const int nd = a->n_det;
    hipError_t e;
    // occupations and coefficients to the device (the host arrays may be
    // reused once the call returns)
    if ((e = hipMemcpyAsync(ws + L.occ, a->occ, (size_t)nd * N * 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ws + L.coef, a->coef, (size_t)nd * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(e, "multidet: upload of occupations");
    uint32_t* st0 = (uint32_t*)(ws + L.st0);
    if ((e = fill_u32(st0, 0u, W, st)) != hipSuccess) return hip_fail(e, "multidet: status clear");
    double* dlog = (double*)(ws + L.logdet);
    int8_t* dsgn = (int8_t*)(ws + L.sign);
    double* ddr = (double*)(ws + L.drift);
    double* dlap = (double*)(ws + L.lap);
    uint32_t* dstat = (uint32_t*)(ws + L.dstatus);
    const int* occ = (const int*)(ws + L.occ);
    for (int s = 0; s < 2; ++s) {
        const int n = n_spin(d, s);
        Job j{};
        j.s = d;
        j.mo = sys->mo[s];
        j.spin = s;
        j.n = n;
        j.mode = a->mode;
        j.gw = 1;
        j.W = W;
        j.R = a->R;
        j.nwin = (int*)(ws + L.base.nwin_off[s]);
        j.win = (int*)(ws + L.base.win_off[s]);
        j.jobslot = ws + L.base.job_off;
        j.f32_tile = F32_TILE_DEFAULT;
        j.status = st0;
        if (n) {
            // the products of the whole orbital set, once
            j.C = ws + L.corb[s];
            ProfScope ps1("screen", st);
            if ((e = launch_screen(j, 0, st)) != hipSuccess) return hip_fail(e, "screen kernel");
            ProfScope ps2(a->mode == QSL_FP64 ? "contract_fp64" : a->mode == QSL_FP32 ? "contract_fp32" : "contract_bf16x3", st);
            if ((e = launch_contract(j, st)) != hipSuccess) return hip_fail(e, "contraction kernel");
        }
        for (int K = 0; K < nd; ++K) {
            Job g = j;
            g.mo.n = n;  // a square Slater matrix from here on
            g.C = ws + L.ck[s];
            g.Dinv = (double*)(ws + L.dinv[s]);
            g.logdet = dlog + (size_t)K * W * 2;
            g.sign = dsgn + (size_t)K * W * 2;
            g.drift = ddr + (size_t)K * W * N * 3;
            g.lap = dlap + (size_t)K * W * N;
            g.status = dstat + (size_t)K * W;
            if (gj_blocked(n)) g.gjws = (double*)(ws + L.base.gj_off[s]);
            if (s == 0 && (e = fill_u32(g.status, 0u, W, st)) != hipSuccess) return hip_fail(e, "multidet: status clear");
            if (n) {
                const int* oK = occ + (size_t)K * N + (s ? d.n_up : 0);
                ProfScope ps("gather_det", st);
                if (a->mode == QSL_FP64)
                    gather_det_kernel<double><<<grid_of(W * 5 * (int64_t)n * n), 256, 0, st>>>(
                        W, n, sys->mo[s].n, oK, (const double*)(ws + L.corb[s]), (double*)g.C);
                else
                    gather_det_kernel<float><<<grid_of(W * 5 * (int64_t)n * n), 256, 0, st>>>(
                        W, n, sys->mo[s].n, oK, (const float*)(ws + L.corb[s]), (float*)g.C);
                if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "multidet: gather kernel");
            }
            {
                ProfScope ps("gauss_jordan", st);
                if ((e = launch_gj(g, st)) != hipSuccess) return hip_fail(e, "inversion kernel");
            }
            if (n) {
                ProfScope ps("drift_lap", st);
                if ((e = launch_epilogue(g, st)) != hipSuccess) return hip_fail(e, "epilogue kernel");
            }
        }
    }
    MDComb c{};
    c.W = W;
    c.N = N;
    c.n_up = d.n_up;
    c.n_det = nd;
    c.coef = (const double*)(ws + L.coef);
    c.logdet = dlog;
    c.sign = dsgn;
    c.drift = ddr;
    c.lap = dlap;
    c.dstatus = dstat;
    c.st0 = st0;
    c.out_logpsi = a->logpsi;
    c.out_sign = a->sign;
    c.out_drift = a->drift;
    c.out_lap = a->lap;
    c.out_status = a->status;
    {
        ProfScope ps("combine_dets", st);
        combine_kernel<<<grid_of(W * N), 256, 0, st>>>(c);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "multidet: combine kernel");
    }
    if (a->det_logdet &&
        (e = hipMemcpyAsync(a->det_logdet, dlog, (size_t)nd * W * 2 * 8, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "multidet: copy of determinant logs");
    if (a->det_sign && (e = hipMemcpyAsync(a->det_sign, dsgn, (size_t)nd * W * 2, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "multidet: copy of determinant signs");
    return QSL_OK;
}

}  // extern "C"
