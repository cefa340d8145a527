// One Monte Carlo step around the Slater-matrix build (section "The quantum
// Monte Carlo method"): the trial wavefunction Psi = e^J Det_up Det_dn with a
// Jastrow factor of electron-electron and electron-nucleus terms (the Psi_T
// equation of the "Critical CPU part" subsection), the drift b = grad Psi /
// Psi (equation (drift)), the local energy E_L = H Psi / Psi (equation
// (localenergy)), the drift-diffusion move (equation (proba)), the branching
// weight (equation (w)) and the reconfiguration of the population at a
// constant number of walkers (subsection "Parallelizing FN-DMC").
//
// Jastrow pair function u(r) = a r / (1 + b r): a = c_ee / 2 for electrons
// of opposite spins, c_ee / 4 for the same spin, a = -c_en Z_alpha for
// electron-nucleus pairs (c = 1 gives the cusp conditions).  Everything here
// is FP64: O(N^2) per walker against the O(N^2 N_basis) products.
#include <math.h>

#include <algorithm>
#include <vector>

#include "qsl_internal.h"

namespace qsl {

constexpr int LE_THREADS = 256;
constexpr int LE_MAX_ELEC = 2048;  // electron positions of a walker staged in LDS (48 KB)

struct LEJob {
    int n_up, n_dn, n_atoms;
    const double* atom_xyz;
    const double* Z;
    double c_ee, b_ee, c_en, b_en, v_nn;
    int64_t W;
    const double* R;       // [W][N][3]
    const double* bd;      // determinant drift [W][N][3]
    const double* ld;      // determinant Laplacian ratio [W][N]
    const double* logdet;  // [W][2]
    const int8_t* sign;    // [W][2]
    double* EL;            // [W]
    double* drift;         // [W][N][3]
    double* logpsi;        // [W] (may be NULL)
    int8_t* psisign;       // [W] (may be NULL)
    double* J;             // [W] (may be NULL)
    double* V;             // [W] (may be NULL)
};

__device__ __forceinline__ void pair_u(double a, double b, double r, double& u, double& du, double& d2u) {
    const double q = 1.0 + b * r;
    u = a * r / q;
    du = a / (q * q);
    d2u = -2.0 * a * b / (q * q * q);
}

// One workgroup per walker: electron i of thread i (strided) sums its
// electron-electron and electron-nucleus pairs for the gradient and
// Laplacian of J, and the pairs j > i for J and the potential.
__global__ __launch_bounds__(LE_THREADS) void local_energy_kernel(LEJob j) {
    extern __shared__ double pos[];  // [N][3]
    __shared__ double red[3][LE_THREADS / 64];
    const int64_t w = blockIdx.x;
    const int N = j.n_up + j.n_dn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double* Rw = j.R + (size_t)w * N * 3;
    for (int q = tid; q < 3 * N; q += LE_THREADS) pos[q] = Rw[q];
    __syncthreads();
    double tsum = 0.0, jsum = 0.0, vsum = 0.0;
    for (int i = tid; i < N; i += LE_THREADS) {
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const bool up = i < j.n_up;
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, l = 0.0;
        for (int k = 0; k < N; ++k) {
            if (k == i) continue;
            const double dx = xi - pos[3 * k], dy = yi - pos[3 * k + 1], dz = zi - pos[3 * k + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double a = j.c_ee * ((up == (k < j.n_up)) ? 0.25 : 0.5);
            double u, du, d2u;
            pair_u(a, j.b_ee, r, u, du, d2u);
            const double ir = 1.0 / r;
            g0 += du * dx * ir;
            g1 += du * dy * ir;
            g2 += du * dz * ir;
            l += d2u + 2.0 * du * ir;
            if (k > i) {
                jsum += u;
                vsum += ir;
            }
        }
        for (int al = 0; al < j.n_atoms; ++al) {
            const double dx = xi - j.atom_xyz[3 * al], dy = yi - j.atom_xyz[3 * al + 1],
                         dz = zi - j.atom_xyz[3 * al + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double Za = j.Z[al];
            double u, du, d2u;
            pair_u(-j.c_en * Za, j.b_en, r, u, du, d2u);
            const double ir = 1.0 / r;
            g0 += du * dx * ir;
            g1 += du * dy * ir;
            g2 += du * dz * ir;
            l += d2u + 2.0 * du * ir;
            jsum += u;
            vsum -= Za * ir;
        }
        const size_t qi = (size_t)w * N + i;
        const double b0 = j.bd[3 * qi], b1 = j.bd[3 * qi + 1], b2 = j.bd[3 * qi + 2];
        // lap_i Psi / Psi = lap J + |grad J|^2 + 2 grad J . b_det + lap_i Det / Det
        tsum += l + (g0 * g0 + g1 * g1 + g2 * g2) + 2.0 * (g0 * b0 + g1 * b1 + g2 * b2) + j.ld[qi];
        j.drift[3 * qi] = g0 + b0;
        j.drift[3 * qi + 1] = g1 + b1;
        j.drift[3 * qi + 2] = g2 + b2;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        tsum += __shfl_xor(tsum, o);
        jsum += __shfl_xor(jsum, o);
        vsum += __shfl_xor(vsum, o);
    }
    if (lane == 0) {
        red[0][wave] = tsum;
        red[1][wave] = jsum;
        red[2][wave] = vsum;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0, jj = 0.0, v = j.v_nn;
        for (int k = 0; k < LE_THREADS / 64; ++k) {
            t += red[0][k];
            jj += red[1][k];
            v += red[2][k];
        }
        j.EL[w] = -0.5 * t + v;
        if (j.J) j.J[w] = jj;
        if (j.V) j.V[w] = v;
        const int8_t su = j.n_up ? j.sign[2 * w] : 1, sd = j.n_dn ? j.sign[2 * w + 1] : 1;
        if (j.psisign) j.psisign[w] = (int8_t)(su * sd);
        if (j.logpsi) j.logpsi[w] = jj + (j.n_up ? j.logdet[2 * w] : 0.0) + (j.n_dn ? j.logdet[2 * w + 1] : 0.0);
    }
}

// R' = (R + tau b) + sqrt(tau) eta, each product and sum rounded on its own.
__global__ void drift_diffuse_kernel(int64_t count, const double* __restrict__ R, const double* __restrict__ b,
                                     const double* __restrict__ eta, double tau, double st, double* __restrict__ out) {
#pragma clang fp contract(off)
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        const double m = tau * b[q];
        const double d = st * eta[q];
        out[q] = (R[q] + m) + d;
    }
}

__global__ void weights_kernel(int64_t W, const double* __restrict__ ELn, const double* __restrict__ ELo,
                               const int8_t* __restrict__ sn, const int8_t* __restrict__ so, double ET, double tau,
                               double* __restrict__ w) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= W) return;
    if (sn[k] == 0 || sn[k] != so[k]) {
        w[k] = 0.0;
        return;
    }
    const double e = (ELn[k] - ET) + (ELo[k] - ET);
    const double v = exp((-0.5 * tau) * e);
    w[k] = isfinite(v) ? v : 0.0;  // a non-finite local energy (or an overflow) drops the walker
}

// The cumulative weights in walker order, by one thread (the order of the
// sums fixes every selection).
__global__ void cumsum_kernel(int64_t W, const double* __restrict__ w, double* __restrict__ cum,
                              double* __restrict__ wsum) {
    if (threadIdx.x != 0) return;
    double c = 0.0;
    for (int64_t k = 0; k < W; ++k) {
        c += w[k];
        cum[k] = c;
    }
    *wsum = c;
}

// Draw m: the first walker whose cumulative weight exceeds u[m] times the
// total (the last walker if rounding leaves none); the population is kept
// when the total is not positive.
__global__ void select_kernel(int64_t W, const double* __restrict__ cum, const double* __restrict__ u,
                              int64_t* __restrict__ idx) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= W) return;
    const double c = cum[W - 1];
    if (!(c > 0.0)) {
        idx[m] = m;
        return;
    }
    const double x = u[m] * c;
    int64_t lo = 0, hi = W - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (x < cum[mid]) hi = mid;
        else lo = mid + 1;
    }
    idx[m] = lo;
}

// dst[m] = src[idx[m]] for records of `width` bytes (8-byte words when the
// width allows).
__global__ void gather_kernel(int64_t W, int64_t width, const int64_t* __restrict__ idx, const void* __restrict__ src,
                              void* __restrict__ dst) {
    const bool words = (width & 7) == 0;
    const int64_t per = words ? width / 8 : width;
    const int64_t total = W * per;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = q / per, c = q % per;
        const int64_t k = idx ? idx[m] : m;
        if (words) ((uint64_t*)dst)[m * per + c] = ((const uint64_t*)src)[k * per + c];
        else ((uint8_t*)dst)[m * per + c] = ((const uint8_t*)src)[k * per + c];
    }
}

static int grid_for(int64_t n, int block) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 65536)); }

static hipError_t launch_gather(int64_t W, int64_t width, const int64_t* idx, const void* src, void* dst, hipStream_t st) {
    if (W <= 0 || width <= 0) return hipSuccess;
    const int64_t per = (width & 7) == 0 ? width / 8 : width;
    gather_kernel<<<grid_for(W * per, 256), 256, 0, st>>>(W, width, idx, src, dst);
    return hipGetLastError();
}

static qsl_status local_energy_impl(qsl_system* sys, const qsl_local_args* a, hipStream_t st) {
    const int N = sys->d.n_up + sys->d.n_dn;
    LEJob j{};
    j.n_up = sys->d.n_up;
    j.n_dn = sys->d.n_dn;
    j.n_atoms = sys->d.n_atoms;
    j.atom_xyz = sys->d.atom_xyz;
    j.Z = sys->atom_Z;
    j.c_ee = sys->c_ee;
    j.b_ee = sys->b_ee;
    j.c_en = sys->c_en;
    j.b_en = sys->b_en;
    j.v_nn = sys->v_nn;
    j.W = a->W;
    j.R = a->R;
    j.bd = a->drift_det;
    j.ld = a->lap_det;
    j.logdet = a->logdet;
    j.sign = a->sign;
    j.EL = a->EL;
    j.drift = a->drift;
    j.logpsi = a->logpsi;
    j.psisign = a->psisign;
    j.J = a->J;
    j.V = a->V;
    ProfScope ps("local_energy", st);
    local_energy_kernel<<<(unsigned)a->W, LE_THREADS, (size_t)N * 3 * sizeof(double), st>>>(j);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QSL_OK : hip_fail(e, "local energy kernel");
}

static qsl_status check_local(const qsl_system* sys, const qsl_local_args* a) {
    if (!sys || !a) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (!sys->jastrow_set) return bad(QSL_ERR_INVALID_ARG, "qsl_set_jastrow was never called for this system");
    if (a->W < 0) return bad(QSL_ERR_INVALID_ARG, "W < 0");
    if (a->W > 0 && (!a->R || !a->drift_det || !a->lap_det || !a->logdet || !a->sign || !a->EL || !a->drift))
        return bad(QSL_ERR_INVALID_ARG, "NULL input or required output");
    if (sys->d.n_up + sys->d.n_dn > LE_MAX_ELEC) return bad(QSL_ERR_UNSUPPORTED, "more electrons than the local energy supports");
    return QSL_OK;
}

}  // namespace qsl

using namespace qsl;

extern "C" {

qsl_status qsl_set_jastrow(qsl_system* sys, const double* Z, double c_ee, double b_ee, double c_en, double b_en) {
    if (!sys || (!Z && sys->d.n_atoms > 0)) return bad(QSL_ERR_INVALID_ARG, "NULL system or charges");
    if (!(b_ee >= 0.0) || !(b_en >= 0.0) || !std::isfinite(c_ee) || !std::isfinite(c_en) || !std::isfinite(b_ee) ||
        !std::isfinite(b_en))
        return bad(QSL_ERR_INVALID_ARG, "Jastrow parameters must be finite, with b >= 0");
    const int na = sys->d.n_atoms;
    std::vector<double> xyz(3 * (size_t)na);
    for (int a = 0; a < na; ++a)
        if (!std::isfinite(Z[a]) || Z[a] < 0) return bad(QSL_ERR_INVALID_ARG, "nuclear charges must be finite and >= 0");
    hipError_t e;
    if (!sys->atom_Z && na > 0) {
        if ((e = hipMalloc(&sys->atom_Z, sizeof(double) * na)) != hipSuccess) return bad(QSL_ERR_OOM, "charges allocation");
    }
    if (na > 0 && (e = hipMemcpy(sys->atom_Z, Z, sizeof(double) * na, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "charges upload");
    if (na > 0 && (e = hipMemcpy(xyz.data(), sys->d.atom_xyz, sizeof(double) * 3 * na, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "atom positions");
    double vnn = 0.0;
    for (int a = 0; a < na; ++a)
        for (int b = a + 1; b < na; ++b) {
            const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1], dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            vnn += Z[a] * Z[b] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    sys->v_nn = vnn;
    sys->c_ee = c_ee;
    sys->b_ee = b_ee;
    sys->c_en = c_en;
    sys->b_en = b_en;
    sys->jastrow_set = true;
    return QSL_OK;
}

qsl_status qsl_local_energy(qsl_system* sys, const qsl_local_args* a, void* stream) {
    qsl_status r = check_local(sys, a);
    if (r != QSL_OK || a->W == 0) return r;
    return local_energy_impl(sys, a, (hipStream_t)stream);
}

qsl_status qsl_drift_diffuse(int64_t count, const double* R, const double* drift, const double* eta, double tau,
                             double* R_out, void* stream) {
    if (count < 0 || !(tau >= 0.0) || !std::isfinite(tau)) return bad(QSL_ERR_INVALID_ARG, "count < 0 or bad tau");
    if (count == 0) return QSL_OK;
    if (!R || !drift || !eta || !R_out) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("drift_diffuse", st);
    drift_diffuse_kernel<<<grid_for(count, 256), 256, 0, st>>>(count, R, drift, eta, tau, std::sqrt(tau), R_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QSL_OK : hip_fail(e, "drift-diffusion kernel");
}

qsl_status qsl_branch_weights(int64_t W, const double* EL_new, const double* EL_old, const int8_t* sign_new,
                              const int8_t* sign_old, double E_T, double tau, double* w, void* stream) {
    if (W < 0 || !std::isfinite(tau) || !std::isfinite(E_T)) return bad(QSL_ERR_INVALID_ARG, "W < 0 or bad tau / E_T");
    if (W == 0) return QSL_OK;
    if (!EL_new || !EL_old || !sign_new || !sign_old || !w) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("branch_weights", st);
    weights_kernel<<<grid_for(W, 256), 256, 0, st>>>(W, EL_new, EL_old, sign_new, sign_old, E_T, tau, w);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QSL_OK : hip_fail(e, "weights kernel");
}

qsl_status qsl_reconfigure(int64_t W, const double* w, const double* u, int64_t* idx, double* wsum, double* cum,
                           void* stream) {
    if (W < 0) return bad(QSL_ERR_INVALID_ARG, "W < 0");
    if (W == 0) return QSL_OK;
    if (!w || !u || !idx || !wsum || !cum) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("reconfigure", st);
    cumsum_kernel<<<1, 64, 0, st>>>(W, w, cum, wsum);
    select_kernel<<<grid_for(W, 256), 256, 0, st>>>(W, cum, u, idx);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QSL_OK : hip_fail(e, "reconfiguration kernels");
}

qsl_status qsl_gather_walkers(int64_t W, int64_t width, const int64_t* idx, const void* src, void* dst, void* stream) {
    if (W < 0 || width < 0) return bad(QSL_ERR_INVALID_ARG, "W or width < 0");
    if (W == 0 || width == 0) return QSL_OK;
    if (!idx || !src || !dst) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (src == dst) return bad(QSL_ERR_INVALID_ARG, "gather needs distinct source and destination");
    hipError_t e = launch_gather(W, width, idx, src, dst, (hipStream_t)stream);
    return e == hipSuccess ? QSL_OK : hip_fail(e, "gather kernel");
}

qsl_status qsl_dmc_workspace_size(int64_t W, int32_t n_elec, size_t* bytes) {
    if (!bytes || W < 0 || n_elec < 0) return bad(QSL_ERR_INVALID_ARG, "NULL bytes or negative size");
    const size_t w8 = round_up((size_t)W * 8, 256), wN = round_up((size_t)W * n_elec * 3 * 8, 256),
                 w1 = round_up((size_t)W, 256);
    *bytes = 4 * w8 + wN + w1 + 256;  // EL', log|Psi'|, w, cumulative w; drift'; sign'
    return QSL_OK;
}

}  // extern "C"

namespace qsl {

// Shared checks of the DMC calls; the plan's system and bound forward.
static qsl_status dmc_check(qsl_plan* plan, const qsl_dmc_args* a, qsl_system** sys, const qsl_fwd_args** f) {
    if (!plan || !a) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    *sys = plan_system(plan, a->sys_index);
    *f = plan_fwd(plan, a->sys_index);
    if (!*sys || !*f) return bad(QSL_ERR_INVALID_ARG, "dmc: system index out of range or never bound");
    if (a->W != plan_walkers(plan, a->sys_index)) return bad(QSL_ERR_SHAPE, "dmc: W differs from the plan");
    if (!(*sys)->jastrow_set) return bad(QSL_ERR_INVALID_ARG, "dmc: qsl_set_jastrow was never called for this system");
    if (!(*f)->drift || !(*f)->lap || !(*f)->logdet || !(*f)->sign)
        return bad(QSL_ERR_INVALID_ARG, "dmc: the plan must be bound with drift, lap, logdet and sign outputs");
    if (!a->R || !a->EL || !a->drift || !a->psisign) return bad(QSL_ERR_INVALID_ARG, "dmc: NULL state");
    if (a->R == (*f)->R) return bad(QSL_ERR_INVALID_ARG, "dmc: the population R must differ from the plan's bound R");
    if ((*sys)->d.n_up + (*sys)->d.n_dn > LE_MAX_ELEC) return bad(QSL_ERR_UNSUPPORTED, "dmc: too many electrons");
    return QSL_OK;
}

}  // namespace qsl

extern "C" {

qsl_status qsl_dmc_init(qsl_plan* plan, const qsl_dmc_args* a, void* stream) {
    qsl_system* sys = nullptr;
    const qsl_fwd_args* f = nullptr;
    qsl_status r = dmc_check(plan, a, &sys, &f);
    if (r != QSL_OK || a->W == 0) return r;
    hipStream_t st = (hipStream_t)stream;
    const int N = sys->d.n_up + sys->d.n_dn;
    hipError_t e = launch_gather(a->W, (int64_t)N * 3 * 8, nullptr, a->R, const_cast<double*>(f->R), st);
    if (e != hipSuccess) return hip_fail(e, "dmc: copy of the population");
    if ((r = qsl_plan_launch(plan, stream)) != QSL_OK) return r;
    qsl_local_args la{};
    la.W = a->W;
    la.R = f->R;
    la.drift_det = f->drift;
    la.lap_det = f->lap;
    la.logdet = f->logdet;
    la.sign = f->sign;
    la.EL = a->EL;
    la.drift = a->drift;
    la.psisign = a->psisign;
    la.logpsi = a->logpsi;
    return local_energy_impl(sys, &la, st);
}

qsl_status qsl_dmc_step(qsl_plan* plan, const qsl_dmc_args* a, void* stream) {
    qsl_system* sys = nullptr;
    const qsl_fwd_args* f = nullptr;
    qsl_status r = dmc_check(plan, a, &sys, &f);
    if (r != QSL_OK || a->W == 0) return r;
    if (!a->eta || !a->u || !a->idx || !a->wsum) return bad(QSL_ERR_INVALID_ARG, "dmc: NULL random numbers or outputs");
    const int N = sys->d.n_up + sys->d.n_dn;
    const int64_t W = a->W;
    size_t need = 0;
    qsl_dmc_workspace_size(W, N, &need);
    if (!a->ws || a->ws_bytes < need) return bad(QSL_ERR_WORKSPACE, "dmc: workspace missing or too small");
    char* ws = (char*)a->ws;
    const size_t w8 = round_up((size_t)W * 8, 256), wN = round_up((size_t)W * N * 3 * 8, 256);
    double* ELn = (double*)ws;
    double* lpn = (double*)(ws + w8);
    double* wt = (double*)(ws + 2 * w8);
    double* cum = (double*)(ws + 3 * w8);
    double* drn = (double*)(ws + 4 * w8);
    int8_t* sgn = (int8_t*)(ws + 4 * w8 + wN);
    hipStream_t st = (hipStream_t)stream;
    double* Rp = const_cast<double*>(f->R);
    // drift-diffusion from the current population into the plan's positions
    if ((r = qsl_drift_diffuse(W * N * 3, a->R, a->drift, a->eta, a->tau, Rp, stream)) != QSL_OK) return r;
    // Slater part at the new positions, then Jastrow, potential, E_L and drift
    if ((r = qsl_plan_launch(plan, stream)) != QSL_OK) return r;
    qsl_local_args la{};
    la.W = W;
    la.R = Rp;
    la.drift_det = f->drift;
    la.lap_det = f->lap;
    la.logdet = f->logdet;
    la.sign = f->sign;
    la.EL = ELn;
    la.drift = drn;
    la.psisign = sgn;
    la.logpsi = lpn;
    if ((r = local_energy_impl(sys, &la, st)) != QSL_OK) return r;
    // branching weights, reconfiguration, and the new population
    if ((r = qsl_branch_weights(W, ELn, a->EL, sgn, a->psisign, a->E_T, a->tau, wt, stream)) != QSL_OK) return r;
    if ((r = qsl_reconfigure(W, wt, a->u, a->idx, a->wsum, cum, stream)) != QSL_OK) return r;
    hipError_t e;
    ProfScope ps("gather", st);
    if ((e = launch_gather(W, (int64_t)N * 24, a->idx, Rp, a->R, st)) != hipSuccess ||
        (e = launch_gather(W, 8, a->idx, ELn, a->EL, st)) != hipSuccess ||
        (e = launch_gather(W, (int64_t)N * 24, a->idx, drn, a->drift, st)) != hipSuccess ||
        (e = launch_gather(W, 1, a->idx, sgn, a->psisign, st)) != hipSuccess ||
        (a->logpsi && (e = launch_gather(W, 8, a->idx, lpn, a->logpsi, st)) != hipSuccess))
        return hip_fail(e, "dmc: gather of the new population");
    return QSL_OK;
}

}  // extern "C"
