// Adjoint of L = sum_w sum_s g[w][s] log|det D^s_w| (not in the paper: the
// chain rule through the MO expansion (mo) and D_ij = phi_i(r_j)).
//
// With G[e][i] = g Dinv[e][i] = dL/dC_1[e][i]:
//   dA^s[i][j] = sum_w sum_e G[e][i] chi_j(r_e)
//   dR_e       = sum_j H[e][j] grad chi_j(r_e),  H[e][j] = sum_i G[e][i] a_ij
// over the screened survivors (held fixed).  The AO values and gradients
// are recomputed here, tile by tile, with the forward's window lists; they
// are never stored by the forward.  One workgroup owns a tile of 32
// electrons and a block of 32 MOs; dA and dR are accumulated with atomics.
#include "qsl_internal.h"

namespace qsl {

constexpr int BW_THREADS = 256;
constexpr int BW_MB = 32;  // MOs per workgroup
constexpr int BW_KW = 8;   // windows per chunk

template <typename T>
__global__ __launch_bounds__(BW_THREADS) void backward_kernel(DevSys s, int spin, int n, int tpw, int ldn,
                                                              const double* __restrict__ R,
                                                              const int* __restrict__ tile_nwin,
                                                              const int* __restrict__ tile_win,
                                                              const T* __restrict__ AT,
                                                              const double* __restrict__ Dinv,
                                                              const double* __restrict__ g,
                                                              double* __restrict__ dR, double* __restrict__ dA) {
    constexpr int KC = BW_KW * WIN;
    __shared__ double epos[TE][3];
    __shared__ int wq[BW_KW];
    __shared__ T G[TE][BW_MB + 1];
    __shared__ T Bv[4][TE][KC + 1];
    __shared__ T red[BW_THREADS / TE][TE][3];

    const int tile = blockIdx.x;
    const int i0 = blockIdx.y * BW_MB;
    const int w = tile / tpw;
    const int e0 = (tile % tpw) * TE;
    const int ne = min(TE, n - e0);
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x;

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)w * N + eoff + e0 + e) * 3 + k] : 0.0;
    }
    const double gw = g[2 * w + spin];
    for (int q = tid; q < TE * BW_MB; q += BW_THREADS) {
        const int e = q / BW_MB, ii = q % BW_MB;
        const bool ok = e < ne && i0 + ii < n;
        G[e][ii] = ok ? (T)(gw * Dinv[((size_t)w * n + e0 + e) * n + i0 + ii]) : T(0);
    }
    const int nwin = tile_nwin[tile];
    const int* wins = tile_win + (size_t)tile * s.n_win;
    T dr[3] = {0, 0, 0};
    bool tie = false;
    __syncthreads();

    for (int c0 = 0; c0 < nwin; c0 += BW_KW) {
        {   // AO value and gradient of (electron, window) into LDS
            const int e = tid & (TE - 1), wl = tid / TE;
            const int q = c0 + wl < nwin ? wins[c0 + wl] : -1;
            if (e == 0) wq[wl] = q;
            T vals[4][WIN];
            for (int d = 0; d < 4; ++d)
                for (int j = 0; j < WIN; ++j) vals[d][j] = T(0);
            if (q >= 0 && e < ne) {
                const int at = s.win_atom[q];
                const double dx = epos[e][0] - s.atom_xyz[3 * at];
                const double dy = epos[e][1] - s.atom_xyz[3 * at + 1];
                const double dz = epos[e][2] - s.atom_xyz[3 * at + 2];
                const double r2 = dist2_exact(dx, dy, dz);
                int prev = -1;
                T gg = 0, g1 = 0, g2 = 0;
                for (int j = 0; j < WIN; ++j) {
                    const int slot = q * WIN + j;
                    const int sh = s.slot_shell[slot];
                    if (sh < 0) continue;
                    if (sh != prev) { shell_radial<T>(s, sh, r2, gg, g1, g2, tie); prev = sh; }
                    T v[5];
                    slot_values<T>(s, slot, (T)dx, (T)dy, (T)dz, gg, g1, g2, v);
                    for (int d = 0; d < 4; ++d) vals[d][j] = v[d];
                }
            }
            for (int d = 0; d < 4; ++d)
                for (int j = 0; j < WIN; ++j) Bv[d][e][wl * WIN + j] = vals[d][j];
        }
        __syncthreads();
        {   // dA[i][slot] += sum_e G[e][i] chi_slot(r_e)
            const int ii = tid & (BW_MB - 1), sg = tid / BW_MB;  // 8 slot groups of 8 slots
            if (i0 + ii < n) {
                for (int j = 0; j < WIN; ++j) {
                    const int c = sg * WIN + j;
                    const int q = wq[c / WIN];
                    if (q < 0) continue;
                    const int ao = s.slot_ao[q * WIN + (c % WIN)];
                    if (ao < 0) continue;
                    T v = 0;
                    for (int e = 0; e < TE; ++e) v += G[e][ii] * Bv[0][e][c];
                    if (dA && v != T(0)) atomicAdd(dA + (size_t)(i0 + ii) * s.n_basis + ao, (double)v);
                }
            }
        }
        {   // H[e][slot] = sum_i G[e][i] a_i,slot ; dR_e += H grad chi
            const int e = tid & (TE - 1), sg = tid / TE;
            for (int j = 0; j < WIN; ++j) {
                const int c = sg * WIN + j;
                const int q = wq[c / WIN];
                if (q < 0) continue;
                const int slot = q * WIN + (c % WIN);
                const T* a = AT + (size_t)slot * ldn + i0;
                T h = 0;
                for (int ii = 0; ii < BW_MB; ++ii) h += G[e][ii] * a[ii];
                dr[0] += h * Bv[1][e][c];
                dr[1] += h * Bv[2][e][c];
                dr[2] += h * Bv[3][e][c];
            }
        }
        __syncthreads();
    }
    {
        const int e = tid & (TE - 1), sg = tid / TE;
        for (int k = 0; k < 3; ++k) red[sg][e][k] = dr[k];
    }
    __syncthreads();
    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        if (e < ne && dR) {
            T v = 0;
            for (int q = 0; q < BW_THREADS / TE; ++q) v += red[q][e][k];
            atomicAdd(dR + ((size_t)w * N + eoff + e0 + e) * 3 + k, (double)v);
        }
    }
}

hipError_t launch_backward(const DevSys& s, const DevMO& mo, int spin, int mode, int64_t W, const double* R,
                           const int* tile_nwin, const int* tile_win, const double* Dinv, const double* g,
                           double* dR, double* dA, hipStream_t st) {
    const int n = n_spin(s, spin);
    const int tpw = tiles_per_walker(n);
    const int64_t tiles = W * tpw;
    if (!tiles || (!dR && !dA)) return hipSuccess;
    dim3 grid((unsigned)tiles, (n + BW_MB - 1) / BW_MB);
    if (mode == QSL_FP64)
        backward_kernel<double><<<grid, BW_THREADS, 0, st>>>(s, spin, n, tpw, mo.ldn, R, tile_nwin, tile_win,
                                                             mo.AT64, Dinv, g, dR, dA);
    else
        backward_kernel<float><<<grid, BW_THREADS, 0, st>>>(s, spin, n, tpw, mo.ldn, R, tile_nwin, tile_win,
                                                            mo.AT32, Dinv, g, dR, dA);
    return hipGetLastError();
}

}  // namespace qsl
