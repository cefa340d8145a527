// Screening and compaction (per tile of 32 electrons of one walker and spin).
//
// An AO window (8 padded slots of one atom) survives for a tile iff some
// electron of the tile keeps some primitive of some shell meeting the window:
// min_k(gamma_k) r^2 <= T, decided in FP64 exactly as the AO evaluation does
// (threshold on the Gaussian part and atomic radius, section "Exploiting the
// highly localized character of atomic basis functions").  Surviving windows
// are written in ascending order with a wavefront ballot + block prefix,
// giving the tile's list of AO indices (the paper's `indices` array, here at
// window granularity and shared by the tile).
#include "qsl_internal.h"

namespace qsl {

constexpr int SCREEN_THREADS = 256;

__global__ __launch_bounds__(SCREEN_THREADS) void screen_kernel(DevSys s, int spin, int n, int tpw,
                                                                 const double* __restrict__ R,
                                                                 int* __restrict__ tile_nwin,
                                                                 int* __restrict__ tile_win,
                                                                 uint32_t* __restrict__ status) {
    __shared__ double ex[TE], ey[TE], ez[TE];
    __shared__ double bb[6];
    __shared__ int wave_cnt[SCREEN_THREADS / 64];
    const int tile = blockIdx.x;
    const int w = tile / tpw;
    const int e0 = (tile % tpw) * TE;
    const int ne = min(TE, n - e0);
    const int N = s.n_up + s.n_dn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int eoff = spin ? s.n_up : 0;

    if (tid < 64) {
        double x = 0, y = 0, z = 0;
        bool ok = tid < ne;
        if (ok) {
            const double* r = R + ((size_t)w * N + eoff + e0 + tid) * 3;
            x = r[0]; y = r[1]; z = r[2];
            ex[tid] = x; ey[tid] = y; ez[tid] = z;
        }
        // bounding box of the tile's electrons
        double lo[3] = {ok ? x : INFINITY, ok ? y : INFINITY, ok ? z : INFINITY};
        double hi[3] = {ok ? x : -INFINITY, ok ? y : -INFINITY, ok ? z : -INFINITY};
        for (int o = 32; o >= 1; o >>= 1)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], __shfl_xor(lo[k], o));
                hi[k] = fmax(hi[k], __shfl_xor(hi[k], o));
            }
        if (tid == 0)
            for (int k = 0; k < 3; ++k) { bb[k] = lo[k]; bb[3 + k] = hi[k]; }
    }
    __syncthreads();

    int base = 0;
    int* out = tile_win + (size_t)tile * s.n_win;
    for (int q0 = 0; q0 < s.n_win; q0 += SCREEN_THREADS) {
        const int q = q0 + tid;
        bool active = false;
        if (q < s.n_win) {
            const int at = s.win_atom[q];
            const double gm = s.win_gmin[q];
            const double qx = s.atom_xyz[3 * at], qy = s.atom_xyz[3 * at + 1], qz = s.atom_xyz[3 * at + 2];
            // conservative prefilter: distance from the atom to the tile's box
            double dx = fmax(fmax(bb[0] - qx, qx - bb[3]), 0.0);
            double dy = fmax(fmax(bb[1] - qy, qy - bb[4]), 0.0);
            double dz = fmax(fmax(bb[2] - qz, qz - bb[5]), 0.0);
            if (gm * (dx * dx + dy * dy + dz * dz) <= s.T * (1.0 + 1e-9)) {
                bool tie = false;
                for (int e = 0; e < ne; ++e) {
                    const double t = __dmul_rn(gm, dist2_exact(ex[e] - qx, ey[e] - qy, ez[e] - qz));
                    active |= t <= s.T;
                    // the smallest exponent of a dropped window decides its
                    // nearest primitive to the threshold
                    tie |= t > s.T && t - s.T <= 1e-12 * s.T;
                }
                if (tie && status) atomicOr(status + w, QSL_STATUS_NEAR_TIE);
            }
        }
        const uint64_t m = __ballot(active);
        if (lane == 0) wave_cnt[wave] = __popcll(m);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int k = 0; k < SCREEN_THREADS / 64; ++k) {
            woff += k < wave ? wave_cnt[k] : 0;
            tot += wave_cnt[k];
        }
        if (active) {
            const int pos = base + woff + __popcll(m & ((1ull << lane) - 1ull));
            out[pos] = q;
        }
        base += tot;
        __syncthreads();
    }
    if (tid == 0) tile_nwin[tile] = base;
}

hipError_t launch_screen(const DevSys& s, int spin, int64_t W, const double* R, int* tile_nwin, int* tile_win,
                         uint32_t* status, hipStream_t st) {
    const int n = n_spin(s, spin);
    const int tpw = tiles_per_walker(n);
    const int64_t tiles = W * tpw;
    if (tiles == 0) return hipSuccess;
    screen_kernel<<<dim3((unsigned)tiles), SCREEN_THREADS, 0, st>>>(s, spin, n, tpw, R, tile_nwin, tile_win, status);
    return hipGetLastError();
}

}  // namespace qsl
