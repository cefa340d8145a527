// Screening and compaction of AO windows for a set of electron positions.
//
// An AO window (8 padded slots of one atom) survives for a set iff some
// electron of the set keeps some primitive of some shell meeting the window:
// min_k(gamma_k) r^2 <= T, decided in FP64 exactly as the AO evaluation does
// (threshold on the Gaussian part and atomic radius, section "Exploiting the
// highly localized character of atomic basis functions").  Surviving windows
// are written in ascending order with a wavefront ballot + block prefix,
// giving the set's list of AO indices (the paper's `indices` array, here at
// window granularity and shared by the set).
//
// Two kinds of sets:
//  electron tiles (forward, adjoint H): electron e of TE consecutive walkers,
//      tile = e * walker_blocks(W) + walker block;
//  walker groups (adjoint dA): electrons [32 t, 32 t + 32) of gw consecutive
//      walkers, group = t * ceil(W / gw) + walker block.
#include "qsl_internal.h"

namespace qsl {

constexpr int SCREEN_THREADS = 256;
static_assert(UNION_MAXWIN / 32 <= SCREEN_THREADS, "one bitmap word per thread");
// positions staged in LDS (the rest are read from L2): a tile has TE, a
// walker group up to gw * TE; the tile kernels keep their LDS small, so
// more of their workgroups share a CU
constexpr int SCREEN_MAXE_GROUP = 2048;

template <int MAXE>
__device__ __forceinline__ void screen_body(const Job& j, bool group, int* __restrict__ tile_nwin,
                                            int* __restrict__ tile_win, uint32_t* __restrict__ status, int bx) {
    const DevSys& s = j.s;
    const int spin = j.spin, n = j.n;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    __shared__ double ex[MAXE], ey[MAXE], ez[MAXE];
    __shared__ double bb[6];
    __shared__ double bred[SCREEN_THREADS / 64][6];
    __shared__ int wave_cnt[SCREEN_THREADS / 64];
    const int tile = bx;
    const int N = s.n_up + s.n_dn;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int eoff = spin ? s.n_up : 0;
    // position k of the set -> (walker, electron); `valid` drops the ragged
    // electrons of the last 32-electron range of a walker group
    int nall, w0, e0, ne, kstride;
    if (group) {
        const int gw = j.gw;
        const int ngw = (int)((W + gw - 1) / gw);
        const int t = tile / ngw, wb = tile % ngw;
        w0 = wb * gw;
        e0 = t * TE;
        ne = min(TE, n - e0);
        nall = (int)min<int64_t>(gw, W - w0) * TE;
        kstride = TE;
    } else {
        const int wbk = walker_blocks(W);
        const int e = tile / wbk, wb = tile % wbk;
        w0 = wb * TE;
        e0 = e;
        ne = 1;
        nall = (int)min<int64_t>(TE, W - w0);
        kstride = 1;
    }
    // tiles read their walkers in the order of wperm (positions w0 + k)
    const int* __restrict__ wp = group ? nullptr : j.wperm;
    auto kw = [&](int k) -> int64_t { return wp ? walker_of(wp, W, e0, w0 + k) : w0 + k / kstride; };
    auto ke = [&](int k) { return e0 + k % kstride; };
    auto valid = [&](int k) { return k % kstride < ne; };
    auto gpos = [&](int k) -> const double* { return R + ((size_t)kw(k) * N + eoff + ke(k)) * 3; };
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = tid; k < nall; k += SCREEN_THREADS) {
        double x = 0, y = 0, z = 0;
        if (valid(k)) {
            const double* r = gpos(k);
            x = r[0]; y = r[1]; z = r[2];
            lo[0] = fmin(lo[0], x); lo[1] = fmin(lo[1], y); lo[2] = fmin(lo[2], z);
            hi[0] = fmax(hi[0], x); hi[1] = fmax(hi[1], y); hi[2] = fmax(hi[2], z);
        }
        if (k < MAXE) { ex[k] = x; ey[k] = y; ez[k] = z; }
    }
    // bounding box of the set's electrons
    for (int o = 32; o >= 1; o >>= 1)
        for (int k = 0; k < 3; ++k) {
            lo[k] = fmin(lo[k], __shfl_xor(lo[k], o));
            hi[k] = fmax(hi[k], __shfl_xor(hi[k], o));
        }
    if (lane == 0)
        for (int k = 0; k < 3; ++k) { bred[wave][k] = lo[k]; bred[wave][3 + k] = hi[k]; }
    __syncthreads();
    if (tid == 0)
        for (int k = 0; k < 3; ++k) {
            double a = INFINITY, b = -INFINITY;
            for (int v = 0; v < SCREEN_THREADS / 64; ++v) { a = fmin(a, bred[v][k]); b = fmax(b, bred[v][3 + k]); }
            bb[k] = a; bb[3 + k] = b;
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
            // conservative prefilter: distance from the atom to the set's box
            double dx = fmax(fmax(bb[0] - qx, qx - bb[3]), 0.0);
            double dy = fmax(fmax(bb[1] - qy, qy - bb[4]), 0.0);
            double dz = fmax(fmax(bb[2] - qz, qz - bb[5]), 0.0);
            if (gm * (dx * dx + dy * dy + dz * dz) <= s.T * (1.0 + 1e-9)) {
                for (int k = 0; k < nall; ++k) {
                    if (!valid(k)) continue;
                    double px, py, pz;
                    if (k < MAXE) { px = ex[k]; py = ey[k]; pz = ez[k]; }
                    else { const double* r = gpos(k); px = r[0]; py = r[1]; pz = r[2]; }
                    const double tt = mul_exact(gm, dist2_exact(px - qx, py - qy, pz - qz));
                    active |= tt <= s.T;
                    // the smallest exponent of a dropped window decides its
                    // nearest primitive to the threshold: flag that walker
                    if (status && tt > s.T && tt - s.T <= 1e-12 * s.T) atomicOr(status + kw(k), QSL_STATUS_NEAR_TIE);
                    if (active && !status) break;
                }
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

__global__ __launch_bounds__(SCREEN_THREADS) void screen_kernel(Job j) {
    screen_body<TE>(j, false, j.nwin, j.win, j.status, blockIdx.x);
}

__global__ __launch_bounds__(SCREEN_THREADS) void screen_group_kernel(Job j) {
    screen_body<SCREEN_MAXE_GROUP>(j, true, j.gnwin, j.gwin, nullptr, blockIdx.x);
}

__global__ __launch_bounds__(SCREEN_THREADS) void screen_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs,
                [&](const Job& j, int bx, int, int) { screen_body<TE>(j, false, j.nwin, j.win, j.status, bx); });
}

__global__ __launch_bounds__(SCREEN_THREADS) void screen_group_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) {
        screen_body<SCREEN_MAXE_GROUP>(j, true, j.gnwin, j.gwin, nullptr, bx);
    });
}

// Blocks of the screening phase of a Job (groups of gw walkers, or tiles).
int screen_blocks(const Job& j, int group) {
    if (!j.n || !j.W) return 0;
    if (!group) return (int)electron_tiles(j.n, j.W);
    return tiles_per_walker(j.n) * (int)((j.W + j.gw - 1) / j.gw);
}

hipError_t launch_screen(const Job& j, int group, hipStream_t st) {
    if (group && j.gw < 1) return hipErrorInvalidValue;
    const int blocks = screen_blocks(j, group);
    if (!blocks) return hipSuccess;
    Job jj = j;
    jj.gx = blocks; jj.gy = 1; jj.gz = 1;
    if (group) screen_group_kernel<<<dim3((unsigned)blocks), SCREEN_THREADS, 0, st>>>(jj);
    else screen_kernel<<<dim3((unsigned)blocks), SCREEN_THREADS, 0, st>>>(jj);
    return hipGetLastError();
}

hipError_t launch_screen_batched(const Job* jobs, const int* prefix, int njobs, int grid, int group,
                                    hipStream_t st) {
    if (group) screen_group_batched<<<dim3((unsigned)grid), SCREEN_THREADS, 0, st>>>(jobs, prefix, njobs);
    else screen_batched<<<dim3((unsigned)grid), SCREEN_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// Walker-group lists as the union of tile lists already built on the same
// positions: electrons [32 t, 32 t + 32) of walkers [w0, w0 + gw) are
// covered by the tiles of those electrons in walker blocks w0 / TE ..
// (w0 + gw - 1) / TE, whose survivors follow the same rule.  The union is
// the group's own list, or a superset when gw is not a multiple of TE (the
// extra windows only carry AO values screened to zero).  One bit per window
// in LDS, compacted in ascending order.
__device__ __forceinline__ void group_union_body(const Job& j, int bx) {
    __shared__ uint32_t bits[UNION_MAXWIN / 32];
    __shared__ int wtot[SCREEN_THREADS / 64];
    const int n = j.n, nwin_all = j.s.n_win;
    const int64_t W = j.W;
    const int gw = j.gw;
    const int ngw = (int)((W + gw - 1) / gw);
    const int t = bx / ngw, wb = bx % ngw;
    const int64_t w0 = (int64_t)wb * gw, wend = min<int64_t>(W, w0 + gw);
    const int e0 = t * TE, ne = min(TE, n - e0);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwords = (nwin_all + 31) / 32;  // <= SCREEN_THREADS
    if (tid < nwords) bits[tid] = 0u;
    __syncthreads();
    const int wbk = walker_blocks(W);
    const int b0 = (int)(w0 / TE), nb = (int)((wend - 1) / TE) - b0 + 1;
    for (int tt = wave; tt < ne * nb; tt += SCREEN_THREADS / 64) {  // one wave per tile
        const int tile = (e0 + tt / nb) * wbk + b0 + tt % nb;
        const int cnt = j.nwin[tile];
        const int* lst = j.win + (size_t)tile * nwin_all;
        for (int q = lane; q < cnt; q += 64) {
            const int wd = lst[q];
            atomicOr(&bits[wd >> 5], 1u << (wd & 31));
        }
    }
    __syncthreads();
    const uint32_t word = tid < nwords ? bits[tid] : 0u;
    const int c = __popc(word);
    int x = c;  // inclusive prefix inside the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    int off = 0;
    for (int v = 0; v < wave; ++v) off += wtot[v];
    int pos = off + x - c;
    int* out = j.gwin + (size_t)bx * nwin_all;
    for (uint32_t wd = word; wd; wd &= wd - 1) out[pos++] = tid * 32 + __builtin_ctz(wd);
    if (tid == SCREEN_THREADS - 1) j.gnwin[bx] = off + x;
}

__global__ __launch_bounds__(SCREEN_THREADS) void group_union_kernel(Job j) { group_union_body(j, blockIdx.x); }

__global__ __launch_bounds__(SCREEN_THREADS) void group_union_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { group_union_body(j, bx); });
}

hipError_t launch_group_union(const Job& j, hipStream_t st) {
    if (j.gw < 1 || j.s.n_win > UNION_MAXWIN) return hipErrorInvalidValue;
    const int blocks = screen_blocks(j, 1);
    if (!blocks) return hipSuccess;
    Job jj = j;
    jj.gx = blocks; jj.gy = 1; jj.gz = 1;
    group_union_kernel<<<dim3((unsigned)blocks), SCREEN_THREADS, 0, st>>>(jj);
    return hipGetLastError();
}

hipError_t launch_group_union_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    group_union_batched<<<dim3((unsigned)grid), SCREEN_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// Walker order of each electron index: the walkers of a segment of 4096 by
// the Morton code of electron e's position (10 bits per axis over the
// system box, positions outside it clamped), ties by walker index, with a
// bitonic sort of (code, index) keys in LDS.  wperm[e][k] = walker at
// position k.  Walkers whose electron e is close in space then share tiles
// and walker groups, whose survivor unions are tighter.
constexpr int WS_SEG = 4096;

__device__ __forceinline__ uint32_t spread10(uint32_t v) {  // bit i -> bit 3 i
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ void wsort_body(const Job& j, int bx) {
    __shared__ uint64_t key[WS_SEG];
    const DevSys& s = j.s;
    const int64_t W = j.W;
    const int nseg = (int)((W + WS_SEG - 1) / WS_SEG);
    const int e = bx / nseg, seg = bx % nseg;
    const int64_t s0 = (int64_t)seg * WS_SEG;
    const int m = (int)min<int64_t>(WS_SEG, W - s0);
    int P = 64;
    while (P < m) P <<= 1;
    const int N = s.n_up + s.n_dn, eoff = j.spin ? s.n_up : 0;
    const int tid = threadIdx.x;
    for (int k = tid; k < P; k += SCREEN_THREADS) {
        uint64_t v = ~0ull;  // padding sorts last
        if (k < m) {
            const double* r = j.R + ((size_t)(s0 + k) * N + eoff + e) * 3;
            uint32_t code = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double u = (r[a] - s.box[a]) / (s.box[3 + a] - s.box[a]) * 1023.0;
                const uint32_t q = u > 0.0 ? (u < 1023.0 ? (uint32_t)u : 1023u) : 0u;  // NaN -> 0
                code |= spread10(q) << a;
            }
            v = ((uint64_t)code << 32) | (uint32_t)k;
        }
        key[k] = v;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += SCREEN_THREADS) {
                const int i = 2 * t - (t & (stride - 1));
                const bool up = (i & size) == 0;
                const uint64_t a = key[i], b = key[i + stride];
                if ((a > b) == up) {
                    key[i] = b;
                    key[i + stride] = a;
                }
            }
            __syncthreads();
        }
    int* out = const_cast<int*>(j.wperm) + (size_t)e * W + s0;
    for (int k = tid; k < m; k += SCREEN_THREADS) out[k] = (int)(s0 + (int64_t)(uint32_t)key[k]);
}

__global__ __launch_bounds__(SCREEN_THREADS) void wsort_kernel(Job j) { wsort_body(j, blockIdx.x); }

__global__ __launch_bounds__(SCREEN_THREADS) void wsort_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { wsort_body(j, bx); });
}

int wsort_blocks(const Job& j) {
    if (!j.n || !j.W || !j.wperm) return 0;
    return j.n * (int)((j.W + WS_SEG - 1) / WS_SEG);
}

hipError_t launch_wsort(const Job& j, hipStream_t st) {
    const int blocks = wsort_blocks(j);
    if (!blocks) return hipSuccess;
    wsort_kernel<<<dim3((unsigned)blocks), SCREEN_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_wsort_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    wsort_batched<<<dim3((unsigned)grid), SCREEN_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// Slot lists of the adjoint's dA by electron: for walker group g (gw
// walkers) of electron index e, the ascending slots whose smallest exponent
// passes the screening test, gmin r^2 <= T in the exact FP64 arithmetic of
// the forward, for at least one walker of the group: every slot with a
// surviving primitive for some walker, and only those (a slot none of whose
// primitives survives for any walker adds nothing).  Candidates are the
// windows of the forward's tile lists of electron e over the group's walker
// blocks; each wave decides whole windows, stopping early once every slot
// of a window is in.  Output: gnwin[group] and gwin[group][WIN * n_win].
constexpr int GS_POS = 512;  // walker positions staged in LDS at a time

__device__ __forceinline__ void group_slots_body(const Job& j, int bx) {
    __shared__ uint32_t bits[UNION_MAXWIN / 32];
    __shared__ int uw[UNION_MAXWIN];
    __shared__ uint8_t sm[UNION_MAXWIN];
    __shared__ double ep[GS_POS][3];
    __shared__ int wtot[SCREEN_THREADS / 64];
    const DevSys& s = j.s;
    const int nwin_all = s.n_win;
    const int64_t W = j.W;
    const int gw = j.gw;
    const int ngw = (int)((W + gw - 1) / gw);
    const int e = bx / ngw, g = bx % ngw;
    const int64_t w0 = (int64_t)g * gw, wend = min<int64_t>(W, w0 + gw);
    const int N = s.n_up + s.n_dn, eoff = j.spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NWAVE = SCREEN_THREADS / 64;
    const double T = s.T;
    const int nwords = (nwin_all + 31) / 32;
    if (tid < nwords) bits[tid] = 0u;
    __syncthreads();
    // candidate windows: the union of the tile lists of electron e
    const int wbk = walker_blocks(W);
    const int b0 = (int)(w0 / TE), nb = (int)((wend - 1) / TE) - b0 + 1;
    for (int tt = wave; tt < nb; tt += NWAVE) {
        const int tile = e * wbk + b0 + tt;
        const int cnt = j.nwin[tile];
        const int* lst = j.win + (size_t)tile * nwin_all;
        for (int q = lane; q < cnt; q += 64) {
            const int wd = lst[q];
            atomicOr(&bits[wd >> 5], 1u << (wd & 31));
        }
    }
    __syncthreads();
    int U;
    {
        const uint32_t word = tid < nwords ? bits[tid] : 0u;
        const int c = __popc(word);
        int x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wtot[wave] = x;
        __syncthreads();
        int off = 0;
        U = 0;
        for (int v = 0; v < NWAVE; ++v) {
            if (v < wave) off += wtot[v];
            U += wtot[v];
        }
        int pos = off + x - c;
        for (uint32_t wd = word; wd; wd &= wd - 1) uw[pos++] = tid * 32 + __builtin_ctz(wd);
    }
    for (int k = tid; k < U; k += SCREEN_THREADS) sm[k] = 0;
    // slot masks, positions staged GS_POS walkers at a time
    const SlotRec* __restrict__ srec = s.slot_rec;
    for (int64_t p0 = w0; p0 < wend; p0 += GS_POS) {
        const int np = (int)min<int64_t>(GS_POS, wend - p0);
        __syncthreads();  // uw / sm written; the previous positions are no longer read
        for (int q = tid; q < np * 3; q += SCREEN_THREADS)
            ep[q / 3][q % 3] = j.R[((size_t)walker_of(j.wperm, W, e, p0 + q / 3) * N + eoff + e) * 3 + q % 3];
        __syncthreads();
        for (int k = wave; k < U; k += NWAVE) {
            const SlotRec* rq = srec + (size_t)uw[k] * WIN;
            uint32_t full = 0;
            double gm[WIN];
#pragma unroll
            for (int jj = 0; jj < WIN; ++jj) {
                gm[jj] = rq[jj].gmin;
                full |= (gm[jj] < INFINITY ? 1u : 0u) << jj;
            }
            uint32_t m = sm[k];
            const double qx = rq->pos[0], qy = rq->pos[1], qz = rq->pos[2];
            for (int wl = 0; wl < np && m != full; wl += 64) {
                uint32_t mine = 0;
                if (wl + lane < np) {
                    const double r2 = dist2_exact(ep[wl + lane][0] - qx, ep[wl + lane][1] - qy, ep[wl + lane][2] - qz);
#pragma unroll
                    for (int jj = 0; jj < WIN; ++jj)
                        if (!((m >> jj) & 1u) && mul_exact(gm[jj], r2) <= T) mine |= 1u << jj;
                }
#pragma unroll
                for (int jj = 0; jj < WIN; ++jj) m |= (__ballot((mine >> jj) & 1u) != 0ull ? 1u : 0u) << jj;
            }
            if (lane == 0) sm[k] = (uint8_t)m;
        }
    }
    __syncthreads();
    // compaction: thread tid takes windows [k0, k1) in order
    const int per = (U + SCREEN_THREADS - 1) / SCREEN_THREADS;
    const int k0 = min(U, tid * per), k1 = min(U, k0 + per);
    int c = 0;
    for (int k = k0; k < k1; ++k) c += __popc((uint32_t)sm[k]);
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();  // wtot of the window compaction is no longer read
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    int off = 0;
    for (int v = 0; v < wave; ++v) off += wtot[v];
    int pos = off + x - c;
    int* out = j.gwin + (size_t)bx * WIN * nwin_all;
    for (int k = k0; k < k1; ++k)
        for (uint32_t mm = sm[k]; mm; mm &= mm - 1) out[pos++] = uw[k] * WIN + __builtin_ctz(mm);
    if (tid == SCREEN_THREADS - 1) j.gnwin[bx] = off + x;
}

__global__ __launch_bounds__(SCREEN_THREADS) void group_slots_kernel(Job j) { group_slots_body(j, blockIdx.x); }

__global__ __launch_bounds__(SCREEN_THREADS) void group_slots_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { group_slots_body(j, bx); });
}

int group_slots_blocks(const Job& j) {
    if (!j.n || !j.W || j.gw < 1) return 0;
    return j.n * (int)((j.W + j.gw - 1) / j.gw);
}

hipError_t launch_group_slots(const Job& j, hipStream_t st) {
    if (j.gw < 1 || j.s.n_win > UNION_MAXWIN) return hipErrorInvalidValue;
    const int blocks = group_slots_blocks(j);
    if (!blocks) return hipSuccess;
    Job jj = j;
    jj.gx = blocks; jj.gy = 1; jj.gz = 1;
    group_slots_kernel<<<dim3((unsigned)blocks), SCREEN_THREADS, 0, st>>>(jj);
    return hipGetLastError();
}

hipError_t launch_group_slots_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    group_slots_batched<<<dim3((unsigned)grid), SCREEN_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

}  // namespace qsl
