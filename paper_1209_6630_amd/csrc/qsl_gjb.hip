// Blocked FP64 Gauss-Jordan for 224 < n <= 1024: log|det|, sign and
// inverse of the Slater matrices too large for the register-resident
// kernel (inversion step, section "Overall performance of QMC=Chem").
//
// The elimination is the same as the unblocked one: at step k the pivot is
// the largest |D[b][k]| over rows b not yet used (smallest b on exact ties),
// pivot rows are never moved, and the inverse is un-permuted at the end.
// It runs on a row-major FP64 copy M[b][a] = D[b][a] in the workspace
// (row b = MO, column a = electron), made by an LDS-tiled transpose of C_1.
//
// Per panel of NB = 32 columns, two kernels:
//  panel   one 512-thread workgroup per matrix reduces the panel columns
//          (each thread holds the panel part of two rows in registers; one
//          barrier per column: every wave publishes its best row, all
//          threads pick the winner from LDS), stores the reduced panel L and
//          copies the panel's pivot rows T[k][a] = M[p_k][a].
//  update  the composite of the panel's NB elementary steps acts on any
//          other column v through its pivot rows only:
//              v <- (v with the panel's pivot rows set to 0) + L v_P.
//          That rank-NB update of the whole matrix runs on
//          v_mfma_f64_16x16x4f64 in output tiles of 16 rows b x 16 columns
//          a.  Eight workgroups per matrix (two halves of the rows b x four
//          contiguous ranges of column tiles); each wave keeps its four
//          16-row strips of L in registers and streams the tiles.
// Then a finish kernel writes D^-1[e][i] = M[p_e][invp(i)] (row p_e of M
// staged in LDS, written out permuted), log|det| and sign.
//
// Traffic: the matrix is read and written once per panel (n^3 / NB x 16
// bytes per matrix); flops 2 n^3 per matrix.  Separate kernels give each
// phase its own register budget and occupancy.
#include <algorithm>

#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(4))) double f64x4;

constexpr int GJB_NB = GJ_PANEL;
constexpr int GJB_COPY_BLOCKS = 8;  // init / finish blocks per matrix

// Launch shapes by the largest n served (NMX = 256 or GJ_NMAX): threads of
// the panel / init / finish workgroups and of the update workgroups, rows
// per panel thread, 16-row strips per update wave, row halves and column
// ranges per matrix in the update.
template <int NMX>
struct GjbCfg {
    static constexpr int PT = NMX >= 512 ? 512 : 256;
    static constexpr int PWAVES = PT / 64;
    static constexpr int RPT = NMX / PT;
    static constexpr int UT = PT;
    static constexpr int UWAVES = UT / 64;
    static constexpr int SPW = 4;
    static constexpr int HALVES = NMX / 16 / UWAVES / SPW;
    static constexpr int CHUNKS = 4;
    static constexpr int UPD_BLOCKS = HALVES * CHUNKS;
    static_assert(HALVES >= 1 && RPT >= 1, "launch shape");
};

struct GjbState {
    double ld;  // sum log|pivot|
    int neg;    // negative pivots
    int flag;   // 0 ok, 1 zero pivot (singular), 2 non-finite pivot
};

// Per-matrix workspace (gj_ws_doubles(n) doubles).
struct GjbView {
    double* M;       // [n][ld] row-major D, then the elimination
    double* Tg;      // [NB][ld] pivot rows of the current panel
    int ld;          // row stride: n rounded up to 16 (128-byte rows)
    int* perm;       // [n] pivot row of step k
    uint8_t* used;   // [n] row already a pivot
    GjbState* st;
};

__device__ __forceinline__ GjbView gjb_view(const Job& j, int w) {
    const int n = j.n;
    GjbView v;
    v.M = j.gjws + (size_t)w * gj_ws_doubles(n);
    v.ld = gj_ld(n);
    v.Tg = v.M + (size_t)v.ld * n;
    v.perm = (int*)(v.Tg + (size_t)v.ld * GJB_NB);
    v.used = (uint8_t*)(v.perm + n);
    v.st = (GjbState*)((char*)v.perm + (((size_t)5 * n + 7) / 8) * 8);
    return v;
}

// Block -> (Job, matrix, sub-block): one Job by value (BATCHED = false), or
// a plan's Jobs through the prefix sums of their matrix counts.  Separate
// instantiations keep one inlined copy of the body per kernel.
template <bool BATCHED, typename F>
__device__ __forceinline__ void gjb_block(const Job& single, const Job* __restrict__ jobs,
                                          const int* __restrict__ prefix, int njobs, int mult, F body) {
    const int b = blockIdx.x / mult, sub = blockIdx.x % mult;
    if constexpr (!BATCHED) {
        if (b < single.W) body(single, b, sub);
    } else {
        if (b >= prefix[njobs]) return;
        const int ji = __builtin_amdgcn_readfirstlane(find_job(prefix, njobs, b));
        body(jobs[ji], b - prefix[ji], sub);
    }
}

// (|value|, row) argmax over the wavefront, smallest row on exact ties;
// uniform result.
__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
    argmax_step<0xB1>(best, bi);
    argmax_step<0x4E>(best, bi);
    argmax_step<0x141>(best, bi);
    argmax_step<0x140>(best, bi);
    double sb = readlane_f64(best, 0);
    int si = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
    for (int rw = 1; rw < 4; ++rw) {
        const double ob = readlane_f64(best, 16 * rw);
        const int oi = __builtin_amdgcn_readlane(bi, 16 * rw);
        if (ob > sb || (ob == sb && oi < si)) { sb = ob; si = oi; }
    }
    best = sb;
    bi = si;
}

// ------------------------------------------------------------------ init
// M[b][a] = D[b][a] = C_1[a][b] promoted to FP64 (32 x 32 tiles through
// LDS: coalesced reads of C_1 rows, coalesced writes of M rows); row flags
// and state reset.
template <int NMX, typename Tin>
__device__ __forceinline__ void gjb_init_body(const Job& j, int w, int sub) {
    constexpr int GJB_PT = GjbCfg<NMX>::PT;
    const int n = j.n;
    const size_t nn = (size_t)n * n;
    const GjbView v = gjb_view(j, w);
    const Tin* __restrict__ C1 = (const Tin*)j.C + (size_t)w * 5 * nn;
    __shared__ double tile[32][33];
    const int tid = threadIdx.x;
    const int nt = (n + 31) >> 5;
    constexpr int RP = GJB_PT / 32;  // tile rows per pass
    const int tx = tid & 31, ty = tid >> 5;
    for (int t = sub; t < nt * nt; t += GJB_COPY_BLOCKS) {
        const int ta = t / nt, tb = t % nt;  // source rows a (C_1), columns b
#pragma unroll
        for (int h = 0; h < 32 / RP; ++h) {
            const int a = 32 * ta + ty + RP * h, b = 32 * tb + tx;
            tile[ty + RP * h][tx] = (a < n && b < n) ? (double)C1[(size_t)a * n + b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 32 / RP; ++h) {
            const int b = 32 * tb + ty + RP * h, a = 32 * ta + tx;
            if (a < n && b < n) v.M[(size_t)b * v.ld + a] = tile[tx][ty + RP * h];
        }
        __syncthreads();
    }
    if (sub == 0) {
        for (int b = tid; b < n; b += GJB_PT) v.used[b] = 0;
        if (tid == 0) {
            v.st->ld = 0.0;
            v.st->neg = 0;
            v.st->flag = 0;
        }
    }
}

template <int NMX, bool BATCHED, typename Tin>
__global__ __launch_bounds__(GjbCfg<NMX>::PT) void gjb_init_kernel(Job single, const Job* jobs, const int* prefix,
                                                                    int njobs) {
    gjb_block<BATCHED>(single, jobs, prefix, njobs, GJB_COPY_BLOCKS,
                       [&](const Job& j, int w, int sub) __attribute__((always_inline)) { gjb_init_body<NMX, Tin>(j, w, sub); });
}

// ----------------------------------------------------------------- panel
template <int NMX>
__device__ __forceinline__ void gjb_panel_body(const Job& j, int w, int k0) {
    using C = GjbCfg<NMX>;
    constexpr int NB = GJB_NB, RPT = C::RPT, GJB_PT = C::PT, GJB_PWAVES = C::PWAVES;
    const int n = j.n;
    if (k0 >= n) return;
    const GjbView v = gjb_view(j, w);
    if (v.st->flag) return;  // singular earlier: nothing left to do
    __shared__ double cand_a[2][GJB_PWAVES];
    __shared__ int cand_i[2][GJB_PWAVES];
    __shared__ double cand_row[2][GJB_PWAVES][NB];
    __shared__ int perm_l[NB];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kn = min(NB, n - k0);

    double P[RPT][NB];  // P[r][k] = M[b][k0 + k], b = tid + 512 r
    bool used[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int b = tid + GJB_PT * r;
        const int bl = min(b, n - 1);  // loads at clamped (valid) addresses, then select
        used[r] = b >= n || v.used[bl];
        const double* row = v.M + (size_t)bl * v.ld + k0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const double x = row[min(k, kn - 1)];
            P[r][k] = (b < n && k < kn) ? x : 0.0;
        }
    }
    double ld = 0.0;
    int neg = 0;
#pragma unroll 1
    for (int k = 0; k < kn; ++k) {
        const int buf = k & 1;
        double x[RPT];  // P[r][k] (k is not a compile-time index: select)
        double best = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            x[r] = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q) x[r] = q == k ? P[r][q] : x[r];
            const double a = fabs(x[r]);
            if (!used[r] && a > best) { best = a; bi = tid + GJB_PT * r; }  // NaN never wins
        }
        wave_argmax(best, bi);
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (tid + GJB_PT * r == bi) {
#pragma unroll
                for (int q = 0; q < NB; ++q) cand_row[buf][wave][q] = P[r][q];
            }
        if (lane == 0) {
            cand_a[buf][wave] = best;
            cand_i[buf][wave] = bi;
        }
        __syncthreads();
        double top = -1.0;
        int p = 0x7fffffff, pw = 0;
#pragma unroll
        for (int q = 0; q < GJB_PWAVES; ++q) {
            const double a = cand_a[buf][q];
            const int i = cand_i[buf][q];
            if (a > top || (a == top && i < p)) { top = a; p = i; pw = q; }
        }
        if (!(top > 0.0) || !isfinite(top)) {  // uniform
            if (tid == 0) v.st->flag = (top > 0.0) ? 2 : 1;  // infinite, or zero / no pivot
            return;
        }
        const double pv = cand_row[buf][pw][k];
        const double inv = 1.0 / pv;
        ld += log(fabs(pv));
        neg += pv < 0.0;
        if (tid == 0) {
            perm_l[k] = p;
            v.perm[k0 + k] = p;
        }
        // pivot row: P *= 1/pv, P[k] = 1/pv; other rows: P -= f * (pivot
        // row), P[k] = -f with f = P[k]/pv (branch-free)
        double f[RPT], m[RPT], pk[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool piv = tid + GJB_PT * r == p;
            f[r] = piv ? 0.0 : x[r] * inv;
            m[r] = piv ? inv : 1.0;
            pk[r] = piv ? inv : -f[r];
            if (piv) {
                used[r] = true;
                v.used[p] = 1;
            }
        }
        // the pivot row in chunks of 8 (bounded live registers)
        static_for<0, NB / 8>([&](auto cc) __attribute__((always_inline)) {
            constexpr int c0 = decltype(cc)::value * 8;
            double pr[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) pr[q] = cand_row[buf][pw][c0 + q];
#pragma unroll
            for (int r = 0; r < RPT; ++r)
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    P[r][c0 + q] = c0 + q == k ? pk[r] : fma(-f[r], pr[q], P[r][c0 + q] * m[r]);
            __builtin_amdgcn_sched_barrier(0);
        });
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int b = tid + GJB_PT * r;
        if (b < n) {
            double* row = v.M + (size_t)b * v.ld + k0;
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (k < kn) row[k] = P[r][k];
        }
    }
    __syncthreads();
    // T[k][a] = M[p_k][a]: the pivot rows, copied before the update
    // overwrites them (rows k >= kn are zero)
    for (int k = 0; k < NB; ++k) {
        const double* src = v.M + (size_t)perm_l[min(k, kn - 1)] * v.ld;
        double* dst = v.Tg + (size_t)k * v.ld;
        for (int a = tid; a < n; a += GJB_PT) dst[a] = k < kn ? src[a] : 0.0;
    }
    if (tid == 0) {
        v.st->ld += ld;
        v.st->neg += neg;
    }
}

template <int NMX, bool BATCHED>
__global__ __launch_bounds__(GjbCfg<NMX>::PT) void gjb_panel_kernel(Job single, const Job* jobs, const int* prefix,
                                                                     int njobs, int k0) {
    gjb_block<BATCHED>(single, jobs, prefix, njobs, 1,
                       [&](const Job& j, int w, int) __attribute__((always_inline)) { gjb_panel_body<NMX>(j, w, k0); });
}

// ---------------------------------------------------------------- update
template <int NMX>
__device__ __forceinline__ void gjb_update_body(const Job& j, int w, int sub, int k0) {
    using C = GjbCfg<NMX>;
    constexpr int NB = GJB_NB, HS = C::SPW, GJB_SPW = C::SPW, GJB_UT = C::UT, GJB_UWAVES = C::UWAVES;
    constexpr int GJB_HALVES = C::HALVES, GJB_CHUNKS = C::CHUNKS;
    const int n = j.n;
    if (k0 >= n) return;
    const GjbView v = gjb_view(j, w);
    if (v.st->flag) return;
    __shared__ unsigned char curpiv[GJ_NMAX];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int half = sub % GJB_HALVES, chunk = sub / GJB_HALVES;
    const int kn = min(NB, n - k0);
    const int ns = (n + 15) >> 4;
    // element q of M: uniform base + 32-bit byte offset (n^2 * 8 < 2^32)
    char* const Mb = (char*)v.M;
    // global (not generic) accesses: a generic load also counts on the LDS
    // counter, and the wait before a tile's products would then take the
    // next tile's loads with it
    auto Mq = [&](uint32_t q) { return gmem((double*)(Mb + q * 8u)); };
    for (int b = tid; b < GJ_NMAX; b += GJB_UT) curpiv[b] = 0;
    __syncthreads();
    if (tid < kn) curpiv[v.perm[k0 + tid]] = 1;
    __syncthreads();
    // this wave's strips of rows b; L[b][k] = M[b][k0 + k] is the MFMA A
    // operand (row b = 16 strip + lane % 16, k = 4 ks + lane / 16)
    int b0s[HS];
    uint32_t keep[HS];  // bit r: output row b0 + lane / 16 + 4 r is kept (not a pivot row)
    double Lr[HS][NB / 4];
#pragma unroll
    for (int u = 0; u < HS; ++u) {
        const int strip = GJB_SPW * GJB_UWAVES * half + wave + GJB_UWAVES * u;
        const int b0 = 16 * strip;
        b0s[u] = b0;
        const int ba = b0 + (lane & 15);
        const int bl = min(ba, n - 1);
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
            const int k = 4 * ks + (lane >> 4);
            const double x = *Mq((uint32_t)(bl * v.ld + k0 + min(k, kn - 1)));
            Lr[u][ks] = (ba < n && k < kn) ? x : 0.0;
        }
        uint32_t kb = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = b0 + (lane >> 4) + 4 * r;
            kb |= (uint32_t)((b < n) && !curpiv[min(b, n - 1)]) << r;
        }
        keep[u] = kb;
    }
    // column tiles chunk, chunk + CHUNKS, ... outside the panel, software
    // pipelined: the next tile's T block and strips are loaded while this
    // tile runs on MFMA and is stored
    // chunk c owns the contiguous tile range [t0, t1), so successive tiles of
    // a wave continue the same rows of M; the panel's two tiles are skipped
    const int t0 = (ns * chunk) / GJB_CHUNKS, t1 = (ns * (chunk + 1)) / GJB_CHUNKS;
    auto skip_panel = [&](int jt) {
        while (jt < t1 && 16 * jt >= k0 && 16 * jt < k0 + NB) ++jt;
        return jt < t1 ? jt : ns;
    };
    // loads at clamped (valid) addresses and no select on the loaded values,
    // so the next tile's loads stay in flight during this tile's products:
    // an output element depends only on its own column of the T block and
    // its own M element, and columns or rows past n are never stored; the
    // panel's pivot rows are zeroed just before the products
    auto load = [&](int jt, int ntv, int ldv, double (&bop)[NB / 4], f64x4 (&acc)[HS]) {
        const int al = min(16 * jt + (lane & 15), ntv - 1);
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) bop[ks] = *gmem(v.Tg + (size_t)(4 * ks + (lane >> 4)) * ldv + al);
#pragma unroll
        for (int u = 0; u < HS; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0s[u] + (lane >> 4) + 4 * r;
                acc[u][r] = *Mq((uint32_t)(min(b, ntv - 1) * ldv + al));
            }
    };
    // one tile: issue the loads of the tile after it into the other register
    // set (on every pass: the last one reloads this tile, unused, so the
    // queue has the same depth on all paths), then its products and stores
    auto step = [&](int& jt, double (&bop)[NB / 4], f64x4 (&acc)[HS], double (&bopn)[NB / 4], f64x4 (&accn)[HS]) {
        int nt = n, ldt = v.ld;
        asm volatile("" : "+s"(nt), "+s"(ldt));  // keep the row offsets below out of registers across tiles
        const int jn = skip_panel(jt + 1);
        load(jn < ns ? jn : jt, nt, ldt, bopn, accn);
#pragma unroll
        for (int u = 0; u < HS; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[u][r] = ((keep[u] >> r) & 1u) ? acc[u][r] : 0.0;
#pragma unroll
        for (int u = 0; u < HS; ++u)
#pragma unroll
            for (int ks = 0; ks < NB / 4; ++ks)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(Lr[u][ks], bop[ks], acc[u], 0, 0, 0);
        const int ac = 16 * jt + (lane & 15);
#pragma unroll
        for (int u = 0; u < HS; ++u) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0s[u] + (lane >> 4) + 4 * r;
                if ((ac < nt) & (b < nt)) *Mq((uint32_t)(b * ldt + ac)) = acc[u][r];
            }
        }
        jt = jn;
    };
    int jt = skip_panel(t0);
    if (jt >= ns) return;
    // two register sets used in turn, so no copy between tiles (a copy of a
    // loaded value waits for its load)
    double bopA[NB / 4], bopB[NB / 4];
    f64x4 accA[HS], accB[HS];
    load(jt, n, v.ld, bopA, accA);
    // wait for the first tile here: the waits at the loop head are merged
    // over both ways in, and a queue holding only these loads would make
    // every pass wait for the whole queue, the next tile's loads included
#pragma unroll
    for (int ks = 0; ks < NB / 4; ++ks) asm volatile("" ::"v"(bopA[ks]));
#pragma unroll
    for (int u = 0; u < HS; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) asm volatile("" ::"v"(accA[u][r]));
#pragma unroll 1
    while (true) {
        step(jt, bopA, accA, bopB, accB);
        if (jt >= ns) break;
        step(jt, bopB, accB, bopA, accA);
        if (jt >= ns) break;
    }
}

template <int NMX, bool BATCHED>
__global__ __launch_bounds__(GjbCfg<NMX>::UT) void gjb_update_kernel(Job single, const Job* jobs, const int* prefix,
                                                                      int njobs, int k0) {
    gjb_block<BATCHED>(single, jobs, prefix, njobs, GjbCfg<NMX>::UPD_BLOCKS,
                       [&](const Job& j, int w, int sub) __attribute__((always_inline)) { gjb_update_body<NMX>(j, w, sub, k0); });
}

// ---------------------------------------------------------------- finish
// D^-1[e][i] = M[p_e][invp(i)]: row p_e of M staged in LDS and written out
// permuted (both sides coalesced); log|det| = sum log|pivot|, sign =
// sign(permutation) prod sign(pivot).
template <int NMX>
__device__ __forceinline__ void gjb_finish_body(const Job& j, int w, int sub) {
    constexpr int GJB_PT = GjbCfg<NMX>::PT;
    const int n = j.n, spin = j.spin;
    const size_t nn = (size_t)n * n;
    const GjbView v = gjb_view(j, w);
    double* __restrict__ Dw = j.Dinv + (size_t)w * nn;
    __shared__ int perm_l[GJ_NMAX];
    __shared__ int invp_l[GJ_NMAX];
    __shared__ unsigned char mark[GJ_NMAX];
    __shared__ double rowbuf[2][GJ_NMAX];
    const int tid = threadIdx.x;
    const int flag = v.st->flag;
    if (flag) {
        for (size_t q = (size_t)sub * GJB_PT + tid; q < nn; q += (size_t)GJB_COPY_BLOCKS * GJB_PT)
            Dw[q] = __longlong_as_double(0x7ff8000000000000ll);
        if (sub == 0 && tid == 0) {
            if (j.logdet) j.logdet[2 * w + spin] = flag == 1 ? -INFINITY : __longlong_as_double(0x7ff8000000000000ll);
            if (j.sign) j.sign[2 * w + spin] = 0;
            if (j.status) atomicOr(j.status + w, flag == 1 ? QSL_STATUS_SINGULAR : QSL_STATUS_NONFINITE);
        }
        return;
    }
    for (int k = tid; k < n; k += GJB_PT) {
        const int p = v.perm[k];
        perm_l[k] = p;
        invp_l[p] = k;
        mark[k] = 0;
    }
    __syncthreads();
    if (sub == 0 && tid == 0) {
        // parity of the pivot permutation by cycle counting
        int cycles = 0;
        for (int i = 0; i < n; ++i) {
            if (mark[i]) continue;
            ++cycles;
            for (int q = i; !mark[q]; q = perm_l[q]) mark[q] = 1;
        }
        const double ld = v.st->ld;
        const int sg = ((v.st->neg + n - cycles) & 1) ? -1 : 1;
        if (j.logdet) j.logdet[2 * w + spin] = ld;
        if (j.sign) j.sign[2 * w + spin] = (int8_t)sg;
        if (j.status && !isfinite(ld)) atomicOr(j.status + w, QSL_STATUS_NONFINITE);
    }
    int buf = 0;
    for (int e = sub; e < n; e += GJB_COPY_BLOCKS) {
        const double* src = v.M + (size_t)perm_l[e] * v.ld;
        for (int a = tid; a < n; a += GJB_PT) rowbuf[buf][a] = src[a];
        __syncthreads();
        double* dst = Dw + (size_t)e * n;
        for (int i = tid; i < n; i += GJB_PT) dst[i] = rowbuf[buf][invp_l[i]];
        buf ^= 1;  // the next row goes to the other buffer: one barrier per row
    }
}

template <int NMX, bool BATCHED>
__global__ __launch_bounds__(GjbCfg<NMX>::PT) void gjb_finish_kernel(Job single, const Job* jobs, const int* prefix,
                                                                      int njobs) {
    gjb_block<BATCHED>(single, jobs, prefix, njobs, GJB_COPY_BLOCKS,
                       [&](const Job& j, int w, int sub) __attribute__((always_inline)) { gjb_finish_body<NMX>(j, w, sub); });
}

// ------------------------------------------------------------- launchers

template <int NMX, bool BATCHED>
static hipError_t gjb_sequence_n(int mode, const Job& single, const Job* jobs, const int* prefix, int njobs,
                                 int matrices, int nmax, hipStream_t st) {
    using C = GjbCfg<NMX>;
    const unsigned m = (unsigned)matrices;
    if (mode == QSL_FP64)
        gjb_init_kernel<NMX, BATCHED, double><<<m * GJB_COPY_BLOCKS, C::PT, 0, st>>>(single, jobs, prefix, njobs);
    else
        gjb_init_kernel<NMX, BATCHED, float><<<m * GJB_COPY_BLOCKS, C::PT, 0, st>>>(single, jobs, prefix, njobs);
    hipError_t e = hipGetLastError();
    for (int k0 = 0; k0 < nmax && e == hipSuccess; k0 += GJB_NB) {
        gjb_panel_kernel<NMX, BATCHED><<<m, C::PT, 0, st>>>(single, jobs, prefix, njobs, k0);
        gjb_update_kernel<NMX, BATCHED><<<m * C::UPD_BLOCKS, C::UT, 0, st>>>(single, jobs, prefix, njobs, k0);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    gjb_finish_kernel<NMX, BATCHED><<<m * GJB_COPY_BLOCKS, C::PT, 0, st>>>(single, jobs, prefix, njobs);
    return hipGetLastError();
}

template <bool BATCHED>
static hipError_t gjb_sequence(int mode, const Job& single, const Job* jobs, const int* prefix, int njobs,
                               int matrices, int nmax, hipStream_t st) {
    if (matrices <= 0 || nmax <= 0) return hipSuccess;
    if (nmax > GJ_NMAX) return hipErrorInvalidValue;
    if (nmax <= 256) return gjb_sequence_n<256, BATCHED>(mode, single, jobs, prefix, njobs, matrices, nmax, st);
    return gjb_sequence_n<GJ_NMAX, BATCHED>(mode, single, jobs, prefix, njobs, matrices, nmax, st);
}

hipError_t launch_gjb(const Job& j, hipStream_t st) {
    if (!gj_blocked(j.n) || j.n > GJ_NMAX || !j.gjws) return hipErrorInvalidValue;
    if (j.W > (int64_t)(0x7fffffff / GjbCfg<GJ_NMAX>::UPD_BLOCKS)) return hipErrorInvalidValue;
    return gjb_sequence<false>(j.mode, j, nullptr, nullptr, 0, (int)j.W, j.n, st);
}

hipError_t launch_gjb_batched(int mode, const Job* jobs, const int* prefix, int njobs, int matrices, int nmax,
                              hipStream_t st) {
    Job dummy{};
    return gjb_sequence<true>(mode, dummy, jobs, prefix, njobs, matrices, nmax, st);
}

}  // namespace qsl
