// Blocked FP64 Gauss-Jordan for 224 < n <= 1024: log|det|, sign and
// inverse of the Slater matrices too large for the register-resident
// kernel (inversion step, section "Overall performance of QMC=Chem").
//
// The elimination is the same as the unblocked one: at step k the pivot is
// the largest |D[b][k]| over rows b not yet used (the smallest b among
// values within 2^-42 relative), pivot rows are never moved, and the
// inverse is un-permuted at the end.
// It runs on a row-major FP64 copy M[b][a] = D[b][a] in the workspace
// (row b = MO, column a = electron), made by an LDS-tiled transpose of C_1.
//
// Panels of NB = 32 columns, two per pass:
//  panel   one workgroup per matrix, one thread per row, reduces the panel
//          columns in registers (one barrier per column), stores the
//          reduced panel L and copies the panel's pivot rows
//          T[k][a] = M[p_k][a].
//  update  the composite of a panel's NB elementary steps acts on any other
//          column v through its pivot rows only:
//              v <- (v with the panel's pivot rows set to 0) + L v_P,
//          on v_mfma_f64_16x16x4f64 in output tiles of 16 rows b x 16
//          columns a; each wave keeps its 16-row strips of L in registers
//          and streams the tiles of a contiguous column range.
// A pass over panels A = [k0, k0 + NB) and B = [k0 + NB, k0 + 2 NB): panel
// A; then B's panel kernel, in which B's columns first take A's steps, B is
// reduced, and A's columns take B's steps, which makes them the final L of
// both (two rank-NB products per row); then every other column takes both
// at once, v <- (v with both panels' pivot rows set to 0)
// + [L_A L_B] [v_PA; v_PB] (rank 2 NB), with v_PA and v_PB the pivot rows
// as they were before the pass.  (B's composite applied after A's is
// exactly that: the rows P_B of A's result are v_PB + L_A[P_B] v_PA, and
// B's steps turn L_A into the final columns of A.)
// Then a finish kernel writes D^-1[e][i] = M[p_e][invp(i)] (row p_e of M
// staged in LDS, written out permuted), log|det| and sign.
//
// Traffic: the matrix is read and written once per pass (n^3 / (2 NB) x 16
// bytes per matrix); flops 2 n^3 per matrix.  Separate kernels give each
// phase its own register budget and occupancy.
#include <algorithm>

#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(2))) unsigned int u32x2;
typedef __attribute__((ext_vector_type(2))) double f64x2;

constexpr int GJB_NB = GJ_PANEL;
constexpr int GJB_COPY_BLOCKS = 8;  // init / finish blocks per matrix

// Launch shapes by the largest n served (NMX = 256 or GJ_NMAX): threads of
// the init / finish workgroups, of the panel workgroup (one row each) and of
// the update workgroups, and column ranges per matrix in the update.
template <int NMX>
struct GjbCfg {
    static constexpr int PT = NMX >= 512 ? 512 : 256;
    static constexpr int PNT = NMX;  // panel: one row per thread
    static constexpr int PWAVES = PNT / 64;
    static constexpr int UT = PT;
    static constexpr int UWAVES = UT / 64;
    static constexpr int CHUNKS = 2;
    static_assert(PNT <= 1024, "launch shape");
};
// The rank-2 NB update of a pass: 16-row strips per wave (two: the strips
// of L hold 2 NB entries per row), row parts and workgroups per matrix.
template <int NMX>
struct GjbUpdCfg {
    static constexpr int SPW = 2;
    static constexpr int PARTS = NMX / 16 / GjbCfg<NMX>::UWAVES / SPW;
    static constexpr int BLOCKS = PARTS * GjbCfg<NMX>::CHUNKS;
    static_assert(PARTS >= 1, "update shape");
};

struct GjbState {
    double ld;  // sum log|pivot|
    int neg;    // negative pivots
    int flag;   // 0 ok, 1 zero pivot (singular), 2 non-finite pivot
};

// Per-matrix workspace (gj_ws_doubles(n) doubles).
struct GjbView {
    double* M;       // [n][ld] row-major D, then the elimination
    double* Tg;      // [2 NB][ld] pivot rows of the current two panels
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
    v.perm = (int*)(v.Tg + (size_t)v.ld * 2 * GJB_NB);
    v.used = (uint8_t*)(v.perm + n);
    v.st = (GjbState*)((char*)v.perm + (((size_t)5 * n + 7) / 8) * 8);
    return v;
}

// Block -> (Job, matrix, sub-block): one Job by value (BATCHED = false), or
// a plan's Jobs through the prefix sums of their matrix counts.  Separate
// instantiations keep one inlined copy of the body per kernel.
// XCD: blocks 8 mult t + o serve matrix 8 t + o % 8, sub-block o / 8 (the
// grid is mult times the matrix count rounded up to 8).  The hardware hands
// consecutive blocks to the eight XCDs in turn, so all sub-blocks of a
// matrix run on one XCD and share its L2 (the update's T block).
template <bool BATCHED, bool XCD = false, typename F>
__device__ __forceinline__ void gjb_block(const Job& single, const Job* __restrict__ jobs,
                                          const int* __restrict__ prefix, int njobs, int mult, F body) {
    const int o = XCD ? (int)(blockIdx.x % (8u * mult)) : 0;
    const int b = XCD ? (int)(blockIdx.x / (8u * mult)) * 8 + o % 8 : (int)(blockIdx.x / mult);
    const int sub = XCD ? o / 8 : (int)(blockIdx.x % mult);
    if constexpr (!BATCHED) {
        if (b < single.W) body(single, b, sub);
    } else {
        if (b >= prefix[njobs]) return;
        const int ji = __builtin_amdgcn_readfirstlane(find_job(prefix, njobs, b));
        body(jobs[ji], b - prefix[ji], sub);
    }
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
// Pivot keys: |value| as its IEEE bits (monotone for |value| >= 0) with the
// low 10 mantissa bits replaced by 1023 - row, so the largest key is the
// largest |value|, and the smallest row among values equal to 2^-42
// relative; 0 for rows not eligible (used, past n, NaN).
__device__ __forceinline__ uint64_t pivot_key(double x, int b, bool eligible) {
    const uint64_t m = (uint64_t)__double_as_longlong(fabs(x));
    return (eligible && !isnan(x)) ? ((m & ~0x3FFull) | (uint64_t)(0x3FF - b)) : 0ull;
}
template <int CTRL>
__device__ __forceinline__ uint64_t key_max_step(uint64_t k) {
    // every lane reads a lane of its own row: no bound control needed
    const uint32_t lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)k, CTRL, 0xf, 0xf, true);
    const uint32_t hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(k >> 32), CTRL, 0xf, 0xf, true);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    return o > k ? o : k;
}
// largest key over each 16-lane row (every lane of the row holds it)
__device__ __forceinline__ uint64_t key_max_row(uint64_t k) {
    k = key_max_step<0xB1>(k);   // quad_perm [1,0,3,2]
    k = key_max_step<0x4E>(k);   // quad_perm [2,3,0,1]
    k = key_max_step<0x141>(k);  // row_half_mirror
    return key_max_step<0x140>(k);  // row_mirror
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t k, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)k, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(k >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
// largest key over the wavefront (uniform)
__device__ __forceinline__ uint64_t key_max_wave(uint64_t k) {
    k = key_max_row(k);
    uint64_t m = readlane_u64(k, 0);
#pragma unroll
    for (int rw = 1; rw < 4; ++rw) {
        const uint64_t o = readlane_u64(k, 16 * rw);
        m = o > m ? o : m;
    }
    return m;
}

// One thread per row b holds M[b][k0 .. k0 + NB) in registers.  The panel's
// columns are unrolled at compile time, so the column being reduced and the
// pivot entry are plain registers (no select over the row), and no column
// leaves the sequence early (a column past the panel or after a failed
// pivot changes nothing that is kept).  Per column: the wave's largest
// pivot key, one barrier, the largest of the waves' keys (16-lane DPP),
// then one FMA per entry, P -= f (pivot row), on every row; the pivot row's
// own scaling by 1/pv is deferred to the store.
// SECOND: the second panel B = [k0, k0 + NB) of a pass, after the first
// A = [k0 - NB, k0).  B's columns first take A's steps (rank NB: the rows
// of A's pivots zeroed, plus L_A times A's pivot rows in B's columns, kept
// in T rows 0 .. NB - 1); after B is reduced, A's columns take B's steps
// (the rows of B's pivots zeroed, plus L_B times the rows P_B of L_A),
// which makes them the final L of both panels.  Both are small products
// per row, done here rather than by two update launches.
template <int NMX, bool SECOND>
__device__ __forceinline__ void gjb_panel_body(const Job& j, int w, int k0, int tofs) {
    using C = GjbCfg<NMX>;
    constexpr int NB = GJB_NB, PNT = C::PNT, PW = C::PWAVES;
    static_assert(PW <= 16 && NMX <= 1024, "keys hold 10-bit rows; waves compared within one 16-lane row");
    const int n = j.n;
    if (k0 >= n) return;
    const GjbView v = gjb_view(j, w);
    if (v.st->flag) return;  // singular earlier: nothing left to do
    __shared__ uint64_t cand_k[2][PW];
    __shared__ double cand_row[2][PW][NB];
    __shared__ int perm_l[NB];
    __shared__ double piv_l[NB];
    // SECOND: T_A[k][q] = M[p^A_k][k0 + q] (A's pivot rows in B's columns),
    // later L_A[p^B_k][q] (B's pivot rows in A's columns); A's pivot rows
    __shared__ double blk[SECOND ? NB : 1][SECOND ? NB : 1];
    __shared__ unsigned char pivA[SECOND ? PNT : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kn = min(NB, n - k0);
    const int b = tid;  // this thread's row
    const int bl = min(b, n - 1);  // loads at clamped (valid) addresses, then select
    bool used = b >= n || v.used[bl];
    double P[NB];  // P[k] = M[b][k0 + k]
    if constexpr (SECOND) {
        pivA[tid] = 0;
        for (int q = tid; q < NB * NB; q += PNT) {
            const int k = q / NB, c = q % NB;
            blk[k][c] = c < kn ? v.Tg[(size_t)k * v.ld + k0 + c] : 0.0;  // A is whole: n > k0
        }
        __syncthreads();
        if (tid < NB) pivA[v.perm[k0 - NB + tid]] = 1;
        __syncthreads();
    }
    {
        // the row's panel entries: 16-byte loads for a whole panel (rows are
        // 128-byte aligned, k0 a multiple of NB), else one clamped load each
        const double* row = v.M + (size_t)bl * v.ld + k0;
        const bool keep = b < n && !(SECOND && pivA[b]);
        if (kn == NB) {
#pragma unroll
            for (int k = 0; k < NB; k += 2) {
                const f64x2 x = *gmem((const f64x2*)(row + k));
                P[k] = keep ? x.x : 0.0;
                P[k + 1] = keep ? x.y : 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const double x = *gmem(row + min(k, kn - 1));
                P[k] = (keep && k < kn) ? x : 0.0;
            }
        }
    }
    if constexpr (SECOND) {
        // + L_A[b][k] T_A[k][.]: L_A is this row's entries in A's columns,
        // taken eight at a time (bounded live registers)
        const double* rowA = v.M + (size_t)bl * v.ld + k0 - NB;
#pragma unroll
        for (int kc = 0; kc < NB; kc += 8) {
            double a[8];
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                const f64x2 x = *gmem((const f64x2*)(rowA + kc + i));
                a[i] = b < n ? x.x : 0.0;
                a[i + 1] = b < n ? x.y : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                static_for<0, NB / 8>([&](auto cc) __attribute__((always_inline)) {
                    constexpr int c0 = decltype(cc)::value * 8;
                    double t[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) t[q] = blk[kc + i][c0 + q];
#pragma unroll
                    for (int q = 0; q < 8; ++q) P[c0 + q] = fma(a[i], t[q], P[c0 + q]);
                    __builtin_amdgcn_sched_barrier(0);
                });
        }
    }
    double sc = 1.0;   // the row's pending scale (1/pv once it is a pivot row)
    bool newpiv = false;  // the row is a pivot row of this panel
    int fail = 0;      // uniform: 1 no pivot (zero column), 2 non-finite pivot
    static_for<0, NB>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value, buf = k & 1;
        const bool live = k < kn && !fail;  // uniform
        const uint64_t wk = key_max_wave(pivot_key(P[k], b, !used));
        if (b == 0x3FF - (int)(wk & 0x3FF) && wk != 0) {
#pragma unroll
            for (int q = 0; q < NB; ++q) cand_row[buf][wave][q] = P[q];
        }
        if (lane == 0) cand_k[buf][wave] = wk;
        __syncthreads();
        uint64_t top = key_max_row(lane < PW ? cand_k[buf][lane] : 0ull);
        top = readlane_u64(top, 0);
        const double topv = __longlong_as_double((long long)(top & ~0x3FFull));
        const int bad = !(topv > 0.0) ? 1 : (!isfinite(topv) ? 2 : 0);
        if (live && bad) {
            if (tid == 0) gmem(v.st)->flag = bad;
            fail = bad;
        }
        const int p = 0x3FF - (int)(top & 0x3FF);  // the pivot row (any row when bad)
        const int pw = min(p >> 6, PW - 1);         // its wave
        const double pv = cand_row[buf][pw][k];
        const double inv = 1.0 / pv;
        const bool go = live && !bad;  // uniform
        if (tid == 0 && go) {
            perm_l[k] = p;
            piv_l[k] = pv;
        }
        const bool piv = go && b == p;
        // other rows: P -= f (pivot row), P[k] = -f with f = P[k] / pv.  The
        // pivot row's scaling by 1/pv is kept aside in sc and applied when
        // the panel is stored: its later updates are the same in the scaled
        // and the unscaled form (f is a ratio of its own entries), and rows
        // not yet used, which decide the pivots, never see it.  Nothing
        // changes unless go.
        const double f = (go && !piv) ? P[k] * inv : 0.0;
        if (go) {
            // the pivot row in chunks of 8 (bounded live registers)
            static_for<0, NB / 8>([&](auto cc) __attribute__((always_inline)) {
                constexpr int c0 = decltype(cc)::value * 8;
                double pr[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) pr[q] = cand_row[buf][pw][c0 + q];
#pragma unroll
                for (int q = 0; q < 8; ++q) P[c0 + q] = fma(-f, pr[q], P[c0 + q]);
                __builtin_amdgcn_sched_barrier(0);
            });
            // the pivot row: 1/pv in column k, i.e. 1 before its scaling
            P[k] = piv ? 1.0 : -f;
        }
        if (piv) {
            used = true;
            newpiv = true;
            sc = inv;
        }
    });
    if (fail) return;
    // the pivot order and row flags, written once the panel is done (a
    // generic store in the column loop would make every later LDS wait
    // include its completion)
    if (tid < kn) gmem(v.perm)[k0 + tid] = perm_l[tid];
    if (newpiv) gmem(v.used)[b] = 1;
#pragma unroll
    for (int k = 0; k < NB; ++k) P[k] *= sc;  // the final L of this panel
    if constexpr (SECOND) {
        // L_A <- (L_A with the rows of B's pivots zeroed) + L_B L_A[P_B]
        __syncthreads();  // every thread is done with T_A
        for (int q = tid; q < NB * NB; q += PNT) {
            const int k = q / NB, c = q % NB;
            blk[k][c] = k < kn ? v.M[(size_t)perm_l[k] * v.ld + k0 - NB + c] : 0.0;
        }
        __syncthreads();
        if (b < n) {
            double* rowA = v.M + (size_t)b * v.ld + k0 - NB;
            // eight of A's columns at a time
#pragma unroll
            for (int c0 = 0; c0 < NB; c0 += 8) {
                double x[8];
#pragma unroll
                for (int q = 0; q < 8; q += 2) {
                    const f64x2 y = *gmem((const f64x2*)(rowA + c0 + q));
                    x[q] = newpiv ? 0.0 : y.x;
                    x[q + 1] = newpiv ? 0.0 : y.y;
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    double t[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) t[q] = blk[k][c0 + q];
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[q] = fma(P[k], t[q], x[q]);
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int q = 0; q < 8; q += 2) *gmem((f64x2*)(rowA + c0 + q)) = f64x2{x[q], x[q + 1]};
            }
        }
    }
    if (b < n) {
        double* row = v.M + (size_t)b * v.ld + k0;
        if (kn == NB) {
#pragma unroll
            for (int k = 0; k < NB; k += 2) *gmem((f64x2*)(row + k)) = f64x2{P[k], P[k + 1]};
        } else {
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (k < kn) *gmem(row + k) = P[k];
        }
    }
    __syncthreads();
    // T[tofs + k][a] = M[p_k][a]: the pivot rows, copied before the updates
    // overwrite them (rows k >= kn are zero)
    // (n <= PNT: one column a per thread; all loads issued before the stores)
    if (tid < n) {
        double t[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) t[k] = *gmem(v.M + (size_t)perm_l[min(k, kn - 1)] * v.ld + tid);
#pragma unroll
        for (int k = 0; k < NB; ++k) *gmem(v.Tg + (size_t)(tofs + k) * v.ld + tid) = k < kn ? t[k] : 0.0;
    }
    // log|pivot| of the panel's columns (one lane each), summed in column order
    if (wave == 0) {
        const double pv = lane < kn ? piv_l[lane] : 1.0;
        const double lg = log(fabs(pv));
        const int neg = __popcll(__ballot(pv < 0.0));
        double ld = 0.0;
        for (int k = 0; k < kn; ++k) ld += readlane_f64(lg, k);
        if (lane == 0) {
            v.st->ld += ld;
            v.st->neg += neg;
        }
    }
}

template <int NMX, bool BATCHED, bool SECOND>
__global__ __launch_bounds__(GjbCfg<NMX>::PNT) void gjb_panel_kernel(Job single, const Job* jobs, const int* prefix,
                                                                      int njobs, int k0, int tofs) {
    gjb_block<BATCHED>(single, jobs, prefix, njobs, 1, [&](const Job& j, int w, int) __attribute__((always_inline)) {
        gjb_panel_body<NMX, SECOND>(j, w, k0, tofs);
    });
}

// ---------------------------------------------------------------- update
// The composite of the elimination steps of the pass's pivots k0 .. k0 +
// NB - 1 (NB = 2 GJB_NB: both panels) applied to every column outside
// [k0, k0 + NB): L is M's columns k0 .. k0 + NB - 1, the pivot rows' entries
// are T's NB rows.
template <int NMX>
__device__ __forceinline__ void gjb_update_body(const Job& j, int w, int sub, int k0) {
    using C = GjbCfg<NMX>;
    using U = GjbUpdCfg<NMX>;
    constexpr int NB = 2 * GJB_NB;
    constexpr int HS = U::SPW, GJB_SPW = U::SPW, GJB_UT = C::UT, GJB_UWAVES = C::UWAVES;
    constexpr int GJB_PARTS = U::PARTS, GJB_CHUNKS = C::CHUNKS;
    const int n = j.n;
    if (k0 >= n) return;
    const int ns = (n + 15) >> 4;  // column tiles
    const GjbView v = gjb_view(j, w);
    if (v.st->flag) return;
    const double* __restrict__ Tg = v.Tg;
    __shared__ unsigned char curpiv[GJ_NMAX];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int part = sub % GJB_PARTS, chunk = sub / GJB_PARTS;
    const int kn = min(NB, n - k0);
    // element q of M: uniform base + 32-bit byte offset (n^2 * 8 < 2^32)
    char* const Mb = (char*)v.M;
    // global (not generic) accesses: a generic load also counts on the LDS
    // counter, and the wait before a tile's products would then take the
    // next tile's loads with it
    auto Mq = [&](uint32_t q) { return gmem((double*)(Mb + q * 8u)); };
    // stores through a buffer resource over M's n rows: a masked element
    // gets an offset past the end, which the hardware drops.  With no branch
    // around them the stores count in the wait before the next tile's
    // products, which then need not wait for them to complete.
    const __amdgpu_buffer_rsrc_t Mr = __builtin_amdgcn_make_buffer_rsrc(v.M, (short)0, n * v.ld * 8, 0x00020000);
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
        const int strip = GJB_SPW * GJB_UWAVES * part + wave + GJB_UWAVES * u;
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
    // chunk c owns a contiguous range [t0, t1) of the tiles, so successive
    // tiles of a wave continue the same rows of M; the pass's four tiles are
    // skipped.  Software pipelined: the next tile's T block and strips are
    // loaded while this tile runs on MFMA and is stored.
    const int t0 = (ns * chunk) / GJB_CHUNKS, t1 = (ns * (chunk + 1)) / GJB_CHUNKS;
    auto skip_panel = [&](int jt) {
        while (jt < t1 && 16 * jt >= k0 && 16 * jt < k0 + NB) ++jt;
        return jt;  // t1 when none is left
    };
    // The T block of a tile (NB rows x 16 columns) is staged in LDS once per
    // workgroup (TE elements per thread), double-buffered: every wave of the
    // workgroup streams the same tiles.  Loads at clamped (valid) addresses
    // and no select on the loaded values, so the next tile's loads stay in
    // flight during this tile's products: an output element depends only on
    // its own column of the T block and its own M element, and columns or
    // rows past n are never stored; the panel's pivot rows are zeroed just
    // before the products.
    constexpr int TE = NB * 16 / GJB_UT;
    static_assert(TE * GJB_UT == NB * 16, "T block per thread");
    __shared__ __attribute__((aligned(16))) double Ts[2][NB][16];
    auto load = [&](int jt, int ntv, int ldv, double (&tv)[TE], f64x4 (&acc)[HS]) {
#pragma unroll
        for (int i = 0; i < TE; ++i) {
            const int e = tid + GJB_UT * i;
            tv[i] = *gmem(Tg + (size_t)(e >> 4) * ldv + min(16 * jt + (e & 15), ntv - 1));
        }
        const int al = min(16 * jt + (lane & 15), ntv - 1);
#pragma unroll
        for (int u = 0; u < HS; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0s[u] + (lane >> 4) + 4 * r;
                acc[u][r] = *Mq((uint32_t)(min(b, ntv - 1) * ldv + al));
            }
    };
    auto put = [&](int buf, const double (&tv)[TE]) {
#pragma unroll
        for (int i = 0; i < TE; ++i) {
            const int e = tid + GJB_UT * i;
            Ts[buf][e >> 4][e & 15] = tv[i];
        }
    };
    // one tile from T block buf: issue the loads of the tile after it (into
    // the other M register set and tv; on every pass: the last one reloads
    // this tile, unused, so the queue has the same depth on all paths), its
    // products and stores, then the next T block into the other buffer
    auto step = [&](int& jt, int buf, f64x4 (&acc)[HS], f64x4 (&accn)[HS]) {
        int nt = n, ldt = v.ld;
        asm volatile("" : "+s"(nt), "+s"(ldt));  // keep the row offsets below out of registers across tiles
        const int jn = skip_panel(jt + 1);
        double tv[TE];
        load(jn < t1 ? jn : jt, nt, ldt, tv, accn);
#pragma unroll
        for (int u = 0; u < HS; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[u][r] = ((keep[u] >> r) & 1u) ? acc[u][r] : 0.0;
        // B operand: T[4 ks + lane / 16][lane % 16]
        const double* tb = &Ts[buf][lane >> 4][lane & 15];
#pragma unroll
        for (int ks = 0; ks < NB / 4; ++ks) {
            const double bop = tb[64 * ks];
#pragma unroll
            for (int u = 0; u < HS; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(Lr[u][ks], bop, acc[u], 0, 0, 0);
        }
        const int ac = 16 * jt + (lane & 15);
#pragma unroll
        for (int u = 0; u < HS; ++u) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0s[u] + (lane >> 4) + 4 * r;
                const uint32_t off = (ac < nt) & (b < nt) ? (uint32_t)(b * ldt + ac) * 8u : 0x80000000u;
                const uint64_t x = (uint64_t)__double_as_longlong(acc[u][r]);
                const u32x2 xv = {(uint32_t)x, (uint32_t)(x >> 32)};
                __builtin_amdgcn_raw_buffer_store_b64(xv, Mr, off, 0, 0);
            }
        }
        put(buf ^ 1, tv);
        __syncthreads();  // the next block is in, and every wave is done with this one
        jt = jn;
    };
    int jt = skip_panel(t0);
    if (jt >= t1) return;
    // two register sets used in turn, so no copy between tiles (a copy of a
    // loaded value waits for its load)
    f64x4 accA[HS], accB[HS];
    {
        double tv[TE];
        load(jt, n, v.ld, tv, accA);
        put(0, tv);
    }
    // wait for the first tile here: the waits at the loop head are merged
    // over both ways in, and a queue holding only these loads would make
    // every pass wait for the whole queue, the next tile's loads included
#pragma unroll
    for (int u = 0; u < HS; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) asm volatile("" ::"v"(accA[u][r]));
    __syncthreads();
#pragma unroll 1
    while (true) {
        step(jt, 0, accA, accB);
        if (jt >= t1) break;
        step(jt, 1, accB, accA);
        if (jt >= t1) break;
    }
}

template <int NMX, bool BATCHED>
__global__ __launch_bounds__(GjbCfg<NMX>::UT) void gjb_update_kernel(Job single, const Job* jobs, const int* prefix,
                                                                      int njobs, int k0) {
    gjb_block<BATCHED, true>(single, jobs, prefix, njobs, GjbUpdCfg<NMX>::BLOCKS,
                             [&](const Job& j, int w, int sub) __attribute__((always_inline)) {
                                 gjb_update_body<NMX>(j, w, sub, k0);
                             });
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
    constexpr int NB = GJB_NB;
    const unsigned bu = ((m + 7) / 8 * 8) * GjbUpdCfg<NMX>::BLOCKS;  // XCD-aware block order
    // two panels per pass: A = [k0, k0 + NB), B = [k0 + NB, k0 + 2 NB)
    for (int k0 = 0; k0 < nmax && e == hipSuccess; k0 += 2 * NB) {
        gjb_panel_kernel<NMX, BATCHED, false><<<m, C::PNT, 0, st>>>(single, jobs, prefix, njobs, k0, 0);
        // B's columns take A's steps, B is reduced, then A's columns take
        // B's steps (they become the final L of A): all in B's panel kernel
        if (k0 + NB < nmax)
            gjb_panel_kernel<NMX, BATCHED, true><<<m, C::PNT, 0, st>>>(single, jobs, prefix, njobs, k0 + NB, NB);
        // every other column takes both panels' steps at once: rank 2 NB,
        // the matrix streamed once per pass
        gjb_update_kernel<NMX, BATCHED><<<bu, C::UT, 0, st>>>(single, jobs, prefix, njobs, k0);
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
    if (j.W > (int64_t)(0x7fffffff / GjbUpdCfg<GJ_NMAX>::BLOCKS) - 8) return hipErrorInvalidValue;
    return gjb_sequence<false>(j.mode, j, nullptr, nullptr, 0, (int)j.W, j.n, st);
}

hipError_t launch_gjb_batched(int mode, const Job* jobs, const int* prefix, int njobs, int matrices, int nmax,
                              hipStream_t st) {
    Job dummy{};
    return gjb_sequence<true>(mode, dummy, jobs, prefix, njobs, matrices, nmax, st);
}

}  // namespace qsl
