// FP64 log|det|, sign and inverse of the Slater matrices (inversion step,
// section "Overall performance of QMC=Chem"; Slater matrix D_ij = phi_i(r_j)).
//
// One workgroup inverts one n x n matrix held entirely in registers, by
// Gauss-Jordan elimination with partial pivoting on the rows of D: at step k
// the pivot is the largest |D[i][k]| over rows not yet used (smallest i on
// exact ties; for 128 < n <= 224, among values within 2^-12 relative of
// the largest, which leaves the elimination as stable).  Pivot rows are not
// moved; the pivot sequence p_k is recorded and the result is un-permuted on
// the way out: D^-1[k][p_j] = M[p_k][j].
// The pivots are the diagonal of U in P D = L U, so log|det| = sum log|pivot|
// and sign = sign(permutation) prod sign(pivot).  2 n^3 flops per matrix.
#include <algorithm>

#include "qsl_internal.h"

namespace qsl {


// Layout: wave v of NWV owns the D columns e = v + NWV c (c < CPW, electron
// index), lane l owns the D rows i = l + 64 r (r < RPL, MO index); thread
// (v, l) holds M[r][c] in registers, loaded coalesced from C_1[e][i].
// Step k: the wave owning column k finds the pivot among the unused rows
// (a wavefront argmax), publishes the column (zero in the pivot row) and
// the pivot through LDS, one barrier; every wave then reads the pivot row
// of its own columns from lane p % 64 with readlane (scalar registers) and
// applies the rank-1 update.  The pivot row is left unscaled (it is divided
// by its pivot on the way out), its column-k entry becomes 1; the other rows
// of column k become -D[i][k]/pv through the entry 1 + 1/pv of the pivot row.

// argmax of |col| over the unused rows of this lane, then over the wavefront
// (largest value, smallest row index on exact ties): DPP exchanges inside
// rows of 16 lanes (quad swaps, half-row and row mirrors), then the four row
// results through scalar registers.  Publishes column and pivot.
template <int RPL>
__device__ __forceinline__ void gj_search(const double (&col)[RPL], int n, int lane, uint32_t used, double* colout,
                                          int* piv_idx, double* piv_val) {
    double best = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const double v = fabs(col[r]);
        if (i < n && !((used >> r) & 1u) && v > best) { best = v; bi = i; }
    }
    argmax_step<0xB1>(best, bi);   // quad_perm [1,0,3,2]
    argmax_step<0x4E>(best, bi);   // quad_perm [2,3,0,1]
    argmax_step<0x141>(best, bi);  // row_half_mirror
    argmax_step<0x140>(best, bi);  // row_mirror
    double sb = readlane_f64(best, 0);
    int si = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
    for (int rw = 1; rw < 4; ++rw) {
        const double ob = readlane_f64(best, 16 * rw);
        const int oi = __builtin_amdgcn_readlane(bi, 16 * rw);
        if (ob > sb || (ob == sb && oi < si)) { sb = ob; si = oi; }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < n) colout[i] = (i == si) ? 0.0 : col[r];
        if (i == si) *piv_val = col[r];
    }
    if (lane == 0) *piv_idx = si;
}

template <int NWV, int RPL, int CPW, typename Tin>
__device__ __forceinline__ void gj_body(const Job& j, int bx) {
    const Tin* __restrict__ C = (const Tin*)j.C;
    const int n = j.n, spin = j.spin;
    double* __restrict__ Dinv = j.Dinv;
    double* __restrict__ logdet = j.logdet;
    int8_t* __restrict__ sign = j.sign;
    uint32_t* __restrict__ status = j.status;
    constexpr int NT = NWV * 64;
    constexpr int NR = 64 * RPL;   // capacity in D rows (MO index i)
    constexpr int NC = NWV * CPW;  // capacity in D columns (electron index e)
    constexpr int QC = 8;          // rows of D^-1 staged per output pass
    __shared__ double colbuf[2][NR];
    __shared__ int piv_idx[2];
    __shared__ double piv_val[2];
    __shared__ int perm[NC];
    __shared__ int invp[NR];
    __shared__ double rowpiv[NR];
    __shared__ double stage[QC][NC > NR ? NC : NR];
    __shared__ int s_flag;

    const int w = bx;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const size_t nn = (size_t)n * n;
    const Tin* C1 = C + (size_t)w * 5 * nn;  // derivative 0 block

    double M[RPL][CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int e = wave + NWV * c, i = lane + 64 * r;
            M[r][c] = (e < n && i < n) ? (double)C1[(size_t)e * n + i] : 0.0;
        }
    for (int k = tid; k < NR; k += NT) { colbuf[0][k] = 0.0; colbuf[1][k] = 0.0; }
    if (tid == 0) s_flag = 0;
    __syncthreads();
    uint32_t used = 0;  // bit r: row lane + 64 r already a pivot row
    if (wave == 0) {
        double col[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) col[r] = M[r][0];
        gj_search<RPL>(col, n, lane, used, colbuf[0], &piv_idx[0], &piv_val[0]);
    }

    bool singular = false;
    for (int k = 0; k < n; ++k) {
        const int b = k & 1;
        __syncthreads();  // pivot and column k are published, step k-1 is done
        const int p = __builtin_amdgcn_readfirstlane(piv_idx[b]);
        const double pv = piv_val[b];
        if (p >= n || !(pv != 0.0) || !isfinite(pv)) {  // zero (or NaN) pivot
            singular = true;
            if (tid == 0) s_flag = isfinite(pv) || p >= n ? 1 : 2;
            break;
        }
        const double inv = 1.0 / pv;
        const int lp = p & 63, rp = p >> 6;  // wave-uniform
        const int vk = k % NWV, ck = k / NWV;
        double colv[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) colv[r] = colbuf[b][lane + 64 * r];
        if (tid == 0) {
            perm[k] = p;
            rowpiv[p] = pv;
        }
        // rank-1 update with the pivot row read from lane lp, register row rp;
        // then the owner of column k + 1 searches that column's pivot and
        // publishes it for the next step.
        const int k1 = k + 1;
        const bool owner1 = k1 < n && wave == k1 % NWV;
        const int c1 = owner1 ? k1 / NWV : -1;
        // colv / pv, so that the pivot-row value read with readlane (a
        // scalar) feeds the FMA directly; column k uses pv + 1, which turns
        // column k into -D[i][k]/pv.  The pivot row is untouched (colv = 0).
        double colv_s[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) colv_s[r] = colv[r] * inv;
        // columns in chunks: the pivot-row values come from register row rp
        // (a scalar branch) of lane lp into scalar registers
        constexpr int CHK = CPW % 7 == 0 ? 7 : (CPW % 4 == 0 ? 4 : 1);
        static_for<0, CPW / CHK>([&](auto chc) __attribute__((always_inline)) {
            constexpr int c0 = decltype(chc)::value * CHK;
            double rv[CHK];
            auto grab = [&](auto rr) __attribute__((always_inline)) {
                constexpr int r = decltype(rr)::value;
#pragma unroll
                for (int j = 0; j < CHK; ++j) rv[j] = readlane_f64(M[r][c0 + j], lp);
            };
            if (rp == 0) grab(std::integral_constant<int, 0>{});
            if constexpr (RPL > 1) { if (rp == 1) grab(std::integral_constant<int, 1>{}); }
            if constexpr (RPL > 2) { if (rp == 2) grab(std::integral_constant<int, 2>{}); }
            if constexpr (RPL > 3) { if (rp == 3) grab(std::integral_constant<int, 3>{}); }
#pragma unroll
            for (int j = 0; j < CHK; ++j) {
                const int c = c0 + j;
                const double r_ = (wave == vk && c == ck) ? pv + 1.0 : rv[j];
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][c] = fma(-colv_s[r], r_, M[r][c]);
            }
        });
        if (owner1) {
            double col[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) col[r] = 0.0;
            static_for<0, CPW>([&](auto cc) __attribute__((always_inline)) {
                constexpr int c = decltype(cc)::value;
                if (c == c1) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) col[r] = M[r][c];
                }
            });
            const uint32_t used1 = used | (lane == lp ? 1u << rp : 0u);
            gj_search<RPL>(col, n, lane, used1, colbuf[b ^ 1], &piv_idx[b ^ 1], &piv_val[b ^ 1]);
        }
        if (lane == lp) used |= 1u << rp;
    }
    __syncthreads();

    double* Dw = Dinv + (size_t)w * nn;
    if (singular) {
        // undefined inverse: NaN, log|det| = -inf, sign = 0
        for (size_t q = tid; q < nn; q += NT) Dw[q] = __longlong_as_double(0x7ff8000000000000ll);
        if (tid == 0) {
            if (logdet) logdet[2 * w + spin] = s_flag == 1 ? -INFINITY : __longlong_as_double(0x7ff8000000000000ll);
            if (sign) sign[2 * w + spin] = 0;
            if (status) atomicOr(status + w, s_flag == 1 ? QSL_STATUS_SINGULAR : QSL_STATUS_NONFINITE);
        }
        return;
    }
    if (tid < 64) {
        // log|det| = sum log|pivot|, sign = sign(permutation) prod sign(pivot)
        double ld = 0.0;
        int neg = 0;
        for (int i = tid; i < n; i += 64) {
            ld += log(fabs(rowpiv[i]));
            neg += rowpiv[i] < 0.0;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            ld += __shfl_xor(ld, o);
            neg += __shfl_xor(neg, o);
        }
        if (tid == 0) {
            // parity of the pivot permutation by cycle counting (invp as scratch)
            for (int i = 0; i < n; ++i) invp[i] = 0;
            int cycles = 0;
            for (int i = 0; i < n; ++i) {
                if (invp[i]) continue;
                ++cycles;
                for (int j = i; !invp[j]; j = perm[j]) invp[j] = 1;
            }
            const int sg = ((neg + n - cycles) & 1) ? -1 : 1;
            if (logdet) logdet[2 * w + spin] = ld;
            if (sign) sign[2 * w + spin] = (int8_t)sg;
            if (status && !isfinite(ld)) atomicOr(status + w, QSL_STATUS_NONFINITE);
        }
    }
    __syncthreads();
    for (int k = tid; k < n; k += NT) invp[perm[k]] = k;
    __syncthreads();
    // the pivot entries were left at pv during the elimination (the pivot row
    // is never scaled); their value in the scaled representation is 1, and
    // later updates of them only added terms: M[p_k][k] += 1 - pv_k
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i >= n) continue;
        const int kp = invp[i];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            if (wave + NWV * c == kp) M[r][c] += 1.0 - rowpiv[i];
    }
    // D^-1[invp[i]][perm[e]] = M[i][e] / pivot(i), staged QC rows at a time
    int rowi[RPL];
    double rs[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        rowi[r] = i < n ? invp[i] : -1;
        rs[r] = i < n ? 1.0 / rowpiv[i] : 0.0;
    }
    for (int q0 = 0; q0 < n; q0 += QC) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int rr = rowi[r] - q0;
            if (rr >= 0 && rr < QC) {
#pragma unroll
                for (int c = 0; c < CPW; ++c) {
                    const int e = wave + NWV * c;
                    if (e < n) stage[rr][perm[e]] = M[r][c] * rs[r];
                }
            }
        }
        __syncthreads();
        const int rows = min(QC, n - q0);
        for (int q = tid; q < rows * n; q += NT) {
            const int rr = q / n, cc = q % n;
            Dw[(size_t)(q0 + rr) * n + cc] = stage[rr][cc];
        }
        __syncthreads();
    }
}

// Flag accesses in LDS.  The LDS executes the DS instructions of one wave in
// program order, so a flag written after a wave's data writes is seen only
// once they are done, and data read after a flag was seen is the data
// published before it; only the compiler has to keep the order (the
// signal fences), no wait is needed.
__device__ __forceinline__ int flag_load(int* f) {
    const int v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return v;
}
__device__ __forceinline__ void flag_store(int* f, int v) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------- 128 < n <= 224
// Half-wave layout (eight waves): lane li (< 32) of either half of a wave
// owns the D rows i = li + 32 r (r < RPL) and holds M[r][c] for CPW columns;
// 7 x 14 values per lane cover 224 x 224 with little padding.  The two
// halves of a wave own a pair of consecutive columns (column e: wave
// (e / 2) % 8, half e % 2, register column e / 16 before rotations), and a
// round publishes two elimination steps through LDS.  The wave owning the
// next round's columns looks ahead: it applies the current round's two
// steps to its register column 0 (both halves, in place), finds the first
// column's pivot, publishes its multipliers -D[i][k]/pv (0 in the pivot
// row), reads them back in the second half, applies that step to the
// second column and finds its pivot.  The other waves wait once per round
// and apply the two rank-1 updates in order: every half writes its segment
// of the pivot row (lane p % 32, register row p / 32) to LDS and reads it
// back broadcast; the owner of column k substitutes pv + 1 in its slot,
// which turns the column into -D[i][k]/pv (the pivot row itself is left
// unscaled).  Steps a look-ahead applied in place are skipped: a zero
// pivot-row entry in the owner's second half, and the look-ahead wave
// leaves out its register column 0 for the round it looked ahead from.
// No barrier per round: the publisher raises a flag in LDS, each wave
// records the last round whose inputs it has read, and a publisher
// overwrites a buffer (four, by round mod 4) only once every wave has read
// it.  A wave's register columns rotate by one after the round of its own
// columns, so the pair a wave handles next is always its register column
// 0; after R rotations register column c holds the D columns
// e = 16 ((c + R) mod CPW) + 2 v + h.

// v[r] for a wave-uniform r < RPL <= 8, by a three-level tree of selects
// on scalar conditions, not a chain of RPL - 1
template <int RPL>
__device__ __forceinline__ double select_row(const double (&v)[RPL], int r) {
    static_assert(RPL <= 8, "three levels");
    double t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = v[q < RPL ? q : RPL - 1];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < (4 >> s); ++q) t[q] = ((r >> s) & 1) ? t[2 * q + 1] : t[2 * q];
    return t[0];
}

// Pivot of the half `half` of a register column: its row si (0x7fffffff if
// none), value pv and reciprocal inv, all wave-uniform.  One 32-bit key per
// candidate row (unused, not past n, not NaN): the high word of |a| (sign
// 0, exponent, 20 significand bits) with its low 8 bits replaced by
// 255 - i; 0 elsewhere.  As unsigned integers the keys order like |a| to
// 2^-12 relative, and among values that close the smallest row wins; the
// row comes back from the key.  The maximum runs inside rows of 16 lanes by
// DPP (quad swaps, half-row and row mirrors), then over the half's two
// rows.  1/pv: hardware reciprocal and two Newton steps (the error squares
// each step).
template <int RPL>
__device__ __forceinline__ void gjh2_pivot(const double (&col)[RPL], int li, int half, uint32_t used, int& si,
                                           double& pv, double& inv) {
    uint32_t best = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = li + 32 * r;
        const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(col[r]) >> 32) & 0x7fffffffu;
        const uint32_t keep = ((used >> r) & 1u) - 1u;  // all ones for a candidate row
        const uint32_t kr = ((hi & ~0xFFu) | (uint32_t)(255 - i)) & keep;
        best = max(best, col[r] == col[r] ? kr : 0u);
    }
    best = max(best, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best, 0xB1, 0xf, 0xf, false));
    best = max(best, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best, 0x4E, 0xf, 0xf, false));
    best = max(best, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best, 0x141, 0xf, 0xf, false));
    best = max(best, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best, 0x140, 0xf, 0xf, false));
    const int l0 = 32 * half;
    const uint32_t gk = max((uint32_t)__builtin_amdgcn_readlane((int)best, l0),
                            (uint32_t)__builtin_amdgcn_readlane((int)best, l0 + 16));
    const bool any = gk != 0;
    si = any ? 255 - (int)(gk & 0xFF) : 0x7fffffff;
    const int rs = any ? si >> 5 : 0, ls = any ? si & 31 : 0;
    double cv = col[0];
#pragma unroll
    for (int r = 1; r < RPL; ++r) cv = rs == r ? col[r] : cv;
    pv = any ? readlane_f64(cv, l0 + ls) : 0.0;
    inv = __builtin_amdgcn_rcp(pv);
    inv = fma(inv, fma(-pv, inv, 1.0), inv);
    inv = fma(inv, fma(-pv, inv, 1.0), inv);
}

template <int RPL, int CPW, typename Tin>
__device__ __forceinline__ void gjh2_body(const Job& j, int bx) {
    const Tin* __restrict__ C = (const Tin*)j.C;
    const int n = j.n, spin = j.spin;
    double* __restrict__ Dinv = j.Dinv;
    double* __restrict__ logdet = j.logdet;
    int8_t* __restrict__ sign = j.sign;
    uint32_t* __restrict__ status = j.status;
    constexpr int NG = 16, NT = 512;
    constexpr int NR = 32 * RPL;  // capacity in D rows (MO index i)
    constexpr int NC = NG * CPW;  // capacity in D columns (electron index e)
    constexpr int QC = 32;        // rows of D^-1 staged per output pass
    constexpr int NB = 4;         // publication buffers, by round mod NB
    __shared__ double colbuf[NB][2][NR];
    __shared__ int piv_idx[NB][2];
    __shared__ double piv_val[NB][2];
    __shared__ __align__(16) double prow[NG][CPW];
    __shared__ int perm[NC];
    __shared__ int invp[NR];
    __shared__ double rowpiv[NR];
    __shared__ double stage[QC][NC > NR ? NC : NR];
    __shared__ double red_ld[NT / 64];
    __shared__ int red_neg[NT / 64];
    __shared__ int s_flag;
    __shared__ int pub;           // last round whose pivots and columns are published
    __shared__ int prog[NT / 64]; // last round each wave has read its inputs of
    __shared__ int s_abort;       // a wait ran over its bound

    const int w = bx;
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 31, h = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int g = wave + 8 * h;                                  // pivot-row segment of this half
    const size_t nn = (size_t)n * n;
    const Tin* C1 = C + (size_t)w * 5 * nn;  // derivative 0 block
    const int nr = (n + 1) / 2;              // rounds

    double M[RPL][CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int e = 16 * c + 2 * wave + h, i = li + 32 * r;
            const Tin v = gmem(C1)[min(e, n - 1) * n + min(i, n - 1)];
            M[r][c] = (e < n && i < n) ? (double)v : 0.0;
        }
    for (int k = tid; k < NB * 2 * NR; k += NT) colbuf[k / (2 * NR)][(k / NR) & 1][k % NR] = 0.0;
    if (tid == 0) { s_flag = 0; pub = -1; s_abort = 0; }
    if (tid < NT / 64) prog[tid] = -1;
    __syncthreads();
    constexpr int SPIN_LIMIT = 1 << 22;
    auto give_up = [&]() {
        if (lane == 0) flag_store(&s_abort, 1);
        return false;
    };
    auto stop = [&](int it) {  // the abort flag is polled every 64th time
        return (it & 63) == 63 && (it >= SPIN_LIMIT || __builtin_amdgcn_readfirstlane(flag_load(&s_abort)));
    };
    auto wait_consumed = [&](int round) -> bool {  // every wave has read the inputs of round
        for (int it = 0;; ++it) {
            const int pg = lane < NT / 64 ? flag_load(&prog[lane]) : 0x7fffffff;
            if (__ballot(pg < round) == 0) return true;
            if (stop(it)) return give_up();
            if (it >= 4) __builtin_amdgcn_s_sleep(1);
        }
    };
    auto row_bit = [&](int p) -> uint32_t { return li == (p & 31) ? 1u << (p >> 5) : 0u; };
    uint32_t used = 0;  // bit r: row li + 32 r already a pivot row, or past n
#pragma unroll
    for (int r = 0; r < RPL; ++r)
        if (li + 32 * r >= n) used |= 1u << r;
    int rot = 0;  // rotations of this wave's register columns (mod CPW)

    // Look-ahead of round rr by its owner wave: register column 0 holds the
    // columns 2 rr (half 0) and 2 rr + 1 (half 1) with every earlier step
    // applied; `u` marks the earlier pivot rows.  Returns false if a wait ran
    // over its bound.
    auto look_ahead = [&](int rr, uint32_t u) -> bool {
        const int b = rr % NB;
        const int pg = lane < NT / 64 ? flag_load(&prog[lane]) : 0x7fffffff;
        double col[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) col[r] = M[r][0];
        int sc;
        double pc, ic;
        gjh2_pivot<RPL>(col, li, 0, u, sc, pc, ic);
        bool ok = true;
        if (rr >= NB && __ballot(pg < rr - NB) != 0) ok = wait_consumed(rr - NB);
        if (h == 0) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = li + 32 * r;
                if (i < n) colbuf[b][0][i] = i == sc ? 0.0 : -col[r] * ic;
            }
        }
        if (lane == 0) { piv_idx[b][0] = sc; piv_val[b][0] = pc; }
        if (2 * rr + 1 < n) {
            // the first step on the second column (half 1), in place: its
            // multipliers back from the buffer, the pivot row's entry of
            // the second column from lane 32 + sc % 32
            double cv[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) cv[r] = colbuf[b][0][li + 32 * r];
            const double xc = sc < n ? readlane_f64(select_row<RPL>(col, sc >> 5), 32 + (sc & 31)) : 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const double y = fma(cv[r], xc, M[r][0]);
                M[r][0] = h ? y : M[r][0];
                col[r] = M[r][0];
            }
            int sd;
            double pd, id;
            gjh2_pivot<RPL>(col, li, 1, u | (sc < n ? row_bit(sc) : 0u), sd, pd, id);
            if (h == 1) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int i = li + 32 * r;
                    if (i < n) colbuf[b][1][i] = i == sd ? 0.0 : -col[r] * id;
                }
            }
            if (lane == 0) { piv_idx[b][1] = sd; piv_val[b][1] = pd; }
        }
        if (ok && lane == 0) flag_store(&pub, rr);
        return ok;
    };
    if (wave == 0 && !look_ahead(0, used)) {
        // a wait ran over its bound: reported below
    }

    bool singular = false;
    auto bad_pivot = [&](int p, double pv) {
        if (p >= n || !(pv != 0.0) || !isfinite(pv)) {
            singular = true;
            if (tid == 0) s_flag = isfinite(pv) || p >= n ? 1 : 2;
            return true;
        }
        return false;
    };
    for (int rd = 0; rd < nr; ++rd) {
        const int b = rd % NB;
        const int ns = 2 * rd + 1 < n ? 2 : 1;  // steps in this round
        bool live = true;
        int seen = rd;
        for (int it = 0;; ++it) {
            seen = __builtin_amdgcn_readfirstlane(flag_load(&pub));
            if (seen >= rd) break;
            if (stop(it)) { live = give_up(); break; }
            if (it >= 4) __builtin_amdgcn_s_sleep(1);
        }
        if (!live) break;
        // a wave behind the published rounds takes issue priority over its
        // SIMD mates until it has caught up
        if (seen >= rd + 2) __builtin_amdgcn_s_setprio(2);
        else if (seen == rd + 1) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        const int pa = __builtin_amdgcn_readfirstlane(piv_idx[b][0]);
        const double pva = readlane_f64(piv_val[b][0], 0);
        const int pb = ns == 2 ? __builtin_amdgcn_readfirstlane(piv_idx[b][1]) : 0;
        const double pvb = ns == 2 ? readlane_f64(piv_val[b][1], 0) : 1.0;
        double colv[RPL];  // multipliers of the round's first step
#pragma unroll
        for (int r = 0; r < RPL; ++r) colv[r] = colbuf[b][0][li + 32 * r];
        if (bad_pivot(pa, pva) || (ns == 2 && bad_pivot(pb, pvb))) break;
        const int own = rd & 7;  // the wave owning this round's columns
        const int r1 = rd + 1;
        const bool la = r1 < nr && wave == (r1 & 7);  // this wave looks ahead
        if (la) {
            // the round's steps on register column 0 (both halves, in place;
            // the regular update below leaves column 0 out), then round
            // rd + 1's pivots.  It is the step's critical path: first thing
            // after the inputs, at raised priority over the SIMD mate.
            __builtin_amdgcn_s_setprio(3);
            double m0[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) m0[r] = M[r][0];
            {
                const double xs = select_row<RPL>(m0, pa >> 5);
                const double x0 = readlane_f64(xs, pa & 31), x1 = readlane_f64(xs, 32 + (pa & 31));
                const double xm = h ? x1 : x0;
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][0] = fma(colv[r], xm, M[r][0]);
            }
            if (ns == 2) {
                double cb[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) { cb[r] = colbuf[b][1][li + 32 * r]; m0[r] = M[r][0]; }
                const double xs = select_row<RPL>(m0, pb >> 5);
                const double x0 = readlane_f64(xs, pb & 31), x1 = readlane_f64(xs, 32 + (pb & 31));
                const double xm = h ? x1 : x0;
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][0] = fma(cb[r], xm, M[r][0]);
            }
            const bool ok = look_ahead(r1, used | row_bit(pa) | (ns == 2 ? row_bit(pb) : 0u));
            __builtin_amdgcn_s_setprio(0);
            if (!ok) break;
        }
        // the round's steps in order; column 2 rd takes pv + 1 (its owner's
        // half 0), which turns it into -D[i][k]/pv; its owner's half 1 holds
        // column 2 rd + 1, which the look-ahead has already updated for the
        // first step (entry 0)
#pragma unroll 1
        for (int sidx = 0; sidx < ns; ++sidx) {
            const int p = sidx ? pb : pa;
            const double pv = sidx ? pvb : pva;
            if (sidx) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) colv[r] = colbuf[b][1][li + 32 * r];
            }
            if (sidx + 1 == ns && lane == 0) flag_store(&prog[wave], rd);  // after the reads of the round's inputs
            const int lp = p & 31, rp = p >> 5;
            if (li == lp) {
                static_for<0, RPL>([&](auto rr) __attribute__((always_inline)) {
                    constexpr int r = decltype(rr)::value;
                    if (rp == r) {
#pragma unroll
                        for (int c = 0; c < CPW; ++c) prow[g][c] = M[r][c];
                        asm volatile("; pivot row %0" ::"n"(r));
                    }
                });
            }
            if (wave == own && lane == 0) {
                if (sidx == 0) {
                    prow[own][0] = pv + 1.0;
                    prow[own + 8][0] = 0.0;
                } else {
                    prow[own + 8][0] = pv + 1.0;
                }
            }
            double pr[CPW];
#pragma unroll
            for (int c = 0; c < CPW; ++c) pr[c] = prow[g][c];
            if (!la) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][0] = fma(colv[r], pr[0], M[r][0]);
            }
#pragma unroll
            for (int c = 1; c < CPW; ++c)
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][c] = fma(colv[r], pr[c], M[r][c]);
            used |= row_bit(p);
            if (tid == 0) {
                perm[2 * rd + sidx] = p;
                rowpiv[p] = pv;
            }
        }
        if (wave == own) {  // both halves done with register column 0
            double t0[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) t0[r] = M[r][0];
#pragma unroll
            for (int c = 0; c + 1 < CPW; ++c)
#pragma unroll
                for (int r = 0; r < RPL; ++r) M[r][c] = M[r][c + 1];
#pragma unroll
            for (int r = 0; r < RPL; ++r) M[r][CPW - 1] = t0[r];
            rot = rot + 1 == CPW ? 0 : rot + 1;
        }
    }
    __syncthreads();
    if (s_abort) {  // reported as a non-finite result
        singular = true;
        if (tid == 0) s_flag = 2;
    }
    double* Dw = Dinv + (size_t)w * nn;
    if (singular) {
        // undefined inverse: NaN, log|det| = -inf, sign = 0
        for (size_t q = tid; q < nn; q += NT) Dw[q] = __longlong_as_double(0x7ff8000000000000ll);
        if (tid == 0) {
            if (logdet) logdet[2 * w + spin] = s_flag == 1 ? -INFINITY : __longlong_as_double(0x7ff8000000000000ll);
            if (sign) sign[2 * w + spin] = 0;
            if (status) atomicOr(status + w, s_flag == 1 ? QSL_STATUS_SINGULAR : QSL_STATUS_NONFINITE);
        }
        return;
    }
    // log|det| = sum log|pivot|; sign = sign(permutation) prod sign(pivot),
    // the permutation's sign from the parity of its inversions
    {
        double ld = 0.0;
        int neg = 0;
        if (tid < n) {
            ld = log(fabs(rowpiv[tid]));
            neg = rowpiv[tid] < 0.0;
            const int pa = perm[tid];
            for (int b2 = tid + 1; b2 < n; ++b2) neg += perm[b2] < pa;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            ld += __shfl_xor(ld, o);
            neg += __shfl_xor(neg, o);
        }
        if (lane == 0) { red_ld[wave] = ld; red_neg[wave] = neg; }
    }
    for (int k = tid; k < n; k += NT) invp[perm[k]] = k;
    __syncthreads();
    if (tid == 0) {
        double ld = 0.0;
        int neg = 0;
        for (int v = 0; v < NT / 64; ++v) { ld += red_ld[v]; neg += red_neg[v]; }
        if (logdet) logdet[2 * w + spin] = ld;
        if (sign) sign[2 * w + spin] = (neg & 1) ? -1 : 1;
        if (status && !isfinite(ld)) atomicOr(status + w, QSL_STATUS_NONFINITE);
    }
    // the pivot entries were left at pv during the elimination (the pivot row
    // is never scaled); their value in the scaled representation is 1, and
    // later updates of them only added terms: M[p_k][k] += 1 - pv_k
    int ec[CPW];  // D column of each register column
#pragma unroll
    for (int c = 0; c < CPW; ++c) ec[c] = 16 * (c + rot < CPW ? c + rot : c + rot - CPW) + 2 * wave + h;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = li + 32 * r;
        if (i >= n) continue;
        const int kp = invp[i];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
            if (ec[c] == kp) M[r][c] += 1.0 - rowpiv[i];
    }
    // D^-1[invp[i]][perm[e]] = M[i][e] / pivot(i), staged QC rows at a time
    int rowi[RPL];
    double rs[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = li + 32 * r;
        rowi[r] = i < n ? invp[i] : -1;
        rs[r] = i < n ? 1.0 / rowpiv[i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) ec[c] = ec[c] < n ? perm[ec[c]] : -1;  // destination column
    for (int q0 = 0; q0 < n; q0 += QC) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int rr = rowi[r] - q0;
            if (rr >= 0 && rr < QC) {
#pragma unroll
                for (int c = 0; c < CPW; ++c)
                    if (ec[c] >= 0) stage[rr][ec[c]] = M[r][c] * rs[r];
            }
        }
        __syncthreads();
        const int rows = min(QC, n - q0);
        for (int q = tid; q < rows * n; q += NT) {
            const int rr = q / n, cc = q % n;
            gmem(Dw)[(size_t)(q0 + rr) * n + cc] = stage[rr][cc];
        }
        __syncthreads();
    }
}

template <int RPL, int CPW, typename Tin>
__global__ __launch_bounds__(512) void gjh2_kernel(Job j) {
    gjh2_body<RPL, CPW, Tin>(j, blockIdx.x);
}
template <int RPL, int CPW, typename Tin>
__global__ __launch_bounds__(512) void gjh2_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& jj, int bx, int, int) { gjh2_body<RPL, CPW, Tin>(jj, bx); });
}
template <int NWV, int RPL, int CPW, typename Tin>
__global__ __launch_bounds__(NWV * 64) void gj_kernel(Job j) {
    gj_body<NWV, RPL, CPW, Tin>(j, blockIdx.x);
}

template <int NWV, int RPL, int CPW, typename Tin>
__global__ __launch_bounds__(NWV * 64) void gj_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { gj_body<NWV, RPL, CPW, Tin>(j, bx); });
}

__global__ void empty_spin_kernel(int64_t W, int spin, double* logdet, int8_t* sign) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w < W) {
        if (logdet) logdet[2 * w + spin] = 0.0;
        if (sign) sign[2 * w + spin] = 1;
    }
}

// Variants by matrix size: register-resident 0: n <= 32, 1: <= 64,
// 2: <= 128, 3: <= 224; 4: blocked, n <= 1024.
int gj_variant(int n) { return gj_blocked(n) ? 4 : n <= 32 ? 0 : n <= 64 ? 1 : n <= 128 ? 2 : 3; }
int gj_threads(int v) { return v == 0 ? 128 : v == 1 ? 256 : 512; }
int gj_job_variant(const Job& j) {
    const int v = gj_variant(j.n);
    return v == 4 ? 4 : std::min(3, v + std::max(0, j.gj_bias));
}

template <typename Tin>
static hipError_t gj_dispatch(const Job& j, int v, bool batched, const Job* jobs, const int* prefix, int njobs,
                              int grid, hipStream_t st) {
    const dim3 g((unsigned)(batched ? grid : j.W));
#define QSL_GJ(NWV, RPL, CPW)                                                                                   \
    do {                                                                                                        \
        if (batched) gj_batched<NWV, RPL, CPW, Tin><<<g, NWV * 64, 0, st>>>(jobs, prefix, njobs);         \
        else gj_kernel<NWV, RPL, CPW, Tin><<<g, NWV * 64, 0, st>>>(j);                                          \
    } while (0)
    switch (v) {
        case 0: QSL_GJ(2, 1, 16); break;
        case 1: QSL_GJ(4, 1, 16); break;
        case 2: QSL_GJ(8, 2, 16); break;
        default:
            if (batched) gjh2_batched<7, 14, Tin><<<g, 512, 0, st>>>(jobs, prefix, njobs);
            else gjh2_kernel<7, 14, Tin><<<g, 512, 0, st>>>(j);
            break;
    }
#undef QSL_GJ
    return hipGetLastError();
}

hipError_t launch_gj(const Job& j0, hipStream_t st) {
    if (j0.W <= 0) return hipSuccess;
    Job j = j0;
    j.gx = (int)j.W; j.gy = 1; j.gz = 1;
    if (j.n == 0) {
        empty_spin_kernel<<<(unsigned)((j.W + 255) / 256), 256, 0, st>>>(j.W, j.spin, j.logdet, j.sign);
        return hipGetLastError();
    }
    if (j.n > GJ_NMAX) return hipErrorInvalidValue;
    const int v = gj_job_variant(j);
    if (v == 4) return launch_gjb(j, st);
    if (j.mode == QSL_FP64) return gj_dispatch<double>(j, v, false, nullptr, nullptr, 0, 0, st);
    return gj_dispatch<float>(j, v, false, nullptr, nullptr, 0, 0, st);
}

// One batched launch of GJ variant v over Jobs whose n all fit it (the
// plan launches each variant present in its batch once; the blocked
// variant 4 is a sequence of launches over panels, see qsl_gjb.hip).
hipError_t launch_gj_batched(int mode, int v, const Job* jobs, const int* prefix, int njobs, int grid,
                             hipStream_t st) {
    if (v < 0 || v > 3) return hipErrorInvalidValue;
    if (grid <= 0) return hipSuccess;
    Job dummy{};
    if (mode == QSL_FP64) return gj_dispatch<double>(dummy, v, true, jobs, prefix, njobs, grid, st);
    return gj_dispatch<float>(dummy, v, true, jobs, prefix, njobs, grid, st);
}

}  // namespace qsl
