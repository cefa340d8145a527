// Adjoint of L = sum_w sum_s g[w][s] log|det D^s_w| (not in the paper: the
// chain rule through the MO expansion (mo) and D_ij = phi_i(r_j)).
//
// With G[e][i] = g Dinv[e][i] = dL/dC_1[e][i]:
//   dR_e       = sum_j H[e][j] grad chi_j(r_e),  H[e][j] = sum_i G[e][i] a_ij
//   dA^s[i][j] = sum_w sum_e G[e][i] chi_j(r_e)
// over the screened survivors (held fixed).  The AO values and gradients are
// recomputed here; the forward never stores them.
//
// Two kernels, both on MFMA in the forward's precision mode:
//  adj_h   one workgroup per tile (one electron index in 32 walkers, as in
//          the forward's contraction): G in LDS,
//          gradients of the tile's surviving AOs into LDS chunk by chunk,
//          H = G A (M = 32 electrons, N = 64 slots, K = MOs), dR = H . grad chi.
//  adj_dA  one workgroup per (electron range t, block of walkers, block of
//          surviving windows, block of MOs).  Electrons with the same index
//          sit in the same region of space across walkers, so the walker
//          block shares one window list.  The dA block (MOs x slots) stays in
//          the accumulators of eight waves while the walkers stream through
//          as the contraction dimension (32 electrons each); one coalesced
//          atomic flush per workgroup (FP32 into a workspace accumulator, or
//          FP64).
#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) double f64x4;


template <int MODE>
using TOf = typename std::conditional<MODE == QSL_FP64, double, float>::type;

// 32 x 32 accumulator block, 16 values per lane.  f32 modes: one 32x32 MFMA
// block (row 8(q/4) + 4(lane/32) + q%4, column lane%32).  FP64: 2 x 2
// blocks of 16x16 (row 16 bi + lane/16 + 4r, column 16 bj + lane%16).
template <int MODE>
struct Blk {
    using T = TOf<MODE>;
    T v[16];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = T(0);
    }
    __device__ __forceinline__ static int row(int q, int lane) {
        if constexpr (MODE == QSL_FP64) return ((q >> 3) << 4) + (lane >> 4) + 4 * (q & 3);
        else return 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
    }
    __device__ __forceinline__ static int col(int q, int lane) {
        if constexpr (MODE == QSL_FP64) return (((q >> 2) & 1) << 4) + (lane & 15);
        else return lane & 31;
    }
};

// acc += A(32 rows) x B(32 cols) over k in [k0, k1) for the FP32 and FP64
// modes; fa(row, k) and fb(k, col) fetch the operands.
template <int MODE, typename FA, typename FB>
__device__ __forceinline__ void mma_f(Blk<MODE>& acc, int k0, int k1, int lane, FA fa, FB fb) {
    if constexpr (MODE == QSL_FP32) {
        f32x16 a16;
#pragma unroll
        for (int q = 0; q < 16; ++q) a16[q] = acc.v[q];
        // two interleaved accumulators: consecutive MFMAs are independent
        f32x16 b16;
#pragma unroll
        for (int q = 0; q < 16; ++q) b16[q] = 0.f;
        const int kk = lane >> 5, rc = lane & 31;
        int k = k0;
        for (; k + 2 < k1; k += 4) {
            a16 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa(rc, k + kk), fb(k + kk, rc), a16, 0, 0, 0);
            b16 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa(rc, k + 2 + kk), fb(k + 2 + kk, rc), b16, 0, 0, 0);
        }
        for (; k < k1; k += 2)
            a16 = __builtin_amdgcn_mfma_f32_32x32x2f32(fa(rc, k + kk), fb(k + kk, rc), a16, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 16; ++q) acc.v[q] = a16[q] + b16[q];
    } else {
        f64x4 a4[2][2];
#pragma unroll
        for (int q = 0; q < 16; ++q) a4[q >> 3][(q >> 2) & 1][q & 3] = acc.v[q];
        const int kk = lane >> 4, rc = lane & 15;
        for (int k = k0; k < k1; k += 4) {
            double a[2], b[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) { a[h] = fa(h * 16 + rc, k + kk); b[h] = fb(k + kk, h * 16 + rc); }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    a4[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], a4[bi][bj], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc.v[q] = a4[q >> 3][(q >> 2) & 1][q & 3];
    }
}

// ---------------------------------------------------------------- adj_h

constexpr int AH_THREADS = 256;
constexpr int AH_KW = 8;                 // windows per chunk
constexpr int AH_KC = AH_KW * WIN;       // 64 slots

template <int MODE>
__device__ __forceinline__ void adj_h_body(const Job& j, int bx, int by) {
    const DevSys& s = j.s;
    const int spin = j.spin, n = j.n, ldn = j.mo.ldn;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    const int* __restrict__ tile_nwin = j.nwin;
    const int* __restrict__ tile_win = j.win;
    const uint16_t* __restrict__ AThi = j.mo.AThi;
    const uint16_t* __restrict__ ATlo = j.mo.ATlo;
    const float* __restrict__ A32 = j.mo.A32;
    const double* __restrict__ A64 = j.mo.A64;
    const double* __restrict__ Dinv = j.Dinv;
    const double* __restrict__ g = j.g;
    double* __restrict__ dR = j.dR;
    using T = TOf<MODE>;
    constexpr bool BF = MODE == QSL_BF16X3;
    constexpr int LDG = ADJ_MB + (BF ? 8 : 1);
    __shared__ double epos[TE][3];
    __shared__ int wq[AH_KW];
    __shared__ __attribute__((aligned(16))) unsigned char gbuf[BF ? 2 * 2 * TE * LDG : sizeof(T) * TE * LDG];
    __shared__ T dX[3][TE][AH_KC + 1];
    __shared__ T Hb[2][TE][AH_KC + 1];

    // row r of the tile is electron eidx of walker wr(r): position w0 + r of
    // the walker order (ne valid rows)
    const int tile = bx;
    const int wbk = walker_blocks(W);
    const int eidx = tile / wbk;
    const int w0 = (tile % wbk) * TE;
    const int ne = (int)min<int64_t>(TE, W - w0);
    auto wr = [&](int r) -> int64_t { return walker_of(j.wperm, W, eidx, w0 + r); };
    const int i0 = by * ADJ_MB;
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    uint16_t* Gh = (uint16_t*)gbuf;
    uint16_t* Gl = Gh + TE * LDG;
    T* Gt = (T*)gbuf;

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)wr(e) * N + eoff + eidx) * 3 + k] : 0.0;
    }
    for (int q = tid; q < TE * ADJ_MB; q += AH_THREADS) {
        const int e = q / ADJ_MB, ii = q % ADJ_MB;
        double v = 0.0;
        if (e < ne && i0 + ii < n) {
            const int64_t w = wr(e);
            const double gw = g[2 * w + spin];
            if (gw != 0.0) v = gw * Dinv[((size_t)w * n + eidx) * n + i0 + ii];
        }
        if constexpr (BF) {
            const float f = (float)v;
            const uint16_t h = bf16_rne(f);
            Gh[e * LDG + ii] = h;
            Gl[e * LDG + ii] = bf16_rne(f - bf16_to_f(h));
        } else {
            Gt[e * LDG + ii] = (T)v;
        }
    }
    const int nwin = tile_nwin[tile];
    const int* wins = tile_win + (size_t)tile * s.n_win;
    // dR partial sums: thread (electron tid % 32, slot group tid / 32 of 8
    // slots per chunk), three components; reduced over the groups at the end
    T dr[3] = {0, 0, 0};

    for (int c0 = 0; c0 < nwin; c0 += AH_KW) {
        __syncthreads();
        {
            const int e = tid & (TE - 1), wl = tid / TE;
            const int q = c0 + wl < nwin ? wins[c0 + wl] : -1;
            if (e == 0) wq[wl] = q;
            T vals[5][WIN];
            bool tie = false;
            if (q >= 0 && e < ne) {
                const double r[3] = {epos[e][0], epos[e][1], epos[e][2]};
                rec_values<T, WIN>(s.win_rec[q], s.T, 0, r, vals, tie);
            } else {
#pragma unroll
                for (int d = 0; d < 5; ++d)
#pragma unroll
                    for (int j = 0; j < WIN; ++j) vals[d][j] = T(0);
            }
#pragma unroll
            for (int j = 0; j < WIN; ++j)
#pragma unroll
                for (int d = 0; d < 3; ++d) dX[d][e][wl * WIN + j] = vals[1 + d][j];
        }
        __syncthreads();
        {   // wave: 32-slot block nb, half kh of the MOs
            const int nb = wave & 1, kh = wave >> 1;
            const int kb = kh * (ADJ_MB / 2), ke = kb + ADJ_MB / 2;
            Blk<MODE> acc;
            acc.zero();
            if constexpr (BF) {
                // the three products in three accumulators (independent chains)
                f32x16 a16, b16, c16;
#pragma unroll
                for (int q = 0; q < 16; ++q) a16[q] = b16[q] = c16[q] = 0.f;
                const int c = nb * 32 + (lane & 31);
                const int qc = wq[c / WIN] < 0 ? 0 : wq[c / WIN];
                const size_t wbase = (size_t)qc * (ldn / 8);
                const int oct = lane >> 5;
                for (int k0 = kb; k0 < ke; k0 += 16) {
                    const int ig = min(i0 + k0 + 8 * oct, ldn - 8);
                    const size_t offb = ((wbase + ig / 8) * WIN + (c % WIN)) * 8;
                    const bf16x8 bh = __builtin_bit_cast(bf16x8, *(const uint4*)(AThi + offb));
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, *(const uint4*)(ATlo + offb));
                    const int off = (lane & 31) * LDG + k0 + 8 * oct;
                    const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const uint4*)(Gh + off));
                    const bf16x8 al = __builtin_bit_cast(bf16x8, *(const uint4*)(Gl + off));
                    a16 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, a16, 0, 0, 0);
                    b16 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, b16, 0, 0, 0);
                    c16 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c16, 0, 0, 0);
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) acc.v[q] = a16[q] + (b16[q] + c16[q]);
            } else {
                int slotc[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = nb * 32 + (MODE == QSL_FP64 ? h * 16 + (lane & 15) : (lane & 31));
                    slotc[h] = (wq[c / WIN] < 0 ? 0 : wq[c / WIN]) * WIN + (c % WIN);
                }
                auto fa = [&](int r, int k) -> T { return Gt[r * LDG + k]; };
                auto fb = [&](int k, int cc) -> T {
                    const int ig = min(i0 + k, ldn - 1);
                    if constexpr (MODE == QSL_FP64) return A64[(size_t)ig * s.n_slots + slotc[cc >> 4]];
                    else return A32[(size_t)ig * s.n_slots + slotc[0]];
                };
                mma_f<MODE>(acc, kb, ke, lane, fa, fb);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) Hb[kh][Blk<MODE>::row(q, lane)][nb * 32 + Blk<MODE>::col(q, lane)] = acc.v[q];
        }
        __syncthreads();
        {
            const int e = tid & (TE - 1), cb = (tid >> 5) * (AH_KC / (AH_THREADS / TE));
#pragma unroll
            for (int c = cb; c < cb + AH_KC / (AH_THREADS / TE); ++c) {
                const T h = Hb[0][e][c] + Hb[1][e][c];
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) dr[comp] += h * dX[comp][e][c];
            }
        }
    }
    // reduce the slot groups (dX is free now) and add to dR
    __syncthreads();
    T* red = &dX[0][0][0];  // [3][groups][TE]
    {
        const int e = tid & (TE - 1), grp = tid >> 5;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) red[(comp * (AH_THREADS / TE) + grp) * TE + e] = dr[comp];
    }
    __syncthreads();
    if (tid < 3 * TE && dR) {
        const int e = tid & (TE - 1), comp = tid >> 5;
        T acc = 0;
#pragma unroll
        for (int grp = 0; grp < AH_THREADS / TE; ++grp) acc += red[(comp * (AH_THREADS / TE) + grp) * TE + e];
        if (e < ne) atomicAdd(dR + ((size_t)wr(e) * N + eoff + eidx) * 3 + comp, (double)acc);
    }
}

// --------------------------------------------------------------- adj_dA

constexpr int AD_THREADS = 512;          // 8 waves

template <int MODE>
struct AdCfg {
    using T = TOf<MODE>;
    static constexpr bool BF = MODE == QSL_BF16X3;
    static constexpr int NWB = MODE == QSL_FP64 ? 16 : 32;   // windows per block
    static constexpr int NS = NWB * WIN;                     // slots per block
    static constexpr int SB = NS / 32;                       // 32-slot blocks
    static constexpr int NBLK = ADJ_NIB * SB;                // 32x32 output blocks
    static constexpr int PB = (NBLK + 7) / 8;                // blocks per wave
    static constexpr int LDGT = BF ? TE + 8 : TE + 1;        // G^T [i][e]
    static constexpr int LDX = BF ? TE + 8 : NS + 1;         // chi: [slot][e] (bf16) or [e][slot]
};

template <int MODE>
__device__ __forceinline__ void adj_da_body(const Job& j, int bx, int by, int bz) {
    const DevSys& s = j.s;
    const int spin = j.spin, n = j.n, gw = j.gw;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    const int* __restrict__ grp_nwin = j.gnwin;
    const int* __restrict__ grp_win = j.gwin;
    const double* __restrict__ Dinv = j.Dinv;
    const double* __restrict__ g = j.g;
    double* __restrict__ dA64 = j.dA64;
    float* __restrict__ dA32 = j.dA32;
    using C = AdCfg<MODE>;
    using T = typename C::T;
    constexpr bool BF = C::BF;
    constexpr int NWB = C::NWB, NS = C::NS, SB = C::SB, NBLK = C::NBLK, PB = C::PB, LDGT = C::LDGT, LDX = C::LDX;
    // BF16X3 double-buffers the electron positions and G: the next walker's
    // are stored after this walker's MFMAs, one barrier per walker
    constexpr int NBUF = BF ? 2 : 1;
    __shared__ double epos[NBUF][TE][3];
    __shared__ int wq[NWB];
    __shared__ __attribute__((aligned(16))) unsigned char gbuf[BF ? NBUF * 2 * 2 * ADJ_MB * LDGT : sizeof(T) * ADJ_MB * LDGT];
    __shared__ __attribute__((aligned(16))) unsigned char xbuf[BF ? 2 * 2 * NS * LDX : sizeof(T) * TE * LDX];

    const int ngw = (int)((W + gw - 1) / gw);
    const int grp = j.t_fix >= 0 ? j.t_fix * ngw + bx : bx;
    const int t = grp / ngw, wb = grp % ngw;
    const int w0 = wb * gw;
    const int nw = (int)min<int64_t>(gw, W - w0);
    const int e0 = t * TE;
    const int ne = min(TE, n - e0);
    const int nwin = grp_nwin[grp];
    const int q0 = by * NWB;
    if (q0 >= nwin) return;
    const int nq = min(NWB, nwin - q0);
    const int i0 = bz * ADJ_MB;
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const double Tscr = readlane_f64(s.T, 0);                    // screening threshold, in scalar registers
    uint16_t* GTh = (uint16_t*)gbuf;  // the current buffer (hi, then lo)
    uint16_t* GTl = GTh + ADJ_MB * LDGT;
    T* GTt = (T*)gbuf;
    double(*ep)[3] = epos[0];
    uint16_t* Xh = (uint16_t*)xbuf;
    uint16_t* Xl = Xh + NS * LDX;
    T* Xt = (T*)xbuf;

    if (tid < NWB) wq[tid] = tid < nq ? grp_win[(size_t)grp * s.n_win + q0 + tid] : -1;
    // the block's windows are the same for every walker of the group: stage
    // their atom positions, slot monomials and shell primitives in LDS once
    constexpr int SPW = WIN;  // local shells per window (shells are consecutive slots)
    __shared__ double lw_pos[NWB][3];
    __shared__ int lw_pow[NWB][WIN];     // a | b<<4 | c<<8, -1 for padding
    __shared__ T lw_f[NWB][WIN];
    __shared__ int8_t lw_sh[NWB][WIN];   // local shell of the slot
    __shared__ int8_t lw_np[NWB][SPW];
    __shared__ double lw_exp[NWB][SPW][QSL_PMAX];
    __shared__ T lw_c[NWB][SPW][QSL_PMAX];
    __syncthreads();
    for (int p = tid; p < NWB * WIN; p += AD_THREADS) {
        const int wli = p / WIN, jj = p % WIN;
        const int q = wq[wli];
        int pw = -1, lsh = 0;
        T f = T(0);
        if (q >= 0) {
            const int slot = q * WIN + jj;
            const int sh = s.slot_shell[slot];
            if (sh >= 0) {
                pw = s.slot_pow[slot] & 0xfff;
                f = (T)s.slot_f[slot];
                lsh = sh - s.slot_shell[q * WIN];
            }
            if (jj == 0) {
                const int at = s.win_atom[q];
                for (int k = 0; k < 3; ++k) lw_pos[wli][k] = s.atom_xyz[3 * at + k];
            }
            // local shell jj of the window (if it exists)
            const int shl = s.slot_shell[q * WIN] + jj;
            int np = 0;
            if (shl < s.n_shells && s.win_atom[q] == s.shell_atom[shl]) {
                np = s.shell_np[shl];
                const int p0 = s.shell_p0[shl];
                for (int k = 0; k < np; ++k) {
                    lw_exp[wli][jj][k] = s.prim_exp[p0 + k];
                    if constexpr (sizeof(T) == 8) lw_c[wli][jj][k] = (T)s.prim_c64[p0 + k];
                    else lw_c[wli][jj][k] = s.prim_c32[p0 + k];
                }
            }
            lw_np[wli][jj] = (int8_t)np;
        }
        lw_pow[wli][jj] = pw;
        lw_f[wli][jj] = f;
        lw_sh[wli][jj] = (int8_t)lsh;
    }
    // BF16X3: X entries that no walker writes (electrons past the tile,
    // windows past the list, padding slots) stay zero from here on
    if constexpr (BF)
        for (int q = tid; q < (int)(sizeof(xbuf) / 4); q += AD_THREADS) ((uint32_t*)xbuf)[q] = 0u;
    // BF16X3: AO values of electron e at the 8 slots of block window wli,
    // written to X; a shell's radial factor is formed at its first slot from
    // its primitives (a primitive past the screening threshold is skipped, by
    // the whole wave when no lane keeps it).  The slot fields and the shell's
    // primitives are loaded at once.
    auto win_vals_bf = [&](int e, int wli) __attribute__((always_inline)) {
        int pws[WIN], lss[WIN];
        float fs[WIN];
#pragma unroll
        for (int jj = 0; jj < WIN; ++jj) {
            pws[jj] = lw_pow[wli][jj];
            lss[jj] = lw_sh[wli][jj];
            fs[jj] = (float)lw_f[wli][jj];
        }
        const double dx = ep[e][0] - lw_pos[wli][0], dy = ep[e][1] - lw_pos[wli][1],
                     dz = ep[e][2] - lw_pos[wli][2];
        const double r2 = dist2_exact(dx, dy, dz);
        const float X = (float)dx, Y = (float)dy, Z = (float)dz;
        int prev = -1;
        float gg = 0.f;
#pragma unroll
        for (int jj = 0; jj < WIN; ++jj) {
            const int pw = pws[jj], ls = lss[jj];
            if (pw < 0) continue;
            if (ls != prev) {
                gg = 0.f;
                const int np = lw_np[wli][ls];
                double exs[QSL_PMAX];
                float cs[QSL_PMAX];
#pragma unroll
                for (int k = 0; k < QSL_PMAX; ++k) {
                    exs[k] = lw_exp[wli][ls][k];
                    cs[k] = (float)lw_c[wli][ls][k];
                }
#pragma unroll
                for (int k = 0; k < QSL_PMAX; ++k) {
                    if (k >= np) break;
                    const double t = mul_exact(exs[k], r2);
                    if (t <= Tscr) gg += cs[k] * exp_t(-(float)t);
                }
                prev = ls;
            }
            const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15;
            const float px = a == 0 ? 1.f : (a == 1 ? X : X * X);
            const float py = b == 0 ? 1.f : (b == 1 ? Y : Y * Y);
            const float pz = c == 0 ? 1.f : (c == 1 ? Z : Z * Z);
            const float v = fs[jj] * px * py * pz * gg;
            const int ci = wli * WIN + jj;
            const uint16_t h = bf16_rne(v);
            Xh[ci * LDX + e] = h;
            Xl[ci * LDX + e] = bf16_rne(v - bf16_to_f(h));
        }
    };
    // FP32 / FP64: AO values of one electron at the 8 slots of block window
    // wli (zeros where the window is past the list)
    auto win_vals = [&](int wli, const double r[3], T vals[WIN]) __attribute__((always_inline)) {
#pragma unroll
        for (int jj = 0; jj < WIN; ++jj) vals[jj] = T(0);
        if (wq[wli] < 0) return;
        const double dx = r[0] - lw_pos[wli][0], dy = r[1] - lw_pos[wli][1], dz = r[2] - lw_pos[wli][2];
        const double r2 = dist2_exact(dx, dy, dz);
        const T X = (T)dx, Y = (T)dy, Z = (T)dz;
        int prev = -1;
        T gg = 0;
        // FP64: slot fields loaded together (in FP32 that costs spills)
        constexpr bool BATCH = MODE == QSL_FP64;
        int pws[BATCH ? WIN : 1], lss[BATCH ? WIN : 1];
        if constexpr (BATCH) {
#pragma unroll
            for (int jj = 0; jj < WIN; ++jj) {
                pws[jj] = lw_pow[wli][jj];
                lss[jj] = lw_sh[wli][jj];
            }
        }
#pragma unroll
        for (int jj = 0; jj < WIN; ++jj) {
            int pw, ls;
            if constexpr (BATCH) {
                pw = pws[jj];
                ls = lss[jj];
            } else {
                pw = lw_pow[wli][jj];
                ls = lw_sh[wli][jj];
            }
            if (pw < 0) continue;
            if (ls != prev) {
                gg = T(0);
                const int np = lw_np[wli][ls];
                for (int k = 0; k < np; ++k) {  // no registers to spare for a batch of loads
                    const double t = mul_exact(lw_exp[wli][ls][k], r2);
                    if (t <= Tscr) gg += lw_c[wli][ls][k] * exp_t(-(T)t);
                }
                prev = ls;
            }
            const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15;
            const T px = a == 0 ? T(1) : (a == 1 ? X : X * X);
            const T py = b == 0 ? T(1) : (b == 1 ? Y : Y * Y);
            const T pz = c == 0 ? T(1) : (c == 1 ? Z : Z * Z);
            vals[jj] = lw_f[wli][jj] * px * py * pz * gg;
        }
    };
    // the dA block in the accumulators: BF16X3 keeps the MFMA operand form
    Blk<MODE> acc[BF ? 1 : PB];
    f32x16 accv[BF ? PB : 1];
#pragma unroll
    for (int k = 0; k < PB; ++k) {
        if constexpr (BF) {
#pragma unroll
            for (int q = 0; q < 16; ++q) accv[k][q] = 0.f;
        } else {
            acc[k].zero();
        }
    }

    // D^-1 block of the next walker, loaded while the current one is used
    // (FP32 / FP64); in BF16X3 the rows of the split G^T (g_split), copied
    // to LDS as they are
    constexpr int GPT = BF ? 1 : (TE * ADJ_MB + AD_THREADS - 1) / AD_THREADS;
    constexpr int GQ = 2 * ADJ_MB * TE / 8;                      // uint4 of G^T hi + lo
    constexpr int GQT = BF ? (GQ + AD_THREADS - 1) / AD_THREADS : 1;
    static_assert(!BF || GQT == 4, "split-G staging is written for 4 rows of 16 bytes per thread");
    double gpre[GPT];
    uint4 gq0{}, gq1{}, gq2{}, gq3{};  // scalars: an array would be moved to LDS
    double gnext = 0.0;
    auto load_gs = [&](int w) __attribute__((always_inline)) {
        const int NIP = (n + ADJ_MB - 1) / ADJ_MB * ADJ_MB;
        const uint16_t* gh = j.gsplit + (((int64_t)w * tiles_per_walker(n) + t) * NIP + i0) * TE;
        const int64_t lo = j.W * gsplit_elems(n);
        auto at = [&](int k) -> const uint4* {
            const int q = tid + k * AD_THREADS;
            const int half = q >= GQ / 2, r = q - half * (GQ / 2);
            return (const uint4*)(gh + (q < GQ ? half * lo + (r >> 2) * TE + (r & 3) * 8 : 0));
        };
        gq0 = __builtin_bit_cast(uint4, *gmem(at(0)));
        gq1 = __builtin_bit_cast(uint4, *gmem(at(1)));
        gq2 = __builtin_bit_cast(uint4, *gmem(at(2)));
        gq3 = __builtin_bit_cast(uint4, *gmem(at(3)));
    };
    auto load_g = [&](int w) __attribute__((always_inline)) {
        if constexpr (BF) {
            load_gs(w);
            return;
        }
        gnext = g[2 * w + spin];
        // uniform base + 32-bit byte offsets (the block spans < 2^32 bytes)
        const char* Db = (const char*)(Dinv + ((size_t)w * n + e0) * n + i0);
#pragma unroll
        for (int k = 0; k < GPT; ++k) {
            const int q = tid + k * AD_THREADS;
            const int e = q / ADJ_MB, ii = q % ADJ_MB;
            const bool ok = q < TE * ADJ_MB && e < ne && i0 + ii < n;
            const uint32_t off = ok ? (uint32_t)(e * n + ii) * 8u : 0u;
            const double x = *(const double*)(Db + off);
            gpre[k] = ok ? x : 0.0;
        }
    };
    // electron coordinates of the tile, loaded one walker ahead with G
    auto load_pos = [&](int w) __attribute__((always_inline)) -> double {
        const int e = tid / 3, k = tid % 3;
        return tid < TE * 3 && e < ne ? gmem(R)[((size_t)w * N + eoff + e0 + e) * 3 + k] : 0.0;
    };
    constexpr bool PF = MODE != QSL_FP64;  // FP64: no registers to spare for the prefetch
    double pnext = PF ? load_pos(w0) : 0.0;
    if constexpr (PF) load_g(w0);
    // BF16X3: copy the prefetched split-G rows into buffer b
    auto put_g = [&](int b) __attribute__((always_inline)) {
        uint16_t* gh = (uint16_t*)gbuf + b * 2 * ADJ_MB * LDGT;
        uint16_t* gl = gh + ADJ_MB * LDGT;
        auto put = [&](int k, const uint4& v) {
            const int q = tid + k * AD_THREADS;
            if (q >= GQ) return;
            const int half = q >= GQ / 2, r = q - half * (GQ / 2);
            *(uint4*)((half ? gl : gh) + (r >> 2) * LDGT + (r & 3) * 8) = v;
        };
        put(0, gq0);
        put(1, gq1);
        put(2, gq2);
        put(3, gq3);
    };
    if constexpr (BF) {  // walker w0 into buffer 0, walker w0 + 1 in flight
        if (tid < TE * 3) epos[0][tid / 3][tid % 3] = pnext;
        put_g(0);
        if (nw > 1) {
            load_g(w0 + 1);
            pnext = load_pos(w0 + 1);
        }
        __syncthreads();
    }
    for (int wl = 0; wl < nw; ++wl) {
        const int w = w0 + wl;
        if constexpr (BF) {
            const int b = wl & 1;
            GTh = (uint16_t*)gbuf + b * 2 * ADJ_MB * LDGT;
            GTl = GTh + ADJ_MB * LDGT;
            ep = epos[b];
        } else {
            __syncthreads();  // previous walker's operands are consumed
            if (tid < TE * 3) epos[0][tid / 3][tid % 3] = PF ? pnext : load_pos(w);
            if constexpr (!PF) load_g(w);
            const double gwv = gnext;
#pragma unroll
            for (int k = 0; k < GPT; ++k) {
                const int q = tid + k * AD_THREADS;
                if (q >= TE * ADJ_MB) continue;
                const int e = q / ADJ_MB, ii = q % ADJ_MB;
                GTt[ii * LDGT + e] = (T)(gwv != 0.0 ? gwv * gpre[k] : 0.0);
            }
            if constexpr (PF) {
                if (wl + 1 < nw) load_g(w + 1);
            }
            // after the G prefetch, so that the G stores above never wait for it
            if (PF && wl + 1 < nw) pnext = load_pos(w + 1);
            __syncthreads();
        }
        // AO values of (electron, window) into LDS.  BF16X3: wave w evaluates
        // the windows of its own slot block (windows w, w + 8, w + 16,
        // w + 24, a mix of slot patterns), which no other wave reads, so no
        // barrier separates its evaluation from its MFMAs: the waves of a
        // SIMD drift apart and one's MFMAs overlap the other's evaluation.
        if constexpr (BF) {
            static_assert(NWB == 4 * (AD_THREADS / 64), "four windows per wave");
            const int e = lane & (TE - 1);
#pragma unroll 1
            for (int it = 0; it < 2; ++it) {
                const int wli = wave + 8 * ((lane >> 5) + 2 * it);
                if (e < ne && wq[wli] >= 0) win_vals_bf(e, wli);
            }
            // this wave's X rows are written before its lanes read them (one
            // wave's LDS operations complete in order; the fence keeps the
            // compiler from moving the reads up)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int p = tid; p < TE * NWB; p += AD_THREADS) {
            const int e = p & (TE - 1), wli = p / TE;
            if constexpr (!BF) {
                T vals[WIN];
                const double r[3] = {ep[e][0], ep[e][1], ep[e][2]};
                if (e < ne) win_vals(wli, r, vals);
                else {
#pragma unroll
                    for (int jj = 0; jj < WIN; ++jj) vals[jj] = T(0);
                }
#pragma unroll
                for (int j = 0; j < WIN; ++j) Xt[e * LDX + wli * WIN + j] = vals[j];
            }
        }
        if constexpr (!BF) __syncthreads();
        if constexpr (BF) {
            // wave w owns slot block w (column c: slot c % 8 of window
            // w + 8 (c / 8)) and every MO block k
            static_assert(SB == 8 && PB == ADJ_NIB && PB == 7, "one slot block per wave, seven MO blocks");
            // Every MO block of the staged G runs, also those past n: their G
            // rows are zeros (g_split pads to whole blocks), and a branch per
            // block costs more registers than the MFMAs it would skip.  Blocks
            // go in groups of two (the last group takes three): a block's
            // products are an MFMA of its partner apart.  The operands of the
            // next group are read while this group's MFMAs run; scheduling
            // barriers keep that order (and the register count) as written.
            // Every index is a compile-time constant, so the accumulators stay
            // in registers.
            if (wave < nq) {
                constexpr int NG = PB / 2;
                constexpr int GMAX = PB - 2 * (NG - 1);
                constexpr int NST = 2 * NG;  // (k-step, group) steps
                const int oct = lane >> 5;
                bf16x8 bh[2], bl[2], ah[2][GMAX], al[2][GMAX];
                const int xrow = (wave + 8 * ((lane & 31) >> 3)) * WIN + (lane & 7);
                static_for<0, 2>([&](auto h) {
                    const int offb = xrow * LDX + 16 * h + 8 * oct;
                    bh[h] = __builtin_bit_cast(bf16x8, *(const uint4*)(Xh + offb));
                    bl[h] = __builtin_bit_cast(bf16x8, *(const uint4*)(Xl + offb));
                });
                auto load = [&](auto st_c) __attribute__((always_inline)) {
                    constexpr int st = decltype(st_c)::value;
                    constexpr int h = st / NG, g = st % NG, kb = 2 * g, kn = g == NG - 1 ? PB - kb : 2;
                    static_for<0, kn>([&](auto u) {
                        const int offa = ((kb + u) * 32 + (lane & 31)) * LDGT + 16 * h + 8 * oct;
                        ah[st & 1][u] = __builtin_bit_cast(bf16x8, *(const uint4*)(GTh + offa));
                        al[st & 1][u] = __builtin_bit_cast(bf16x8, *(const uint4*)(GTl + offa));
                    });
                };
                load(std::integral_constant<int, 0>{});
                static_for<0, NST>([&](auto st_c) {
                    constexpr int st = decltype(st_c)::value;
                    if constexpr (st + 1 < NST) load(std::integral_constant<int, st + 1>{});
                    __builtin_amdgcn_sched_barrier(0);
                    constexpr int h = st / NG, g = st % NG, kb = 2 * g, kn = g == NG - 1 ? PB - kb : 2;
                    constexpr int bb = st & 1;
                    static_for<0, kn>([&](auto u) {
                        accv[kb + u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bb][u], bh[h], accv[kb + u], 0, 0, 0);
                    });
                    static_for<0, kn>([&](auto u) {
                        accv[kb + u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bb][u], bl[h], accv[kb + u], 0, 0, 0);
                    });
                    static_for<0, kn>([&](auto u) {
                        accv[kb + u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bb][u], bh[h], accv[kb + u], 0, 0, 0);
                    });
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
            if (wl + 1 < nw) {  // walker w + 1 into the other buffers, w + 2 in flight
                if (tid < TE * 3) epos[(wl + 1) & 1][tid / 3][tid % 3] = pnext;
                put_g((wl + 1) & 1);
                if (wl + 2 < nw) {
                    load_g(w + 2);
                    pnext = load_pos(w + 2);
                }
            }
            // the one barrier per walker: this walker's MFMAs are done with G
            // and the next walker's positions and G are visible
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < PB; ++k) {
                const int b = wave + 8 * k;
                if (b >= NBLK) continue;
                const int ib = b / SB, sb = b % SB;
                if (i0 + ib * 32 >= n || sb * 32 >= nq * WIN) continue;
                auto fa = [&](int r, int kk) -> T { return GTt[(ib * 32 + r) * LDGT + kk]; };
                auto fb = [&](int kk, int cc) -> T { return Xt[kk * LDX + sb * 32 + cc]; };
                mma_f<MODE>(acc[k], 0, TE, lane, fa, fb);
            }
        }
    }
    // one coalesced flush: the lanes of one accumulator register cover
    // consecutive slots of one MO row
#pragma unroll
    for (int k = 0; k < PB; ++k) {
        const int b = wave + 8 * k;
        if (b >= NBLK) continue;
        const int ib = b / SB, sb = b % SB;
        // (BF16X3: slot block sb starts with window sb)
        if (i0 + ib * 32 >= n || (BF ? sb >= nq : sb * 32 >= nq * WIN)) continue;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = i0 + ib * 32 + Blk<MODE>::row(q, lane);
            const int c = sb * 32 + Blk<MODE>::col(q, lane);
            // BF16X3 columns: slot c % 8 of window sb + 8 ((c % 32) / 8)
            const int wc = BF ? sb + 8 * ((c & 31) >> 3) : c / WIN;
            const int qw = wq[wc];
            T v;
            if constexpr (BF) v = accv[k][q];
            else v = acc[k].v[q];
            if (i >= n || qw < 0 || v == T(0)) continue;
            const int ao = s.slot_ao[qw * WIN + (c % WIN)];
            if (ao < 0) continue;
            if (j.dApart) {
                // this (walker group, MO, AO) has one writer per launch
                T* pt = (T*)j.dApart + ((size_t)wb * n + i) * s.n_basis + ao;
                *pt += v;
            } else if constexpr (MODE == QSL_FP64) {
                if (dA64) atomicAdd(dA64 + (size_t)i * s.n_basis + ao, v);
            } else {
                if (dA32) atomicAdd(dA32 + (size_t)i * s.n_basis + ao, v);
            }
        }
    }
}

// ------------------------------------------------- dA by electron (FP32)
// dA[i][slot] += sum over the walkers w of a group of
//   G_w[e][i] chi_slot(r_we),   G_w = g_w D_w^-1 (0 where g_w = 0),
// for one electron index e at a time: its walkers share one exact slot list
// (group_slots), so the products run over those slots only.  One 256-thread
// workgroup per (electron, walker group, chunk stride, 224 MOs); it takes
// the chunks cs, cs + DE_NCH, ... of 128 slots of the list.  Per chunk the
// 224 x 128 block of dA stays in the accumulators (wave v: slot block v,
// seven MO blocks) while the group's walkers stream through 32 at a time as
// the contraction dimension (v_mfma_f32_32x32x2f32, k-step s taking walkers
// 2s and 2s + 1); one atomic flush per chunk into the FP32 accumulator.
// Per batch of 32 walkers: the G rows (FP32, written by the epilogue or the
// g32 pre-pass) are copied from global memory straight into LDS while the
// AO values of the batch are evaluated (each thread keeps the record of its
// slot in registers for the whole chunk), then the 16 k-steps run.
constexpr int DE_NS = 128;  // slots per chunk (four waves x 32)
constexpr int DE_MB = ADJ_MB;  // MOs per workgroup (seven blocks of 32)
constexpr int DE_KW = 32;   // walkers per batch
constexpr int DE_NCH = 4;   // chunk stride: workgroups per (electron, group, MO block)
constexpr int DE_THREADS = 256;
constexpr int DE_GP = DE_KW * DE_MB / 4;  // 16-byte pieces of a batch's G rows
constexpr int DE_LDX = DE_NS + 32;        // AO value rows: walkers 2s and 2s + 1 in other banks
static_assert(DE_NS == (DE_THREADS / 64) * 32, "one 32-slot block per wave");
static_assert(DE_NCH == 4, "the block mapping puts the four chunk strides of a group on one XCD");
static_assert(DE_GP % DE_THREADS == 0, "whole passes of the G copy");

// A slot record in registers: what the value of the AO needs.
struct SlotRegs {
    double x, y, z;
    double ex[QSL_PMAX];
    float c[QSL_PMAX];
    float f;
    int pw, np;
    __device__ __forceinline__ void load(const SlotRec& r) {
        x = r.pos[0]; y = r.pos[1]; z = r.pos[2];
#pragma unroll
        for (int k = 0; k < QSL_PMAX; ++k) {
            ex[k] = r.ex[k];
            c[k] = r.c32[k];
        }
        f = r.f32; pw = r.pw; np = r.np;
    }
    // Value at electron p (FP32 AO arithmetic, FP64 screening as in the
    // forward).
    __device__ __forceinline__ float value(double T_thr, double px, double py, double pz) const {
        const double dx = px - x, dy = py - y, dz = pz - z;
        const double r2 = dist2_exact(dx, dy, dz);
        float g = 0.f;
#pragma unroll
        for (int k = 0; k < QSL_PMAX; ++k) {
            if (k < np) {
                const double t = mul_exact(ex[k], r2);
                if (t <= T_thr) g += c[k] * exp_t(-(float)t);
            }
        }
        float p1, p2, p3, d, d2;
        axis_pow(pw & 15, (float)dx, p1, d, d2);
        axis_pow((pw >> 4) & 15, (float)dy, p2, d, d2);
        axis_pow((pw >> 8) & 15, (float)dz, p3, d, d2);
        return (f * p2 * p3) * p1 * g;
    }
};

__device__ __forceinline__ void adj_dae_body(const Job& j, int bx, int by) {
    const DevSys& s = j.s;
    const int n = j.n, gw = j.gw, spin = j.spin;
    const int64_t W = j.W;
    const int ngw = (int)((W + gw - 1) / gw);
    // blocks 32 t + o: group 8 t + o % 8, chunk stride o / 8.  The hardware
    // hands consecutive blocks to the eight XCDs in turn, and every Job's
    // block count is a multiple of 32 (adj_dae_grid), so the four chunk
    // workgroups of a group run on one XCD and read its G rows through one L2.
    const int o = bx & 31;
    const int grp = (bx >> 5) * 8 + (o & 7), cs = o >> 3;
    if (grp >= j.n * ngw) return;
    const int e = grp / ngw, g = grp % ngw;
    const int nsl = j.gnwin[grp];
    if (cs * DE_NS >= nsl) return;
    const int* __restrict__ sl = j.gwin + (size_t)grp * WIN * s.n_win;
    const int64_t w0 = (int64_t)g * gw;
    const int nw = (int)min<int64_t>(gw, W - w0);
    const int i0 = by * DE_MB;
    const int ldg = g32_ld(n);
    const int N = s.n_up + s.n_dn, eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double Tscr = readlane_f64(s.T, 0);
    const float* __restrict__ G32 = j.g32;
    const SlotRec* __restrict__ srec = s.slot_rec;
    float* __restrict__ dA32 = j.dA32;

    __shared__ double ep[DE_KW][3];
    __shared__ int wl[DE_KW];  // the batch's walkers (Job.wperm order)
    __shared__ __attribute__((aligned(16))) float X[DE_KW * DE_LDX];
    __shared__ __attribute__((aligned(16))) float G[DE_KW * DE_MB];
    __shared__ int qao[DE_NS];
    // walker of position wb + tid of the group (tid < 32) and coordinate
    // tid of batch wb (tid < 96; -1 past the group)
    auto walker_at = [&](int wb) -> int {
        return wb + tid < nw ? (int)walker_of(j.wperm, W, e, w0 + wb + tid) : -1;
    };
    auto pos_of = [&](int wb) -> double {
        const int k = tid / 3;
        return wb + k < nw ? j.R[((size_t)walker_of(j.wperm, W, e, w0 + wb + k) * N + eoff + e) * 3 + tid % 3] : 0.0;
    };

    for (int c0 = cs * DE_NS; c0 < nsl; c0 += DE_NCH * DE_NS) {
        const int cnt = min(DE_NS, nsl - c0);
        __syncthreads();  // the previous chunk's flush is done with qao
        if (tid < DE_NS) qao[tid] = tid < cnt ? s.slot_ao[sl[c0 + tid]] : -1;
        // this thread's slot (slots past the chunk repeat its last; their
        // values are not computed)
        const int ql = tid & (DE_NS - 1);
        const bool live = ql < cnt;
        SlotRegs rg;
        rg.load(srec[sl[c0 + min(ql, cnt - 1)]]);
        f32x16 acc[DE_MB / 32];
#pragma unroll
        for (int mb = 0; mb < DE_MB / 32; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mb][r] = 0.f;
        double pnext = tid < DE_KW * 3 ? pos_of(0) : 0.0;
        int wnext = tid < DE_KW ? walker_at(0) : 0;
        for (int wb = 0; wb < nw; wb += DE_KW) {
            const int kw = min(DE_KW, nw - wb);
            __syncthreads();  // the previous batch's products are done with X, G, ep and wl; qao is visible
            if (tid < DE_KW * 3) ep[tid / 3][tid % 3] = pnext;
            if (tid < DE_KW) wl[tid] = wnext;
            __syncthreads();  // positions and walkers of the batch visible
            // G rows of the batch straight into LDS: piece p = 56 row + c of
            // 16 bytes; rows past the group repeat its last walker (their
            // AO values are zero)
#pragma unroll
            for (int ps = 0; ps < DE_GP / DE_THREADS; ++ps) {
                const int p = ps * DE_THREADS + tid;
                const int row = min(p / (DE_MB / 4), kw - 1), c = p % (DE_MB / 4);
                const float* src = G32 + ((size_t)wl[row] * n + e) * ldg + i0 + 4 * c;
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (__attribute__((address_space(3))) void*)&G[(ps * DE_THREADS + wave * 64) * 4],
                                                 16, 0, 0);
            }
            if (wb + DE_KW < nw) {
                if (tid < DE_KW * 3) pnext = pos_of(wb + DE_KW);
                if (tid < DE_KW) wnext = walker_at(wb + DE_KW);
            }
            // AO values: thread (slot tid % 128, walkers of parity tid / 128)
#pragma unroll 1
            for (int k = tid >> 7; k < DE_KW; k += 2) {
                float v = 0.f;
                if (live && k < kw) v = rg.value(Tscr, ep[k][0], ep[k][1], ep[k][2]);
                X[k * DE_LDX + ql] = v;
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's copies into LDS have landed
            __syncthreads();
            if (wave * 32 < cnt) {
                const int h = lane >> 5, c = lane & 31;
                // every MO block runs: G is zero past n, so blocks there add
                // zeros (per-block branches kept the compiler from batching
                // the operand reads).  The operands of k-step s + 1 are read
                // before the MFMAs of k-step s.
                constexpr int NMB = DE_MB / 32;
                float a[2][NMB], bv[2];
                auto fetch = [&](int s2, int q) __attribute__((always_inline)) {
                    const int k = 2 * s2 + h;
                    bv[q] = X[k * DE_LDX + wave * 32 + c];
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb) a[q][mb] = G[k * DE_MB + mb * 32 + c];
                };
                fetch(0, 0);
#pragma unroll
                for (int s2 = 0; s2 < DE_KW / 2; ++s2) {
                    if (s2 + 1 < DE_KW / 2) fetch(s2 + 1, (s2 + 1) & 1);
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb)
                        acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s2 & 1][mb], bv[s2 & 1], acc[mb], 0, 0, 0);
                    // schedule: the next k-step's LDS reads, then this one's MFMAs
                    if (s2 + 1 < DE_KW / 2) __builtin_amdgcn_sched_group_barrier(0x100, NMB + 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, NMB, 0);
                }
            }
        }
        // flush: lanes of one register cover 32 consecutive slots of one MO
        // row; row di of the lane's base row adds di N_b to its address (the
        // base and row limit are made opaque here, so that the 112 row
        // offsets are not computed ahead of the loop and held in registers)
        if (wave * 32 < cnt) {
            const int col = wave * 32 + (lane & 31);
            const int ao = col < cnt ? qao[col] : -1;
            int nbas = __builtin_amdgcn_readfirstlane(s.n_basis);
            int lim = n - i0 - 4 * (lane >> 5);  // rows di < lim exist
            asm volatile("" : "+s"(nbas));
            asm volatile("" : "+v"(lim));
            float* rowp = dA32 + (size_t)(i0 + 4 * (lane >> 5)) * nbas + max(ao, 0);
#pragma unroll
            for (int mb = 0; mb < DE_MB / 32; ++mb) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int di = mb * 32 + 8 * (r >> 2) + (r & 3);
                    const float v = acc[mb][r];
                    if (di < lim && ao >= 0 && v != 0.f) atomicAdd(rowp + (size_t)di * nbas, v);
                }
            }
        }
    }
}

// The same dA with the products on split-bf16 MFMA (FP32 tile 2): G and
// the AO values are split exactly into three bf16 each (x = hi + mid + lo)
// and dA += the six leading products on v_mfma_f32_32x32x16_bf16 (K = 16
// walkers), FP32 accumulation; per product 2^-23 relative next to the
// 2^-24 of an FP32 one.  The batch's G rows pass through registers into
// three transposed bf16 planes [plane][MO][walker] (shared by the four
// waves); each wave splits the AO values of its own 32 slots when it forms
// its operand.
constexpr int DS_GW = DE_KW + 8;        // bf16 row stride (walkers) of the G planes
constexpr int DS_PL = DE_MB * DS_GW;    // elements per plane
constexpr int DS_UNITS = (DE_MB / 4) * (DE_KW / 2);  // (MO quad, walker pair) units of the G split
constexpr int DS_PASS = (DS_UNITS + DE_THREADS - 1) / DE_THREADS;

__device__ __forceinline__ void adj_dae_s3_body(const Job& j, int bx, int by) {
    typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
    const DevSys& s = j.s;
    const int n = j.n, gw = j.gw, spin = j.spin;
    const int64_t W = j.W;
    const int ngw = (int)((W + gw - 1) / gw);
    // the XCD-aware block mapping of adj_dae_body
    const int o = bx & 31;
    const int grp = (bx >> 5) * 8 + (o & 7), cs = o >> 3;
    if (grp >= j.n * ngw) return;
    const int e = grp / ngw, g = grp % ngw;
    const int nsl = j.gnwin[grp];
    if (cs * DE_NS >= nsl) return;
    const int* __restrict__ sl = j.gwin + (size_t)grp * WIN * s.n_win;
    const int64_t w0 = (int64_t)g * gw;
    const int nw = (int)min<int64_t>(gw, W - w0);
    const int i0 = by * DE_MB;
    const int ldg = g32_ld(n);
    const int N = s.n_up + s.n_dn, eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double Tscr = readlane_f64(s.T, 0);
    const float* __restrict__ G32 = j.g32;
    const SlotRec* __restrict__ srec = s.slot_rec;
    float* __restrict__ dA32 = j.dA32;

    __shared__ double ep[DE_KW][3];
    __shared__ int wl[DE_KW];
    __shared__ __attribute__((aligned(16))) float X[DE_KW * DE_LDX];
    __shared__ __attribute__((aligned(16))) uint16_t G3[3 * DS_PL];
    __shared__ int qao[DE_NS];
    auto walker_at = [&](int wb) -> int {
        return wb + tid < nw ? (int)walker_of(j.wperm, W, e, w0 + wb + tid) : -1;
    };
    auto pos_of = [&](int wb) -> double {
        const int k = tid / 3;
        return wb + k < nw ? j.R[((size_t)walker_of(j.wperm, W, e, w0 + wb + k) * N + eoff + e) * 3 + tid % 3] : 0.0;
    };

    for (int c0 = cs * DE_NS; c0 < nsl; c0 += DE_NCH * DE_NS) {
        const int cnt = min(DE_NS, nsl - c0);
        __syncthreads();  // the previous chunk's flush is done with qao
        if (tid < DE_NS) qao[tid] = tid < cnt ? s.slot_ao[sl[c0 + tid]] : -1;
        const int ql = tid & (DE_NS - 1);
        const bool live = ql < cnt;
        SlotRegs rg;
        rg.load(srec[sl[c0 + min(ql, cnt - 1)]]);
        f32x16 acc[DE_MB / 32];
#pragma unroll
        for (int mb = 0; mb < DE_MB / 32; ++mb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mb][r] = 0.f;
        double pnext = tid < DE_KW * 3 ? pos_of(0) : 0.0;
        int wnext = tid < DE_KW ? walker_at(0) : 0;
        for (int wb = 0; wb < nw; wb += DE_KW) {
            const int kw = min(DE_KW, nw - wb);
            __syncthreads();  // the previous batch's products are done with X, G3, ep and wl
            if (tid < DE_KW * 3) ep[tid / 3][tid % 3] = pnext;
            if (tid < DE_KW) wl[tid] = wnext;
            __syncthreads();  // positions and walkers of the batch visible
            // G rows into registers: unit u = (MO quad u / 16, walker pair
            // u % 16), its 16-byte pieces of both walkers' rows (rows past the
            // group repeat its last walker: their AO values are zero)
            float4 ga[DS_PASS], gb[DS_PASS];
#pragma unroll
            for (int ps = 0; ps < DS_PASS; ++ps) {
                const int u = ps * DE_THREADS + tid;
                const int kp = u % (DE_KW / 2), mq = min(u / (DE_KW / 2), DE_MB / 4 - 1);
                const int r0 = min(2 * kp, kw - 1), r1 = min(2 * kp + 1, kw - 1);
                ga[ps] = *(const float4*)(G32 + ((size_t)wl[r0] * n + e) * ldg + i0 + 4 * mq);
                gb[ps] = *(const float4*)(G32 + ((size_t)wl[r1] * n + e) * ldg + i0 + 4 * mq);
            }
            if (wb + DE_KW < nw) {
                if (tid < DE_KW * 3) pnext = pos_of(wb + DE_KW);
                if (tid < DE_KW) wnext = walker_at(wb + DE_KW);
            }
            // AO values (FP32): thread (slot tid % 128, walkers of parity tid / 128)
#pragma unroll 1
            for (int k = tid >> 7; k < DE_KW; k += 2) {
                float v = 0.f;
                if (live && k < kw) v = rg.value(Tscr, ep[k][0], ep[k][1], ep[k][2]);
                X[k * DE_LDX + ql] = v;
            }
            // the G planes: per unit and MO, one packed pair (walkers 2 kp,
            // 2 kp + 1) per plane; sixteen lanes fill one row's 64 bytes
#pragma unroll
            for (int ps = 0; ps < DS_PASS; ++ps) {
                const int u = ps * DE_THREADS + tid;
                if (u < DS_UNITS) {
                    const int kp = u % (DE_KW / 2), mq = u / (DE_KW / 2);
                    const float va[4] = {ga[ps].x, ga[ps].y, ga[ps].z, ga[ps].w};
                    const float vb[4] = {gb[ps].x, gb[ps].y, gb[ps].z, gb[ps].w};
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        uint32_t h3, m3, l3;
                        bf16_split3_pair(va[t], vb[t], h3, m3, l3);
                        const int off = (4 * mq + t) * DS_GW + 2 * kp;
                        *(uint32_t*)&G3[off] = h3;
                        *(uint32_t*)&G3[DS_PL + off] = m3;
                        *(uint32_t*)&G3[2 * DS_PL + off] = l3;
                    }
                }
            }
            __syncthreads();
            if (wave * 32 < cnt) {
                const int h = lane >> 5, c = lane & 31;
                constexpr int NMB = DE_MB / 32;
#pragma unroll
                for (int kb = 0; kb < DE_KW / 16; ++kb) {
                    // this wave's operand: slot wave * 32 + c, walkers
                    // 16 kb + 8 h .. + 7, split into three planes
                    uint32_t xh[4], xm[4], xl[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = 16 * kb + 8 * h + 2 * i;
                        bf16_split3_pair(X[k * DE_LDX + wave * 32 + c], X[(k + 1) * DE_LDX + wave * 32 + c], xh[i],
                                         xm[i], xl[i]);
                    }
                    const bf16x8 bh = __builtin_bit_cast(bf16x8, uint4{xh[0], xh[1], xh[2], xh[3]});
                    const bf16x8 bm = __builtin_bit_cast(bf16x8, uint4{xm[0], xm[1], xm[2], xm[3]});
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, uint4{xl[0], xl[1], xl[2], xl[3]});
                    // MO blocks two at a time, so that consecutive products go
                    // to different accumulators
#pragma unroll
                    for (int m0 = 0; m0 < NMB; m0 += 2) {
                        constexpr int P = 2;
                        bf16x8 gh[P], gm[P], gl[P];
#pragma unroll
                        for (int q = 0; q < P; ++q) {
                            const int mb = min(m0 + q, NMB - 1);
                            const int off = (mb * 32 + c) * DS_GW + 16 * kb + 8 * h;
                            gh[q] = __builtin_bit_cast(bf16x8, *(const uint4*)&G3[off]);
                            gm[q] = __builtin_bit_cast(bf16x8, *(const uint4*)&G3[DS_PL + off]);
                            gl[q] = __builtin_bit_cast(bf16x8, *(const uint4*)&G3[2 * DS_PL + off]);
                        }
#define QSL_DS3(GA, XB)                                                                                    \
    _Pragma("unroll") for (int q = 0; q < P; ++q) if (m0 + q < NMB) acc[m0 + q] =                          \
        __builtin_amdgcn_mfma_f32_32x32x16_bf16(GA[q], XB, acc[m0 + q], 0, 0, 0);
                        QSL_DS3(gl, bh)
                        QSL_DS3(gm, bm)
                        QSL_DS3(gh, bl)
                        QSL_DS3(gm, bh)
                        QSL_DS3(gh, bm)
                        QSL_DS3(gh, bh)
#undef QSL_DS3
                    }
                }
            }
        }
        // flush, as adj_dae_body
        if (wave * 32 < cnt) {
            const int col = wave * 32 + (lane & 31);
            const int ao = col < cnt ? qao[col] : -1;
            int nbas = __builtin_amdgcn_readfirstlane(s.n_basis);
            int lim = n - i0 - 4 * (lane >> 5);  // rows di < lim exist
            asm volatile("" : "+s"(nbas));
            asm volatile("" : "+v"(lim));
            float* rowp = dA32 + (size_t)(i0 + 4 * (lane >> 5)) * nbas + max(ao, 0);
#pragma unroll
            for (int mb = 0; mb < DE_MB / 32; ++mb) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int di = mb * 32 + 8 * (r >> 2) + (r & 3);
                    const float v = acc[mb][r];
                    if (di < lim && ao >= 0 && v != 0.f) atomicAdd(rowp + (size_t)di * nbas, v);
                }
            }
        }
    }
}

__global__ __launch_bounds__(DE_THREADS, 2) void adj_dae_kernel(Job j) { adj_dae_body(j, blockIdx.x, blockIdx.y); }

__global__ __launch_bounds__(DE_THREADS, 2) void adj_dae_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) { adj_dae_body(j, bx, by); });
}

__global__ __launch_bounds__(DE_THREADS, 2) void adj_dae_s3_kernel(Job j) { adj_dae_s3_body(j, blockIdx.x, blockIdx.y); }

__global__ __launch_bounds__(DE_THREADS, 2) void adj_dae_s3_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) { adj_dae_s3_body(j, bx, by); });
}

void adj_dae_grid(Job& j) {
    j.gx = (j.n * (int)((j.W + j.gw - 1) / j.gw) + 7) / 8 * 32;  // whole runs of 8 groups x 4 chunk strides
    j.gy = (j.n + DE_MB - 1) / DE_MB;
    j.gz = 1;
}

hipError_t launch_adj_dae(const Job& j0, hipStream_t st) {
    Job j = j0;
    if (j.gw < 1 || j.mode != QSL_FP32 || !j.by_e || (j.n && j.W && j.dA32 && !j.g32)) return hipErrorInvalidValue;
    adj_dae_grid(j);
    if (!j.n || !j.W || !j.dA32) return hipSuccess;
    if (j.f32_tile == 2) adj_dae_s3_kernel<<<dim3((unsigned)j.gx, j.gy), DE_THREADS, 0, st>>>(j);
    else adj_dae_kernel<<<dim3((unsigned)j.gx, j.gy), DE_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_adj_dae_batched(int tile, const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    if (tile == 2) adj_dae_s3_batched<<<grid, DE_THREADS, 0, st>>>(jobs, prefix, njobs);
    else adj_dae_batched<<<grid, DE_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------- G split
// G = g D^-1 (0 where g = 0) rounded to FP32 and split hi = bf16(G),
// lo = bf16(G - hi) (the arithmetic the dA kernel applied per window block
// before), stored transposed per electron tile: [w][t][i][32 electrons],
// i < round_up(n, ADJ_MB), hi array then lo array.  One thread per 8
// electrons of one (walker, tile, MO).
__device__ __forceinline__ void gsplit_body(const Job& j, int bx) {
    const int n = j.n;
    const int T = (n + TE - 1) / TE, NIP = (n + ADJ_MB - 1) / ADJ_MB * ADJ_MB;
    const int64_t q = (int64_t)bx * 256 + threadIdx.x;
    if (q >= j.W * T * NIP * 4) return;
    // four consecutive lanes fill one 64-byte row (32 electrons) of one MO
    const int e8 = (int)(q & 3);
    const int64_t rest = q >> 2;
    const int ii = (int)(rest % NIP);
    const int64_t wt = rest / NIP;
    const int64_t w = wt / T;
    const int t = (int)(wt % T);
    const double gw = j.g[2 * w + j.spin];
    uint32_t hv[4], lv[4];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
        float f[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = t * TE + e8 * 8 + u + k;
            double v = 0.0;
            if (e < n && ii < n && gw != 0.0) v = gw * gmem(j.Dinv)[((size_t)w * n + e) * n + ii];
            f[k] = (float)v;
        }
        bf16_split2(f[0], f[1], hv[u / 2], lv[u / 2]);
    }
    uint16_t* gh = j.gsplit + (wt * NIP + ii) * TE + e8 * 8;
    uint16_t* gl = gh + j.W * gsplit_elems(n);
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    *gmem((u32x4*)gh) = u32x4{hv[0], hv[1], hv[2], hv[3]};
    *gmem((u32x4*)gl) = u32x4{lv[0], lv[1], lv[2], lv[3]};
}

__global__ __launch_bounds__(256) void gsplit_kernel(Job j) { gsplit_body(j, blockIdx.x); }

__global__ __launch_bounds__(256) void gsplit_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { gsplit_body(j, bx); });
}

int gsplit_blocks(const Job& j) {
    return (int)((j.W * (int64_t)tiles_per_walker(j.n) * ((j.n + ADJ_MB - 1) / ADJ_MB * ADJ_MB) * 4 + 255) / 256);
}

hipError_t launch_gsplit(const Job& j0, hipStream_t st) {
    Job j = j0;
    j.gx = gsplit_blocks(j); j.gy = 1; j.gz = 1;
    if (!j.gx || !j.gsplit) return hipSuccess;
    gsplit_kernel<<<(unsigned)j.gx, 256, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_gsplit_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    gsplit_batched<<<grid, 256, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

template <int MODE>
__global__ __launch_bounds__(AH_THREADS) void adj_h_kernel(Job j) {
    adj_h_body<MODE>(j, blockIdx.x, blockIdx.y);
}

template <int MODE>
__global__ __launch_bounds__(AH_THREADS) void adj_h_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) { adj_h_body<MODE>(j, bx, by); });
}

template <int MODE>
__global__ __launch_bounds__(AD_THREADS) void adj_da_kernel(Job j) {
    adj_da_body<MODE>(j, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int MODE>
__global__ __launch_bounds__(AD_THREADS) void adj_da_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs,
                    [&](const Job& j, int bx, int by, int bz) { adj_da_body<MODE>(j, bx, by, bz); });
}

void adj_h_grid(Job& j) {
    j.gx = (int)electron_tiles(j.n, j.W);
    j.gy = (j.n + ADJ_MB - 1) / ADJ_MB;
    j.gz = 1;
}

void adj_da_grid(Job& j) {
    const int nwb = j.mode == QSL_FP64 ? AdCfg<QSL_FP64>::NWB : AdCfg<QSL_FP32>::NWB;
    j.gx = (j.t_fix >= 0 ? 1 : tiles_per_walker(j.n)) * (int)((j.W + j.gw - 1) / j.gw);
    j.gy = (j.s.n_win + nwb - 1) / nwb;
    j.gz = (j.n + ADJ_MB - 1) / ADJ_MB;
}

hipError_t launch_adj_h(const Job& j0, hipStream_t st) {
    Job j = j0;
    adj_h_grid(j);
    if (!j.n || !j.W || !j.dR) return hipSuccess;
    const dim3 grid((unsigned)j.gx, j.gy);
    if (j.mode == QSL_FP64) adj_h_kernel<QSL_FP64><<<grid, AH_THREADS, 0, st>>>(j);
    else if (j.mode == QSL_FP32) adj_h_kernel<QSL_FP32><<<grid, AH_THREADS, 0, st>>>(j);
    else adj_h_kernel<QSL_BF16X3><<<grid, AH_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_adj_da(const Job& j0, hipStream_t st) {
    Job j = j0;
    if (j.gw < 1) return hipErrorInvalidValue;
    adj_da_grid(j);
    if (!j.n || !j.W || (!j.dA64 && !j.dA32 && !j.dApart)) return hipSuccess;
    const dim3 grid((unsigned)j.gx, j.gy, j.gz);
    if (j.mode == QSL_FP64) adj_da_kernel<QSL_FP64><<<grid, AD_THREADS, 0, st>>>(j);
    else if (j.mode == QSL_FP32) adj_da_kernel<QSL_FP32><<<grid, AD_THREADS, 0, st>>>(j);
    else adj_da_kernel<QSL_BF16X3><<<grid, AD_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_adj_h_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                   hipStream_t st) {
    if (mode == QSL_FP64) adj_h_batched<QSL_FP64><<<grid, AH_THREADS, 0, st>>>(jobs, prefix, njobs);
    else if (mode == QSL_FP32) adj_h_batched<QSL_FP32><<<grid, AH_THREADS, 0, st>>>(jobs, prefix, njobs);
    else adj_h_batched<QSL_BF16X3><<<grid, AH_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

hipError_t launch_adj_da_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                    hipStream_t st) {
    if (mode == QSL_FP64) adj_da_batched<QSL_FP64><<<grid, AD_THREADS, 0, st>>>(jobs, prefix, njobs);
    else if (mode == QSL_FP32) adj_da_batched<QSL_FP32><<<grid, AD_THREADS, 0, st>>>(jobs, prefix, njobs);
    else adj_da_batched<QSL_BF16X3><<<grid, AD_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

}  // namespace qsl
