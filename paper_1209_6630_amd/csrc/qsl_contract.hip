// Fused AO evaluation + AO->MO products C_n = A B_n, n = 1..5 (equation (abc)).
//
// One workgroup owns a tile (one electron index of one spin in 32
// consecutive walkers: positions that share their neighbourhood, so the
// tile's union of surviving windows stays close to one electron's) and a
// block of MO columns.  It walks the tile's surviving AO windows in chunks:
// each thread evaluates the five AO quantities (value, gradient, Laplacian;
// AO equations for chi and g) of one electron at the 8 slots of one window
// straight into LDS, so B never reaches HBM, then the four waves run the
// contraction on MFMA with the 5 x 32 rows (derivative, electron) as the M
// dimension and MOs as N.  Zero rows/columns of the screened B cost MFMA
// work but no memory traffic.  In the f32 modes each wave holds two MO
// sub-blocks, so one evaluation of the AOs serves 256 MOs; a sub-block past
// n is skipped.
//
// Precision modes:
//   FP64   AO eval FP64, v_mfma_f64_16x16x4f64, 64 MOs per workgroup.
//   FP32   AO eval FP32, over the tile's surviving slots rather than whole
//          windows (below), 256 MOs per workgroup; the products by default
//          as six v_mfma_f32_32x32x16_bf16 products of exact three-way bf16
//          splits of the FP32 operands (tile 2), or on v_mfma_f32_32x32x2f32
//          (tiles 0 and 1).
//   BF16X3 AO eval FP32, each operand split x = hi + lo (bf16, round to
//          nearest even), C += Bhi Ahi + Bhi Alo + Blo Ahi on
//          v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;

constexpr int CT_WAVES = 4;

template <int MODE>
struct CT {
    // windows per chunk, MO columns per wave, MO columns per workgroup
    static constexpr int KW = MODE == QSL_FP64 ? 4 : 8;
    static constexpr int KC = KW * WIN;
    static constexpr int NBW = MODE == QSL_FP64 ? 16 : 32;
    static constexpr int MSUB = MODE == QSL_FP64 ? 1 : 2;  // MO sub-blocks per wave
    static constexpr int NSB = CT_WAVES * NBW;      // MOs per sub-block
    static constexpr int NB = MSUB * NSB;
    static constexpr int THREADS = CT_WAVES * 64;
    // AO evaluation: slots of one window per thread (8, or 4 when the
    // workgroup has twice as many threads as (electron, window) pairs)
    static constexpr int SPT = THREADS >= 2 * TE * KW ? WIN / 2 : WIN;
    using T = typename std::conditional<MODE == QSL_FP64, double, float>::type;
    // LDS row stride (elements) of one electron's chunk of B
    static constexpr int LD = MODE == QSL_BF16X3 ? KC + 8 : (MODE == QSL_FP32 ? KC + 4 : KC + 2);
};

// ---------------------------------------------------------------- FP32
// The FP32 products take the tile's surviving slots as their K dimension,
// not whole windows: a window of 8 slots holds two or three shells of one
// atom, and a shell whose smallest exponent fails the FP64 test for every
// electron of the tile contributes exact zeros.  The tile's window list is
// filtered 32 windows at a time (one distance per electron and window, one
// compare per slot, a wavefront OR over the 32 electrons) into an ascending
// ring of slot indices; chunks of 64 slots are evaluated into LDS (one
// thread per slot and eight electrons) and contracted with
// v_mfma_f32_32x32x2f32, k-step t taking chunk slots t and 32 + t.
// Three workgroup shapes (tuning): tile 0 holds two 32-MO sub-blocks per
// wave (256 MOs, 160 accumulators, two workgroups per CU), tile 1 one (128
// MOs, 80 accumulators, three per CU; the AOs are evaluated once per 128
// MOs).  Tile 2 is tile 0 with the products on v_mfma_f32_32x32x16_bf16: both
// FP32 operands split exactly into three bf16 (x = hi + mid + lo), C += the
// six products hi.hi, hi.mid, mid.hi, hi.lo, mid.mid, lo.hi with FP32
// accumulation.  The three dropped products are below 2^-23 relative of
// each term, next to the 2^-24 of an FP32 product; the bf16 products take
// 2.7 times fewer matrix-core cycles than the FP32 ones and, unlike them,
// run beside the VALU work of the AO evaluation.
template <int TILE>
struct F32T {
    static constexpr int MSUB = TILE == 1 ? 1 : 2;
    static constexpr int NB = MSUB * CT_WAVES * 32;
    static constexpr int MINB = TILE == 1 ? 3 : 2;
};
constexpr int F32_BATCH = 32;   // windows filtered at a time
constexpr int F32_KC = 64;      // slots per chunk
constexpr int F32_RING = 512;   // ring of slot indices (>= 8 * F32_BATCH + F32_KC)
constexpr int F32_LD = F32_KC + 4;
constexpr int F32_LD3 = F32_KC + 8;  // bf16 row stride of tile 2's B planes

// Value, gradient and Laplacian of slot record r at electron p (FP32 AO
// arithmetic, FP64 screening), with the near-tie flag.  The primitives are
// read from the record one at a time (few registers; they stay in L1).
__device__ __forceinline__ void slot_values(const SlotRec& r, double T_thr, const double p[3], float v[5],
                                            bool& tie) {
    const double dx = p[0] - r.pos[0], dy = p[1] - r.pos[1], dz = p[2] - r.pos[2];
    const double r2 = dist2_exact(dx, dy, dz);
    const float X = (float)dx, Y = (float)dy, Z = (float)dz;
    const double tieb = 1e-12 * T_thr;
    float g = 0.f, g1 = 0.f, g2 = 0.f;
    const int np = r.np;
#pragma unroll 1
    for (int k = 0; k < np; ++k) {
        const double gk = r.ex[k];
        const double t = mul_exact(gk, r2);
        tie |= fabs(t - T_thr) <= tieb;
        if (t <= T_thr) {
            const float ek = r.c32[k] * exp_t(-(float)t);
            const float gT = (float)gk;
            g += ek;
            g1 += -2.f * gT * ek;
            g2 += ek * (4.f * gT * gT * (float)r2 - 6.f * gT);
        }
    }
    const int pw = r.pw;
    const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15, l = (pw >> 12) & 15;
    float px, ddx, d2x, py, ddy, d2y, pz, ddz, d2z;
    axis_pow(a, X, px, ddx, d2x);
    axis_pow(b, Y, py, ddy, d2y);
    axis_pow(c, Z, pz, ddz, d2z);
    const float f = r.f32;
    const float fyz = f * py * pz, fxz = f * px * pz, fxy = f * px * py;
    const float P = fyz * px;
    const float pg1 = P * g1;
    v[0] = P * g;
    v[1] = fyz * ddx * g + pg1 * X;
    v[2] = fxz * ddy * g + pg1 * Y;
    v[3] = fxy * ddz * g + pg1 * Z;
    v[4] = (d2x * fyz + d2y * fxz + d2z * fxy) * g + (float)(2 * l) * pg1 + P * g2;
}

// The part of a slot record the evaluation reads for every electron, held
// in registers for a chunk: position, the first three primitives, factor,
// powers, count (a shell with more primitives reads the rest from memory).
constexpr int SR_NP = 3;
struct SlotR {
    double x, y, z;
    double ex[SR_NP];
    float c[SR_NP];
    float f;
    int pw, np;
    __device__ __forceinline__ void load(const SlotRec* r) {
        typedef __attribute__((ext_vector_type(2))) double f64x2;
        typedef __attribute__((ext_vector_type(4))) float f32x4v;
        typedef __attribute__((ext_vector_type(4))) int i32x4;
        const f64x2 p01 = *gmem((const f64x2*)&r->pos[0]);
        const f64x2 p2g = *gmem((const f64x2*)&r->pos[2]);
        const f64x2 e01 = *gmem((const f64x2*)&r->ex[0]);
        const f64x2 e23 = *gmem((const f64x2*)&r->ex[2]);
        const f32x4v cc = *gmem((const f32x4v*)&r->c32[0]);
        const i32x4 tl = *gmem((const i32x4*)&r->f32);
        x = p01.x; y = p01.y; z = p2g.x;
        ex[0] = e01.x; ex[1] = e01.y; ex[2] = e23.x;
        c[0] = cc.x; c[1] = cc.y; c[2] = cc.z;
        f = __int_as_float(tl.x); pw = tl.y; np = tl.z;
    }
};
static_assert(offsetof(SlotRec, pos) == 0 && offsetof(SlotRec, ex) == 32 && offsetof(SlotRec, c32) == 96 &&
                  offsetof(SlotRec, f32) == 128 && offsetof(SlotRec, pw) == 132 && offsetof(SlotRec, np) == 136,
              "slot record layout read by SlotR::load");

// slot_values on a record held (in part) in registers.
__device__ __forceinline__ void slot_values_r(const SlotR& r, const SlotRec* __restrict__ rec, double T_thr,
                                              const double p[3], float v[5], bool& tie) {
    const double dx = p[0] - r.x, dy = p[1] - r.y, dz = p[2] - r.z;
    const double r2 = dist2_exact(dx, dy, dz);
    const float X = (float)dx, Y = (float)dy, Z = (float)dz;
    const double tieb = 1e-12 * T_thr;
    float g = 0.f, g1 = 0.f, g2 = 0.f;
    auto prim = [&](double gk, float ck) __attribute__((always_inline)) {
        const double t = mul_exact(gk, r2);
        tie |= fabs(t - T_thr) <= tieb;
        if (t <= T_thr) {
            const float ek = ck * exp_t(-(float)t);
            const float gT = (float)gk;
            g += ek;
            g1 += -2.f * gT * ek;
            g2 += ek * (4.f * gT * gT * (float)r2 - 6.f * gT);
        }
    };
#pragma unroll
    for (int k = 0; k < SR_NP; ++k)
        if (k < r.np) prim(r.ex[k], r.c[k]);
#pragma unroll 1
    for (int k = SR_NP; k < r.np; ++k) prim(gmem(rec)->ex[k], gmem(rec)->c32[k]);
    const int pw = r.pw;
    const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15, l = (pw >> 12) & 15;
    float px, ddx, d2x, py, ddy, d2y, pz, ddz, d2z;
    axis_pow(a, X, px, ddx, d2x);
    axis_pow(b, Y, py, ddy, d2y);
    axis_pow(c, Z, pz, ddz, d2z);
    const float f = r.f;
    const float fyz = f * py * pz, fxz = f * px * pz, fxy = f * px * py;
    const float P = fyz * px;
    const float pg1 = P * g1;
    v[0] = P * g;
    v[1] = fyz * ddx * g + pg1 * X;
    v[2] = fxz * ddy * g + pg1 * Y;
    v[3] = fxy * ddz * g + pg1 * Z;
    v[4] = (d2x * fyz + d2y * fxz + d2z * fxy) * g + (float)(2 * l) * pg1 + P * g2;
}

// Tile 2's products over one chunk: k-block q (16 ring slots) gives the
// lanes of half h the slots 16 q + 8 h .. + 7.  One (k-block, sub-block) at
// a time: its coefficient triples (8 bytes per slot and MO, loaded one unit
// ahead) are repacked into the three bf16 operand planes with byte permutes;
// B is read one plane at a time for the five quantities, so consecutive
// products go to five different accumulators.
template <int MSUB>
__device__ __forceinline__ void contract_s3_products(const Job& j, const uint16_t* B3, const int* ringo,
                                                     const uint64_t* ringm, int head, int tail, int n0, int nsub,
                                                     int nmo, int ldn, int wave, int lane, f32x16 (&acc)[MSUB][5]) {
    constexpr int NSB = CT_WAVES * 32, PL = 5 * TE * F32_LD3;  // plane size in elements
    constexpr int NQ = F32_KC / 16;
    const int h = lane >> 5;
    const char* __restrict__ a3b = (const char*)j.mo.A3;
    uint64_t cr[8];
    // uniform base + 32-bit byte offset: one address register per load;
    // entries past the list hold row 0 and no MO block (their B values are
    // zero)
    auto load_c = [&](int q, int sb) __attribute__((always_inline)) {
        const int pos = head + 16 * q + 8 * h;  // a multiple of 8: the ring reads are aligned
        const int4 s0 = *(const int4*)&ringo[pos & (F32_RING - 1)];
        const int4 s1 = *(const int4*)&ringo[(pos + 4) & (F32_RING - 1)];
        const int ov[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        const int mcol = min(n0 + sb * NSB + wave * 32, ldn - 32) + (lane & 31);
#pragma unroll
        for (int t = 0; t < 8; ++t) cr[t] = *gmem((const uint64_t*)(a3b + (size_t)(uint32_t)((ov[t] + mcol) * 8)));
    };
    load_c(0, 0);
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        uint64_t gm = 0;  // MO blocks with a non-zero coefficient on this half's 8 slots
        {
            const int pos = head + 16 * q + 8 * h;
#pragma unroll
            for (int t = 0; t < 8; t += 2) {
                const uint4 m2 = *(const uint4*)&ringm[(pos + t) & (F32_RING - 1)];
                gm |= ((uint64_t)m2.y << 32 | m2.x) | ((uint64_t)m2.w << 32 | m2.z);
            }
        }
#pragma unroll
        for (int sb = 0; sb < MSUB; ++sb) {
            uint32_t x[4], y[4], z[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t a0 = (uint32_t)cr[2 * i], a1 = (uint32_t)cr[2 * i + 1];
                const uint32_t b0 = (uint32_t)(cr[2 * i] >> 32), b1 = (uint32_t)(cr[2 * i + 1] >> 32);
                x[i] = __builtin_amdgcn_perm(a1, a0, 0x05040100u);  // hi
                y[i] = __builtin_amdgcn_perm(a1, a0, 0x07060302u);  // mid
                z[i] = __builtin_amdgcn_perm(b1, b0, 0x05040100u);  // lo
            }
            const bf16x8 ch = __builtin_bit_cast(bf16x8, uint4{x[0], x[1], x[2], x[3]});
            const bf16x8 cm = __builtin_bit_cast(bf16x8, uint4{y[0], y[1], y[2], y[3]});
            const bf16x8 cl = __builtin_bit_cast(bf16x8, uint4{z[0], z[1], z[2], z[3]});
            __builtin_amdgcn_sched_barrier(0);  // the planes are made before cr is reloaded
            if (sb + 1 < MSUB) load_c(q, sb + 1);
            else if (q + 1 < NQ) load_c(q + 1, 0);
            // work: inside n, and (block-sparse A) some non-zero coefficient
            // of the wave's 32 MOs on the k-block's 16 slots
            const int mb0 = n0 + sb * NSB + wave * 32;
            if (sb >= nsub || mb0 >= nmo || __ballot((gm >> ((mb0 >> 5) & 63)) & 1ull) == 0ull) continue;
            const int off = (lane & 31) * F32_LD3 + 16 * q + 8 * h;
            bf16x8 b[5];
#pragma unroll
            for (int d = 0; d < 5; ++d) b[d] = __builtin_bit_cast(bf16x8, *(const uint4*)(B3 + 2 * PL + d * TE * F32_LD3 + off));
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], ch, acc[sb][d], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int d = 0; d < 5; ++d) b[d] = __builtin_bit_cast(bf16x8, *(const uint4*)(B3 + PL + d * TE * F32_LD3 + off));
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], cm, acc[sb][d], 0, 0, 0);
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], ch, acc[sb][d], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int d = 0; d < 5; ++d) b[d] = __builtin_bit_cast(bf16x8, *(const uint4*)(B3 + d * TE * F32_LD3 + off));
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], cl, acc[sb][d], 0, 0, 0);
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], cm, acc[sb][d], 0, 0, 0);
#pragma unroll
            for (int d = 0; d < 5; ++d) acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[d], ch, acc[sb][d], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int TILE>
__device__ __forceinline__ void contract_f32_body(const Job& j, int bx, int by, int tid_in) {
    const DevSys& s = j.s;
    // n electrons of the spin (rows of a tile's C), nmo MOs (columns; n for
    // a Slater matrix, more for the orbital set of several determinants)
    const int spin = j.spin, n = j.n, nmo = j.mo.n, ldn = j.mo.ldn;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    const float* __restrict__ AT32 = j.mo.AT32;
    const SlotRec* __restrict__ srec = s.slot_rec;
    uint32_t* __restrict__ status = j.status;
    constexpr int MSUB = F32T<TILE>::MSUB, NSB = CT_WAVES * 32, LD = F32_LD, KC = F32_KC;

    __shared__ double epos[TE][3];
    // B: FP32 [5][TE][LD], or (tile 2) its three bf16 planes [3][5][TE][LD3]
    __shared__ __attribute__((aligned(16))) unsigned char Bbuf[TILE == 2 ? 3 * 5 * TE * F32_LD3 * 2 : 5 * TE * LD * 4];
    float* B = (float*)Bbuf;
    uint16_t* B3 = (uint16_t*)Bbuf;
    __shared__ __attribute__((aligned(16))) int ring[F32_RING];
    __shared__ __attribute__((aligned(16))) int ringo[F32_RING];  // slot * ldn: the slot's coefficient row
    __shared__ __attribute__((aligned(16))) uint64_t ringm[F32_RING];  // the slot's MO-block mask
    __shared__ uint32_t wmask[F32_BATCH];
    __shared__ int s_tail;
    __shared__ int wt[TE];  // the tile's walkers (Job.wperm order)

    const int tile = bx;
    const int n0 = by * MSUB * NSB;
    const int wbk = walker_blocks(W);
    const int eidx = tile / wbk;
    const int w0 = (tile % wbk) * TE;
    const int ne = (int)min<int64_t>(TE, W - w0);
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = tid_in, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double Tscr = s.T;

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)walker_of(j.wperm, W, eidx, w0 + e) * N + eoff + eidx) * 3 + k] : 0.0;
    }
    if (tid < TE) wt[tid] = tid < ne ? (int)walker_of(j.wperm, W, eidx, w0 + tid) : 0;
    if (tid == 0) s_tail = 0;
    const int nwin = j.nwin[tile];
    const int* __restrict__ wins = j.win + (size_t)tile * s.n_win;
    const int nsub = min(MSUB, (nmo - n0 + NSB - 1) / NSB);
    f32x16 acc[MSUB][5];
#pragma unroll
    for (int sb = 0; sb < MSUB; ++sb)
#pragma unroll
        for (int d = 0; d < 5; ++d)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[sb][d][r] = 0.f;
    uint32_t tiebits = 0;  // near ties seen by this thread, one bit per electron it evaluates
    bool ftie = false;     // a near tie in the slot filter for electron lane % 32
    __syncthreads();

    int head = 0, tail = 0, b0 = 0;
    while (b0 < nwin || head < tail) {
        if (tail - head < KC && b0 < nwin) {
            // ---- filter: windows b0 .. b0 + 31 of the tile's list
            const int e = lane & (TE - 1);
#pragma unroll
            for (int it = 0; it < F32_BATCH / 8; ++it) {
                const int wl = it * 8 + wave * 2 + (lane >> 5);
                const int q = b0 + wl < nwin ? wins[b0 + wl] : -1;
                uint32_t m = 0;
                if (q >= 0 && e < ne) {
                    const SlotRec* rq = srec + (size_t)q * WIN;
                    const double r2 = dist2_exact(epos[e][0] - rq->pos[0], epos[e][1] - rq->pos[1],
                                                  epos[e][2] - rq->pos[2]);
#pragma unroll
                    for (int jj = 0; jj < WIN; ++jj) {
                        const double t = mul_exact(rq[jj].gmin, r2);
                        if (t <= Tscr) m |= 1u << jj;
                        else ftie |= t - Tscr <= 1e-12 * Tscr;
                    }
                }
                uint32_t wm = 0;
#pragma unroll
                for (int jj = 0; jj < WIN; ++jj) {
                    const uint64_t bal = __ballot((m >> jj) & 1u);
                    const uint32_t half = (uint32_t)(lane < 32 ? bal : (bal >> 32));
                    wm |= (half != 0u ? 1u : 0u) << jj;
                }
                if ((lane & 31) == 0) wmask[wl] = wm;
            }
            __syncthreads();
            if (wave == 0 && lane < F32_BATCH) {
                const uint32_t m = b0 + lane < nwin ? wmask[lane] : 0u;
                const int q = b0 + lane < nwin ? wins[b0 + lane] : 0;
                const int c = __popc(m);
                int x = c;  // inclusive prefix over the 32 windows
#pragma unroll
                for (int o = 1; o < 32; o <<= 1) {
                    const int y = __shfl_up(x, o, 32);
                    if (lane >= o) x += y;
                }
                int pos = tail + x - c;
                for (uint32_t mm = m; mm; mm &= mm - 1) {
                    const int sl = q * WIN + __builtin_ctz(mm);
                    ring[pos & (F32_RING - 1)] = sl;
                    ringo[pos & (F32_RING - 1)] = sl * ldn;
                    ringm[pos & (F32_RING - 1)] = j.mo.blkmask[sl];
                    ++pos;
                }
                if (lane == F32_BATCH - 1) s_tail = tail + x;
            }
            __syncthreads();
            tail = s_tail;
            b0 += F32_BATCH;
            continue;
        }
        // ---- chunk [head, head + 64): AO values into LDS
        const int cnt = min(KC, tail - head);
        {
            const int kk = tid & (KC - 1), eg = tid >> 6;
            const bool live = kk < cnt;
            const int slot = live ? ring[(head + kk) & (F32_RING - 1)] : 0;
            if constexpr (TILE == 2) {
                // the last chunk: entries past the list become row 0 with no
                // MO block (the filter is done, nothing is appended after)
                if (!live && eg == 0) {
                    ringo[(head + kk) & (F32_RING - 1)] = 0;
                    ringm[(head + kk) & (F32_RING - 1)] = 0ull;
                }
            }
            SlotR r;
            r.load(srec + slot);
#pragma unroll 1
            for (int i = 0; i < 8; ++i) {
                const int e = eg + 4 * i;
                bool tie = false;
                float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
                if (live && e < ne) {
                    const double p[3] = {epos[e][0], epos[e][1], epos[e][2]};
                    slot_values_r(r, srec + slot, Tscr, p, v, tie);
                }
                tiebits |= (tie ? 1u : 0u) << i;
                if constexpr (TILE == 2) {
                    // quantities two at a time (packed conversions), each
                    // half written to its own plane row
                    uint32_t hv[3], mv[3], lv[3];
#pragma unroll
                    for (int d2 = 0; d2 < 3; ++d2)
                        bf16_split3_pair(v[2 * d2], 2 * d2 + 1 < 5 ? v[2 * d2 + 1] : 0.f, hv[d2], mv[d2], lv[d2]);
#pragma unroll
                    for (int d = 0; d < 5; ++d) {
                        const int sh = 16 * (d & 1);
                        B3[((0 * 5 + d) * TE + e) * F32_LD3 + kk] = (uint16_t)(hv[d >> 1] >> sh);
                        B3[((1 * 5 + d) * TE + e) * F32_LD3 + kk] = (uint16_t)(mv[d >> 1] >> sh);
                        B3[((2 * 5 + d) * TE + e) * F32_LD3 + kk] = (uint16_t)(lv[d >> 1] >> sh);
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < 5; ++d) B[(d * TE + e) * LD + kk] = v[d];
                }
            }
        }
        __syncthreads();
        if constexpr (TILE == 2) {
            contract_s3_products<MSUB>(j, B3, ringo, ringm, head, tail, n0, nsub, nmo, ldn, wave, lane, acc);
        } else
        // ---- products: k-step t of group u takes chunk slots 4u + t (lanes
        // 0..31) and 32 + 4u + t (lanes 32..63); the coefficients of the
        // next group are loaded during this group's MFMAs
        {
            const int h = lane >> 5;
            float bq[MSUB][4], bn[MSUB][4];
            const float* __restrict__ Acol[MSUB];
#pragma unroll
            for (int sb = 0; sb < MSUB; ++sb) Acol[sb] = AT32 + min(n0 + sb * NSB + wave * 32, ldn - 32) + (lane & 31);
            auto load_b = [&](int u) __attribute__((always_inline)) {
                const int pos = head + h * 32 + 4 * u;
                const int4 so = *(const int4*)&ringo[pos & (F32_RING - 1)];
                // entries past the list point at row 0 (their B values are zero)
                const int ov[4] = {pos + 0 < tail ? so.x : 0, pos + 1 < tail ? so.y : 0, pos + 2 < tail ? so.z : 0,
                                   pos + 3 < tail ? so.w : 0};
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb)
#pragma unroll
                    for (int t = 0; t < 4; ++t) bn[sb][t] = gmem(Acol[sb])[ov[t]];
            };
            load_b(0);
#pragma unroll
            for (int u = 0; u < KC / 8; ++u) {
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb)
#pragma unroll
                    for (int t = 0; t < 4; ++t) bq[sb][t] = bn[sb][t];
                if (u + 1 < KC / 8) load_b(u + 1);
                f32x4 a[5];
#pragma unroll
                for (int d = 0; d < 5; ++d)
                    a[d] = *(const f32x4*)&B[(d * TE + (lane & 31)) * LD + h * 32 + 4 * u];
                // the group's eight slots (four per half-wave): the MO blocks
                // with a non-zero coefficient on any of them (a block with
                // none adds exact zeros, so its MFMAs are skipped: localised
                // MOs give block-sparse A)
                uint64_t gm = 0;
                {
                    const int pos = head + h * 32 + 4 * u;
#pragma unroll
                    for (int t = 0; t < 4; ++t) gm |= pos + t < tail ? ringm[(pos + t) & (F32_RING - 1)] : 0ull;
                }
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) {
                    if (sb >= nsub) break;
                    const int mb0 = n0 + sb * NSB + wave * 32;
                    if (mb0 >= nmo) continue;  // this wave's 32 MOs are all padding
                    if (__ballot((gm >> ((mb0 >> 5) & 63)) & 1ull) == 0ull) continue;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int d = 0; d < 5; ++d)
                            acc[sb][d] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[d][t], bq[sb][t], acc[sb][d], 0, 0, 0);
                }
            }
        }
        __syncthreads();
        head += KC;
    }

    // near ties flag the walkers of the electrons concerned
    if (status) {
        const int eg = tid >> 6;
        for (uint32_t tb = tiebits; tb; tb &= tb - 1) {
            const int e = eg + 4 * __builtin_ctz(tb);
            if (e < ne) atomicOr(status + wt[e], QSL_STATUS_NEAR_TIE);
        }
        if (ftie && (lane & 31) < ne) atomicOr(status + wt[lane & 31], QSL_STATUS_NEAR_TIE);
    }
    // ---- store C[w][d][e][mo]
    float* C = (float*)j.C;
#pragma unroll
    for (int sb = 0; sb < MSUB; ++sb) {
        const int mo = n0 + sb * NSB + wave * 32 + (lane & 31);
        if (mo < nmo) {
#pragma unroll
            for (int d = 0; d < 5; ++d)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int el = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    // ordinary stores: the L2 merges the partial lines at the
                    // ends of a wave's 128-byte segments of a C row
                    if (el < ne) gmem(C)[(((size_t)wt[el] * 5 + d) * n + eidx) * nmo + mo] = acc[sb][d][r];
                }
        }
    }
}

template <int MODE>
__device__ __forceinline__ void contract_body(const Job& j, int bx, int by, int tid_in) {
    if constexpr (MODE == QSL_FP32) {
        contract_f32_body<0>(j, bx, by, tid_in);
    } else {
    const DevSys& s = j.s;
    const int spin = j.spin, n = j.n, nmo = j.mo.n, ldn = j.mo.ldn;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    const int* __restrict__ tile_nwin = j.nwin;
    const int* __restrict__ tile_win = j.win;
    const double* __restrict__ AT64 = j.mo.AT64;
    const uint16_t* __restrict__ Ahi = j.mo.Ahi;
    const uint16_t* __restrict__ Alo = j.mo.Alo;
    void* __restrict__ Cout = j.C;
    uint32_t* __restrict__ status = j.status;
    using P = CT<MODE>;
    using T = typename P::T;
    constexpr int KW = P::KW, KC = P::KC, LD = P::LD, SPT = P::SPT;

    __shared__ double epos[TE][3];
    __shared__ int wq[KW];
    // B chunk in LDS: [5][32 electrons][LD]
    constexpr int BELEMS = 5 * TE * LD;
    __shared__ __attribute__((aligned(16))) unsigned char bbuf[MODE == QSL_BF16X3 ? 2 * BELEMS * 2 : BELEMS * sizeof(T)];

    // tiles are numbered e * walker_blocks(W) + walker block, so that
    // concurrently resident workgroups share the same AO windows of A; row r
    // of the tile is walker w0 + r (ne valid rows)
    const int tile = bx;
    const int n0 = by * P::NB;
    const int wbk = walker_blocks(W);
    const int eidx = tile / wbk;
    const int w0 = (tile % wbk) * TE;
    const int ne = (int)min<int64_t>(TE, W - w0);
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = tid_in, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)(w0 + e) * N + eoff + eidx) * 3 + k] : 0.0;
    }
    const int nwin = tile_nwin[tile];
    const int* wins = tile_win + (size_t)tile * s.n_win;

    constexpr int MSUB = P::MSUB, NSB = P::NSB;
    const int nsub = min(MSUB, (nmo - n0 + NSB - 1) / NSB);  // sub-blocks below nmo (uniform)
    f32x16 acc32[MSUB][5];
    f64x4 acc64[MSUB][5][2];
#pragma unroll
    for (int sb = 0; sb < MSUB; ++sb) {
        if constexpr (MODE == QSL_FP64) {
            for (int d = 0; d < 5; ++d)
                for (int h = 0; h < 2; ++h) acc64[sb][d][h] = f64x4{0, 0, 0, 0};
        } else {
            for (int d = 0; d < 5; ++d)
                for (int r = 0; r < 16; ++r) acc32[sb][d][r] = 0.f;
        }
    }
    bool tie = false;
    // the records of a chunk's windows in LDS (two buffers, by chunk parity):
    // the AO evaluation reads them many times per thread, from LDS rather
    // than through dependent global loads; chunk c + 1 is copied during the
    // products of chunk c
    // (the f32 modes keep the record prefix they read, RQ pieces of 16 bytes,
    // back to back; a wave's direct global-to-LDS load fills 64 consecutive
    // pieces, no registers involved)
    constexpr int RQ = MODE == QSL_FP64 ? WINREC_Q64 : WINREC_Q32;
    constexpr int NPASS = (KW * RQ + P::THREADS - 1) / P::THREADS;
    __shared__ __attribute__((aligned(16))) uint4 wrecq[2][NPASS * P::THREADS];
    auto rec = [&](int buf, int wl) -> const WinRec& { return *(const WinRec*)&wrecq[buf][wl * RQ]; };
    auto fetch_recs = [&](int buf, int c0) __attribute__((always_inline)) {
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
            const int q = ps * P::THREADS + tid;
            const int wl = q / RQ;
            const int wi = gmem(wins)[q < KW * RQ && c0 + wl < nwin ? c0 + wl : 0];
            // lane l of wave v writes piece ps * THREADS + 64 v + l
            __builtin_amdgcn_global_load_lds((const void*)((const uint4*)&s.win_rec[wi] + q % RQ),
                                             (__attribute__((address_space(3))) void*)&wrecq[buf][ps * P::THREADS + wave * 64],
                                             16, 0, 0);
        }
    };
    if (nwin > 0) fetch_recs(0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the direct loads into LDS are done
    __syncthreads();

    for (int c0 = 0; c0 < nwin; c0 += KW) {
        const int buf = (c0 / KW) & 1;
        // ---- phase R: AO values of (electron e, window wl, slots js..js+SPT)
        // into LDS
        if (tid < TE * KW * (WIN / SPT)) {
            const int e = tid & (TE - 1), wl = (tid / TE) % KW, js = (tid / (TE * KW)) * SPT;
            const int q = c0 + wl < nwin ? gmem(wins)[c0 + wl] : -1;
            if (e == 0 && js == 0) wq[wl] = q < 0 ? 0 : q;
            T vals[5][SPT];
#pragma unroll
            for (int d = 0; d < 5; ++d)
#pragma unroll
                for (int j = 0; j < SPT; ++j) vals[d][j] = T(0);
            if (q >= 0 && e < ne) {
                const double r[3] = {epos[e][0], epos[e][1], epos[e][2]};
                rec_values<T, SPT>(rec(buf, wl), s.T, js, r, vals, tie);
            }
            if constexpr (MODE == QSL_BF16X3) {
                uint16_t* bh = (uint16_t*)bbuf;
                uint16_t* bl = bh + BELEMS;
#pragma unroll
                for (int d = 0; d < 5; ++d) {
                    uint32_t hv[SPT / 2], lv[SPT / 2];
#pragma unroll
                    for (int p = 0; p < SPT / 2; ++p) bf16_split2(vals[d][2 * p], vals[d][2 * p + 1], hv[p], lv[p]);
                    uint16_t* ph = bh + (d * TE + e) * LD + wl * WIN + js;
                    uint16_t* pl = bl + (d * TE + e) * LD + wl * WIN + js;
                    if constexpr (SPT == WIN) {
                        *(uint4*)ph = uint4{hv[0], hv[1], hv[2], hv[3]};
                        *(uint4*)pl = uint4{lv[0], lv[1], lv[2], lv[3]};
                    } else {
                        *(uint2*)ph = uint2{hv[0], hv[1]};
                        *(uint2*)pl = uint2{lv[0], lv[1]};
                    }
                }
            } else {
                T* bt = (T*)bbuf;
#pragma unroll
                for (int d = 0; d < 5; ++d)
#pragma unroll
                    for (int j = 0; j < SPT; ++j) bt[(d * TE + e) * LD + wl * WIN + js + j] = vals[d][j];
            }
        }
        __syncthreads();

        // ---- phase M: MFMA over the chunk (the next chunk's records load
        // meanwhile; pieces of windows past the list are never read)
        if (c0 + KW < nwin) fetch_recs(buf ^ 1, c0 + KW);
        if constexpr (MODE == QSL_BF16X3) {
            const uint16_t* bh = (const uint16_t*)bbuf;
            const uint16_t* bl = bh + BELEMS;
            const int oct = lane >> 5;
            // A fragments of every sub-block, one k-step ahead (software
            // pipelined: the next k-step's loads are in flight during this
            // k-step's products); a sub-block wholly past n reads a valid
            // row and is skipped
            bf16x8 ah[MSUB], al[MSUB];
            auto load_a = [&](int ks) __attribute__((always_inline)) {
                const size_t wbase = (size_t)wq[ks * 2 + oct] * ldn;
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) {
                    const int mo = min(n0 + sb * NSB + wave * 32, ldn - 32) + (lane & 31);
                    const size_t off = (wbase + mo) * WIN;
                    // global (not generic) loads: the wait before the products
                    // can leave the next k-step's loads in flight
                    ah[sb] = __builtin_bit_cast(bf16x8, *gmem((const uint4*)(Ahi + off)));
                    al[sb] = __builtin_bit_cast(bf16x8, *gmem((const uint4*)(Alo + off)));
                }
            };
            load_a(0);
#pragma unroll
            for (int ks = 0; ks < KC / 16; ++ks) {
                bf16x8 xh[5], xl[5];
#pragma unroll
                for (int d = 0; d < 5; ++d) {
                    const int off = (d * TE + (lane & 31)) * LD + ks * 16 + oct * 8;
                    xh[d] = __builtin_bit_cast(bf16x8, *(const uint4*)(bh + off));
                    xl[d] = __builtin_bit_cast(bf16x8, *(const uint4*)(bl + off));
                }
                bf16x8 cah[MSUB], cal[MSUB];
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) { cah[sb] = ah[sb]; cal[sb] = al[sb]; }
                if (ks + 1 < KC / 16) load_a(ks + 1);
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) {
                    if (sb >= nsub) break;
                    if (n0 + sb * NSB + wave * 32 >= nmo) continue;  // this wave's 32 MOs are all padding
                    const bf16x8 bah = cah[sb], bal = cal[sb];
                    // the three products of one accumulator are dependent:
                    // issue them five accumulators apart
#pragma unroll
                    for (int d = 0; d < 5; ++d)
                        acc32[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[d], bah, acc32[sb][d], 0, 0, 0);
#pragma unroll
                    for (int d = 0; d < 5; ++d)
                        acc32[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[d], bal, acc32[sb][d], 0, 0, 0);
#pragma unroll
                    for (int d = 0; d < 5; ++d)
                        acc32[sb][d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[d], bah, acc32[sb][d], 0, 0, 0);
                }
            }
        } else {
            const double* bt = (const double*)bbuf;
            const int kk = lane >> 4;
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int c = ks * 4 + kk;
                const int slot = wq[c / WIN] * WIN + (c % WIN);
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) {
                    if (sb >= nsub) break;
                    const int mo = n0 + sb * NSB + wave * 16 + (lane & 15);
                    const double b = AT64[(size_t)slot * ldn + mo];
                    for (int d = 0; d < 5; ++d)
                        for (int h = 0; h < 2; ++h) {
                            const double a = bt[(d * TE + h * 16 + (lane & 15)) * LD + c];
                            acc64[sb][d][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc64[sb][d][h], 0, 0, 0);
                        }
                }
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the next chunk's records are in LDS
        __syncthreads();
    }

    // a near tie of a kept primitive flags the walker of the thread's row
    if (tie && status) atomicOr(status + w0 + (tid & (TE - 1)), QSL_STATUS_NEAR_TIE);
    // ---- store C[w][d][e][mo]
#pragma unroll
    for (int sb = 0; sb < MSUB; ++sb) {
        if constexpr (MODE == QSL_FP64) {
            double* C = (double*)Cout;
            const int mo = n0 + sb * NSB + wave * 16 + (lane & 15);
            if (mo < nmo) {
                for (int d = 0; d < 5; ++d)
                    for (int h = 0; h < 2; ++h)
                        for (int r = 0; r < 4; ++r) {
                            // v_mfma_f64_16x16x4f64 result: row (lane / 16) + 4 r, column lane % 16
                            const int el = h * 16 + (lane >> 4) + 4 * r;
                            if (el < ne) gmem(C)[(((size_t)(w0 + el) * 5 + d) * n + eidx) * nmo + mo] = acc64[sb][d][h][r];
                        }
            }
        } else {
            float* C = (float*)Cout;
            const int mo = n0 + sb * NSB + wave * 32 + (lane & 31);
            if (mo < nmo) {
                for (int d = 0; d < 5; ++d)
                    for (int r = 0; r < 16; ++r) {
                        const int el = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        if (el < ne) gmem(C)[(((size_t)(w0 + el) * 5 + d) * n + eidx) * nmo + mo] = acc32[sb][d][r];
                    }
            }
        }
    }
    }  // FP64 / BF16X3
}

template <int MODE>
__global__ __launch_bounds__(CT_WAVES * 64, 2) void contract_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs,
                [&](const Job& j, int bx, int by, int) __attribute__((always_inline)) {
                    contract_body<MODE>(j, bx, by, threadIdx.x);
                });
}

__global__ __launch_bounds__(CT_WAVES * 64, F32T<1>::MINB) void contract_batched_f32t1(const Job* jobs,
                                                                                       const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) __attribute__((always_inline)) {
        contract_f32_body<1>(j, bx, by, threadIdx.x);
    });
}

__global__ __launch_bounds__(CT_WAVES * 64, F32T<2>::MINB) void contract_batched_f32t2(const Job* jobs,
                                                                                       const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) __attribute__((always_inline)) {
        contract_f32_body<2>(j, bx, by, threadIdx.x);
    });
}

// Persistent form: `gridDim.x` resident workgroups take the items of the
// work list in order from a device counter (zeroed before the launch) until
// it passes the last; every workgroup leaves once the counter does.
template <int MODE, int TILE>
__device__ __forceinline__ void contract_persist_body(const Job* __restrict__ jobs, const int* __restrict__ prefix,
                                                      int njobs, unsigned* __restrict__ queue) {
    __shared__ int s_item;
    const int total = prefix[njobs];
    for (;;) {
        __syncthreads();  // the previous item's LDS is no longer read
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int b = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar registers
        if (b >= total) break;
        // the thread index, opaque per item: values derived from it are not
        // hoisted out of the loop (held across the body, they would spill)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int ji = __builtin_amdgcn_readfirstlane(find_job(prefix, njobs, b));
        const Job& j = jobs[ji];
        const int lb = b - prefix[ji];
        if constexpr (MODE == QSL_FP32) contract_f32_body<TILE>(j, lb % j.gx, (lb / j.gx) % j.gy, tid);
        else contract_body<MODE>(j, lb % j.gx, (lb / j.gx) % j.gy, tid);
    }
}

template <int MODE>
__global__ __launch_bounds__(CT_WAVES * 64, 2) void contract_persist(const Job* jobs, const int* prefix, int njobs,
                                                                     unsigned* queue) {
    contract_persist_body<MODE, 0>(jobs, prefix, njobs, queue);
}

__global__ __launch_bounds__(CT_WAVES * 64, F32T<1>::MINB) void contract_persist_f32t1(const Job* jobs,
                                                                                       const int* prefix, int njobs,
                                                                                       unsigned* queue) {
    contract_persist_body<QSL_FP32, 1>(jobs, prefix, njobs, queue);
}

__global__ __launch_bounds__(CT_WAVES * 64, F32T<2>::MINB) void contract_persist_f32t2(const Job* jobs,
                                                                                       const int* prefix, int njobs,
                                                                                       unsigned* queue) {
    contract_persist_body<QSL_FP32, 2>(jobs, prefix, njobs, queue);
}

// Grid of the contraction phase of a Job: tiles x MO blocks.
void contract_grid(Job& j) {
    const int nb = j.mode == QSL_FP64 ? CT<QSL_FP64>::NB
                                      : (j.mode == QSL_FP32 ? (j.f32_tile == 1 ? F32T<1>::NB : F32T<0>::NB)
                                                            : CT<QSL_BF16X3>::NB);
    j.gx = (int)electron_tiles(j.n, j.W);
    j.gy = (j.mo.n + nb - 1) / nb;  // MO blocks (n for a Slater matrix)
    j.gz = 1;
}

// The Job of a per-system launch into device memory (with the block prefix
// {0, grid}), so the contraction reads it as a batched launch does (passed
// by value, its fields would crowd the registers).
__global__ void store_job_kernel(Job j, Job* dst, int* prefix) {
    if (threadIdx.x == 0) {
        *dst = j;
        prefix[0] = 0;
        prefix[1] = j.gx * j.gy * j.gz;
    }
}

hipError_t launch_contract(const Job& j0, hipStream_t st) {
    Job j = j0;
    contract_grid(j);
    if (!j.n || !j.W) return hipSuccess;
    if (!j.jobslot) return hipErrorInvalidValue;  // every caller's workspace holds one
    Job* dj = (Job*)j.jobslot;
    int* pre = (int*)((char*)j.jobslot + sizeof(Job));
    store_job_kernel<<<1, 64, 0, st>>>(j, dj, pre);
    return launch_contract_batched(j.mode, j.f32_tile, nullptr, dj, pre, 1, j.gx * j.gy, st);
}

int contract_per_cu(int mode, int tile) { return mode == QSL_FP32 && tile == 1 ? F32T<1>::MINB : 2; }

hipError_t launch_contract_batched(int mode, int tile, unsigned* queue, const Job* jobs, const int* prefix, int njobs,
                                   int grid, hipStream_t st) {
    constexpr int T = CT_WAVES * 64;
    if (grid <= 0) return hipSuccess;
    const bool t1 = mode == QSL_FP32 && tile == 1, t2 = mode == QSL_FP32 && tile == 2;
    if (queue) {
        if (mode == QSL_FP64) contract_persist<QSL_FP64><<<grid, T, 0, st>>>(jobs, prefix, njobs, queue);
        else if (t1) contract_persist_f32t1<<<grid, T, 0, st>>>(jobs, prefix, njobs, queue);
        else if (t2) contract_persist_f32t2<<<grid, T, 0, st>>>(jobs, prefix, njobs, queue);
        else if (mode == QSL_FP32) contract_persist<QSL_FP32><<<grid, T, 0, st>>>(jobs, prefix, njobs, queue);
        else contract_persist<QSL_BF16X3><<<grid, T, 0, st>>>(jobs, prefix, njobs, queue);
    } else {
        if (mode == QSL_FP64) contract_batched<QSL_FP64><<<grid, T, 0, st>>>(jobs, prefix, njobs);
        else if (t1) contract_batched_f32t1<<<grid, T, 0, st>>>(jobs, prefix, njobs);
        else if (t2) contract_batched_f32t2<<<grid, T, 0, st>>>(jobs, prefix, njobs);
        else if (mode == QSL_FP32) contract_batched<QSL_FP32><<<grid, T, 0, st>>>(jobs, prefix, njobs);
        else contract_batched<QSL_BF16X3><<<grid, T, 0, st>>>(jobs, prefix, njobs);
    }
    return hipGetLastError();
}

}  // namespace qsl
