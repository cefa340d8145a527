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
//   FP32   AO eval FP32, v_mfma_f32_32x32x2f32, 256 MOs per workgroup.
//   BF16X3 AO eval FP32, each operand split x = hi + lo (bf16, round to
//          nearest even), C += Bhi Ahi + Bhi Alo + Blo Ahi on
//          v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
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

template <int MODE>
__device__ __forceinline__ void contract_body(const Job& j, int bx, int by) {
    const DevSys& s = j.s;
    const int spin = j.spin, n = j.n, ldn = j.mo.ldn;
    const int64_t W = j.W;
    const double* __restrict__ R = j.R;
    const int* __restrict__ tile_nwin = j.nwin;
    const int* __restrict__ tile_win = j.win;
    const double* __restrict__ AT64 = j.mo.AT64;
    const float* __restrict__ AT32 = j.mo.AT32;
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
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)(w0 + e) * N + eoff + eidx) * 3 + k] : 0.0;
    }
    const int nwin = tile_nwin[tile];
    const int* wins = tile_win + (size_t)tile * s.n_win;

    constexpr int MSUB = P::MSUB, NSB = P::NSB;
    const int nsub = min(MSUB, (n - n0 + NSB - 1) / NSB);  // sub-blocks below n (uniform)
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
                    if (n0 + sb * NSB + wave * 32 >= n) continue;  // this wave's 32 MOs are all padding
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
        } else if constexpr (MODE == QSL_FP32) {
            const float* bt = (const float*)bbuf;
            const int kk = lane >> 5;
            for (int ks = 0; ks < KC / 2; ++ks) {
                const int c = ks * 2 + kk;
                const int slot = wq[c / WIN] * WIN + (c % WIN);
                float a[5];
#pragma unroll
                for (int d = 0; d < 5; ++d) a[d] = bt[(d * TE + (lane & 31)) * LD + c];
#pragma unroll
                for (int sb = 0; sb < MSUB; ++sb) {
                    if (sb >= nsub) break;
                    if (n0 + sb * NSB + wave * 32 >= n) continue;  // this wave's 32 MOs are all padding
                    const int mo = n0 + sb * NSB + wave * 32 + (lane & 31);
                    const float b = AT32[(size_t)slot * ldn + mo];
#pragma unroll
                    for (int d = 0; d < 5; ++d)
                        acc32[sb][d] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[d], b, acc32[sb][d], 0, 0, 0);
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
            if (mo < n) {
                for (int d = 0; d < 5; ++d)
                    for (int h = 0; h < 2; ++h)
                        for (int r = 0; r < 4; ++r) {
                            // v_mfma_f64_16x16x4f64 result: row (lane / 16) + 4 r, column lane % 16
                            const int el = h * 16 + (lane >> 4) + 4 * r;
                            if (el < ne) gmem(C)[(((size_t)(w0 + el) * 5 + d) * n + eidx) * n + mo] = acc64[sb][d][h][r];
                        }
            }
        } else {
            float* C = (float*)Cout;
            const int mo = n0 + sb * NSB + wave * 32 + (lane & 31);
            if (mo < n) {
                for (int d = 0; d < 5; ++d)
                    for (int r = 0; r < 16; ++r) {
                        const int el = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        if (el < ne) gmem(C)[(((size_t)(w0 + el) * 5 + d) * n + eidx) * n + mo] = acc32[sb][d][r];
                    }
            }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(CT_WAVES * 64, 2) void contract_kernel(Job j) {
    contract_body<MODE>(j, blockIdx.x, blockIdx.y);
}

template <int MODE>
__global__ __launch_bounds__(CT_WAVES * 64, 2) void contract_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs,
                [&](const Job& j, int bx, int by, int) __attribute__((always_inline)) { contract_body<MODE>(j, bx, by); });
}

// Grid of the contraction phase of a Job: tiles x MO blocks.
void contract_grid(Job& j) {
    const int nb = j.mode == QSL_FP64 ? CT<QSL_FP64>::NB : CT<QSL_FP32>::NB;
    j.gx = (int)electron_tiles(j.n, j.W);
    j.gy = (j.n + nb - 1) / nb;
    j.gz = 1;
}

hipError_t launch_contract(const Job& j0, hipStream_t st) {
    Job j = j0;
    contract_grid(j);
    if (!j.n || !j.W) return hipSuccess;
    const dim3 g((unsigned)j.gx, j.gy);
    constexpr int T = CT_WAVES * 64;
    if (j.mode == QSL_FP64) contract_kernel<QSL_FP64><<<g, T, 0, st>>>(j);
    else if (j.mode == QSL_FP32) contract_kernel<QSL_FP32><<<g, T, 0, st>>>(j);
    else contract_kernel<QSL_BF16X3><<<g, T, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_contract_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                   hipStream_t st) {
    constexpr int T = CT_WAVES * 64;
    if (mode == QSL_FP64) contract_batched<QSL_FP64><<<grid, T, 0, st>>>(jobs, prefix, njobs);
    else if (mode == QSL_FP32) contract_batched<QSL_FP32><<<grid, T, 0, st>>>(jobs, prefix, njobs);
    else contract_batched<QSL_BF16X3><<<grid, T, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

}  // namespace qsl
