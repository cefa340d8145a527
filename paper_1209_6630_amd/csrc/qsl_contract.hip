// Fused AO evaluation + AO->MO products C_n = A B_n, n = 1..5 (equation (abc)).
//
// One workgroup owns a tile of 32 electrons of one walker and spin and a
// block of MO columns.  It walks the tile's surviving AO windows in chunks:
// each thread evaluates the five AO quantities (value, gradient, Laplacian;
// AO equations for chi and g) of one electron at the 8 slots of one window
// straight into LDS, so B never reaches HBM, then the four waves run the
// contraction on MFMA with the 5 x 32 rows (derivative, electron) as the M
// dimension and MOs as N.  Zero rows/columns of the screened B cost MFMA
// work but no memory traffic.
//
// Precision modes:
//   FP64   AO eval FP64, v_mfma_f64_16x16x4f64, 64 MOs per workgroup.
//   FP32   AO eval FP32, v_mfma_f32_32x32x2f32, 128 MOs per workgroup.
//   BF16X3 AO eval FP32, each operand split x = hi + lo (bf16, round to
//          nearest even), C += Bhi Ahi + Bhi Alo + Blo Ahi on
//          v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
#include "qsl_internal.h"

namespace qsl {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) double f64x4;

constexpr int CT_THREADS = 256;

template <int MODE>
struct CT {
    // windows per chunk, MO columns per wave
    static constexpr int KW = MODE == QSL_FP64 ? 4 : 8;
    static constexpr int KC = KW * WIN;
    static constexpr int NBW = MODE == QSL_FP64 ? 16 : 32;
    static constexpr int NB = 4 * NBW;
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
    constexpr int KW = P::KW, KC = P::KC, LD = P::LD;

    __shared__ double epos[TE][3];
    __shared__ int wq[KW];
    // B chunk in LDS: [5][32 electrons][LD]
    constexpr int BELEMS = 5 * TE * LD;
    __shared__ __attribute__((aligned(16))) unsigned char bbuf[MODE == QSL_BF16X3 ? 2 * BELEMS * 2 : BELEMS * sizeof(T)];

    // tiles are numbered t * W + w (electron range t of walker w), so that
    // concurrently resident workgroups share the same AO windows of A
    const int tile = bx;
    const int n0 = by * P::NB;
    const int w = (int)(tile % W);
    const int e0 = (int)(tile / W) * TE;
    const int ne = min(TE, n - e0);
    const int N = s.n_up + s.n_dn;
    const int eoff = spin ? s.n_up : 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform

    if (tid < TE * 3) {
        const int e = tid / 3, k = tid % 3;
        epos[e][k] = e < ne ? R[((size_t)w * N + eoff + e0 + e) * 3 + k] : 0.0;
    }
    const int nwin = tile_nwin[tile];
    const int* wins = tile_win + (size_t)tile * s.n_win;

    f32x16 acc32[5];
    f64x4 acc64[5][2];
    if constexpr (MODE == QSL_FP64) {
        for (int d = 0; d < 5; ++d)
            for (int h = 0; h < 2; ++h) acc64[d][h] = f64x4{0, 0, 0, 0};
    } else {
        for (int d = 0; d < 5; ++d)
            for (int r = 0; r < 16; ++r) acc32[d][r] = 0.f;
    }
    bool tie = false;
    __syncthreads();

    for (int c0 = 0; c0 < nwin; c0 += KW) {
        // ---- phase R: AO values of (electron e, window wl) into LDS
        if (tid < TE * KW) {
            const int e = tid & (TE - 1), wl = tid / TE;
            const int q = c0 + wl < nwin ? wins[c0 + wl] : -1;
            if (e == 0) wq[wl] = q < 0 ? 0 : q;
            T vals[5][WIN];
            for (int d = 0; d < 5; ++d)
                for (int j = 0; j < WIN; ++j) vals[d][j] = T(0);
            if (q >= 0 && e < ne) {
                const int at = s.win_atom[q];
                const double dx = epos[e][0] - s.atom_xyz[3 * at];
                const double dy = epos[e][1] - s.atom_xyz[3 * at + 1];
                const double dz = epos[e][2] - s.atom_xyz[3 * at + 2];
                const double r2 = dist2_exact(dx, dy, dz);
                int prev = -1;
                T g = 0, g1 = 0, g2 = 0;
                for (int j = 0; j < WIN; ++j) {
                    const int slot = q * WIN + j;
                    const int sh = s.slot_shell[slot];
                    if (sh < 0) continue;
                    if (sh != prev) {
                        shell_radial<T>(s, sh, r2, g, g1, g2, tie);
                        prev = sh;
                    }
                    T v[5];
                    slot_values<T>(s, slot, (T)dx, (T)dy, (T)dz, g, g1, g2, v);
                    for (int d = 0; d < 5; ++d) vals[d][j] = v[d];
                }
            }
            if constexpr (MODE == QSL_BF16X3) {
                uint16_t* bh = (uint16_t*)bbuf;
                uint16_t* bl = bh + BELEMS;
                for (int d = 0; d < 5; ++d) {
                    uint16_t h[WIN], lo[WIN];
                    for (int j = 0; j < WIN; ++j) {
                        h[j] = bf16_rne(vals[d][j]);
                        lo[j] = bf16_rne(vals[d][j] - bf16_to_f(h[j]));
                    }
                    uint4 hv, lv;
                    hv.x = h[0] | ((uint32_t)h[1] << 16); hv.y = h[2] | ((uint32_t)h[3] << 16);
                    hv.z = h[4] | ((uint32_t)h[5] << 16); hv.w = h[6] | ((uint32_t)h[7] << 16);
                    lv.x = lo[0] | ((uint32_t)lo[1] << 16); lv.y = lo[2] | ((uint32_t)lo[3] << 16);
                    lv.z = lo[4] | ((uint32_t)lo[5] << 16); lv.w = lo[6] | ((uint32_t)lo[7] << 16);
                    *(uint4*)(bh + (d * TE + e) * LD + wl * WIN) = hv;
                    *(uint4*)(bl + (d * TE + e) * LD + wl * WIN) = lv;
                }
            } else {
                T* bt = (T*)bbuf;
                for (int d = 0; d < 5; ++d)
                    for (int j = 0; j < WIN; ++j) bt[(d * TE + e) * LD + wl * WIN + j] = vals[d][j];
            }
        }
        __syncthreads();

        // ---- phase M: MFMA over the chunk
        if constexpr (MODE == QSL_BF16X3) {
            const uint16_t* bh = (const uint16_t*)bbuf;
            const uint16_t* bl = bh + BELEMS;
            const int mo = n0 + wave * 32 + (lane & 31);
            const int oct = lane >> 5;
            for (int ks = 0; ks < KC / 16; ++ks) {
                const size_t off = ((size_t)wq[ks * 2 + oct] * ldn + mo) * WIN;
                const uint4 ah = *(const uint4*)(Ahi + off);
                const uint4 al = *(const uint4*)(Alo + off);
                const bf16x8 bah = __builtin_bit_cast(bf16x8, ah);
                const bf16x8 bal = __builtin_bit_cast(bf16x8, al);
                for (int d = 0; d < 5; ++d) {
                    const int off = (d * TE + (lane & 31)) * LD + ks * 16 + oct * 8;
                    const bf16x8 xh = __builtin_bit_cast(bf16x8, *(const uint4*)(bh + off));
                    const bf16x8 xl = __builtin_bit_cast(bf16x8, *(const uint4*)(bl + off));
                    acc32[d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, bah, acc32[d], 0, 0, 0);
                    acc32[d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, bal, acc32[d], 0, 0, 0);
                    acc32[d] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl, bah, acc32[d], 0, 0, 0);
                }
            }
        } else if constexpr (MODE == QSL_FP32) {
            const float* bt = (const float*)bbuf;
            const int mo = n0 + wave * 32 + (lane & 31);
            const int kk = lane >> 5;
            for (int ks = 0; ks < KC / 2; ++ks) {
                const int c = ks * 2 + kk;
                const int slot = wq[c / WIN] * WIN + (c % WIN);
                const float b = AT32[(size_t)slot * ldn + mo];
                for (int d = 0; d < 5; ++d) {
                    const float a = bt[(d * TE + (lane & 31)) * LD + c];
                    acc32[d] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc32[d], 0, 0, 0);
                }
            }
        } else {
            const double* bt = (const double*)bbuf;
            const int mo = n0 + wave * 16 + (lane & 15);
            const int kk = lane >> 4;
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int c = ks * 4 + kk;
                const int slot = wq[c / WIN] * WIN + (c % WIN);
                const double b = AT64[(size_t)slot * ldn + mo];
                for (int d = 0; d < 5; ++d)
                    for (int h = 0; h < 2; ++h) {
                        const double a = bt[(d * TE + h * 16 + (lane & 15)) * LD + c];
                        acc64[d][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc64[d][h], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }

    if (tie && status) atomicOr(status + w, QSL_STATUS_NEAR_TIE);
    // ---- store C[w][d][e][mo]
    if constexpr (MODE == QSL_FP64) {
        double* C = (double*)Cout;
        const int mo = n0 + wave * 16 + (lane & 15);
        if (mo < n) {
            for (int d = 0; d < 5; ++d)
                for (int h = 0; h < 2; ++h)
                    for (int r = 0; r < 4; ++r) {
                        // v_mfma_f64_16x16x4f64 result: row (lane / 16) + 4 r, column lane % 16
                        const int el = h * 16 + (lane >> 4) + 4 * r;
                        if (el < ne) C[(((size_t)w * 5 + d) * n + e0 + el) * n + mo] = acc64[d][h][r];
                    }
        }
    } else {
        float* C = (float*)Cout;
        const int mo = n0 + wave * 32 + (lane & 31);
        if (mo < n) {
            for (int d = 0; d < 5; ++d)
                for (int r = 0; r < 16; ++r) {
                    const int el = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    if (el < ne) C[(((size_t)w * 5 + d) * n + e0 + el) * n + mo] = acc32[d][r];
                }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(CT_THREADS) void contract_kernel(Job j) {
    contract_body<MODE>(j, blockIdx.x, blockIdx.y);
}

template <int MODE>
__global__ __launch_bounds__(CT_THREADS) void contract_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int by, int) { contract_body<MODE>(j, bx, by); });
}

// Grid of the contraction phase of a Job: tiles x MO blocks.
void contract_grid(Job& j) {
    const int nb = j.mode == QSL_FP64 ? CT<QSL_FP64>::NB : CT<QSL_FP32>::NB;
    j.gx = (int)(j.W * tiles_per_walker(j.n));
    j.gy = (j.n + nb - 1) / nb;
    j.gz = 1;
}

hipError_t launch_contract(const Job& j0, hipStream_t st) {
    Job j = j0;
    contract_grid(j);
    if (!j.n || !j.W) return hipSuccess;
    const dim3 g((unsigned)j.gx, j.gy);
    if (j.mode == QSL_FP64) contract_kernel<QSL_FP64><<<g, CT_THREADS, 0, st>>>(j);
    else if (j.mode == QSL_FP32) contract_kernel<QSL_FP32><<<g, CT_THREADS, 0, st>>>(j);
    else contract_kernel<QSL_BF16X3><<<g, CT_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_contract_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                      hipStream_t st) {
    if (mode == QSL_FP64) contract_batched<QSL_FP64><<<grid, CT_THREADS, 0, st>>>(jobs, prefix, njobs);
    else if (mode == QSL_FP32) contract_batched<QSL_FP32><<<grid, CT_THREADS, 0, st>>>(jobs, prefix, njobs);
    else contract_batched<QSL_BF16X3><<<grid, CT_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

}  // namespace qsl
