// Small kernels: padded MO-coefficient copies and the drift/Laplacian
// epilogue.
#include "qsl_internal.h"

namespace qsl {

// A^s (n x N_b, row-major, leading dimension ld, FP64) -> the library's
// padded copies: AT64/AT32 [slot][ldn], A64/A32 [ldn][slot], and hi/lo bf16
// splits (hi = bf16(x), lo = bf16(x - hi) of the FP32 value x) packed per
// window: Ahi/Alo [window][ldn][8], AThi/ATlo [window][ldn/8][8][8]; and
// the exact three-way bf16 split of the FP32 value, A3 [slot][ldn].
__global__ void build_mo_kernel(DevSys s, int n, int ldn, const double* __restrict__ A, int64_t ld,
                                double* AT64, float* AT32, uint16_t* Ahi, uint16_t* Alo, uint16_t* AThi,
                                uint16_t* ATlo, double* A64, float* A32, uint64_t* A3) {
    const int64_t total = (int64_t)s.n_slots * ldn;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int slot = (int)(q / ldn), mo = (int)(q % ldn);
        const int ao = s.slot_ao[slot];
        const double v = (ao >= 0 && mo < n) ? A[(int64_t)mo * ld + ao] : 0.0;
        const float f = (float)v;
        const uint16_t h = bf16_rne(f);
        const uint16_t l = bf16_rne(f - bf16_to_f(h));
        const int win = slot / WIN, j = slot % WIN;
        // bf16 copies packed per window: the MFMA fragments of one window
        // (8 slots of consecutive MOs, or 8 MOs of its 8 slots) are
        // contiguous
        const int64_t pk = ((int64_t)win * ldn + mo) * WIN + j;                        // [win][mo][j]
        AT64[q] = v;
        AT32[q] = f;
        const int64_t pt = (((int64_t)win * (ldn / 8) + mo / 8) * WIN + j) * 8 + mo % 8;  // [win][mo/8][j][mo%8]
        Ahi[pk] = h;
        Alo[pk] = l;
        AThi[pt] = h;
        ATlo[pt] = l;
        A64[(int64_t)mo * s.n_slots + slot] = v;
        A32[(int64_t)mo * s.n_slots + slot] = f;
        uint16_t h3, m3, l3;
        bf16_split3(f, h3, m3, l3);
        A3[q] = (uint64_t)h3 | ((uint64_t)m3 << 16) | ((uint64_t)l3 << 32);
    }
}

// Block occupancy of the FP32 copy: one wavefront per slot, lane l tests
// the MOs l, l + 64, ...; bit b of the slot's mask is set when a non-zero
// coefficient lies in MO block b (32 MOs).  With more than 64 blocks every
// bit is set (no block is skipped).
__global__ void mo_mask_kernel(int n_slots, int n, int ldn, const float* __restrict__ AT32,
                               uint64_t* __restrict__ mask) {
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (slot >= n_slots) return;
    const int nblk = (n + 31) / 32;
    uint64_t m = 0;
    for (int mo = lane; mo < n; mo += 64)
        if (AT32[(size_t)slot * ldn + mo] != 0.f) m |= 1ull << (mo >> 5);
    for (int o = 32; o >= 1; o >>= 1) m |= __shfl_xor(m, o);
    if (lane == 0) mask[slot] = nblk > 64 ? ~0ull : m;
}

hipError_t launch_build_mo(const DevSys& s, DevMO& mo, const double* A, int64_t ld, hipStream_t st) {
    const int64_t total = (int64_t)s.n_slots * mo.ldn;
    if (!total) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    build_mo_kernel<<<blocks, 256, 0, st>>>(s, mo.n, mo.ldn, A, ld, mo.AT64, mo.AT32, mo.Ahi, mo.Alo, mo.AThi,
                                            mo.ATlo, mo.A64, mo.A32, mo.A3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mo_mask_kernel<<<(s.n_slots + 3) / 4, 256, 0, st>>>(s.n_slots, mo.n, mo.ldn, mo.AT32, mo.blkmask);
    return hipGetLastError();
}

// dA (caller, FP64) = [dA +] the FP32 accumulator of the adjoint kernel.
__global__ void finalize_dA_kernel(const float* __restrict__ a32, double* __restrict__ dA, int64_t count,
                                   int accumulate) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        dA[q] = (accumulate ? dA[q] : 0.0) + (double)a32[q];
}

hipError_t launch_finalize_dA(const float* dA32, double* dA, int64_t count, int accumulate, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((count + 255) / 256, 8192);
    finalize_dA_kernel<<<blocks, 256, 0, st>>>(dA32, dA, count, accumulate);
    return hipGetLastError();
}

// dA (caller, FP64) = [dA +] sum over p = 0, 1, ... of the partial sums
// part[p] (the deterministic dA: the same order on every call).
template <typename T>
__global__ void reduce_dA_kernel(const T* __restrict__ part, int npart, int64_t count, double* __restrict__ dA,
                                 int accumulate) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        double acc = accumulate ? dA[q] : 0.0;
        for (int p = 0; p < npart; ++p) acc += (double)part[(size_t)p * count + q];
        dA[q] = acc;
    }
}

hipError_t launch_reduce_dA(const void* part, bool fp64, int npart, int64_t count, double* dA, int accumulate,
                            hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((count + 255) / 256, 8192);
    if (fp64) reduce_dA_kernel<double><<<blocks, 256, 0, st>>>((const double*)part, npart, count, dA, accumulate);
    else reduce_dA_kernel<float><<<blocks, 256, 0, st>>>((const float*)part, npart, count, dA, accumulate);
    return hipGetLastError();
}

// drift[e] = sum_i Dinv[e][i] C_{2..4}[e][i], lap[e] = sum_i Dinv[e][i] C_5[e][i]
// (the determinant's "vector products"), one wavefront per electron.
template <typename Tc>
__device__ __forceinline__ void epilogue_body(const Job& j, int bx) {
    const Tc* __restrict__ C = (const Tc*)j.C;
    const double* __restrict__ Dinv = j.Dinv;
    const int n = j.n, spin = j.spin, N = j.s.n_up + j.s.n_dn, e_off = j.spin ? j.s.n_up : 0;
    const int64_t W = j.W;
    double* __restrict__ drift = j.drift;
    double* __restrict__ lap = j.lap;
    const double* __restrict__ logdet = j.logdet;
    uint32_t* __restrict__ status = j.status;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)bx * 4 + (threadIdx.x >> 6);
    if (row >= W * n) return;
    const int64_t w = row / n;
    const int e = (int)(row % n);
    const double* d = Dinv + (w * n + e) * n;
    const size_t nn = (size_t)n * n;
    const Tc* Cw = C + (size_t)w * 5 * nn + (size_t)e * n;
    // G row of the dA by electron (FP32 mode with that adjoint)
    float* __restrict__ grow = j.g32 ? j.g32 + (size_t)(w * n + e) * g32_ld(n) : nullptr;
    const double gv = grow ? j.g[2 * w + spin] : 0.0;
    double acc[4] = {0, 0, 0, 0};
    // four strides of 64 per pass, their loads issued together (clamped
    // addresses; past n nothing is added)
    for (int i0 = 0; i0 < n; i0 += 256) {
        double di[4];
        Tc cv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = min(i0 + 64 * u + lane, n - 1);
            di[u] = gmem(d)[i];
#pragma unroll
            for (int c = 0; c < 4; ++c) cv[u][c] = gmem(Cw)[(size_t)(c + 1) * nn + i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + 64 * u + lane < n) {
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = fma(di[u], (double)cv[u][c], acc[c]);
                if (grow) gmem(grow)[i0 + 64 * u + lane] = gv != 0.0 ? (float)(gv * di[u]) : 0.f;
            }
    }
    if (grow)
        for (int i = n + lane; i < g32_ld(n); i += 64) gmem(grow)[i] = 0.f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += __shfl_xor(acc[c], o);
    if (lane == 0) {
        const int64_t ge = w * N + e_off + e;
        if (drift)
            for (int c = 0; c < 3; ++c) drift[ge * 3 + c] = acc[c];
        if (lap) lap[ge] = acc[3];
        bool fin = isfinite(acc[0]) && isfinite(acc[1]) && isfinite(acc[2]) && isfinite(acc[3]);
        bool sing = logdet && isinf(logdet[2 * w + spin]) && logdet[2 * w + spin] < 0;
        if (!fin && !sing && status) atomicOr(status + w, QSL_STATUS_NONFINITE);
    }
}

template <typename Tc>
__global__ __launch_bounds__(256) void epilogue_kernel(Job j) {
    epilogue_body<Tc>(j, blockIdx.x);
}

template <typename Tc>
__global__ __launch_bounds__(256) void epilogue_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { epilogue_body<Tc>(j, bx); });
}

int epilogue_blocks(const Job& j) { return (int)((j.W * j.n + 3) / 4); }

// G = g D^-1 rounded to FP32 (0 where g = 0, and past n), [W][n][g32_ld(n)]:
// the dA by electron's operand, for walkers bound without the epilogue.
__device__ __forceinline__ void g32_body(const Job& j, int bx) {
    const int n = j.n, ld = g32_ld(n);
    const int64_t q = (int64_t)bx * 256 + threadIdx.x;
    if (q >= j.W * n * ld) return;
    const int i = (int)(q % ld);
    const int64_t we = q / ld;  // w * n + e
    const double gv = j.g[2 * (we / n) + j.spin];
    float v = 0.f;
    if (i < n && gv != 0.0) v = (float)(gv * gmem(j.Dinv)[we * n + i]);
    gmem(j.g32)[q] = v;
}

__global__ __launch_bounds__(256) void g32_kernel(Job j) { g32_body(j, blockIdx.x); }

__global__ __launch_bounds__(256) void g32_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { g32_body(j, bx); });
}

int g32_blocks(const Job& j) { return (int)((j.W * j.n * g32_ld(j.n) + 255) / 256); }

hipError_t launch_g32(const Job& j, hipStream_t st) {
    if (!j.g32 || !j.n || !j.W) return hipSuccess;
    g32_kernel<<<(unsigned)g32_blocks(j), 256, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_g32_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    g32_batched<<<grid, 256, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

hipError_t launch_epilogue(const Job& j0, hipStream_t st) {
    Job j = j0;
    j.gx = epilogue_blocks(j); j.gy = 1; j.gz = 1;
    if (!j.gx) return hipSuccess;
    if (j.mode == QSL_FP64) epilogue_kernel<double><<<(unsigned)j.gx, 256, 0, st>>>(j);
    else epilogue_kernel<float><<<(unsigned)j.gx, 256, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_epilogue_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                      hipStream_t st) {
    if (mode == QSL_FP64) epilogue_batched<double><<<grid, 256, 0, st>>>(jobs, prefix, njobs);
    else epilogue_batched<float><<<grid, 256, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// Drift and Laplacian together with the split-BF16 G^T of the dA adjoint
// (plans in BF16X3 that run both): one workgroup per (walker, electron tile
// of 32) reads the tile's D^-1 rows once for both.  The drift / Laplacian
// arithmetic is the plain epilogue's lane for lane (same sums, same order),
// and G = g D^-1 rounded to FP32 and split like gsplit_body, so the results
// are bit-identical to the two separate kernels.  The G^T tile [i][32] is
// transposed through LDS in chunks of 256 MOs: wave v fills the columns of
// its 8 electrons, then the chunk goes out as 16-byte rows.
constexpr int EPG_THREADS = 512;  // 8 waves, 4 electron rows each

template <typename Tc>
__device__ __forceinline__ void epilogue_g_body(const Job& j, int bx) {
    const Tc* __restrict__ C = (const Tc*)j.C;
    const double* __restrict__ Dinv = j.Dinv;
    const int n = j.n, spin = j.spin, N = j.s.n_up + j.s.n_dn, e_off = spin ? j.s.n_up : 0;
    const int T = tiles_per_walker(n), NIP = (n + ADJ_MB - 1) / ADJ_MB * ADJ_MB;
    const int64_t w = bx / T;
    const int t = bx % T;
    if (w >= j.W) return;
    constexpr int RW = TE / (EPG_THREADS / 64);  // electrons per wave
    constexpr int CH = 256;         // MOs per chunk
    constexpr int LDT = TE + 2;     // LDS row (uint16): 68 bytes, rows on distinct banks
    __shared__ __attribute__((aligned(16))) uint16_t th[CH][LDT], tl[CH][LDT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double gw = j.g[2 * w + spin];
    const size_t nn = (size_t)n * n;
    uint16_t* gh = j.gsplit + (w * T + t) * (int64_t)NIP * TE;
    uint16_t* gl = gh + j.W * gsplit_elems(n);
    double acc[RW][4];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    for (int i0 = 0; i0 < NIP; i0 += CH) {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int el = wave * RW + r, e = t * TE + el;
            const bool ev = e < n;
            const double* d = Dinv + (w * n + (ev ? e : 0)) * n;
            const Tc* Cw = C + (size_t)w * 5 * nn + (size_t)(ev ? e : 0) * n;
            double di[4];
            Tc cv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = min(i0 + 64 * u + lane, n - 1);
                di[u] = gmem(d)[i];
#pragma unroll
                for (int c = 0; c < 4; ++c) cv[u][c] = gmem(Cw)[(size_t)(c + 1) * nn + i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + 64 * u + lane;
                if (ev && i < n) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[r][c] = fma(di[u], (double)cv[u][c], acc[r][c]);
                }
                double v = 0.0;
                if (ev && i < n && gw != 0.0) v = gw * di[u];
                const float f = (float)v;
                const uint16_t h = bf16_rne(f);
                th[64 * u + lane][el] = h;
                tl[64 * u + lane][el] = bf16_rne(f - bf16_to_f(h));
            }
        }
        __syncthreads();
        // rows i0 .. i0 + rows - 1 of the tile, hi then lo: 4 pieces of 16
        // bytes per row
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        const int rows = min(CH, NIP - i0);
        for (int q = threadIdx.x; q < rows * 8; q += EPG_THREADS) {
            const int half = q >= rows * 4, qq = q - half * rows * 4;
            const int row = qq >> 2, part = qq & 3;
            const uint32_t* src = (const uint32_t*)((half ? tl[row] : th[row]) + part * 8);
            const u32x4 v = u32x4{src[0], src[1], src[2], src[3]};
            *gmem((u32x4*)((half ? gl : gh) + (int64_t)(i0 + row) * TE + part * 8)) = v;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += __shfl_xor(acc[r][c], o);
        const int e = t * TE + wave * RW + r;
        if (lane == 0 && e < n) {
            const int64_t ge = w * N + e_off + e;
            if (j.drift)
                for (int c = 0; c < 3; ++c) j.drift[ge * 3 + c] = acc[r][c];
            if (j.lap) j.lap[ge] = acc[r][3];
            const bool fin = isfinite(acc[r][0]) && isfinite(acc[r][1]) && isfinite(acc[r][2]) && isfinite(acc[r][3]);
            const bool sing = j.logdet && isinf(j.logdet[2 * w + spin]) && j.logdet[2 * w + spin] < 0;
            if (!fin && !sing && j.status) atomicOr(j.status + w, QSL_STATUS_NONFINITE);
        }
    }
}

__global__ __launch_bounds__(EPG_THREADS) void epilogue_g_kernel(Job j) { epilogue_g_body<float>(j, blockIdx.x); }

__global__ __launch_bounds__(EPG_THREADS) void epilogue_g_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { epilogue_g_body<float>(j, bx); });
}

int epilogue_g_blocks(const Job& j) { return (int)(j.W * tiles_per_walker(j.n)); }

hipError_t launch_epilogue_g(const Job& j0, hipStream_t st) {
    Job j = j0;
    j.gx = epilogue_g_blocks(j); j.gy = 1; j.gz = 1;
    if (!j.gx || !j.gsplit || !j.g || j.mode == QSL_FP64) return hipErrorInvalidValue;
    epilogue_g_kernel<<<(unsigned)j.gx, EPG_THREADS, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_epilogue_g_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    epilogue_g_batched<<<grid, EPG_THREADS, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

// dR through the forward's drift.  By Jacobi's formula the derivative of
// log|det D^s| in r_e is sum_i D^-1[e][i] grad phi_i(r_e), the drift of the
// "vector products" equations, so dR[w][e] = g[w][s] drift[w][e] for the
// electrons e of spin s (exactly 0 where g = 0: a singular walker's drift is
// NaN).  One thread per component.
__device__ __forceinline__ void dr_drift_body(const Job& j, int bx) {
    const int64_t q = (int64_t)bx * 256 + threadIdx.x;
    const int64_t per_w = (int64_t)j.n * 3;
    if (q >= j.W * per_w) return;
    const int64_t w = q / per_w;
    const int64_t r = q - w * per_w;  // e * 3 + component within the spin
    const int N = j.s.n_up + j.s.n_dn;
    const int64_t at = w * N * 3 + (j.spin ? (int64_t)j.s.n_up * 3 : 0) + r;
    const double gw = j.g[2 * w + j.spin];
    j.dR[at] = gw != 0.0 ? gw * j.drift[at] : 0.0;
}

__global__ __launch_bounds__(256) void dr_drift_kernel(Job j) { dr_drift_body(j, blockIdx.x); }

__global__ __launch_bounds__(256) void dr_drift_batched(const Job* jobs, const int* prefix, int njobs) {
    batch_block(jobs, prefix, njobs, [&](const Job& j, int bx, int, int) { dr_drift_body(j, bx); });
}

int dr_drift_blocks(const Job& j) { return (int)((j.W * j.n * 3 + 255) / 256); }

hipError_t launch_dr_drift(const Job& j0, hipStream_t st) {
    Job j = j0;
    j.gx = dr_drift_blocks(j); j.gy = 1; j.gz = 1;
    if (!j.gx || !j.dR || !j.drift) return hipSuccess;
    dr_drift_kernel<<<(unsigned)j.gx, 256, 0, st>>>(j);
    return hipGetLastError();
}

hipError_t launch_dr_drift_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    dr_drift_batched<<<grid, 256, 0, st>>>(jobs, prefix, njobs);
    return hipGetLastError();
}

}  // namespace qsl
