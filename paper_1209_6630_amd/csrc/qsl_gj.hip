// FP64 log|det|, sign and inverse of the Slater matrices (inversion step,
// section "Overall performance of QMC=Chem"; Slater matrix D_ij = phi_i(r_j)).
//
// One workgroup inverts one n x n matrix held entirely in registers:
// thread (pr, pc) of a PR x PC grid owns D[i][e] for i = pc + PC c (MO rows)
// and e = pr + PR r (electron columns), loaded coalesced from C_1[e][i].
// Gauss-Jordan elimination with partial pivoting on the rows of D: at step
// k the pivot is the largest |D[i][k]| over rows not yet used (smallest i on
// exact ties), found by one thread row with a wavefront shuffle reduction.
// Pivot rows are not moved; the pivot sequence p_k is recorded and the
// result is un-permuted on the way out: D^-1[k][p_j] = M[p_k][j].  The pivots
// are the diagonal of U in P D = L U, so log|det| = sum log|pivot| and
// sign = sign(permutation) prod sign(pivot).  2 n^3 flops per matrix.
#include "qsl_internal.h"

namespace qsl {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Pivot search over column k (register row RK of thread row k % PR) among
// the rows not yet used; publishes the pivot and the column (with a zero in
// the pivot row, which the update must leave untouched).
template <int PC, int CPT>
__device__ __forceinline__ void gj_search(const double (&col)[CPT], int n, int pc, uint32_t used,
                                          double* colout, int* piv_idx, double* piv_val) {
    double best = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = pc + PC * c;
        const double v = fabs(col[c]);
        if (i < n && !((used >> c) & 1u) && v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = PC / 2; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = pc + PC * c;
        if (i < n) colout[i] = (i == bi) ? 0.0 : col[c];
        if (i == bi) *piv_val = col[c];
    }
    if (pc == 0) *piv_idx = bi;
}

template <int PR, int PC, int RPT, int CPT, typename Tin>
__global__ __launch_bounds__(PR* PC) void gj_kernel(const Tin* __restrict__ C, int n, int spin,
                                                    double* __restrict__ Dinv, double* __restrict__ logdet,
                                                    int8_t* __restrict__ sign, uint32_t* __restrict__ status) {
    constexpr int NT = PR * PC;
    constexpr int NR = PC * CPT;  // capacity in D rows (MO index i)
    constexpr int NC = PR * RPT;  // capacity in D columns (electron index e)
    constexpr int QC = 8;         // rows of D^-1 staged per output pass
    __shared__ double colbuf[2][NR];
    __shared__ double rowbuf[2][NC];
    __shared__ int piv_idx[2];
    __shared__ double piv_val[2];
    __shared__ int perm[NC];
    __shared__ int invp[NR];
    __shared__ double rowpiv[NR];
    __shared__ double stage[QC][NC > NR ? NC : NR];
    __shared__ int s_flag;

    const int w = blockIdx.x;
    const int tid = threadIdx.x, pr = tid / PC, pc = tid % PC;
    const size_t nn = (size_t)n * n;
    const Tin* C1 = C + (size_t)w * 5 * nn;  // derivative 0 block

    double M[RPT][CPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int e = pr + PR * r, i = pc + PC * c;
            M[r][c] = (e < n && i < n) ? (double)C1[(size_t)e * n + i] : 0.0;
        }
    for (int k = tid; k < NR; k += NT) { colbuf[0][k] = 0.0; colbuf[1][k] = 0.0; }
    for (int k = tid; k < NC; k += NT) { rowbuf[0][k] = 0.0; rowbuf[1][k] = 0.0; }
    if (tid == 0) s_flag = 0;
    __syncthreads();
    uint32_t used = 0;  // bit c: row pc + PC c already a pivot row
    if (pr == 0) {
        double col[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) col[c] = M[0][c];
        gj_search<PC, CPT>(col, n, pc, used, colbuf[0], &piv_idx[0], &piv_val[0]);
    }

    bool singular = false;
    for (int k = 0; k < n; ++k) {
        const int b = k & 1;
        __syncthreads();  // pivot, column k and the previous update are visible
        const int p = __builtin_amdgcn_readfirstlane(piv_idx[b]);
        const double pv = piv_val[b];
        if (p >= n || !(pv != 0.0) || !isfinite(pv)) {  // zero (or NaN) pivot
            singular = true;
            if (tid == 0) s_flag = isfinite(pv) || p >= n ? 1 : 2;
            break;
        }
        const double inv = 1.0 / pv;
        const int cp = p / PC;  // wave-uniform
        const bool own_p = pc == p % PC;
        // the pivot row, normalised; entry k carries 1 + 1/pv so that the
        // update turns column k into -D[i][k]/pv
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (c == cp) {
                if (own_p) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) {
                        const int e = pr + PR * r;
                        if (e < n) rowbuf[b][e] = e == k ? 1.0 + inv : M[r][c] * inv;
                    }
                    used |= 1u << c;
                }
            }
        }
        if (tid == 0) {
            perm[k] = p;
            rowpiv[p] = pv;
        }
        __syncthreads();
        // rank-1 update; the pivot row keeps its values (scaled by pv), its
        // column-k entry becomes 1 (i.e. 1/pv after the final row scaling)
        const int rk = k / PR, kk = k % PR;
        const int k1 = k + 1, rk1 = k1 / PR, kk1 = k1 % PR;
        double col[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) col[c] = 0.0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const double rv = rowbuf[b][pr + PR * r];
#pragma unroll
            for (int c = 0; c < CPT; ++c) M[r][c] = fma(-colbuf[b][pc + PC * c], rv, M[r][c]);
            if (r == rk) {
#pragma unroll
                for (int c = 0; c < CPT; ++c)
                    if (c == cp && pr == kk && own_p) M[r][c] = 1.0;
            }
            if (r == rk1) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) col[c] = M[r][c];
            }
        }
        if (k1 < n && pr == kk1) gj_search<PC, CPT>(col, n, pc, used, colbuf[b ^ 1], &piv_idx[b ^ 1], &piv_val[b ^ 1]);
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
    // D^-1[invp[i]][perm[e]] = M[i][e] / pivot(i), staged QC rows at a time
    int rowi[CPT];
    double rs[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = pc + PC * c;
        rowi[c] = i < n ? invp[i] : -1;
        rs[c] = i < n ? 1.0 / rowpiv[i] : 0.0;
    }
    int cole[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int e = pr + PR * r;
        cole[r] = e < n ? perm[e] : -1;
    }
    for (int q0 = 0; q0 < n; q0 += QC) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int rr = rowi[c] - q0;
            if (rr >= 0 && rr < QC) {
#pragma unroll
                for (int r = 0; r < RPT; ++r)
                    if (cole[r] >= 0) stage[rr][cole[r]] = M[r][c] * rs[c];
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

__global__ void empty_spin_kernel(int64_t W, int spin, double* logdet, int8_t* sign) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w < W) {
        if (logdet) logdet[2 * w + spin] = 0.0;
        if (sign) sign[2 * w + spin] = 1;
    }
}

template <typename Tin>
static hipError_t gj_dispatch(const Tin* C, int n, int64_t W, int spin, double* Dinv, double* logdet, int8_t* sign,
                              uint32_t* status, hipStream_t st) {
    const dim3 g((unsigned)W);
    if (n <= 32) gj_kernel<8, 32, 4, 1, Tin><<<g, 256, 0, st>>>(C, n, spin, Dinv, logdet, sign, status);
    else if (n <= 64) gj_kernel<16, 32, 4, 2, Tin><<<g, 512, 0, st>>>(C, n, spin, Dinv, logdet, sign, status);
    else if (n <= 128) gj_kernel<16, 32, 8, 4, Tin><<<g, 512, 0, st>>>(C, n, spin, Dinv, logdet, sign, status);
    else gj_kernel<16, 32, 14, 7, Tin><<<g, 512, 0, st>>>(C, n, spin, Dinv, logdet, sign, status);
    return hipGetLastError();
}

hipError_t launch_gj(int mode, const void* C, int n, int64_t W, int spin, double* Dinv, double* logdet,
                     int8_t* sign, uint32_t* status, hipStream_t st) {
    if (W <= 0) return hipSuccess;
    if (n == 0) {
        empty_spin_kernel<<<(unsigned)((W + 255) / 256), 256, 0, st>>>(W, spin, logdet, sign);
        return hipGetLastError();
    }
    if (n > GJ_NMAX) return hipErrorInvalidValue;
    if (mode == QSL_FP64) return gj_dispatch<double>((const double*)C, n, W, spin, Dinv, logdet, sign, status, st);
    return gj_dispatch<float>((const float*)C, n, W, spin, Dinv, logdet, sign, status, st);
}

}  // namespace qsl
