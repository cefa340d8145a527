// Internal definitions of the gfx950 Slater-matrix builder (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "../../include/qslater.h"

namespace qsl {

// Electrons per tile: one MFMA row block of 32.
constexpr int TE = 32;
// AO slots per window: the AOs of every atom are padded to a multiple of 8
// slots, so a window belongs to exactly one atom and is one 8-wide k-group of
// a bf16 MFMA operand.
constexpr int WIN = 8;
// Largest Slater matrix inverted in registers by one workgroup.
constexpr int GJ_REG_NMAX = 224;   // largest n of the register-resident inversion
constexpr int GJ_BLOCKED_FROM = GJ_REG_NMAX + 1;  // n from which the blocked inversion is used
__host__ __device__ inline bool gj_blocked(int n) { return n >= GJ_BLOCKED_FROM; }
constexpr int GJ_NMAX = 1024;      // largest n of the blocked inversion
constexpr int GJ_PANEL = 32;       // panel width of the blocked inversion
// Blocked inversion workspace per matrix: the copy of D with rows padded to
// gj_ld(n) doubles (128-byte aligned rows), the pivot rows of two panels,
// the pivot order, row flags and state; a multiple of 16 doubles.
__host__ __device__ inline int gj_ld(int n) { return (n + 15) & ~15; }
__host__ __device__ inline size_t gj_ws_doubles(int n) {
    const size_t ld = (size_t)gj_ld(n);
    return (ld * n + ld * 2 * GJ_PANEL + ((size_t)5 * n + 40) / 8 + 15) & ~(size_t)15;
}

// Everything the AO evaluation of one window needs, in one record (built
// once per system), so that an evaluation is one level of loads after the
// window index instead of a chain through slot, shell and primitive tables.
// Slot j: pw = a | b<<4 | c<<8 | l<<12 | (its shell's index within the
// window)<<16, -1 for padding; the shell's primitives are repeated per slot.
struct WinRec {
    double pos[3];
    double pad0;
    int pw[WIN];
    int np[WIN];
    float f32[WIN];
    double ex[WIN][QSL_PMAX];
    float c32[WIN][QSL_PMAX];
    // FP64-only fields last: the f32 modes read a prefix of the record
    double f64[WIN];
    double c64[WIN][QSL_PMAX];
};
// 16-byte pieces of a record read in FP32 / split-BF16 (prefix) or FP64 mode
constexpr int WINREC_Q32 = (int)(offsetof(WinRec, f64) / 16);
constexpr int WINREC_Q64 = (int)(sizeof(WinRec) / 16);
static_assert(offsetof(WinRec, f64) % 16 == 0 && sizeof(WinRec) % 16 == 0, "records are copied in 16-byte pieces");

// Everything the AO evaluation of one slot needs (the FP32 contraction
// evaluates slot by slot): atom position, the smallest exponent of the
// slot's shell (its survival test), the shell's primitives, the Cartesian
// factor and powers pw = a | b<<4 | c<<8 | l<<12 (-1 for padding).
struct SlotRec {
    double pos[3];
    double gmin;
    double ex[QSL_PMAX];
    float c32[QSL_PMAX];
    float f32;
    int pw;
    int np;
    int pad;
};
static_assert(sizeof(SlotRec) % 16 == 0, "slot records are loaded in 16-byte pieces");

// Device view of a system, passed to kernels by value.
struct DevSys {
    int n_atoms, n_shells, n_slots, n_win, n_basis;
    int n_up, n_dn;
    double T;
    double box[6];            // lo x, y, z, hi x, y, z: the atoms' box widened by 8 bohr (walker order keys)
    const double* atom_xyz;   // [n_atoms*3]
    const double* atom_gmin;  // [n_atoms] min exponent of the atom
    const int* shell_atom;    // [n_shells]
    const int* shell_l;       // [n_shells]
    const int* shell_p0;      // [n_shells] first primitive
    const int* shell_np;      // [n_shells]
    const double* prim_exp;   // [n_prim]
    const double* prim_c64;   // [n_prim] normalised weights
    const float* prim_c32;    // [n_prim]
    const int* slot_shell;    // [n_slots] shell of the slot, -1 for padding
    const int* slot_pow;      // [n_slots] a | b<<4 | c<<8 | l<<12
    const double* slot_f;     // [n_slots] Cartesian factor
    const int* slot_ao;       // [n_slots] ABI AO index, -1 for padding
    const WinRec* win_rec;    // [n_win]
    const int* win_atom;      // [n_win]
    const double* win_gmin;   // [n_win] min exponent over shells meeting the window
    const SlotRec* slot_rec;  // [n_slots]
};

// MO coefficient copies of one spin, padded: n rows -> ldn (multiple of 128).
struct DevMO {
    int n = 0, ldn = 0;
    bool set = false;
    double* AT64 = nullptr;     // [n_slots][ldn]
    float* AT32 = nullptr;      // [n_slots][ldn]
    uint16_t* Ahi = nullptr;    // bf16 bits [n_win][ldn][8 slots]
    uint16_t* Alo = nullptr;
    uint16_t* AThi = nullptr;   // bf16 bits [n_win][ldn/8][8 slots][8 MOs]
    uint16_t* ATlo = nullptr;
    double* A64 = nullptr;      // [ldn][n_slots]
    float* A32 = nullptr;       // [ldn][n_slots]
    // [n_slots][ldn]: the FP32 value x as bf16 bits hi | mid << 16 | lo << 32
    // with x = hi + mid + lo exactly (each rounded to nearest even)
    uint64_t* A3 = nullptr;
    // [n_slots]: bit b set when some MO of block [32 b, 32 b + 32) has a
    // non-zero coefficient on the slot (all bits set past 64 blocks)
    uint64_t* blkmask = nullptr;
};

}  // namespace qsl

struct qsl_system {
    qsl::DevSys d{};
    qsl::DevMO mo[2];
    void* dev_block = nullptr;  // one allocation holding all device tables
    int device = 0;
    int n_prim = 0;
    // host copies of the AO order
    std::vector<int> ao_atom, ao_shell;
    std::vector<int8_t> ao_nxyz;
    std::vector<int> slot_ao;
    // MO copies per spin: capacity (padded rows) and a separate allocation
    // when an orbital set larger than the spin's electrons was set
    int mo_cap[2] = {0, 0};
    void* mo_block[2] = {nullptr, nullptr};
    int64_t mo_generation = 0;  // raised when the MO copies move or change shape (plans rebuild their Jobs)
    // Jastrow factor and nuclear charges (qsl_set_jastrow)
    bool jastrow_set = false;
    double* atom_Z = nullptr;  // device [n_atoms]
    double c_ee = 0, b_ee = 1, c_en = 0, b_en = 1;
    double v_nn = 0;           // nuclear repulsion
};

namespace qsl {

void set_error(const std::string& msg);

inline int n_spin(const DevSys& s, int spin) { return spin ? s.n_dn : s.n_up; }
__host__ __device__ inline int tiles_per_walker(int n) { return (n + TE - 1) / TE; }
// Forward (and adjoint-H) tiles: one electron index across TE consecutive
// walkers; tile = e * walker_blocks(W) + walker block.  Electron e of every
// walker sits near the same atoms, so the tile's surviving windows are few.
__host__ __device__ inline int walker_blocks(int64_t W) { return (int)((W + TE - 1) / TE); }
__host__ __device__ inline int64_t electron_tiles(int n, int64_t W) { return (int64_t)n * walker_blocks(W); }

// ------------------------------------------------------------------ device

// Exact FP64 squared distance, evaluated as (dx*dx + dy*dy) + dz*dz with
// every product and sum rounded on its own, so that every screening decision
// is identical in every precision mode (and to a plain IEEE evaluation on the
// host).  HIP compiles with FP contraction on, and __dmul_rn / __dadd_rn are
// plain operators in this toolchain, so they would be fused into FMAs once
// inlined; contraction is switched off for this scope instead.
__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}
// gamma * r^2 of the screening test, rounded on its own (never fused with a
// later subtraction).
__device__ __forceinline__ double mul_exact(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

__device__ __forceinline__ double exp_t(double x) { return exp(x); }
// e^x for the FP32 AO evaluation (x = -gamma r^2 in [-T, 0]): 2^(x log2 e)
// with the product split exactly into h + l by an FMA remainder (log2 e
// itself as a float pair), the hardware 2^h (v_exp_f32) and the first-order
// factor 1 + l ln 2 for the small rest (|l| < 2^-17 here, so l^2 is below
// the float rounding).  A few ulp, against about 20 instructions of expf.
__device__ __forceinline__ float exp_t(float x) {
    constexpr float L2E = 1.44269502f;         // log2(e) rounded to float
    constexpr float L2E_LO = 1.92596299e-8f;   // log2(e) - L2E
    const float h = x * L2E;
    const float l = fmaf(x, L2E_LO, fmaf(x, L2E, -h));
    return __builtin_amdgcn_exp2f(h) * fmaf(l, 0.693147181f, 1.0f);
}

// x^a, a x^(a-1) and a (a-1) x^(a-2) of one Cartesian axis, a <= 2.
template <typename T>
__device__ __forceinline__ void axis_pow(int a, T x, T& p, T& dp, T& d2) {
    p = a == 0 ? T(1) : (a == 1 ? x : x * x);
    dp = a == 0 ? T(0) : (a == 1 ? T(1) : T(2) * x);
    d2 = a == 2 ? T(2) : T(0);
}

// Value, gradient and Laplacian (out[0..4]) of the CNT slots js.. of window
// record r for one electron at p (zeros for padding slots), with the near-tie
// flag of the kept-primitive tests.
template <typename T, int CNT>
__device__ __forceinline__ void rec_values(const WinRec& r, double T_thr, int js, const double p[3],
                                           T vals[5][CNT], bool& tie) {
    const double dx = p[0] - r.pos[0], dy = p[1] - r.pos[1], dz = p[2] - r.pos[2];
    const double r2 = dist2_exact(dx, dy, dz);
    const T X = (T)dx, Y = (T)dy, Z = (T)dz;
    const double tieb = 1e-12 * T_thr;
    // the slot fields first, all loads issued together
    int pws[CNT];
#pragma unroll
    for (int j = 0; j < CNT; ++j) pws[j] = r.pw[js + j];
    int prev = -1;
    T g = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int j = 0; j < CNT; ++j) {
        const int pw = pws[j];
#pragma unroll
        for (int d = 0; d < 5; ++d) vals[d][j] = T(0);
        if (pw < 0) continue;
        const int ls = pw >> 16;
        if (ls != prev) {
            g = T(0); g1 = T(0); g2 = T(0);
            const int np = r.np[js + j];
            // every primitive slot of the shell loaded at once (np <= QSL_PMAX)
            double exs[QSL_PMAX];
            T cs[QSL_PMAX];
#pragma unroll
            for (int k = 0; k < QSL_PMAX; ++k) {
                exs[k] = r.ex[js + j][k];
                if constexpr (sizeof(T) == 8) cs[k] = (T)r.c64[js + j][k];
                else cs[k] = r.c32[js + j][k];
            }
#pragma unroll
            for (int k = 0; k < QSL_PMAX; ++k) {
                if (k >= np) break;
                const double gk = exs[k];
                const double t = mul_exact(gk, r2);
                tie |= fabs(t - T_thr) <= tieb;
                if (t <= T_thr) {
                    const T c = cs[k];
                    const T ek = c * exp_t(-(T)t);
                    const T gT = (T)gk;
                    g += ek;
                    g1 += T(-2) * gT * ek;
                    g2 += ek * (T(4) * gT * gT * (T)r2 - T(6) * gT);
                }
            }
            prev = ls;
        }
        const int a = pw & 15, b = (pw >> 4) & 15, c = (pw >> 8) & 15, l = (pw >> 12) & 15;
        T px, ddx, d2x, py, ddy, d2y, pz, ddz, d2z;
        axis_pow(a, X, px, ddx, d2x);
        axis_pow(b, Y, py, ddy, d2y);
        axis_pow(c, Z, pz, ddz, d2z);
        T f;
        if constexpr (sizeof(T) == 8) f = (T)r.f64[js + j];
        else f = r.f32[js + j];
        const T fyz = f * py * pz, fxz = f * px * pz, fxy = f * px * py;
        const T P = fyz * px;
        const T pg1 = P * g1;
        vals[0][j] = P * g;
        vals[1][j] = fyz * ddx * g + pg1 * X;
        vals[2][j] = fxz * ddy * g + pg1 * Y;
        vals[3][j] = fxy * ddz * g + pg1 * Z;
        vals[4][j] = (d2x * fyz + d2y * fxz + d2z * fxy) * g + T(2 * l) * pg1 + P * g2;
    }
}

// bf16 round-to-nearest-even of a float, as raw bits (the gfx950 hardware
// conversion v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t bf16_rne(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Split of two floats x = hi + lo with hi = bf16(x), lo = bf16(x - hi), as
// packed bf16 pairs (first value in the low half): two packed conversions.
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2_t;
__device__ __forceinline__ void bf16_split2(float a, float b, uint32_t& hi, uint32_t& lo) {
    const uint32_t h = __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)a, (__bf16)b});
    const float ra = a - __uint_as_float(h << 16);
    const float rb = b - __uint_as_float(h & 0xffff0000u);
    hi = h;
    lo = __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)ra, (__bf16)rb});
}

// The same split of two floats at once, as packed bf16 pairs (a in the low
// half): three packed conversions.
__device__ __forceinline__ void bf16_split3_pair(float a, float b, uint32_t& hi, uint32_t& mid, uint32_t& lo) {
    hi = __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)a, (__bf16)b});
    const float ra = a - __uint_as_float(hi << 16), rb = b - __uint_as_float(hi & 0xffff0000u);
    mid = __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)ra, (__bf16)rb});
    const float sa = ra - __uint_as_float(mid << 16), sb = rb - __uint_as_float(mid & 0xffff0000u);
    lo = __builtin_bit_cast(uint32_t, bf16x2_t{(__bf16)sa, (__bf16)sb});
}

// Exact three-way split of a float: x = hi + mid + lo, each bf16 rounded to
// nearest even from the remainder of the previous ones (x has 24 significand
// bits, each part takes 8, so the last remainder is exact).
__device__ __forceinline__ void bf16_split3(float x, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
    hi = bf16_rne(x);
    const float r1 = x - bf16_to_f(hi);
    mid = bf16_rne(r1);
    lo = bf16_rne(r1 - bf16_to_f(mid));
}

// One (system, spin) unit of work of a kernel phase: everything the kernel
// bodies read.  A per-system launch passes one Job by value; a batched
// launch walks the blocks of several Jobs (an uneven batch of systems) with
// one deterministic schedule, so both compute the same values.
struct Job {
    DevSys s;
    DevMO mo;
    int spin, n, mode, gw;
    int gj_bias;             // Gauss-Jordan block shape: the smallest holding n, + gj_bias
    int64_t W;
    const double* R;
    int* nwin;               // per tile (gw = 1) surviving-window counts and lists
    int* win;
    int* gnwin;              // per walker group (gw walkers) counts and lists
    int* gwin;
    void* C;
    double* logdet;
    int8_t* sign;
    double* Dinv;
    double* drift;
    double* lap;
    uint32_t* status;
    const double* g;
    double* dR;
    double* dA64;
    float* dA32;
    double* gjws;            // blocked inversion (gj_blocked(n)): W x gj_ws_doubles(n)
    uint16_t* gsplit;        // BF16X3 adjoint: W x gsplit_elems(n) hi, then as many lo
    void* jobslot;           // per-system launches: device copy of the Job and its block prefix
    int f32_tile;            // FP32 products: 0 = 256 MOs per workgroup, 1 = 128, 2 = 256 on split bf16
    // Deterministic dA: one launch per electron range t_fix (-1: one launch
    // for all ranges, atomic flush), each walker group adding its block into
    // its own partial sum dApart[wb][n][N_b] (float, or double in FP64) with
    // plain loads and stores; the partials are reduced in a fixed order.
    void* dApart;
    int t_fix = -1;
    // dA by electron index: gnwin / gwin hold, per (electron, walker group
    // of gw walkers), the count and ascending list of the group's slots;
    // g32 = G = g D^-1 in FP32, [W][n][g32_ld(n)] (0 where g = 0 and past
    // n), written by the epilogue or a pre-pass
    int by_e;
    float* g32;
    // FP32 with the dA by electron: the walkers of each electron index in
    // space-filling-curve order, wperm[e][k] = walker at position k; tile
    // (e, b) and walker group (e, g) take positions [32 b, 32 b + 32) and
    // [g gw, (g + 1) gw) (NULL: walker order)
    const int* wperm;
    int gx, gy, gz;          // the Job's grid in the current phase
};
// Bytes of the device Job copy of a per-system launch (Job, then two ints).
constexpr size_t JOBSLOT_BYTES = (sizeof(Job) + 2 * sizeof(int) + 255) / 256 * 256;

// Block b of a batched launch -> (Job, block coordinates within the Job).
__device__ __forceinline__ int find_job(const int* __restrict__ prefix, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Block blockIdx.x of a batched launch (grid = prefix[njobs] blocks)
// -> body(job, bx, by, bz).  The hardware dispatcher hands out blocks in
// index order, so the work list is the queue: the plan orders Jobs by
// falling cost per block and the long blocks start first.
template <typename F>
__device__ __forceinline__ void batch_block(const Job* __restrict__ jobs, const int* __restrict__ prefix,
                                            int njobs, F body) {
    const int b = blockIdx.x;
    if (b >= prefix[njobs]) return;
    const int ji = __builtin_amdgcn_readfirstlane(find_job(prefix, njobs, b));
    const Job& j = jobs[ji];
    const int lb = b - prefix[ji];
    body(j, lb % j.gx, (lb / j.gx) % j.gy, lb / (j.gx * j.gy));
}

// The same pointer in the global address space: its loads and stores are
// global (not generic) instructions, so waits for them leave LDS traffic
// and younger loads alone.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Compile-time loop: f(integral_constant<int, I>) for I in [I0, N).
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Wavefront helpers of the pivot searches.
__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const uint64_t u = __double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint64_t u = __double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

template <int CTRL>
__device__ __forceinline__ void argmax_step(double& best, int& bi) {
    const double ob = dpp_f64<CTRL>(best);
    const int oi = __builtin_amdgcn_update_dpp(0, bi, CTRL, 0xf, 0xf, false);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
}

// Timing of kernel launches with HIP events (enabled by qsl_profile_enable).
struct ProfScope {
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
};

// ------------------------------------------------------------ host helpers
qsl_status hip_fail(hipError_t e, const char* what);
qsl_status bad(qsl_status code, const std::string& msg);
size_t round_up(size_t x, size_t a);
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t st);
// Default walkers per dA group: they share one window list.
int bw_group(int64_t W, bool by_e);
// The adjoint's dA runs by electron index (walker groups of one electron,
// an exact slot list per group, walkers as the contraction dimension) in
// FP32 unless the deterministic reduction is asked for; by 32-electron
// ranges otherwise.
inline bool dA_by_electron(int mode, bool det) { return mode == QSL_FP32 && !det; }

// Workspace of one system: byte offsets of the per-spin tile and group
// window lists and of the FP32 dA accumulator.
// MOs per workgroup of the adjoint kernels (7 blocks of 32).
constexpr int ADJ_MB = 224;
constexpr int ADJ_NIB = ADJ_MB / 32;
// Split-BF16 G^T of the dA adjoint, per walker and spin: for each electron
// tile t (32 electrons) and MO i < round_up(n, ADJ_MB), 32 values (one per
// electron of the tile), hi array then lo array.
__host__ __device__ inline int64_t gsplit_elems(int n) {
    return (int64_t)((n + TE - 1) / TE) * ((n + ADJ_MB - 1) / ADJ_MB * ADJ_MB) * TE;
}

struct WsLayout {
    size_t job_off;  // the device Job copy of per-system launches
    size_t nwin_off[2], win_off[2], dA32_off[2], gnwin_off[2], gwin_off[2], gj_off[2], gs_off[2], g32_off[2];
    size_t perm_off[2];  // walker order per electron (FP32), [n][W] int
    size_t fwd_total;  // end of the forward's regions (tile lists, blocked-inversion copy)
    size_t total;      // end of the adjoint's regions
};
WsLayout ws_layout(const DevSys& d, int64_t W, int gw, int mode, bool by_e);
// The Job of spin s of a forward / adjoint call on workspace ws.
// The FP32 products' default tile (per-system calls and a new plan): the
// split-bf16 products, as accurate as FP32 MFMA and faster.
constexpr int F32_TILE_DEFAULT = 2;
Job fwd_job(qsl_system* sys, const qsl_fwd_args* a, const WsLayout& L, char* ws, int s, bool sorted = false);
Job bwd_job(qsl_system* sys, const qsl_bwd_args* a, const WsLayout& L, char* ws, int s, int gw, bool by_e);

// ------------------------------------------------------------- launchers

// Every phase has a per-Job launcher (grid = the Job's own blocks) and a
// batched launcher whose grid covers the blocks of jobs[0..njobs) given the
// block prefix sums `prefix` (device memory, njobs + 1 entries; grid =
// prefix[njobs]) of the Job grids that the *_grid / *_blocks helpers define.

// Screening: group = 0 gives per-tile window lists (nwin/win, near-tie
// status), group = 1 per walker-group lists (gnwin/gwin, gw walkers);
// group index = t * ceil(W / gw) + walker block.
int screen_blocks(const Job& j, int group);
// Walker-group lists as the union of the tile lists (same blocks as group
// screening); for systems of at most UNION_MAXWIN windows.
constexpr int UNION_MAXWIN = 8192;
hipError_t launch_group_union(const Job& j, hipStream_t st);
hipError_t launch_group_union_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
// Walker k of electron e in the order of Job.wperm.
__device__ __forceinline__ int64_t walker_of(const int* __restrict__ wperm, int64_t W, int e, int64_t k) {
    return wperm ? (int64_t)wperm[(size_t)e * W + k] : k;
}
// Walker order of each electron index (Job.wperm): one block per (electron,
// segment of 4096 walkers) sorting them by the Morton code of the
// electron's position in the system box (ties by walker index).
int wsort_blocks(const Job& j);
hipError_t launch_wsort(const Job& j, hipStream_t st);
hipError_t launch_wsort_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
// Slot lists of the dA by electron (Job.by_e): one block per (electron,
// walker group), from the tile lists; systems of at most UNION_MAXWIN windows.
int group_slots_blocks(const Job& j);
hipError_t launch_group_slots(const Job& j, hipStream_t st);
hipError_t launch_group_slots_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
hipError_t launch_screen(const Job& j, int group, hipStream_t st);
hipError_t launch_screen_batched(const Job* jobs, const int* prefix, int njobs, int grid, int group,
                                    hipStream_t st);
// Fused AO evaluation + the five AO->MO products C_n = A B_n.
void contract_grid(Job& j);
hipError_t launch_contract(const Job& j, hipStream_t st);
// tile: the FP32 workgroup shape (Job.f32_tile); queue: NULL for one
// workgroup per item, else a zeroed device counter that `grid` resident
// workgroups draw items from (persistent launch).
hipError_t launch_contract_batched(int mode, int tile, unsigned* queue, const Job* jobs, const int* prefix, int njobs,
                                   int grid, hipStream_t st);
// Workgroups of one contraction launch that fit on a CU at once.
int contract_per_cu(int mode, int tile);
// Gauss-Jordan inversion, log|det| and sign (one block per matrix; the
// block shape depends on n, so a batched launch serves one variant).
int gj_variant(int n);
int gj_threads(int v);
int gj_job_variant(const Job& j);  // gj_variant(n) + gj_bias, clamped; 4 = blocked
// Blocked inversion (variant 4, 224 < n <= 1024): the launch sequence of one
// Job, or of the Jobs of a plan (prefix counts matrices, nmax = largest n).
hipError_t launch_gjb(const Job& j, hipStream_t st);
hipError_t launch_gjb_batched(int mode, const Job* jobs, const int* prefix, int njobs, int matrices, int nmax,
                              hipStream_t st);
hipError_t launch_gj(const Job& j, hipStream_t st);
hipError_t launch_gj_batched(int mode, int v, const Job* jobs, const int* prefix, int njobs, int grid,
                             hipStream_t st);
// Row length of the FP32 G of the dA by electron: whole blocks of 224 MOs.
__host__ __device__ inline int g32_ld(int n) { return (n + ADJ_MB - 1) / ADJ_MB * ADJ_MB; }
// G = g D^-1 in FP32 (Job.g32) for walkers bound without the epilogue.
int g32_blocks(const Job& j);
hipError_t launch_g32(const Job& j, hipStream_t st);
hipError_t launch_g32_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
// Drift and Laplacian (four electrons per block); with Job.g32 set the same
// pass writes G = g D^-1 in FP32 for the dA by electron.
int epilogue_blocks(const Job& j);
// dR of one spin from the forward's drift: dR[w][e] = g[w][s] drift[w][e].
int dr_drift_blocks(const Job& j);
hipError_t launch_dr_drift(const Job& j, hipStream_t st);
hipError_t launch_dr_drift_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
hipError_t launch_epilogue(const Job& j, hipStream_t st);
hipError_t launch_epilogue_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                      hipStream_t st);
// Drift and Laplacian plus the split-BF16 G^T (Job.g, Job.gsplit; f32 C):
// one block per (walker, electron tile).
int epilogue_g_blocks(const Job& j);
hipError_t launch_epilogue_g(const Job& j, hipStream_t st);
hipError_t launch_epilogue_g_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
// Adjoint: H = G A and dR per tile; dA per walker group.
void adj_h_grid(Job& j);
void adj_da_grid(Job& j);
// G = g D^-1 of the dA adjoint as its BF16 hi/lo pair, transposed per
// electron tile (Job.gsplit); BF16X3 mode.
int gsplit_blocks(const Job& j);
hipError_t launch_gsplit(const Job& j, hipStream_t st);
hipError_t launch_gsplit_batched(const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
hipError_t launch_adj_h(const Job& j, hipStream_t st);
hipError_t launch_adj_da(const Job& j, hipStream_t st);
hipError_t launch_adj_h_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                   hipStream_t st);
hipError_t launch_adj_da_batched(int mode, const Job* jobs, const int* prefix, int njobs, int grid,
                                    hipStream_t st);
// dA by electron (FP32, Job.by_e): grid (electron x walker group x chunk
// stride, MO blocks of 224) over the group slot lists.
void adj_dae_grid(Job& j);
hipError_t launch_adj_dae(const Job& j, hipStream_t st);
hipError_t launch_adj_dae_batched(int tile, const Job* jobs, const int* prefix, int njobs, int grid, hipStream_t st);
hipError_t launch_finalize_dA(const float* dA32, double* dA, int64_t count, int accumulate, hipStream_t st);
// dA = [dA +] sum_p part[p] (p ascending; float or double partials).
hipError_t launch_reduce_dA(const void* part, bool fp64, int npart, int64_t count, double* dA, int accumulate,
                            hipStream_t st);
hipError_t launch_build_mo(const DevSys& s, DevMO& mo, const double* A_dev, int64_t ld,
                           hipStream_t st);

}  // namespace qsl

struct qsl_plan;

namespace qsl {
// The plan's system i and its bound forward arguments (NULL when out of
// range or never bound).
qsl_system* plan_system(qsl_plan* p, int i);
const qsl_fwd_args* plan_fwd(const qsl_plan* p, int i);
int64_t plan_walkers(const qsl_plan* p, int i);

}  // namespace qsl
