// Host side of the C ABI: validation, normalisation of the contraction
// weights, the padded AO-slot layout, device tables and the orchestration
// of the kernels on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qsl_internal.h"

namespace qsl {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

qsl_status hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QSL_ERR_HIP;
}

qsl_status bad(qsl_status code, const std::string& msg) {
    set_error(msg);
    return code;
}

// (2m-1)!! for m = 0..2
static double odd_fact(int m) { return m == 2 ? 3.0 : 1.0; }

// Cartesian powers of component c of a shell with angular momentum l.
static void powers(int l, int c, int p[3]) {
    static const int P1[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const int P2[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
    for (int k = 0; k < 3; ++k) p[k] = l == 0 ? 0 : (l == 1 ? P1[c][k] : P2[c][k]);
}

// Byte arena: host staging of all device tables, copied in one transfer.
struct Arena {
    std::vector<char> buf;
    size_t add(const void* src, size_t bytes) {
        size_t off = (buf.size() + 255) & ~size_t(255);
        buf.resize(off + std::max<size_t>(bytes, 1));
        if (bytes) memcpy(buf.data() + off, src, bytes);
        return off;
    }
    size_t reserve(size_t bytes) {
        size_t off = (buf.size() + 255) & ~size_t(255);
        buf.resize(off + std::max<size_t>(bytes, 1));
        return off;
    }
};

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_f64_kernel(double* p, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Kernels instead of hipMemsetAsync so that callers may capture the
// sequence into a graph.
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    fill_u32_kernel<<<blocks, 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    fill_f64_kernel<<<blocks, 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------- profiling
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof_pending;
struct ProfAgg {
    std::string name;
    int64_t launches;
    double ms;
};
static std::vector<ProfAgg> g_prof_agg;

// Set while an allocation-free call enqueues: its launches are not timed
// (timing creates events).
static thread_local bool g_prof_suspend = false;

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    if (!g_prof_on || g_prof_suspend) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;  // no events in graphs
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
    hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
    if (!a) return;
    hipEventRecord(b, st);
    g_prof_pending.push_back({name, a, b});
}


// Walkers per dA group: they share one window list (screened together).
// Default walkers per dA group: by electron, the groups are long (the
// flush is one atomic per dA entry and group); by 32-electron range, the
// group's window union stays small.
int bw_group(int64_t W, bool by_e) { return (int)std::min<int64_t>(W, by_e ? 1024 : 128); }

// Workspace layout.  The forward's regions come first: per spin,
// tile_nwin[T_s] and tile_win[T_s][n_win], and the FP64 copy of the blocked
// inversion; then the adjoint's: the lists per walker group of gw walkers
// (windows per 32-electron range, or slots per electron with by_e), the
// FP32 dA accumulator and the split-BF16 G.  A forward-only workspace ends
// at fwd_total.
WsLayout ws_layout(const DevSys& d, int64_t W, int gw, int mode, bool by_e) {
    WsLayout L{};
    size_t off = 0;
    L.job_off = off;
    off += JOBSLOT_BYTES;
    for (int s = 0; s < 2; ++s) {
        L.perm_off[s] = off;
        if (mode == QSL_FP32) off = round_up(off + (size_t)n_spin(d, s) * W * sizeof(int), 256);
    }
    for (int s = 0; s < 2; ++s) {
        int n = n_spin(d, s);
        size_t tiles = n ? (size_t)electron_tiles(n, W) : 0;
        L.nwin_off[s] = off;
        off = round_up(off + tiles * sizeof(int), 256);
        L.win_off[s] = off;
        off = round_up(off + tiles * (size_t)d.n_win * sizeof(int), 256);
    }
    for (int s = 0; s < 2; ++s) {
        const size_t n = (size_t)n_spin(d, s);
        L.gj_off[s] = off;
        if (gj_blocked((int)n)) off = round_up(off + (size_t)W * gj_ws_doubles((int)n) * sizeof(double), 256);
    }
    L.fwd_total = std::max<size_t>(off, 256);
    for (int s = 0; s < 2; ++s) {
        int n = n_spin(d, s);
        const size_t ngw = (size_t)((W + gw - 1) / std::max(gw, 1));
        size_t groups = n ? (by_e ? (size_t)n : (size_t)tiles_per_walker(n)) * ngw : 0;
        const size_t cap = by_e ? (size_t)WIN * d.n_win : (size_t)d.n_win;
        L.gnwin_off[s] = off;
        off = round_up(off + groups * sizeof(int), 256);
        L.gwin_off[s] = off;
        off = round_up(off + groups * cap * sizeof(int), 256);
    }
    for (int s = 0; s < 2; ++s) {
        L.dA32_off[s] = off;
        off = round_up(off + (size_t)n_spin(d, s) * d.n_basis * sizeof(float), 256);
    }
    for (int s = 0; s < 2; ++s) {
        const int n = n_spin(d, s);
        L.gs_off[s] = off;
        if (mode == QSL_BF16X3 && n) off = round_up(off + (size_t)W * gsplit_elems(n) * 2 * sizeof(uint16_t), 256);
    }
    for (int s = 0; s < 2; ++s) {
        const int n = n_spin(d, s);
        L.g32_off[s] = off;
        if (by_e && n) off = round_up(off + (size_t)W * n * g32_ld(n) * sizeof(float), 256);
    }
    L.total = std::max<size_t>(off, 256);
    return L;
}

// The Job of one spin of a forward call: inputs, workspace lists, outputs.
Job fwd_job(qsl_system* sys, const qsl_fwd_args* a, const WsLayout& L, char* ws, int s, bool sorted) {
    Job j{};
    j.s = sys->d;
    j.mo = sys->mo[s];
    j.spin = s;
    j.n = n_spin(sys->d, s);
    j.mode = a->mode;
    j.gw = 1;
    j.W = a->W;
    j.R = a->R;
    j.nwin = (int*)(ws + L.nwin_off[s]);
    j.win = (int*)(ws + L.win_off[s]);
    j.jobslot = ws + L.job_off;
    if (sorted && a->mode == QSL_FP32) j.wperm = (const int*)(ws + L.perm_off[s]);
    j.f32_tile = F32_TILE_DEFAULT;
    j.C = a->C[s];
    if (gj_blocked(j.n)) j.gjws = (double*)(ws + L.gj_off[s]);
    j.logdet = a->logdet;
    j.sign = a->sign;
    j.Dinv = a->Dinv[s];
    j.drift = a->drift;
    j.lap = a->lap;
    j.status = a->status;
    return j;
}

// The Job of one spin of an adjoint call.
Job bwd_job(qsl_system* sys, const qsl_bwd_args* a, const WsLayout& L, char* ws, int s, int gw, bool by_e) {
    Job j{};
    j.s = sys->d;
    j.mo = sys->mo[s];
    j.spin = s;
    j.n = n_spin(sys->d, s);
    j.mode = a->mode;
    j.gw = gw;
    j.by_e = by_e ? 1 : 0;
    // FP32: the walker order of the tiles, as the forward's (the dA by
    // electron's groups and the tile kernels read it)
    if (a->mode == QSL_FP32) j.wperm = (const int*)(ws + L.perm_off[s]);
    j.W = a->W;
    j.R = a->R;
    j.nwin = (int*)(ws + L.nwin_off[s]);
    j.win = (int*)(ws + L.win_off[s]);
    j.gnwin = (int*)(ws + L.gnwin_off[s]);
    j.gwin = (int*)(ws + L.gwin_off[s]);
    j.Dinv = const_cast<double*>(a->Dinv[s]);
    j.g = a->g_logdet;
    j.dR = a->dR;
    j.drift = const_cast<double*>(a->drift);  // read only by the backward
    if (a->dA[s]) {
        if (a->mode == QSL_FP64) j.dA64 = a->dA[s];
        else j.dA32 = (float*)(ws + L.dA32_off[s]);
        if (a->mode == QSL_BF16X3) j.gsplit = (uint16_t*)(ws + L.gs_off[s]);
        if (by_e) j.g32 = (float*)(ws + L.g32_off[s]);
    }
    j.f32_tile = F32_TILE_DEFAULT;
    return j;
}

}  // namespace qsl

using namespace qsl;

extern "C" {

const char* qsl_status_string(qsl_status s) {
    switch (s) {
        case QSL_OK: return "ok";
        case QSL_ERR_INVALID_ARG: return "invalid argument";
        case QSL_ERR_UNSUPPORTED: return "unsupported";
        case QSL_ERR_SHAPE: return "shape mismatch";
        case QSL_ERR_WORKSPACE: return "workspace too small";
        case QSL_ERR_HIP: return "HIP runtime error";
        case QSL_ERR_OOM: return "out of device memory";
    }
    return "unknown status";
}

const char* qsl_last_error(void) { return g_last_error.c_str(); }

qsl_status qsl_profile_enable(int32_t on) {
    g_prof_on = on != 0;
    return QSL_OK;
}

qsl_status qsl_profile_read(qsl_kernel_time* out, int32_t capacity, int32_t* count, int32_t reset) {
    if (!count) return bad(QSL_ERR_INVALID_ARG, "NULL count");
    for (auto& r : g_prof_pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "profile event");
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.a, r.b);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
        bool found = false;
        for (auto& g : g_prof_agg)
            if (g.name == r.name) { g.launches++; g.ms += ms; found = true; break; }
        if (!found) g_prof_agg.push_back({r.name, 1, (double)ms});
    }
    g_prof_pending.clear();
    int n = 0;
    for (auto& g : g_prof_agg) {
        if (out && n < capacity) {
            memset(out[n].name, 0, sizeof(out[n].name));
            strncpy(out[n].name, g.name.c_str(), sizeof(out[n].name) - 1);
            out[n].launches = g.launches;
            out[n].total_ms = g.ms;
        }
        ++n;
    }
    *count = n;
    if (reset) g_prof_agg.clear();
    return QSL_OK;
}

qsl_status qsl_system_create(const qsl_system_desc* d, qsl_system** out) {
    try {
        set_error("");
        if (!d || !out) return bad(QSL_ERR_INVALID_ARG, "NULL descriptor or output");
        *out = nullptr;
        if (d->flags != 0) return bad(QSL_ERR_INVALID_ARG, "flags must be 0");
        if (d->n_atoms < 0 || d->n_shells < 0) return bad(QSL_ERR_INVALID_ARG, "negative counts");
        if (d->n_up < 0 || d->n_dn < 0 || d->n_up < d->n_dn)
            return bad(QSL_ERR_INVALID_ARG, "need n_up >= n_dn >= 0");
        if (d->n_atoms && !d->atom_xyz) return bad(QSL_ERR_INVALID_ARG, "NULL atom_xyz");
        if (d->n_shells && (!d->shell_atom || !d->shell_l || !d->shell_nprim || !d->prim_exp || !d->prim_coef))
            return bad(QSL_ERR_INVALID_ARG, "NULL shell or primitive array");
        for (int i = 0; i < 3 * d->n_atoms; ++i)
            if (!std::isfinite(d->atom_xyz[i])) return bad(QSL_ERR_INVALID_ARG, "non-finite atom coordinate");
        const double T = d->screen_T > 0 ? d->screen_T : 30.0;
        int n_prim = 0;
        for (int s = 0; s < d->n_shells; ++s) {
            int a = d->shell_atom[s], l = d->shell_l[s], np = d->shell_nprim[s];
            if (a < 0 || a >= d->n_atoms) return bad(QSL_ERR_INVALID_ARG, "shell_atom out of range");
            if (s && a < d->shell_atom[s - 1]) return bad(QSL_ERR_INVALID_ARG, "shell_atom must be non-decreasing");
            if (l < 0) return bad(QSL_ERR_INVALID_ARG, "negative l");
            if (l > QSL_LMAX) return bad(QSL_ERR_UNSUPPORTED, "angular momentum above 2");
            if (np < 1) return bad(QSL_ERR_INVALID_ARG, "shell without primitives");
            if (np > QSL_PMAX) return bad(QSL_ERR_UNSUPPORTED, "more than QSL_PMAX primitives");
            n_prim += np;
        }
        for (int k = 0; k < n_prim; ++k) {
            if (!(d->prim_exp[k] > 0) || !std::isfinite(d->prim_exp[k]))
                return bad(QSL_ERR_INVALID_ARG, "exponents must be positive and finite");
            if (!std::isfinite(d->prim_coef[k])) return bad(QSL_ERR_INVALID_ARG, "non-finite weight");
        }

        qsl_system* S = new qsl_system();
        S->n_prim = n_prim;
        hipGetDevice(&S->device);

        // shells: first primitive, normalised weights
        std::vector<int> p0(d->n_shells), sh_np(d->n_shells), sh_l(d->n_shells), sh_at(d->n_shells);
        std::vector<double> c64(n_prim), ex(d->prim_exp, d->prim_exp + n_prim);
        std::vector<float> c32(n_prim);
        int off = 0;
        for (int s = 0; s < d->n_shells; ++s) {
            int l = d->shell_l[s], np = d->shell_nprim[s];
            p0[s] = off; sh_np[s] = np; sh_l[s] = l; sh_at[s] = d->shell_atom[s];
            // overlap of two unit-norm primitives x^l e^{-g r^2}: (2 sqrt(g_k g_m)/(g_k+g_m))^(l+3/2)
            double S2 = 0.0;
            for (int k = 0; k < np; ++k)
                for (int m = 0; m < np; ++m) {
                    double gk = ex[off + k], gm = ex[off + m];
                    S2 += d->prim_coef[off + k] * d->prim_coef[off + m] *
                          pow(2.0 * sqrt(gk * gm) / (gk + gm), l + 1.5);
                }
            for (int k = 0; k < np; ++k) {
                double gk = ex[off + k];
                double Nk = pow(2.0 * gk / M_PI, 0.75) * pow(4.0 * gk, 0.5 * l) / sqrt(odd_fact(l));
                c64[off + k] = d->prim_coef[off + k] * Nk / sqrt(S2);
                c32[off + k] = (float)c64[off + k];
            }
            off += np;
        }

        // AO order, padded slots and windows
        std::vector<double> atom_gmin(std::max(d->n_atoms, 1), std::numeric_limits<double>::infinity());
        for (int s = 0; s < d->n_shells; ++s)
            for (int k = 0; k < sh_np[s]; ++k)
                atom_gmin[sh_at[s]] = std::min(atom_gmin[sh_at[s]], ex[p0[s] + k]);
        std::vector<int> slot_shell, slot_pow, slot_ao;
        std::vector<double> slot_f;
        int ao = 0, s = 0;
        for (int a = 0; a < d->n_atoms; ++a) {
            size_t start = slot_shell.size();
            for (; s < d->n_shells && sh_at[s] == a; ++s) {
                int l = sh_l[s];
                for (int c = 0; c < (l + 1) * (l + 2) / 2; ++c) {
                    int p[3];
                    powers(l, c, p);
                    slot_shell.push_back(s);
                    slot_pow.push_back(p[0] | (p[1] << 4) | (p[2] << 8) | (l << 12));
                    slot_f.push_back(sqrt(odd_fact(l) / (odd_fact(p[0]) * odd_fact(p[1]) * odd_fact(p[2]))));
                    slot_ao.push_back(ao);
                    S->ao_atom.push_back(a);
                    S->ao_shell.push_back(s);
                    for (int k = 0; k < 3; ++k) S->ao_nxyz.push_back((int8_t)p[k]);
                    ++ao;
                }
            }
            while ((slot_shell.size() - start) % WIN) {
                slot_shell.push_back(-1); slot_pow.push_back(0); slot_f.push_back(0.0); slot_ao.push_back(-1);
            }
        }
        // Windows ordered by their slot pattern (shells, valid slots), atom
        // order within a pattern: every ascending window list (a tile's, a
        // walker group's) then holds windows of one pattern side by side,
        // and the AO passes, which give the two half-waves of a wave two
        // windows, branch alike in both halves.
        {
            const int nw0 = (int)slot_shell.size() / WIN;
            std::vector<int> key(nw0), perm(nw0);
            for (int q = 0; q < nw0; ++q) {
                int nv = 0, shl = slot_shell[q * WIN];
                for (int j = 0; j < WIN; ++j) {
                    if (slot_shell[q * WIN + j] < 0) continue;
                    ++nv;
                    shl = slot_shell[q * WIN + j];
                }
                key[q] = (shl - slot_shell[q * WIN]) * (WIN + 1) + nv;
                perm[q] = q;
            }
            std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
            auto permute = [&](auto& v) {
                const auto o = v;
                for (int q = 0; q < nw0; ++q)
                    for (int j = 0; j < WIN; ++j) v[(size_t)q * WIN + j] = o[(size_t)perm[q] * WIN + j];
            };
            permute(slot_shell);
            permute(slot_pow);
            permute(slot_f);
            permute(slot_ao);
        }
        const int n_slots = (int)slot_shell.size(), n_win = n_slots / WIN;
        std::vector<int> win_atom(std::max(n_win, 1));
        std::vector<double> win_gmin(std::max(n_win, 1), std::numeric_limits<double>::infinity());
        for (int q = 0; q < n_win; ++q) {
            for (int j = 0; j < WIN; ++j) {
                int sh = slot_shell[q * WIN + j];
                if (sh < 0) continue;
                win_atom[q] = sh_at[sh];
                for (int k = 0; k < sh_np[sh]; ++k) win_gmin[q] = std::min(win_gmin[q], ex[p0[sh] + k]);
            }
        }
        S->slot_ao = slot_ao;
        std::vector<WinRec> win_rec(std::max(n_win, 1));
        for (int q = 0; q < n_win; ++q) {
            WinRec& r = win_rec[q];
            memset(&r, 0, sizeof r);
            const int at = win_atom[q];
            for (int k = 0; k < 3; ++k) r.pos[k] = d->atom_xyz[3 * at + k];
            const int sh0 = slot_shell[q * WIN];
            for (int j = 0; j < WIN; ++j) {
                const int sh = slot_shell[q * WIN + j];
                if (sh < 0) { r.pw[j] = -1; continue; }
                r.pw[j] = (slot_pow[q * WIN + j] & 0xffff) | ((sh - sh0) << 16);
                r.f32[j] = (float)slot_f[q * WIN + j];
                r.f64[j] = slot_f[q * WIN + j];
                r.np[j] = sh_np[sh];
                for (int k = 0; k < sh_np[sh]; ++k) {
                    r.ex[j][k] = ex[p0[sh] + k];
                    r.c32[j][k] = c32[p0[sh] + k];
                    r.c64[j][k] = c64[p0[sh] + k];
                }
            }
        }

        std::vector<SlotRec> slot_rec(std::max(n_slots, 1));
        for (int q = 0; q < n_slots; ++q) {
            SlotRec& r = slot_rec[q];
            memset(&r, 0, sizeof r);
            const int sh = slot_shell[q];
            r.pw = -1;
            r.gmin = std::numeric_limits<double>::infinity();
            const int at = win_atom[q / WIN];
            for (int k = 0; k < 3; ++k) r.pos[k] = d->atom_xyz[3 * at + k];
            if (sh < 0) continue;
            r.pw = slot_pow[q] & 0xffff;
            r.f32 = (float)slot_f[q];
            r.np = sh_np[sh];
            for (int k = 0; k < sh_np[sh]; ++k) {
                r.ex[k] = ex[p0[sh] + k];
                r.c32[k] = c32[p0[sh] + k];
                r.gmin = std::min(r.gmin, r.ex[k]);
            }
        }

        // device tables in one allocation
        Arena ar;
        size_t o_xyz = ar.add(d->atom_xyz, sizeof(double) * 3 * d->n_atoms);
        size_t o_agm = ar.add(atom_gmin.data(), sizeof(double) * atom_gmin.size());
        size_t o_sat = ar.add(sh_at.data(), sizeof(int) * sh_at.size());
        size_t o_sl = ar.add(sh_l.data(), sizeof(int) * sh_l.size());
        size_t o_sp0 = ar.add(p0.data(), sizeof(int) * p0.size());
        size_t o_snp = ar.add(sh_np.data(), sizeof(int) * sh_np.size());
        size_t o_ex = ar.add(ex.data(), sizeof(double) * ex.size());
        size_t o_c64 = ar.add(c64.data(), sizeof(double) * c64.size());
        size_t o_c32 = ar.add(c32.data(), sizeof(float) * c32.size());
        size_t o_ssh = ar.add(slot_shell.data(), sizeof(int) * slot_shell.size());
        size_t o_spw = ar.add(slot_pow.data(), sizeof(int) * slot_pow.size());
        size_t o_sf = ar.add(slot_f.data(), sizeof(double) * slot_f.size());
        size_t o_sao = ar.add(slot_ao.data(), sizeof(int) * slot_ao.size());
        size_t o_wat = ar.add(win_atom.data(), sizeof(int) * win_atom.size());
        size_t o_wgm = ar.add(win_gmin.data(), sizeof(double) * win_gmin.size());
        size_t o_wrec = ar.add(win_rec.data(), sizeof(WinRec) * win_rec.size());
        size_t o_srec = ar.add(slot_rec.data(), sizeof(SlotRec) * slot_rec.size());
        // MO copies per spin
        size_t o_mo[2][10];
        int ldn[2];
        for (int sp = 0; sp < 2; ++sp) {
            int n = sp ? d->n_dn : d->n_up;
            ldn[sp] = n ? (int)round_up(n, 128) : 0;
            size_t cells = (size_t)n_slots * ldn[sp];
            o_mo[sp][0] = ar.reserve(cells * 8);
            o_mo[sp][1] = ar.reserve(cells * 4);
            for (int k = 2; k < 6; ++k) o_mo[sp][k] = ar.reserve(cells * 2);
            o_mo[sp][6] = ar.reserve(cells * 8);
            o_mo[sp][7] = ar.reserve(cells * 4);
            o_mo[sp][8] = ar.reserve((size_t)n_slots * 8);
            o_mo[sp][9] = ar.reserve(cells * 8);
        }
        void* blk = nullptr;
        hipError_t e = hipMalloc(&blk, ar.buf.size());
        if (e != hipSuccess) {
            delete S;
            set_error(std::string("hipMalloc of system tables: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? QSL_ERR_OOM : QSL_ERR_HIP;
        }
        e = hipMemcpy(blk, ar.buf.data(), ar.buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) { hipFree(blk); delete S; return hip_fail(e, "upload of system tables"); }
        S->dev_block = blk;
        char* b = (char*)blk;
        DevSys& D = S->d;
        D.n_atoms = d->n_atoms; D.n_shells = d->n_shells; D.n_slots = n_slots; D.n_win = n_win;
        D.n_basis = ao; D.n_up = d->n_up; D.n_dn = d->n_dn; D.T = T;
        for (int k = 0; k < 3; ++k) {
            D.box[k] = INFINITY;
            D.box[3 + k] = -INFINITY;
        }
        for (int a = 0; a < d->n_atoms; ++a)
            for (int k = 0; k < 3; ++k) {
                D.box[k] = std::min(D.box[k], d->atom_xyz[3 * a + k] - 8.0);
                D.box[3 + k] = std::max(D.box[3 + k], d->atom_xyz[3 * a + k] + 8.0);
            }
        D.atom_xyz = (const double*)(b + o_xyz); D.atom_gmin = (const double*)(b + o_agm);
        D.shell_atom = (const int*)(b + o_sat); D.shell_l = (const int*)(b + o_sl);
        D.shell_p0 = (const int*)(b + o_sp0); D.shell_np = (const int*)(b + o_snp);
        D.prim_exp = (const double*)(b + o_ex); D.prim_c64 = (const double*)(b + o_c64);
        D.prim_c32 = (const float*)(b + o_c32);
        D.slot_shell = (const int*)(b + o_ssh); D.slot_pow = (const int*)(b + o_spw);
        D.slot_f = (const double*)(b + o_sf); D.slot_ao = (const int*)(b + o_sao);
        D.win_atom = (const int*)(b + o_wat); D.win_gmin = (const double*)(b + o_wgm);
        D.win_rec = (const WinRec*)(b + o_wrec);
        D.slot_rec = (const SlotRec*)(b + o_srec);
        for (int sp = 0; sp < 2; ++sp) {
            DevMO& m = S->mo[sp];
            m.n = sp ? d->n_dn : d->n_up;
            m.ldn = ldn[sp];
            m.AT64 = (double*)(b + o_mo[sp][0]);
            m.AT32 = (float*)(b + o_mo[sp][1]);
            m.Ahi = (uint16_t*)(b + o_mo[sp][2]);
            m.Alo = (uint16_t*)(b + o_mo[sp][3]);
            m.AThi = (uint16_t*)(b + o_mo[sp][4]);
            m.ATlo = (uint16_t*)(b + o_mo[sp][5]);
            m.A64 = (double*)(b + o_mo[sp][6]);
            m.A32 = (float*)(b + o_mo[sp][7]);
            m.blkmask = (uint64_t*)(b + o_mo[sp][8]);
            m.A3 = (uint64_t*)(b + o_mo[sp][9]);
            m.set = (m.n == 0);
            S->mo_cap[sp] = ldn[sp];
        }
        *out = S;
        return QSL_OK;
    } catch (const std::bad_alloc&) {
        return bad(QSL_ERR_OOM, "host allocation failed");
    } catch (...) {
        return bad(QSL_ERR_INVALID_ARG, "unexpected exception");
    }
}

qsl_status qsl_system_destroy(qsl_system* sys) {
    if (!sys) return QSL_OK;
    if (sys->dev_block) hipFree(sys->dev_block);
    if (sys->atom_Z) hipFree(sys->atom_Z);
    for (int sp = 0; sp < 2; ++sp)
        if (sys->mo_block[sp]) hipFree(sys->mo_block[sp]);
    delete sys;
    return QSL_OK;
}

int64_t qsl_n_basis(const qsl_system* sys) { return sys ? sys->d.n_basis : -1; }

qsl_status qsl_ao_info(const qsl_system* sys, int32_t* ao_atom, int32_t* ao_shell, int8_t* ao_nxyz) {
    if (!sys) return bad(QSL_ERR_INVALID_ARG, "NULL system");
    int nb = sys->d.n_basis;
    for (int j = 0; j < nb; ++j) {
        if (ao_atom) ao_atom[j] = sys->ao_atom[j];
        if (ao_shell) ao_shell[j] = sys->ao_shell[j];
        if (ao_nxyz)
            for (int k = 0; k < 3; ++k) ao_nxyz[3 * j + k] = sys->ao_nxyz[3 * j + k];
    }
    return QSL_OK;
}

}  // extern "C"

namespace qsl {

// Copies of n_rows MO coefficient rows of one spin: in the system's own
// tables when they hold round_up(n_rows, 128) rows, else in a separate
// allocation (an orbital set larger than the spin's electrons).
static qsl_status set_mo_rows(qsl_system* sys, int32_t spin, const double* A, int n_rows, int64_t ld,
                              int32_t on_device, void* stream) {
    DevMO& m = sys->mo[spin];
    const int need = (int)round_up((size_t)n_rows, 128);
    if (need > sys->mo_cap[spin]) {
        const size_t cells = (size_t)sys->d.n_slots * need;
        // FP64, FP32, four bf16, the [ldn][slot] FP64 / FP32 copies, the
        // block masks and the three-way bf16 split
        const size_t o32 = round_up(cells * 8, 256), o16 = o32 + round_up(cells * 4, 256),
                     oa64 = o16 + 4 * round_up(cells * 2, 256), oa32 = oa64 + round_up(cells * 8, 256),
                     omask = oa32 + round_up(cells * 4, 256), oa3 = omask + round_up((size_t)sys->d.n_slots * 8, 256),
                     total = oa3 + round_up(cells * 8, 256);
        void* blk = nullptr;
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);  // earlier calls may still read the old copies
        if (e != hipSuccess) return hip_fail(e, "orbitals: synchronize");
        if ((e = hipMalloc(&blk, total)) != hipSuccess) return bad(QSL_ERR_OOM, "orbitals: allocation of MO copies");
        if (sys->mo_block[spin]) hipFree(sys->mo_block[spin]);
        sys->mo_block[spin] = blk;
        char* b = (char*)blk;
        m.AT64 = (double*)b;
        m.AT32 = (float*)(b + o32);
        m.Ahi = (uint16_t*)(b + o16);
        m.Alo = (uint16_t*)(b + o16 + round_up(cells * 2, 256));
        m.AThi = (uint16_t*)(b + o16 + 2 * round_up(cells * 2, 256));
        m.ATlo = (uint16_t*)(b + o16 + 3 * round_up(cells * 2, 256));
        m.A64 = (double*)(b + oa64);
        m.A32 = (float*)(b + oa32);
        m.blkmask = (uint64_t*)(b + omask);
        m.A3 = (uint64_t*)(b + oa3);
        sys->mo_cap[spin] = need;
        ++sys->mo_generation;
    }
    if (m.n != n_rows || m.ldn != need) ++sys->mo_generation;
    m.n = n_rows;
    m.ldn = need;
    m.set = false;
    if (n_rows == 0) {
        m.set = true;
        return QSL_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    const double* src = A;
    double* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
        size_t bytes = sizeof(double) * (size_t)m.n * ld;
        e = hipMalloc(&tmp, bytes);
        if (e != hipSuccess) return hip_fail(e, "staging of A");
        e = hipMemcpy(tmp, A, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) { hipFree(tmp); return hip_fail(e, "copy of A"); }
        src = tmp;
    }
    e = launch_build_mo(sys->d, m, src, ld, st);
    if (e != hipSuccess) { if (tmp) hipFree(tmp); return hip_fail(e, "MO copy kernel"); }
    if (tmp) {
        e = hipStreamSynchronize(st);
        hipFree(tmp);
        if (e != hipSuccess) return hip_fail(e, "set_mo synchronize");
    }
    m.set = true;
    return QSL_OK;
}

}  // namespace qsl

extern "C" {

qsl_status qsl_set_mo(qsl_system* sys, int32_t spin, const double* A, int64_t ld, int32_t on_device,
                      void* stream) {
    if (!sys) return bad(QSL_ERR_INVALID_ARG, "NULL system");
    if (spin != 0 && spin != 1) return bad(QSL_ERR_INVALID_ARG, "spin must be 0 or 1");
    const int n = n_spin(sys->d, spin);
    if (n == 0) return set_mo_rows(sys, spin, A, 0, ld, on_device, stream);
    if (!A) return bad(QSL_ERR_INVALID_ARG, "NULL A");
    if (ld < sys->d.n_basis) return bad(QSL_ERR_INVALID_ARG, "ld < N_basis");
    return set_mo_rows(sys, spin, A, n, ld, on_device, stream);
}

qsl_status qsl_set_orbitals(qsl_system* sys, int32_t spin, const double* A, int32_t n_orb, int64_t ld,
                            int32_t on_device, void* stream) {
    if (!sys) return bad(QSL_ERR_INVALID_ARG, "NULL system");
    if (spin != 0 && spin != 1) return bad(QSL_ERR_INVALID_ARG, "spin must be 0 or 1");
    if (n_orb < n_spin(sys->d, spin)) return bad(QSL_ERR_INVALID_ARG, "n_orb below the spin's electron count");
    if (n_orb > 0 && !A) return bad(QSL_ERR_INVALID_ARG, "NULL A");
    if (ld < sys->d.n_basis) return bad(QSL_ERR_INVALID_ARG, "ld < N_basis");
    return set_mo_rows(sys, spin, A, n_orb, ld, on_device, stream);
}

qsl_status qsl_workspace_size(const qsl_system* sys, int64_t W, int32_t mode, int32_t what, size_t* bytes) {
    if (!sys || !bytes) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (W < 0) return bad(QSL_ERR_INVALID_ARG, "W < 0");
    if (mode < QSL_FP64 || mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "bad mode");
    if (what < QSL_WS_FORWARD || what > QSL_WS_BOTH) return bad(QSL_ERR_INVALID_ARG, "bad workspace selector");
    const bool by_e = dA_by_electron(mode, false) && sys->d.n_win <= UNION_MAXWIN;
    const WsLayout L = ws_layout(sys->d, W, bw_group(W, by_e), mode, by_e);
    *bytes = (what & QSL_WS_BACKWARD) ? L.total : L.fwd_total;
    return QSL_OK;
}

}  // extern "C"

namespace qsl {

// Argument checks of a forward call (everything but the workspace).
static qsl_status forward_check(qsl_system* sys, const qsl_fwd_args* a) {
    if (!sys || !a) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (a->W < 0) return bad(QSL_ERR_INVALID_ARG, "W < 0");
    if (a->mode < QSL_FP64 || a->mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "bad mode");
    if (a->W == 0) return QSL_OK;
    if (!a->R) return bad(QSL_ERR_INVALID_ARG, "NULL R");
    const DevSys& d = sys->d;
    for (int s = 0; s < 2; ++s) {
        int n = n_spin(d, s);
        if (!n) continue;
        if (!sys->mo[s].set) return bad(QSL_ERR_INVALID_ARG, "MO coefficients of a spin were never set");
        if (sys->mo[s].n != n)
            return bad(QSL_ERR_SHAPE, "the MO set of a spin has more rows than electrons (qsl_set_orbitals): "
                                      "use qsl_multidet_forward");
        if (!a->C[s] || !a->Dinv[s]) return bad(QSL_ERR_INVALID_ARG, "C and Dinv outputs are required");
        if (n > GJ_NMAX) return bad(QSL_ERR_UNSUPPORTED, "more electrons of one spin than the inversion supports");
    }
    return QSL_OK;
}

// The forward's launches on workspace ws (at least the forward's part of
// ws_layout); enqueues kernels only.
static qsl_status forward_enqueue(qsl_system* sys, const qsl_fwd_args* a, char* ws, hipStream_t st) {
    const WsLayout L = ws_layout(sys->d, a->W, 1, a->mode, false);  // the forward's part only
    hipError_t e;
    if (a->status && (e = fill_u32(a->status, 0u, a->W, st)) != hipSuccess) return hip_fail(e, "status clear");
    for (int s = 0; s < 2; ++s) {
        // FP32: each electron index's walkers in space-filling-curve order,
        // so the tiles' survivor unions are tighter
        Job j = fwd_job(sys, a, L, ws, s, /*sorted=*/true);
        if (j.n) {
            if (j.wperm) {
                ProfScope ps("walker_order", st);
                if ((e = launch_wsort(j, st)) != hipSuccess) return hip_fail(e, "walker order kernel");
            }
            {
                ProfScope ps("screen", st);
                if ((e = launch_screen(j, 0, st)) != hipSuccess) return hip_fail(e, "screen kernel");
            }
            {
                ProfScope ps(a->mode == QSL_FP64 ? "contract_fp64" : a->mode == QSL_FP32 ? "contract_fp32" : "contract_bf16x3", st);
                if ((e = launch_contract(j, st)) != hipSuccess) return hip_fail(e, "contraction kernel");
            }
        }
        {
            ProfScope ps("gauss_jordan", st);
            if ((e = launch_gj(j, st)) != hipSuccess) return hip_fail(e, "inversion kernel");
        }
        if (j.n && (a->drift || a->lap)) {
            ProfScope ps("drift_lap", st);
            if ((e = launch_epilogue(j, st)) != hipSuccess) return hip_fail(e, "epilogue kernel");
        }
    }
    return QSL_OK;
}

// Workspace of qsl_forward_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself
// to a kernel (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[QSL_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

static qsl_status scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "noalloc: hipGetDevice");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return bad(QSL_ERR_UNSUPPORTED, "noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "noalloc: hipGetSymbolAddress");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QSL_OK;
}

}  // namespace qsl

extern "C" {

qsl_status qsl_forward(qsl_system* sys, const qsl_fwd_args* a, void* stream) {
    qsl_status r = forward_check(sys, a);
    if (r != QSL_OK || a->W == 0) return r;
    WsLayout L = ws_layout(sys->d, a->W, 1, a->mode, false);
    if (!a->ws || a->ws_bytes < L.fwd_total) return bad(QSL_ERR_WORKSPACE, "workspace missing or too small");
    return forward_enqueue(sys, a, (char*)a->ws, (hipStream_t)stream);
}

qsl_status qsl_forward_noalloc(qsl_system* sys, const qsl_fwd_args* a, void* stream) {
    qsl_status r = forward_check(sys, a);
    if (r != QSL_OK || a->W == 0) return r;
    const WsLayout L = ws_layout(sys->d, a->W, 1, a->mode, false);
    if (L.fwd_total > (size_t)QSL_NOALLOC_SCRATCH_BYTES)
        return bad(QSL_ERR_WORKSPACE, "noalloc: the forward of this many walkers needs " + std::to_string(L.fwd_total) +
                                          " bytes of workspace, more than the " +
                                          std::to_string((size_t)QSL_NOALLOC_SCRATCH_BYTES) + " of the static scratch");
    void* ws = nullptr;
    if ((r = scratch_address(&ws)) != QSL_OK) return r;
    g_prof_suspend = true;
    r = forward_enqueue(sys, a, (char*)ws, (hipStream_t)stream);
    g_prof_suspend = false;
    return r;
}

qsl_status qsl_backward(qsl_system* sys, const qsl_bwd_args* a, void* stream) {
    if (!sys || !a) return bad(QSL_ERR_INVALID_ARG, "NULL argument");
    if (a->W < 0) return bad(QSL_ERR_INVALID_ARG, "W < 0");
    if (a->mode < QSL_FP64 || a->mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "bad mode");
    const DevSys& d = sys->d;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    const int N = d.n_up + d.n_dn;
    for (int s = 0; s < 2; ++s) {
        // FP64 accumulates into dA directly; with no walkers, dA = 0 in every mode
        if (a->dA[s] && !a->accumulate_dA && n_spin(d, s) && (a->mode == QSL_FP64 || a->W == 0)) {
            if ((e = fill_f64(a->dA[s], 0.0, (int64_t)n_spin(d, s) * d.n_basis, st)) != hipSuccess)
                return hip_fail(e, "dA clear");
        }
    }
    if (a->W == 0) return QSL_OK;
    if (!a->R || !a->g_logdet) return bad(QSL_ERR_INVALID_ARG, "NULL R or g_logdet");
    for (int s = 0; s < 2; ++s) {
        if (!n_spin(d, s)) continue;
        if (!sys->mo[s].set) return bad(QSL_ERR_INVALID_ARG, "MO coefficients of a spin were never set");
        if (sys->mo[s].n != n_spin(d, s))
            return bad(QSL_ERR_SHAPE, "the MO set of a spin has more rows than electrons (qsl_set_orbitals)");
        if (!a->Dinv[s]) return bad(QSL_ERR_INVALID_ARG, "NULL Dinv");
    }
    const bool by_e = dA_by_electron(a->mode, false) && d.n_win <= UNION_MAXWIN;
    const int gw = bw_group(a->W, by_e);
    WsLayout L = ws_layout(d, a->W, gw, a->mode, by_e);
    if (!a->ws || a->ws_bytes < L.total) return bad(QSL_ERR_WORKSPACE, "workspace missing or too small");
    char* ws = (char*)a->ws;
    // with the drift, dR is written whole (every electron of both spins)
    if (a->dR && !a->drift && (e = fill_f64(a->dR, 0.0, a->W * N * 3, st)) != hipSuccess)
        return hip_fail(e, "dR clear");
    for (int s = 0; s < 2; ++s) {
        Job j = bwd_job(sys, a, L, ws, s, gw, by_e);
        if (!j.n) continue;
        if (j.wperm) {  // the walker order of the tiles (as the forward's)
            ProfScope ps("walker_order", st);
            if ((e = launch_wsort(j, st)) != hipSuccess) return hip_fail(e, "walker order kernel");
        }
        const bool f32acc = j.dA32 != nullptr;
        if (f32acc && (e = fill_u32((uint32_t*)j.dA32, 0u, (int64_t)j.n * d.n_basis, st)) != hipSuccess)
            return hip_fail(e, "dA accumulator clear");
        if (a->dR && a->drift) {
            ProfScope ps("dR_drift", st);
            if ((e = launch_dr_drift(j, st)) != hipSuccess) return hip_fail(e, "dR kernel");
        } else if (a->dR) {
            {
                ProfScope ps("screen", st);
                if ((e = launch_screen(j, 0, st)) != hipSuccess) return hip_fail(e, "screen kernel");
            }
            ProfScope ps("adjoint_h", st);
            if ((e = launch_adj_h(j, st)) != hipSuccess) return hip_fail(e, "adjoint H kernel");
        }
        if (a->dA[s] && by_e) {
            // the tile lists (as the forward screens them), then the slot
            // lists of the (electron, walker group) pairs
            if (!(a->dR && !a->drift)) {
                ProfScope ps("screen", st);
                if ((e = launch_screen(j, 0, st)) != hipSuccess) return hip_fail(e, "screen kernel");
            }
            {
                ProfScope ps("screen_group", st);
                if ((e = launch_group_slots(j, st)) != hipSuccess) return hip_fail(e, "group slot kernel");
            }
            {
                ProfScope ps("g32", st);
                if ((e = launch_g32(j, st)) != hipSuccess) return hip_fail(e, "G kernel");
            }
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_dae(j, st)) != hipSuccess) return hip_fail(e, "adjoint dA kernel");
        } else if (a->dA[s]) {
            {
                ProfScope ps("screen_group", st);
                if ((e = launch_screen(j, 1, st)) != hipSuccess) return hip_fail(e, "group screen kernel");
            }
            if (j.gsplit) {
                ProfScope ps("g_split", st);
                if ((e = launch_gsplit(j, st)) != hipSuccess) return hip_fail(e, "G split kernel");
            }
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_da(j, st)) != hipSuccess) return hip_fail(e, "adjoint dA kernel");
        }
        if (f32acc && (e = launch_finalize_dA(j.dA32, a->dA[s], (int64_t)j.n * d.n_basis, a->accumulate_dA, st)) != hipSuccess)
            return hip_fail(e, "dA finalize");
    }
    return QSL_OK;
}

}  // extern "C"
