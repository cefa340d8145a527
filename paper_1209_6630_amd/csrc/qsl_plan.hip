// Plans: the forward and the adjoint of an uneven batch of systems, one
// batched launch per kernel phase over a device work list, optionally
// captured into a HIP graph, plus the autotuner over the plan's runtime
// parameters with its JSON cache.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "qsl_internal.h"

namespace qsl {

// Kernel phases of a launch, in order.
enum Phase {
    PH_SCREEN = 0,   // per-tile window lists (forward; reused by the adjoint)
    PH_CONTRACT,     // AO evaluation + the five products
    PH_GJ0,          // Gauss-Jordan, one phase per block shape
    PH_GJ1,
    PH_GJ2,
    PH_GJ3,
    PH_GJ4,          // blocked (n > 224)
    PH_EPILOGUE,     // drift and Laplacian
    PH_EPI_G,        // drift and Laplacian with the split-BF16 G^T (BF16X3 with dA)
    PH_DR,           // dR = g drift (drift bound)
    PH_ADJ_H,        // H = G A, dR (no drift bound)
    PH_SCREEN_G,     // per walker-group window lists
    PH_GSPLIT,       // split-BF16 G^T for dA (BF16X3)
    PH_ADJ_DA,       // dA by 32-electron range
    PH_SLOTS_G,      // dA by electron: the (electron, walker group) slot lists
    PH_G32,          // dA by electron: G = g D^-1 in FP32 where no epilogue writes it
    PH_ADJ_DAE,      // dA by electron
    PH_SORT,         // walker order per electron index (FP32 with the dA by electron; runs first)
    PH_COUNT
};

struct PhaseList {
    std::vector<Job> jobs;      // host copies, grids set for the phase
    std::vector<int> prefix;    // block prefix sums (njobs + 1)
    size_t jobs_off = 0, prefix_off = 0;
    int blocks() const { return prefix.empty() ? 0 : prefix.back(); }
};

}  // namespace qsl

using namespace qsl;

struct qsl_plan {
    int n_sys = 0, mode = 0;
    uint32_t flags = 0;
    int device = 0;
    std::vector<qsl_system*> sys;
    std::vector<int64_t> W;
    std::vector<qsl_fwd_args> fwd;
    std::vector<qsl_bwd_args> bwd;
    std::vector<char> bound, has_bwd;
    qsl_tuning tune{1, 0, 0, F32_TILE_DEFAULT, 0, 0};
    int n_cu = 256;  // compute units (the persistent launch's grid)
    // workspace: the persistent launch's item counter, then per system window
    // lists and dA accumulators, then the deterministic dA's partial sums
    void* ws = nullptr;
    size_t ws_cap = 0;
    std::vector<size_t> ws_off;
    std::vector<WsLayout> lay;
    std::vector<int> gw;
    // per-job (system, spin) Jobs and the device work lists of the phases
    std::vector<Job> fjobs, bjobs;
    PhaseList ph[PH_COUNT];
    std::vector<PhaseList> da_t;  // deterministic dA: the adjoint dA launch of each electron range
    void* lists = nullptr;
    size_t lists_cap = 0;
    bool dirty = true;
    std::vector<int64_t> mo_gen;  // the systems' MO generations the Jobs were built from
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace qsl {

static void drop_graph(qsl_plan* p) {
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// The plan's dA runs by electron (FP32 without det_dA, systems whose
// windows fit the slot screen's bitmap) or by 32-electron range.
static bool plan_by_e(const qsl_plan* p, int i) {
    return dA_by_electron(p->mode, p->tune.det_dA != 0) && p->sys[i]->d.n_win <= UNION_MAXWIN;
}

static int plan_gw(const qsl_plan* p, int i) {
    const int64_t W = std::max<int64_t>(p->W[i], 1);
    return p->tune.adj_group > 0 ? (int)std::min<int64_t>(p->tune.adj_group, W) : bw_group(W, plan_by_e(p, i));
}

// Jobs in falling order of n (the larger systems' blocks start first);
// ties keep the (system, spin) order.
static void sort_jobs(std::vector<Job>& v) {
    std::stable_sort(v.begin(), v.end(), [](const Job& a, const Job& b) { return a.n > b.n; });
}

static void set_prefix(PhaseList& L) {
    L.prefix.assign(1, 0);
    for (const Job& j : L.jobs) L.prefix.push_back(L.prefix.back() + j.gx * j.gy * j.gz);
}

// Workspace, Jobs and device work lists for the current bindings and tuning.
static qsl_status prepare(qsl_plan* p, hipStream_t st) {
    for (int i = 0; i < p->n_sys; ++i) {
        if (!p->bound[i]) return bad(QSL_ERR_INVALID_ARG, "plan: system " + std::to_string(i) + " was never bound");
        for (int s = 0; s < 2; ++s)
            if (p->sys[i]->mo[s].n != n_spin(p->sys[i]->d, s))
                return bad(QSL_ERR_SHAPE, "plan: the MO set of a spin has more rows than electrons");
    }
    p->mo_gen.resize(p->n_sys);
    for (int i = 0; i < p->n_sys; ++i) p->mo_gen[i] = p->sys[i]->mo_generation;
    hipError_t e;
    // nothing of an earlier launch may still read the buffers replaced here
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "plan: stream synchronize");
    drop_graph(p);
    p->lay.resize(p->n_sys);
    p->ws_off.resize(p->n_sys);
    p->gw.resize(p->n_sys);
    size_t total = 256;  // the item counter
    for (int i = 0; i < p->n_sys; ++i) {
        p->gw[i] = plan_gw(p, i);
        p->lay[i] = ws_layout(p->sys[i]->d, p->W[i], p->gw[i], p->mode, plan_by_e(p, i));
        p->ws_off[i] = total;
        total = round_up(total + p->lay[i].total, 256);
    }
    // deterministic dA: one partial sum [n][N_b] per walker group and spin
    const bool det = p->tune.det_dA != 0;
    std::vector<size_t> part_off(2 * p->n_sys, 0);
    const size_t elem = p->mode == QSL_FP64 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < p->n_sys && det; ++i) {
        if (!p->has_bwd[i]) continue;
        const int64_t ngw = (p->W[i] + p->gw[i] - 1) / p->gw[i];
        for (int s = 0; s < 2; ++s) {
            if (!p->bwd[i].dA[s]) continue;
            part_off[2 * i + s] = total;
            total = round_up(total + (size_t)ngw * n_spin(p->sys[i]->d, s) * p->sys[i]->d.n_basis * elem, 256);
        }
    }
    if (total > p->ws_cap) {
        if (p->ws) hipFree(p->ws);
        p->ws = nullptr;
        p->ws_cap = 0;
        if ((e = hipMalloc(&p->ws, total)) != hipSuccess) return bad(QSL_ERR_OOM, "plan: workspace allocation");
        p->ws_cap = total;
    }
    char* ws = (char*)p->ws;
    p->fjobs.clear();
    p->bjobs.clear();
    for (int i = 0; i < p->n_sys; ++i)
        for (int s = 0; s < 2; ++s) {
            Job f = fwd_job(p->sys[i], &p->fwd[i], p->lay[i], ws + p->ws_off[i], s, /*sorted=*/true);
            f.gj_bias = p->tune.gj_bias;
            f.f32_tile = p->tune.contract_tile;
            p->fjobs.push_back(f);
            if (p->has_bwd[i]) {
                Job b = bwd_job(p->sys[i], &p->bwd[i], p->lay[i], ws + p->ws_off[i], s, p->gw[i], plan_by_e(p, i));
                b.f32_tile = p->tune.contract_tile;
                if (det && part_off[2 * i + s] && (b.dA64 || b.dA32)) b.dApart = ws + part_off[2 * i + s];
                p->bjobs.push_back(b);
            }
        }
    for (auto& L : p->ph) { L.jobs.clear(); L.prefix.clear(); }
    p->da_t.clear();
    for (const Job& f : p->fjobs) {
        if (!f.n || !f.W) continue;
        Job j = f;
        if (f.wperm) {
            j.gx = wsort_blocks(j); j.gy = 1; j.gz = 1;
            p->ph[PH_SORT].jobs.push_back(j);
            j = f;
        }
        j.gx = screen_blocks(j, 0); j.gy = 1; j.gz = 1;
        p->ph[PH_SCREEN].jobs.push_back(j);
        j = f;
        contract_grid(j);
        p->ph[PH_CONTRACT].jobs.push_back(j);
        j = f;
        j.gx = (int)j.W; j.gy = 1; j.gz = 1;
        p->ph[PH_GJ0 + gj_job_variant(j)].jobs.push_back(j);
        if (f.drift || f.lap) {
            j = f;
            // BF16X3 with dA: the epilogue also writes the adjoint's split G
            // (it reads the same D^-1 rows), and g_split does not run
            const Job* bg = nullptr;
            if (f.mode == QSL_BF16X3)
                for (const Job& b : p->bjobs)
                    if (b.gsplit && b.g && (b.dA64 || b.dA32) && b.Dinv == f.Dinv && b.spin == f.spin && b.W == f.W &&
                        b.n == f.n)
                        bg = &b;
            if (bg) {
                j.g = bg->g;
                j.gsplit = bg->gsplit;
                j.gx = epilogue_g_blocks(j); j.gy = 1; j.gz = 1;
                p->ph[PH_EPI_G].jobs.push_back(j);
            } else {
                // FP32 with the dA by electron: the epilogue also writes G
                for (const Job& b : p->bjobs)
                    if (b.g32 && b.by_e && (b.dA64 || b.dA32) && b.Dinv == f.Dinv && b.spin == f.spin &&
                        b.W == f.W && b.n == f.n) {
                        j.g = b.g;
                        j.g32 = b.g32;
                    }
                j.gx = epilogue_blocks(j); j.gy = 1; j.gz = 1;
                p->ph[PH_EPILOGUE].jobs.push_back(j);
            }
        }
    }
    auto g_fused = [&](const Job& b) {
        for (const Job& e : p->ph[PH_EPI_G].jobs)
            if (e.gsplit == b.gsplit) return true;
        return false;
    };
    for (const Job& b : p->bjobs) {
        if (!b.n || !b.W) continue;
        Job j = b;
        if (j.dR && j.drift) {
            j.gx = dr_drift_blocks(j); j.gy = 1; j.gz = 1;
            p->ph[PH_DR].jobs.push_back(j);
        } else if (j.dR) {
            adj_h_grid(j);
            p->ph[PH_ADJ_H].jobs.push_back(j);
        }
        if ((b.dA64 || b.dA32) && b.by_e) {
            j = b;
            j.gx = group_slots_blocks(j); j.gy = 1; j.gz = 1;
            p->ph[PH_SLOTS_G].jobs.push_back(j);
            bool g_written = false;
            for (const Job& ej : p->ph[PH_EPILOGUE].jobs) g_written |= ej.g32 == b.g32;
            if (!g_written) {
                j = b;
                j.gx = g32_blocks(j); j.gy = 1; j.gz = 1;
                p->ph[PH_G32].jobs.push_back(j);
            }
            j = b;
            adj_dae_grid(j);
            p->ph[PH_ADJ_DAE].jobs.push_back(j);
        } else if (b.dA64 || b.dA32) {
            j = b;
            j.gx = screen_blocks(j, 1); j.gy = 1; j.gz = 1;
            p->ph[PH_SCREEN_G].jobs.push_back(j);
            if (b.gsplit && !g_fused(b)) {
                j = b;
                j.gx = gsplit_blocks(j); j.gy = 1; j.gz = 1;
                p->ph[PH_GSPLIT].jobs.push_back(j);
            }
            if (b.dApart) {
                // electron range t of every Job in launch t (ascending)
                const int T = tiles_per_walker(b.n);
                if ((int)p->da_t.size() < T) p->da_t.resize(T);
                for (int t = 0; t < T; ++t) {
                    j = b;
                    j.t_fix = t;
                    adj_da_grid(j);
                    p->da_t[t].jobs.push_back(j);
                }
            } else {
                j = b;
                adj_da_grid(j);
                p->ph[PH_ADJ_DA].jobs.push_back(j);
            }
        }
    }
    size_t bytes = 0;
    auto place = [&](PhaseList& L) {
        sort_jobs(L.jobs);
        set_prefix(L);
        L.jobs_off = bytes;
        bytes = round_up(bytes + L.jobs.size() * sizeof(Job), 256);
        L.prefix_off = bytes;
        bytes = round_up(bytes + L.prefix.size() * sizeof(int), 256);
    };
    for (auto& L : p->ph) place(L);
    for (auto& L : p->da_t) place(L);
    if (bytes > p->lists_cap) {
        if (p->lists) hipFree(p->lists);
        p->lists = nullptr;
        p->lists_cap = 0;
        if ((e = hipMalloc(&p->lists, bytes)) != hipSuccess) return bad(QSL_ERR_OOM, "plan: work list allocation");
        p->lists_cap = bytes;
    }
    std::vector<char> host(bytes, 0);
    auto put = [&](const PhaseList& L) {
        if (!L.jobs.empty()) memcpy(host.data() + L.jobs_off, L.jobs.data(), L.jobs.size() * sizeof(Job));
        memcpy(host.data() + L.prefix_off, L.prefix.data(), L.prefix.size() * sizeof(int));
    };
    for (auto& L : p->ph) put(L);
    for (auto& L : p->da_t) put(L);
    if (bytes && (e = hipMemcpy(p->lists, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "plan: work list upload");
    p->dirty = false;
    return QSL_OK;
}

static const Job* dev_jobs(const qsl_plan* p, const PhaseList& L) {
    return (const Job*)((const char*)p->lists + L.jobs_off);
}
static const int* dev_prefix(const qsl_plan* p, const PhaseList& L) {
    return (const int*)((const char*)p->lists + L.prefix_off);
}
static const Job* dev_jobs(const qsl_plan* p, int ph) { return dev_jobs(p, p->ph[ph]); }
static const int* dev_prefix(const qsl_plan* p, int ph) { return dev_prefix(p, p->ph[ph]); }

static const char* contract_name(int mode) {
    return mode == QSL_FP64 ? "contract_fp64" : mode == QSL_FP32 ? "contract_fp32" : "contract_bf16x3";
}

// Enqueue one launch of the plan on st (no synchronisation, no allocation:
// safe under stream capture).
static qsl_status enqueue(qsl_plan* p, hipStream_t st) {
    hipError_t e;
    const bool batched = p->tune.batched != 0;
    const int mode = p->mode;
    // clears
    for (int i = 0; i < p->n_sys; ++i) {
        const qsl_fwd_args& f = p->fwd[i];
        if (f.status && f.W && (e = fill_u32(f.status, 0u, f.W, st)) != hipSuccess) return hip_fail(e, "status clear");
        if (!p->has_bwd[i]) continue;
        const qsl_bwd_args& b = p->bwd[i];
        const DevSys& d = p->sys[i]->d;
        // with the drift, dR is written whole
        if (b.dR && !b.drift && b.W && (e = fill_f64(b.dR, 0.0, b.W * (d.n_up + d.n_dn) * 3, st)) != hipSuccess)
            return hip_fail(e, "dR clear");
    }
    for (int i = 0, k = 0; i < p->n_sys; ++i) {
        if (!p->has_bwd[i]) continue;
        for (int s = 0; s < 2; ++s, ++k) {
            const Job& j = p->bjobs[k];
            const int64_t cnt = (int64_t)j.n * j.s.n_basis;
            if (j.dApart) {
                const int64_t words = cnt * ((j.W + j.gw - 1) / j.gw) * (mode == QSL_FP64 ? 2 : 1);
                if ((e = fill_u32((uint32_t*)j.dApart, 0u, words, st)) != hipSuccess) return hip_fail(e, "dA clear");
                continue;
            }
            if (j.dA32 && (e = fill_u32((uint32_t*)j.dA32, 0u, cnt, st)) != hipSuccess) return hip_fail(e, "dA clear");
            if (j.dA64 && !p->bwd[i].accumulate_dA && (e = fill_f64(j.dA64, 0.0, cnt, st)) != hipSuccess)
                return hip_fail(e, "dA clear");
        }
    }
    // forward
    if (batched) {
        auto& WS = p->ph[PH_SORT];
        if (WS.blocks()) {
            ProfScope ps("walker_order", st);
            if ((e = launch_wsort_batched(dev_jobs(p, PH_SORT), dev_prefix(p, PH_SORT), (int)WS.jobs.size(), WS.blocks(),
                                          st)) != hipSuccess)
                return hip_fail(e, "walker order kernel");
        }
        auto& S = p->ph[PH_SCREEN];
        if (S.blocks()) {
            ProfScope ps("screen", st);
            if ((e = launch_screen_batched(dev_jobs(p, PH_SCREEN), dev_prefix(p, PH_SCREEN), (int)S.jobs.size(),
                                           S.blocks(), 0, st)) != hipSuccess)
                return hip_fail(e, "screen kernel");
        }
        auto& C = p->ph[PH_CONTRACT];
        if (C.blocks()) {
            ProfScope ps(contract_name(mode), st);
            const int tile = p->tune.contract_tile;
            unsigned* queue = nullptr;
            int grid = C.blocks();
            if (p->tune.persistent) {
                queue = (unsigned*)p->ws;
                grid = std::min(grid, p->n_cu * contract_per_cu(mode, tile));
                if ((e = fill_u32(queue, 0u, 1, st)) != hipSuccess) return hip_fail(e, "item counter clear");
            }
            if ((e = launch_contract_batched(mode, tile, queue, dev_jobs(p, PH_CONTRACT), dev_prefix(p, PH_CONTRACT),
                                             (int)C.jobs.size(), grid, st)) != hipSuccess)
                return hip_fail(e, "contraction kernel");
        }
        for (int v = 0; v <= 4; ++v) {
            auto& G = p->ph[PH_GJ0 + v];
            if (!G.blocks()) continue;
            ProfScope ps("gauss_jordan", st);
            if (v == 4) {
                int nmax = 0;
                for (const Job& j : G.jobs) nmax = std::max(nmax, j.n);
                e = launch_gjb_batched(mode, dev_jobs(p, PH_GJ4), dev_prefix(p, PH_GJ4), (int)G.jobs.size(),
                                       G.blocks(), nmax, st);
            } else {
                e = launch_gj_batched(mode, v, dev_jobs(p, PH_GJ0 + v), dev_prefix(p, PH_GJ0 + v),
                                      (int)G.jobs.size(), G.blocks(), st);
            }
            if (e != hipSuccess) return hip_fail(e, "inversion kernel");
        }
    } else {
        for (const Job& j : p->ph[PH_SORT].jobs) {
            ProfScope ps("walker_order", st);
            if ((e = launch_wsort(j, st)) != hipSuccess) return hip_fail(e, "walker order kernel");
        }
        for (const Job& j : p->ph[PH_SCREEN].jobs) {
            ProfScope ps("screen", st);
            if ((e = launch_screen(j, 0, st)) != hipSuccess) return hip_fail(e, "screen kernel");
        }
        for (const Job& j : p->ph[PH_CONTRACT].jobs) {
            ProfScope ps(contract_name(mode), st);
            if ((e = launch_contract(j, st)) != hipSuccess) return hip_fail(e, "contraction kernel");
        }
        for (int v = 0; v <= 4; ++v)
            for (const Job& j : p->ph[PH_GJ0 + v].jobs) {
                ProfScope ps("gauss_jordan", st);
                if ((e = launch_gj(j, st)) != hipSuccess) return hip_fail(e, "inversion kernel");
            }
    }
    // spins without electrons: log|det| = 0, sign = +1
    for (const Job& j : p->fjobs)
        if (!j.n && j.W && (e = launch_gj(j, st)) != hipSuccess) return hip_fail(e, "empty spin kernel");
    auto& E = p->ph[PH_EPILOGUE];
    if (batched && E.blocks()) {
        ProfScope ps("drift_lap", st);
        if ((e = launch_epilogue_batched(mode, dev_jobs(p, PH_EPILOGUE), dev_prefix(p, PH_EPILOGUE),
                                         (int)E.jobs.size(), E.blocks(), st)) != hipSuccess)
            return hip_fail(e, "epilogue kernel");
    } else if (!batched) {
        for (const Job& j : E.jobs) {
            ProfScope ps("drift_lap", st);
            if ((e = launch_epilogue(j, st)) != hipSuccess) return hip_fail(e, "epilogue kernel");
        }
    }
    auto& EG = p->ph[PH_EPI_G];
    if (batched && EG.blocks()) {
        ProfScope ps("drift_lap_g", st);
        if ((e = launch_epilogue_g_batched(dev_jobs(p, PH_EPI_G), dev_prefix(p, PH_EPI_G), (int)EG.jobs.size(),
                                           EG.blocks(), st)) != hipSuccess)
            return hip_fail(e, "epilogue kernel");
    } else if (!batched) {
        for (const Job& j : EG.jobs) {
            ProfScope ps("drift_lap_g", st);
            if ((e = launch_epilogue_g(j, st)) != hipSuccess) return hip_fail(e, "epilogue kernel");
        }
    }
    // adjoint (the tile lists of the forward's screening are reused)
    auto& DRp = p->ph[PH_DR];
    if (batched && DRp.blocks()) {
        ProfScope ps("dR_drift", st);
        if ((e = launch_dr_drift_batched(dev_jobs(p, PH_DR), dev_prefix(p, PH_DR), (int)DRp.jobs.size(), DRp.blocks(),
                                         st)) != hipSuccess)
            return hip_fail(e, "dR kernel");
    } else if (!batched) {
        for (const Job& j : DRp.jobs) {
            ProfScope ps("dR_drift", st);
            if ((e = launch_dr_drift(j, st)) != hipSuccess) return hip_fail(e, "dR kernel");
        }
    }
    auto& H = p->ph[PH_ADJ_H];
    auto& SG = p->ph[PH_SCREEN_G];
    auto& DA = p->ph[PH_ADJ_DA];
    if (batched) {
        if (H.blocks()) {
            ProfScope ps("adjoint_h", st);
            if ((e = launch_adj_h_batched(mode, dev_jobs(p, PH_ADJ_H), dev_prefix(p, PH_ADJ_H), (int)H.jobs.size(),
                                          H.blocks(), st)) != hipSuccess)
                return hip_fail(e, "adjoint H kernel");
        }
        // the adjoint's walker-group lists: the union of the forward's tile
        // lists (same positions), or a screening of their own for systems
        // with more windows than the union bitmap holds
        // (tiles in a walker order of their own (FP32) cannot give the
        // unions of consecutive walkers: those groups are screened directly)
        bool small = true;
        for (const Job& j : SG.jobs) small = small && j.s.n_win <= UNION_MAXWIN && !j.wperm;
        if (SG.blocks()) {
            ProfScope ps("screen_group", st);
            e = small ? launch_group_union_batched(dev_jobs(p, PH_SCREEN_G), dev_prefix(p, PH_SCREEN_G),
                                                   (int)SG.jobs.size(), SG.blocks(), st)
                      : launch_screen_batched(dev_jobs(p, PH_SCREEN_G), dev_prefix(p, PH_SCREEN_G), (int)SG.jobs.size(),
                                              SG.blocks(), 1, st);
            if (e != hipSuccess) return hip_fail(e, "group screen kernel");
        }
        auto& SL = p->ph[PH_SLOTS_G];
        if (SL.blocks()) {
            ProfScope ps("screen_group", st);
            if ((e = launch_group_slots_batched(dev_jobs(p, PH_SLOTS_G), dev_prefix(p, PH_SLOTS_G), (int)SL.jobs.size(),
                                                SL.blocks(), st)) != hipSuccess)
                return hip_fail(e, "group slot kernel");
        }
        auto& G3 = p->ph[PH_G32];
        if (G3.blocks()) {
            ProfScope ps("g32", st);
            if ((e = launch_g32_batched(dev_jobs(p, PH_G32), dev_prefix(p, PH_G32), (int)G3.jobs.size(), G3.blocks(),
                                        st)) != hipSuccess)
                return hip_fail(e, "G kernel");
        }
        auto& DE = p->ph[PH_ADJ_DAE];
        if (DE.blocks()) {
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_dae_batched(p->tune.contract_tile, dev_jobs(p, PH_ADJ_DAE), dev_prefix(p, PH_ADJ_DAE), (int)DE.jobs.size(),
                                            DE.blocks(), st)) != hipSuccess)
                return hip_fail(e, "adjoint dA kernel");
        }
        auto& GS = p->ph[PH_GSPLIT];
        if (GS.blocks()) {
            ProfScope ps("g_split", st);
            if ((e = launch_gsplit_batched(dev_jobs(p, PH_GSPLIT), dev_prefix(p, PH_GSPLIT), (int)GS.jobs.size(),
                                           GS.blocks(), st)) != hipSuccess)
                return hip_fail(e, "G split kernel");
        }
        if (DA.blocks()) {
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_da_batched(mode, dev_jobs(p, PH_ADJ_DA), dev_prefix(p, PH_ADJ_DA),
                                           (int)DA.jobs.size(), DA.blocks(), st)) != hipSuccess)
                return hip_fail(e, "adjoint dA kernel");
        }
        for (const PhaseList& L : p->da_t) {
            if (!L.blocks()) continue;
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_da_batched(mode, dev_jobs(p, L), dev_prefix(p, L), (int)L.jobs.size(), L.blocks(),
                                           st)) != hipSuccess)
                return hip_fail(e, "adjoint dA kernel");
        }
    } else {
        for (const Job& j : H.jobs) {
            ProfScope ps("adjoint_h", st);
            if ((e = launch_adj_h(j, st)) != hipSuccess) return hip_fail(e, "adjoint H kernel");
        }
        for (const Job& j : SG.jobs) {
            ProfScope ps("screen_group", st);
            e = j.s.n_win <= UNION_MAXWIN && !j.wperm ? launch_group_union(j, st) : launch_screen(j, 1, st);
            if (e != hipSuccess) return hip_fail(e, "group screen kernel");
        }
        for (const Job& j : p->ph[PH_SLOTS_G].jobs) {
            ProfScope ps("screen_group", st);
            if ((e = launch_group_slots(j, st)) != hipSuccess) return hip_fail(e, "group slot kernel");
        }
        for (const Job& j : p->ph[PH_G32].jobs) {
            ProfScope ps("g32", st);
            if ((e = launch_g32(j, st)) != hipSuccess) return hip_fail(e, "G kernel");
        }
        for (const Job& j : p->ph[PH_ADJ_DAE].jobs) {
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_dae(j, st)) != hipSuccess) return hip_fail(e, "adjoint dA kernel");
        }
        for (const Job& j : p->ph[PH_GSPLIT].jobs) {
            ProfScope ps("g_split", st);
            if ((e = launch_gsplit(j, st)) != hipSuccess) return hip_fail(e, "G split kernel");
        }
        for (const Job& j : DA.jobs) {
            ProfScope ps("adjoint_dA", st);
            if ((e = launch_adj_da(j, st)) != hipSuccess) return hip_fail(e, "adjoint dA kernel");
        }
        for (const PhaseList& L : p->da_t)
            for (const Job& j : L.jobs) {
                ProfScope ps("adjoint_dA", st);
                if ((e = launch_adj_da(j, st)) != hipSuccess) return hip_fail(e, "adjoint dA kernel");
            }
    }
    // FP32 dA accumulators -> the caller's FP64 dA
    for (int i = 0, k = 0; i < p->n_sys; ++i) {
        if (!p->has_bwd[i]) continue;
        for (int s = 0; s < 2; ++s, ++k) {
            const Job& j = p->bjobs[k];
            if (j.dApart && j.n) {
                if ((e = launch_reduce_dA(j.dApart, mode == QSL_FP64, (int)((j.W + j.gw - 1) / j.gw),
                                          (int64_t)j.n * j.s.n_basis, p->bwd[i].dA[s], p->bwd[i].accumulate_dA, st)) !=
                    hipSuccess)
                    return hip_fail(e, "dA reduction");
                continue;
            }
            if (!j.dA32 || !j.n) continue;
            if ((e = launch_finalize_dA(j.dA32, p->bwd[i].dA[s], (int64_t)j.n * j.s.n_basis, p->bwd[i].accumulate_dA,
                                        st)) != hipSuccess)
                return hip_fail(e, "dA finalize");
        }
    }
    return QSL_OK;
}

static qsl_status launch_plan(qsl_plan* p, hipStream_t st) {
    hipError_t e;
    for (int i = 0; i < p->n_sys && !p->dirty; ++i)
        if (i >= (int)p->mo_gen.size() || p->mo_gen[i] != p->sys[i]->mo_generation) p->dirty = true;
    if (p->dirty) {
        qsl_status r = prepare(p, st);
        if (r != QSL_OK) return r;
    }
    if (!(p->flags & QSL_PLAN_GRAPH)) return enqueue(p, st);
    if (!p->exec) {
        if (!p->cap_stream && (e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "plan: capture stream");
        if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "plan: begin capture");
        qsl_status r = enqueue(p, p->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->cap_stream, &g);
        if (r != QSL_OK) {
            if (g) hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return hip_fail(e, "plan: end capture");
        p->graph = g;
        if ((e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess) {
            drop_graph(p);
            return hip_fail(e, "plan: graph instantiate");
        }
    }
    if ((e = hipGraphLaunch(p->exec, st)) != hipSuccess) return hip_fail(e, "plan: graph launch");
    return QSL_OK;
}

// ------------------------------------------------------------- autotuner

static std::string tune_key(const qsl_plan* p) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream k;
    k << arch << "|mode" << p->mode;
    for (int i = 0; i < p->n_sys; ++i) {
        const DevSys& d = p->sys[i]->d;
        k << "|" << d.n_up << "x" << d.n_dn << "b" << d.n_basis << "a" << d.n_atoms << "w" << p->W[i]
          << (p->has_bwd[i] ? "fb" : "f");
    }
    return k.str();
}

static bool parse_int(const std::string& line, const char* name, int* out) {
    const std::string pat = std::string("\"") + name + "\":";
    size_t q = line.find(pat);
    if (q == std::string::npos) return false;
    *out = atoi(line.c_str() + q + pat.size());
    return true;
}

// The cache file holds one entry per line:
// {"key": "...", "batched": 1, "adj_group": 64, "gj_bias": 0, "contract_tile": 0,
//  "persistent": 0, "det_dA": 0, "ms": 1.25},  (on one line)
static bool cache_lookup(const char* path, const std::string& key, qsl_tuning* t) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string pat = "{\"key\": \"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(pat) == std::string::npos) continue;
        qsl_tuning r{};
        if (parse_int(line, "batched", &r.batched) && parse_int(line, "adj_group", &r.adj_group) &&
            parse_int(line, "gj_bias", &r.gj_bias)) {
            // fields added later read as 0 when an entry lacks them
            parse_int(line, "contract_tile", &r.contract_tile);
            parse_int(line, "persistent", &r.persistent);
            parse_int(line, "det_dA", &r.det_dA);
            *t = r;
            return true;
        }
    }
    return false;
}

static bool cache_store(const char* path, const std::string& key, const qsl_tuning& t, double ms) {
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        const std::string pat = "{\"key\": \"" + key + "\"";
        while (f && std::getline(f, line))
            if (line.rfind("{\"key\": ", 0) == 0 && line.find(pat) == std::string::npos) {
                if (!line.empty() && line.back() == ',') line.pop_back();
                keep.push_back(line);
            }
    }
    char buf[512];
    snprintf(buf, sizeof buf,
             "{\"key\": \"%s\", \"batched\": %d, \"adj_group\": %d, \"gj_bias\": %d, \"contract_tile\": %d, "
             "\"persistent\": %d, \"det_dA\": %d, \"ms\": %.6f}",
             key.c_str(), t.batched, t.adj_group, t.gj_bias, t.contract_tile, t.persistent, t.det_dA, ms);
    keep.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return false;
        o << "{\"qslater_autotune\": [\n";
        for (size_t i = 0; i < keep.size(); ++i) o << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        o << "]}\n";
        if (!o) return false;
    }
    return rename(tmp.c_str(), path) == 0;
}

// Host copies of the outputs the self-check compares: the first and last
// (up to) 8 walkers of every system, and dA in full.
struct Snapshot {
    std::vector<std::vector<double>> v;  // one vector per compared array
    std::vector<std::vector<int8_t>> sign;
};

static hipError_t copy_rows(std::vector<double>& out, const double* dev, int64_t W, size_t per_walker) {
    if (!dev || W <= 0) return hipSuccess;
    const int64_t k = std::min<int64_t>(W, 8);
    const size_t old = out.size();
    out.resize(old + 2 * k * per_walker);
    hipError_t e = hipMemcpy(out.data() + old, dev, k * per_walker * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    return hipMemcpy(out.data() + old + k * per_walker, dev + (W - k) * per_walker, k * per_walker * sizeof(double),
                     hipMemcpyDeviceToHost);
}

static hipError_t snapshot(const qsl_plan* p, Snapshot& S) {
    S.v.clear();
    S.sign.clear();
    hipError_t e;
    for (int i = 0; i < p->n_sys; ++i) {
        const qsl_fwd_args& f = p->fwd[i];
        const DevSys& d = p->sys[i]->d;
        const int N = d.n_up + d.n_dn;
        std::vector<double> a;
        if ((e = copy_rows(a, f.logdet, f.W, 2)) != hipSuccess) return e;
        S.v.push_back(std::move(a));
        for (int s = 0; s < 2; ++s) {
            std::vector<double> b;
            const size_t n = s ? d.n_dn : d.n_up;
            if ((e = copy_rows(b, f.Dinv[s], f.W, n * n)) != hipSuccess) return e;
            S.v.push_back(std::move(b));
        }
        std::vector<double> c;
        if ((e = copy_rows(c, f.drift, f.W, (size_t)N * 3)) != hipSuccess) return e;
        if ((e = copy_rows(c, f.lap, f.W, (size_t)N)) != hipSuccess) return e;
        S.v.push_back(std::move(c));
        if (f.sign && f.W) {
            std::vector<int8_t> sg((size_t)f.W * 2);
            if ((e = hipMemcpy(sg.data(), f.sign, sg.size(), hipMemcpyDeviceToHost)) != hipSuccess) return e;
            S.sign.push_back(std::move(sg));
        }
        if (!p->has_bwd[i]) continue;
        const qsl_bwd_args& b = p->bwd[i];
        std::vector<double> r;
        if ((e = copy_rows(r, b.dR, b.W, (size_t)N * 3)) != hipSuccess) return e;
        S.v.push_back(std::move(r));
        for (int s = 0; s < 2; ++s) {
            const size_t n = s ? d.n_dn : d.n_up;
            std::vector<double> da(b.dA[s] ? n * d.n_basis : 0);
            if (!da.empty() && (e = hipMemcpy(da.data(), b.dA[s], da.size() * sizeof(double), hipMemcpyDeviceToHost)) !=
                                   hipSuccess)
                return e;
            S.v.push_back(std::move(da));
        }
    }
    return hipSuccess;
}

// Candidate vs default: every compared array within rel * (its largest
// |entry| in the default run); dA arrays (the last two of a system with an
// adjoint) within dA_rel.  Non-finite entries must match exactly.
static bool same_results(const qsl_plan* p, const Snapshot& ref, const Snapshot& got) {
    if (ref.v.size() != got.v.size() || ref.sign != got.sign) return false;
    const double rel = 1e-9, dA_rel = p->mode == QSL_FP64 ? 1e-10 : 1e-4;
    size_t k = 0;
    for (int i = 0; i < p->n_sys; ++i) {
        const size_t per = p->has_bwd[i] ? 7 : 4;
        for (size_t a = 0; a < per; ++a, ++k) {
            const auto& x = ref.v[k];
            const auto& y = got.v[k];
            if (x.size() != y.size()) return false;
            const bool is_dA = p->has_bwd[i] && a >= 5;
            double m = 0.0;
            for (double t : x)
                if (isfinite(t)) m = std::max(m, fabs(t));
            const double tol = (is_dA ? dA_rel : rel) * m;
            for (size_t q = 0; q < x.size(); ++q) {
                if (!isfinite(x[q]) || !isfinite(y[q])) {
                    if (!(isnan(x[q]) && isnan(y[q])) && x[q] != y[q]) return false;
                    continue;
                }
                if (fabs(x[q] - y[q]) > tol) return false;
            }
        }
    }
    return true;
}

static qsl_status time_plan(qsl_plan* p, hipStream_t st, int reps, double* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    qsl_status r = QSL_OK;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) hipEventDestroy(a);
        return hip_fail(e, "autotune: event create");
    }
    if ((r = launch_plan(p, st)) == QSL_OK) {  // warm-up (and capture)
        hipEventRecord(a, st);
        for (int k = 0; k < reps && r == QSL_OK; ++k) r = launch_plan(p, st);
        hipEventRecord(b, st);
        if (r == QSL_OK && (e = hipEventSynchronize(b)) != hipSuccess) r = hip_fail(e, "autotune: event sync");
        float t = 0.0f;
        if (r == QSL_OK && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess) r = hip_fail(e, "autotune: elapsed");
        *ms = (double)t / reps;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return r;
}

static qsl_status autotune_run(qsl_plan* p, hipStream_t st, const std::string& key, const char* cache_path,
                               const qsl_tuning saved, qsl_tuning* chosen);

qsl_system* plan_system(qsl_plan* p, int i) { return p && i >= 0 && i < p->n_sys ? p->sys[i] : nullptr; }
const qsl_fwd_args* plan_fwd(const qsl_plan* p, int i) {
    return p && i >= 0 && i < p->n_sys && p->bound[i] ? &p->fwd[i] : nullptr;
}
int64_t plan_walkers(const qsl_plan* p, int i) { return p && i >= 0 && i < p->n_sys ? p->W[i] : -1; }

}  // namespace qsl

extern "C" {

qsl_status qsl_plan_create(int32_t n_sys, qsl_system* const* sys, const int64_t* W, int32_t mode, uint32_t flags,
                           qsl_plan** out) {
    if (!out || !sys || !W || n_sys < 1) return bad(QSL_ERR_INVALID_ARG, "plan: NULL argument or n_sys < 1");
    *out = nullptr;
    if (mode < QSL_FP64 || mode > QSL_BF16X3) return bad(QSL_ERR_INVALID_ARG, "plan: bad mode");
    if (flags & ~QSL_PLAN_GRAPH) return bad(QSL_ERR_INVALID_ARG, "plan: unknown flags");
    for (int i = 0; i < n_sys; ++i) {
        if (!sys[i]) return bad(QSL_ERR_INVALID_ARG, "plan: NULL system");
        if (W[i] < 0) return bad(QSL_ERR_INVALID_ARG, "plan: W < 0");
        for (int s = 0; s < 2; ++s)
            if (n_spin(sys[i]->d, s) > GJ_NMAX)
                return bad(QSL_ERR_UNSUPPORTED, "plan: more electrons of one spin than the inversion supports");
    }
    qsl_plan* p = new (std::nothrow) qsl_plan();
    if (!p) return bad(QSL_ERR_OOM, "plan: host allocation");
    p->n_sys = n_sys;
    p->mode = mode;
    p->flags = flags;
    hipGetDevice(&p->device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && ncu > 0)
        p->n_cu = ncu;
    p->sys.assign(sys, sys + n_sys);
    p->W.assign(W, W + n_sys);
    p->fwd.assign(n_sys, qsl_fwd_args{});
    p->bwd.assign(n_sys, qsl_bwd_args{});
    p->bound.assign(n_sys, 0);
    p->has_bwd.assign(n_sys, 0);
    *out = p;
    return QSL_OK;
}

qsl_status qsl_plan_bind(qsl_plan* p, int32_t i, const qsl_fwd_args* f, const qsl_bwd_args* b) {
    if (!p || !f) return bad(QSL_ERR_INVALID_ARG, "plan bind: NULL argument");
    if (i < 0 || i >= p->n_sys) return bad(QSL_ERR_INVALID_ARG, "plan bind: system index out of range");
    if (f->W != p->W[i] || f->mode != p->mode) return bad(QSL_ERR_SHAPE, "plan bind: forward W or mode differ");
    const DevSys& d = p->sys[i]->d;
    if (f->W && !f->R) return bad(QSL_ERR_INVALID_ARG, "plan bind: NULL R");
    for (int s = 0; s < 2; ++s) {
        if (!n_spin(d, s) || !f->W) continue;
        if (!p->sys[i]->mo[s].set) return bad(QSL_ERR_INVALID_ARG, "plan bind: MO coefficients of a spin never set");
        if (p->sys[i]->mo[s].n != n_spin(d, s))
            return bad(QSL_ERR_SHAPE, "plan bind: the MO set of a spin has more rows than electrons");
        if (!f->C[s] || !f->Dinv[s]) return bad(QSL_ERR_INVALID_ARG, "plan bind: C and Dinv outputs are required");
    }
    if (b) {
        if (b->W != p->W[i] || b->mode != p->mode) return bad(QSL_ERR_SHAPE, "plan bind: adjoint W or mode differ");
        if (b->R != f->R) return bad(QSL_ERR_INVALID_ARG, "plan bind: the adjoint must use the forward's R");
        if (b->W && !b->g_logdet) return bad(QSL_ERR_INVALID_ARG, "plan bind: NULL g_logdet");
        for (int s = 0; s < 2; ++s)
            if (n_spin(d, s) && b->W && !b->Dinv[s]) return bad(QSL_ERR_INVALID_ARG, "plan bind: NULL Dinv");
    }
    p->fwd[i] = *f;
    p->fwd[i].ws = nullptr;
    p->fwd[i].ws_bytes = 0;
    p->has_bwd[i] = b ? 1 : 0;
    if (b) {
        p->bwd[i] = *b;
        p->bwd[i].ws = nullptr;
        p->bwd[i].ws_bytes = 0;
        // the adjoint runs after the forward: its drift gives dR
        if (!p->bwd[i].drift) p->bwd[i].drift = f->drift;
    }
    p->bound[i] = 1;
    p->dirty = true;
    return QSL_OK;
}

qsl_status qsl_plan_set_tuning(qsl_plan* p, const qsl_tuning* t) {
    if (!p || !t) return bad(QSL_ERR_INVALID_ARG, "plan tuning: NULL argument");
    auto flag = [](int32_t v) { return v == 0 || v == 1; };
    if (!flag(t->batched) || t->adj_group < 0 || t->adj_group > 4096 || !flag(t->gj_bias) || t->contract_tile < 0 ||
        t->contract_tile > 2 ||
        !flag(t->persistent) || !flag(t->det_dA))
        return bad(QSL_ERR_INVALID_ARG, "plan tuning: value out of range");
    p->tune = *t;
    p->dirty = true;
    return QSL_OK;
}

qsl_status qsl_plan_get_tuning(const qsl_plan* p, qsl_tuning* t) {
    if (!p || !t) return bad(QSL_ERR_INVALID_ARG, "plan tuning: NULL argument");
    *t = p->tune;
    return QSL_OK;
}

qsl_status qsl_plan_launch(qsl_plan* p, void* stream) {
    if (!p) return bad(QSL_ERR_INVALID_ARG, "plan launch: NULL plan");
    return launch_plan(p, (hipStream_t)stream);
}

qsl_status qsl_plan_destroy(qsl_plan* p) {
    if (!p) return QSL_OK;
    if (p->cap_stream) hipStreamSynchronize(p->cap_stream);
    drop_graph(p);
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    if (p->ws) hipFree(p->ws);
    if (p->lists) hipFree(p->lists);
    delete p;
    return QSL_OK;
}

qsl_status qsl_autotune(qsl_plan* p, const char* cache_path, void* stream, qsl_tuning* chosen) {
    if (!p) return bad(QSL_ERR_INVALID_ARG, "autotune: NULL plan");
    for (int i = 0; i < p->n_sys; ++i)
        if (!p->bound[i]) return bad(QSL_ERR_INVALID_ARG, "autotune: a system was never bound");
    hipStream_t st = (hipStream_t)stream;
    const std::string key = tune_key(p);
    qsl_tuning t{};
    if (cache_path && cache_lookup(cache_path, key, &t)) {
        qsl_status r = qsl_plan_set_tuning(p, &t);
        if (r == QSL_OK && chosen) *chosen = t;
        return r;
    }
    const qsl_tuning saved = p->tune;
    // Every tuning run overwrites dA (the reference and each candidate must
    // produce the same dA, not add to it); the caller's accumulate flags come
    // back on every return path, and the graph is captured anew.
    std::vector<int32_t> acc(p->n_sys, 0);
    for (int i = 0; i < p->n_sys; ++i) {
        acc[i] = p->bwd[i].accumulate_dA;
        p->bwd[i].accumulate_dA = 0;
    }
    auto restore = [&](qsl_status r) {
        for (int i = 0; i < p->n_sys; ++i) p->bwd[i].accumulate_dA = acc[i];
        if (r != QSL_OK) p->tune = saved;
        p->dirty = true;
        return r;
    };
    return restore(autotune_run(p, st, key, cache_path, saved, chosen));
}

}  // extern "C"

namespace qsl {

static qsl_status autotune_run(qsl_plan* p, hipStream_t st, const std::string& key, const char* cache_path,
                               const qsl_tuning saved, qsl_tuning* chosen) {
    hipError_t e;
    // the reference of the self-check is the default tuning with the
    // candidate's FP32 contraction tile (the tiles round differently: FP32
    // or split-bf16 products), run once per tile; every candidate keeps the
    // caller's choice of the deterministic dA
    const qsl_tuning base{1, 0, 0, F32_TILE_DEFAULT, 0, saved.det_dA};
    Snapshot refs[3], got;
    bool have_ref[3] = {false, false, false};
    auto reference = [&](int tile) -> qsl_status {
        if (have_ref[tile]) return QSL_OK;
        p->tune = base;
        p->tune.contract_tile = tile;
        p->dirty = true;
        qsl_status q = launch_plan(p, st);
        if (q != QSL_OK) return q;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "autotune: sync");
        if ((e = snapshot(p, refs[tile])) != hipSuccess) return hip_fail(e, "autotune: copy");
        have_ref[tile] = true;
        return QSL_OK;
    };
    qsl_status r = reference(base.contract_tile);
    if (r != QSL_OK) return r;
    int64_t wmax = 1;
    int nmax = 0;
    for (int i = 0; i < p->n_sys; ++i) {
        wmax = std::max(wmax, p->W[i]);
        nmax = std::max(nmax, std::max(p->sys[i]->d.n_up, p->sys[i]->d.n_dn));
    }
    bool any_bwd = false;
    for (char h : p->has_bwd) any_bwd |= h != 0;
    std::vector<qsl_tuning> cands;
    for (int bt = 1; bt >= 0; --bt)
        for (int gb = 0; gb <= 1; ++gb) {
            if (gb && gj_variant(nmax) >= 3) continue;  // no larger block shape
            const int groups[] = {0, 16, 32, 64, 128, 256, 512, 1024};
            for (int g : groups) {
                if (!any_bwd && g) continue;
                if (g > 16 && g >= 2 * wmax) continue;  // the same as a smaller group for every system
                cands.push_back(qsl_tuning{bt, g, gb, base.contract_tile, 0, saved.det_dA});
            }
        }
    double best_ms = 1e300;
    qsl_tuning best = base;
    bool found = false;
    auto trial = [&](const qsl_tuning& c) -> qsl_status {
        qsl_status q0 = reference(c.contract_tile);
        if (q0 != QSL_OK) return q0;
        p->tune = c;
        p->dirty = true;
        double ms = 0.0;
        qsl_status q = time_plan(p, st, 3, &ms);
        if (q != QSL_OK) return q;
        if ((e = snapshot(p, got)) != hipSuccess) return hip_fail(e, "autotune: copy");
        if (!same_results(p, refs[c.contract_tile], got)) return QSL_OK;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
            found = true;
        }
        return QSL_OK;
    };
    // coordinate descent: the launch and group shapes first, then the
    // contraction's tile and persistent launch around the best of those
    for (const qsl_tuning& c : cands)
        if ((r = trial(c)) != QSL_OK) return r;
    if (found) {
        const qsl_tuning b0 = best;
        const int tiles = p->mode == QSL_FP32 ? 2 : 0;  // the tile is an FP32 choice
        for (int tile = 0; tile <= tiles; ++tile)
            for (int pers = 0; pers <= (b0.batched ? 1 : 0); ++pers) {
                if (tiles && tile == b0.contract_tile && pers == b0.persistent) continue;  // b0 itself
                if (!tiles && !pers) continue;
                qsl_tuning c = b0;
                c.contract_tile = tiles ? tile : b0.contract_tile;
                c.persistent = pers;
                if ((r = trial(c)) != QSL_OK) return r;
            }
    }
    if (!found) {
        p->tune = saved;
        p->dirty = true;
        return bad(QSL_ERR_UNSUPPORTED, "autotune: no candidate passed the self-check");
    }
    p->tune = best;
    p->dirty = true;
    if (cache_path && !cache_store(cache_path, key, best, best_ms))
        return bad(QSL_ERR_INVALID_ARG, std::string("autotune: cannot write ") + cache_path);
    if (chosen) *chosen = best;
    return QSL_OK;
}

}  // namespace qsl
