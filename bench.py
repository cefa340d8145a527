#!/usr/bin/env python3
"""Benchmark: walker Slater-builds per second, forward + adjoint, on one GPU.

A step is one pass of the whole hot path over one batch of walkers:
screening, fused AO evaluation + AO->MO products (FP32 products, as the
paper computes them in single precision: each FP32 operand split exactly
into three bf16 and the six leading products taken on bf16 MFMA with FP32
accumulation, as accurate as FP32 MFMA and faster; the FP32-MFMA tiles are
timed among the launch forms), FP64
Gauss-Jordan log|det| / sign / inverse, drift and Laplacian, then the
adjoint (AO recomputation, dR and dA).  The headline workload is the
synthetic 434-electron peptide-shaped system (134 atoms, 1270 AOs, 217 x
1270 MO coefficients per spin) with 4096 walkers; the step is one replay of
the plan's HIP graph, inputs resident in HBM.

Beside it (in "also"), each with its own roofline and, for the reduced
precisions, the error of every output against the FP64 run on the same
walkers: the same system with split-BF16 products and in plain FP64; the
1731-electron system (531 atoms, 5055 AOs, 866/865 MOs, 512 walkers) in FP32
and FP64; and the uneven batch of 512 walkers each of the 44-, 158- and
434-electron systems in one autotuned FP32 plan.  Per-kernel times come from
a second, eager pass of the same steps with HIP events around every launch
on the launch stream.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker Slater-builds/sec fwd+adjoint at 434e/1731e; mixed-prec vs FP64 at stated err"
PEAK = {"bf16x3": ("mfma", 2500.0), "fp32": ("mfma", 157.3), "fp64": ("mfma", 78.6)}
PEAK_FP64 = 78.6
HBM_PEAK = 8000.0  # GB/s
DTYPE = {"bf16x3": "bf16x3+f32acc/f64", "fp32": "f32/f64", "fp64": "f64"}
# FP32 mode with the split-bf16 products (contraction tile 2, the default):
# each FP32 operand as three bf16, six bf16 MFMA products, FP32 accumulation
DTYPE_F32_SPLIT = "bf16x6+f32acc/f64"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def survivors_per_electron(sysm, R, max_walkers=64):
    """Mean surviving AOs per electron (the cost model of the flop counts):
    a shell survives when its smallest exponent times r^2 is <= T."""
    Rs = R[:max_walkers].reshape(-1, 3)
    off = np.concatenate([[0], np.cumsum(sysm.shell_nprim)])
    gmin = np.array([sysm.prim_exp[off[s]:off[s + 1]].min() for s in range(sysm.n_shells)])
    nao = (sysm.shell_l + 1) * (sysm.shell_l + 2) // 2
    Q = sysm.atom_xyz[sysm.shell_atom]
    tot = 0
    for c0 in range(0, Rs.shape[0], 4096):
        d = Rs[c0:c0 + 4096, None, :] - Q[None]
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        tot += int(((gmin[None] * r2 <= sysm.screen_T) * nao[None]).sum())
    return tot / Rs.shape[0]


def work_per_step(sysm, nnz, W, mode, tile=2):
    """Algorithmic work of one step per kernel kind: (amount, bound, peak, unit).
    The FP32 contraction on split-bf16 products (tile 2) is priced against
    the bf16 MFMA peak, the dtype its MFMAs run in."""
    ns = [sysm.n_up, sysm.n_dn]
    contract = sum(10.0 * n * n * nnz * W for n in ns)   # 5 products x 2 flops x MOs x survivors
    gj = sum(2.0 * n ** 3 * W for n in ns)                 # 2 n^3 per matrix
    adjoint = sum(2.0 * n * n * nnz * W for n in ns)       # H or dA: 2 flops per (electron, survivor, MO)
    cb = 8 if mode == "fp64" else 4
    epi = sum((8.0 * n * n + 4 * cb * n * n + 32.0 * n) * W for n in ns)  # Dinv + 4 C blocks read, drift/lap

    def gsplit_bytes(D_read):
        return sum(((8.0 * n * n if D_read else 0.0) + 4.0 * -(-n // 32) * 32 * -(-n // 224) * 224) * W for n in ns)
    # FP32 dA by electron: G = g D^-1 in FP32, rows of whole 224-MO blocks,
    # written by the drift / Laplacian epilogue (D^-1 read once for both)
    g32 = sum(4.0 * n * -(-n // 224) * 224 * W for n in ns) if mode == "fp32" else 0.0
    cpeak = PEAK["bf16x3"] if mode == "fp32" and tile == 2 else PEAK[mode]
    return {
        f"contract_{mode}": (contract, cpeak[0], cpeak[1], "TFLOP/s"),
        # n <= 224: register-resident elimination on FP64 vector FMAs; larger
        # n: blocked, with the rank-32 updates on FP64 MFMA
        "gauss_jordan": (gj, "mfma" if max(ns) > 224 else "alu", PEAK_FP64, "TFLOP/s"),
        "adjoint_h": (adjoint, PEAK[mode][0], PEAK[mode][1], "TFLOP/s"),
        # the FP32 dA by electron follows the contraction's tile
        "adjoint_dA": (adjoint, cpeak[0], cpeak[1], "TFLOP/s"),
        "drift_lap": (epi + g32, "hbm", HBM_PEAK, "GB/s"),
        "g32": (sum(8.0 * n * n * W for n in ns) + g32, "hbm", HBM_PEAK, "GB/s"),
        # dR = g drift: drift read, dR written, g read per component
        "dR_drift": (sum(56.0 * n * W for n in ns), "hbm", HBM_PEAK, "GB/s"),
        # split-BF16 G^T: D^-1 read, hi + lo written over the padded tiles
        "g_split": (gsplit_bytes(D_read=True), "hbm", HBM_PEAK, "GB/s"),
        # drift / Laplacian that also writes the split G^T (D^-1 read once)
        "drift_lap_g": (epi + gsplit_bytes(D_read=False), "hbm", HBM_PEAK, "GB/s"),
    }


class Workload:
    """Systems (config name, W) in one mode: a graph plan and an eager plan
    bound to the same device buffers (forward + adjoint of every system)."""

    def __init__(self, config, W, mode, more=(), autotune=False):
        import torch
        import qsl_synth as q
        from paper_1209_6630_amd.api import Plan, System
        self.config, self.W, self.mode = config, W, mode
        self.items = []
        dev = "cuda"
        for name, Wx in [(config, W), *more]:
            sysm, A_up, A_dn, R_np = q.make_config(name, W=Wx)
            S = System.from_synth(sysm)
            S.set_mo(0, A_up)
            S.set_mo(1, A_dn)
            it = dict(name=name, W=Wx, sysm=sysm, R_np=R_np, S=S, R=torch.from_numpy(R_np).to(dev),
                      out=S.alloc_outputs(Wx, mode),
                      g=torch.ones((Wx, 2), dtype=torch.float64, device=dev),
                      dR=torch.empty((Wx, S.n_elec, 3), dtype=torch.float64, device=dev),
                      dA=(torch.empty((S.n_up, S.n_basis), dtype=torch.float64, device=dev),
                          torch.empty((S.n_dn, S.n_basis), dtype=torch.float64, device=dev)))
            self.items.append(it)
        first = self.items[0]
        self.sysm, self.R_np, self.S = first["sysm"], first["R_np"], first["S"]
        self.out, self.dR, self.dA = first["out"], first["dR"], first["dA"]
        self.plans = {}
        self.tuning = None
        for graph in (True, False):
            P = Plan([it["S"] for it in self.items], [it["W"] for it in self.items], mode, graph=graph)
            for i, it in enumerate(self.items):
                P.bind(i, it["R"], it["out"], g=it["g"], dR=it["dR"], dA=it["dA"])
            if autotune:
                if self.tuning is None:
                    self.tuning = P.autotune(None)
                else:
                    P.tuning = self.tuning
            self.plans[graph] = P
        torch.cuda.synchronize()

    def work(self):
        """Algorithmic work per step of every kernel kind, summed over the
        systems of the plan."""
        total = {}
        for it in self.items:
            nnz = survivors_per_electron(it["sysm"], it["R_np"])
            it["nnz"] = nnz
            for k, (amt, bound, peak, unit) in work_per_step(it["sysm"], nnz, it["W"], self.mode,
                                                             self.tile()).items():
                if k in total:
                    total[k] = (total[k][0] + amt,) + total[k][1:]
                else:
                    total[k] = (amt, bound, peak, unit)
        return total

    def tile(self):
        """The FP32 contraction tile of the timed plan."""
        return self.plans[True].tuning["contract_tile"]

    def dtype(self):
        return DTYPE_F32_SPLIT if self.mode == "fp32" and self.tile() == 2 else DTYPE[self.mode]

    def time(self, steps, warmup):
        """K graph replays bracketed by synchronisations -> ms per step;
        then K eager launches with kernel timing -> per-kernel totals."""
        import torch
        from paper_1209_6630_amd import _lib
        Pg, Pe = self.plans[True], self.plans[False]
        for _ in range(warmup):
            Pg.launch()
        Pe.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            Pg.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        _lib.profile_enable(True)
        _lib.profile_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            Pe.launch()
        torch.cuda.synchronize()
        ms_eager = (time.perf_counter() - t0) * 1e3 / steps
        prof = _lib.profile_read(reset=True)
        _lib.profile_enable(False)
        return ms, ms_eager, prof

    def time_tunings(self, variants, steps):
        """Graph replays of the plan under each variant of its tuning (a dict
        of changed fields) -> ms per step; the tuning is restored after."""
        import torch
        P = self.plans[True]
        base = P.tuning
        out = {}
        for name, delta in variants.items():
            P.tuning = {**base, **delta}
            P.launch()  # re-plans and captures (untimed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                P.launch()
            torch.cuda.synchronize()
            out[name] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
        P.tuning = base
        P.launch()
        torch.cuda.synchronize()
        return out

    def close(self):
        for P in self.plans.values():
            P.close()
        self.plans = {}
        for it in self.items:
            it["S"].close()
        self.items = []
        self.out = self.dR = self.dA = self.S = None


def kernel_table(prof, steps, kinds):
    kernels = {}
    for name, (launches, tot) in prof.items():
        e = {"launches": launches, "avg_ms": tot / max(launches, 1), "ms_per_step": tot / steps}
        if name in kinds:
            work, bound, peak, unit = kinds[name]
            achieved = work / (tot / steps * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
            e.update(bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak)
        kernels[name] = e
    return kernels


def err_vs_fp64(mixed, ref):
    """Mixed precision against the FP64 run on the same walkers (g = 1 for
    every walker), each as median / p99 / max over walkers (and spins):
      logdet   |d logdet|;
      C_n      normwise relative difference of each of the five products
               (values, three gradient components, Laplacian) per walker and
               spin, ||dC_n||_F / ||C_n||_F over the [e][i] block;
      Dinv     normwise relative difference per walker and spin;
      drift, lap, dR   per walker, max over electrons of |d x| / max(1, |x|);
      dA       normwise relative difference per spin (one value each).
    Ill-conditioned walkers amplify the product error by the condition
    number of D, hence the long tails of log|det|, D^-1 and what follows from
    D^-1.  mixed / ref: dicts of the forward outputs plus dR, dA_up, dA_dn."""
    import torch

    def q3(x):
        x = x[torch.isfinite(x)].double()
        if x.numel() == 0:
            return [0.0, 0.0, 0.0]
        return [float(torch.quantile(x, 0.5)), float(torch.quantile(x, 0.99)), float(x.max())]

    def blockwise(a, b, dims):
        r = []
        for c0 in range(0, b.shape[0], 128):
            x, y = a[c0:c0 + 128].double(), b[c0:c0 + 128].double()
            r.append(torch.linalg.vector_norm(x - y, dim=dims) / torch.linalg.vector_norm(y, dim=dims))
        return torch.cat(r)

    ok = torch.isfinite(ref["logdet"]) & torch.isfinite(mixed["logdet"])
    res = {"logdet_abs": q3((mixed["logdet"] - ref["logdet"]).abs()[ok])}
    for n, name in enumerate(("C_value", "C_dx", "C_dy", "C_dz", "C_lap")):
        vals = [blockwise(mixed[k][:, n], ref[k][:, n], (1, 2)) for k in ("C_up", "C_dn") if ref[k].numel()]
        res[name + "_normwise_rel"] = q3(torch.cat(vals))
    vals = [blockwise(mixed[k], ref[k], (1, 2)) for k in ("Dinv_up", "Dinv_dn") if ref[k].numel()]
    res["Dinv_normwise_rel"] = q3(torch.cat(vals))
    for k, dims in (("drift", (1, 2)), ("lap", (1,)), ("dR", (1, 2))):
        if k not in mixed or k not in ref:
            continue
        d = (mixed[k] - ref[k]).abs() / torch.clamp(ref[k].abs(), min=1.0)
        res[k + "_rel"] = q3(torch.amax(d, dim=dims))
    if "dA_up" in mixed:
        res["dA_normwise_rel"] = [float(torch.linalg.vector_norm(mixed[k] - ref[k]) / torch.linalg.vector_norm(ref[k]))
                                  for k in ("dA_up", "dA_dn") if ref[k].numel()]
    res["sign_mismatch"] = int((mixed["sign"] != ref["sign"]).sum())
    return res


def cpu_baseline(sysm, A_up, A_dn, R, workload, target_s=12.0, target_1core_s=6.0):
    """The FP64 oracle, forward + adjoint, on a bounded sample of walkers:
    on every host thread (OpenMP over walkers), and on one thread (the
    per-core figure the paper's tables give)."""
    import oracle
    oracle.load()
    nthr = oracle.max_threads()
    W = R.shape[0]

    def run(ws, threads):
        t0 = time.perf_counter()
        out = oracle.forward(sysm, A_up, A_dn, R[:ws], nthreads=threads)
        g = np.ones((ws, 2))
        oracle.backward(sysm, A_up, A_dn, R[:ws], out["Dinv_up"], out["Dinv_dn"], g, nthreads=threads)
        return time.perf_counter() - t0

    cal = max(1, min(W, nthr))
    t = run(cal, nthr)
    n = int(min(W, max(cal, round(cal * target_s / max(t, 1e-3)))))
    n = max(cal, (n // cal) * cal)
    log(f"cpu baseline: calibration {cal} walkers {t:.2f}s -> sample {n} walkers")
    t = run(n, nthr)
    # one thread: as many walkers as take about target_1core_s at the rate
    # just measured divided by the thread count
    n1 = int(max(1, min(W, round(target_1core_s * n / t / nthr))))
    t1 = run(n1, 1)
    return {"value": n / t, "unit": "walker Slater-builds/s", "cores": nthr, "kind": "oracle",
            "sample": f"{n} of the {W} walkers of the {workload} workload, FP64 forward + adjoint, "
                      f"OpenMP over walkers on {nthr} threads, {t:.1f} s",
            "one_core": {"value": n1 / t1, "unit": "walker Slater-builds/s", "cores": 1,
                         "sample": f"{n1} walkers of the same workload on one thread, {t1:.1f} s"}}


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "traffic_434e_W4096_fp32.md")
KERNEL_SOURCES = {
    "contract": ["qsl_contract.hip", "qsl_internal.h"],
    "gauss_jordan": ["qsl_gj.hip", "qsl_internal.h"],
    "adjoint_dA": ["qsl_backward.hip", "qsl_internal.h"],
    "drift_lap": ["qsl_misc.hip", "qsl_internal.h"],
}


def sources_digest(kind):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1209_6630_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (its `traffic-json:` line), scaled by the
    copy-kernel calibration there; None when there is no entry for this
    workload and kernel, or the kernel's sources changed since."""
    kind = "contract" if kernel.startswith("contract_") else kernel
    if kind not in KERNEL_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic-json:"):
            doc = json.loads(line.split(":", 1)[1])
            e = doc.get("kernels", {}).get(kernel)
            if doc.get("workload") == workload and e and e.get("sources_sha256") == sources_digest(kind):
                return e["hbm_bytes_per_launch"]
    return None


def dmc_line(config, W, mode, steps, warmup=2, tau=1e-4):
    """Time per fixed-node DMC step of the whole population (the analogue of
    the paper's time per QMC step): drift-diffusion move, the Slater build
    by a forward-only plan replayed from its HIP graph, Jastrow factor, local
    energy and drift, branching weights, reconfiguration and gather.  The
    random deviates of every step are drawn beforehand and resident on the
    GPU.  tau is small enough that the synthetic trial function's drifts
    (up to a few thousand bohr^-1 near its nodes) move an electron by less
    than a bohr, so the population stays spread over its walkers."""
    import torch
    import qsl_synth as q
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import DMC, System
    sysm, A_up, A_dn, R = q.make_config(config, W=W)
    S = System.from_synth(sysm)
    S.set_mo(0, A_up)
    S.set_mo(1, A_dn)
    S.set_jastrow(q.nuclear_charges(sysm))
    N = sysm.n_elec
    dmc = DMC(S, torch.from_numpy(R).cuda(), mode=mode, tau=tau, E_T=0.0, graph=True)
    EL0 = dmc.EL.cpu().numpy()
    dmc.E_T = float(EL0[np.isfinite(EL0)].mean())
    rnd = [q.dmc_randoms(W, N, seed=5, step=k) for k in range(warmup + steps)]
    eta = [torch.from_numpy(e).cuda() for e, _ in rnd]
    u = [torch.from_numpy(x).cuda() for _, x in rnd]
    for k in range(warmup):
        dmc.step(eta[k], u[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        dmc.step(eta[k], u[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    _lib.profile_enable(True)
    _lib.profile_read(reset=True)
    for k in range(warmup, warmup + steps):
        dmc.step(eta[k], u[k])
    torch.cuda.synchronize()
    prof = _lib.profile_read(reset=True)
    _lib.profile_enable(False)
    EL = dmc.EL.cpu().numpy()
    parents = int(np.unique(dmc.idx.cpu().numpy()).size)
    dmc.close()
    S.close()
    fin = np.isfinite(EL)
    return {"workload": f"dmc-step-{config}-W{W}-{mode}", "value": W / (ms * 1e-3), "unit": "walker DMC steps/s",
            "ms_per_step": ms, "steps": steps, "dtype": DTYPE_F32_SPLIT if mode == "fp32" else DTYPE[mode],
            "tau": tau, "E_T": dmc.E_T, "mean_local_energy": float(EL[fin].mean()) if fin.any() else None,
            "finite_local_energies": int(fin.sum()), "distinct_parents_last_step": parents,
            "timed": "DMC steps (plan graph replay inside), deviates resident on the GPU",
            "kernels_ms_per_step": {k: round(v[1] / steps, 3) for k, v in prof.items()},
            "context": "paper Table 3: 0.0119 s per walker step on one Sandy Bridge core for its 434-electron "
                       "beta-strand (other basis and molecule)"}


def sparse_a_line(config, W, radii, steps=3):
    """The paper's dense-versus-sparse A question on MFMA: FP32 contraction
    time of the same walkers with dense MO coefficients and with localised
    ones (zero beyond a radius of each MO's centre, block-sparse along the
    chain) whose all-zero 32-MO blocks the products skip; forward-only plan,
    eager launches with kernel timing."""
    import torch
    import qsl_synth as q
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import Plan, System
    sysm, A_up, A_dn, R_np = q.make_config(config, W=W)
    S = System.from_synth(sysm)
    R = torch.from_numpy(R_np).cuda()
    out = S.alloc_outputs(W, "fp32")
    rows = []
    for rad in [None] + list(radii):
        au, ad = (A_up, A_dn) if rad is None else q.localize_mos(sysm, A_up, A_dn, rad)
        S.set_mo(0, au)
        S.set_mo(1, ad)
        P = Plan([S], [W], "fp32", graph=False)
        P.bind(0, R, out)
        P.launch()
        torch.cuda.synchronize()
        _lib.profile_enable(True)
        _lib.profile_read(reset=True)
        for _ in range(steps):
            P.launch()
        torch.cuda.synchronize()
        prof = _lib.profile_read(reset=True)
        _lib.profile_enable(False)
        P.close()
        n = sysm.n_up
        blk = np.mean([(au[b:b + 32] != 0).any(0) for b in range(0, n, 32)])
        rows.append({"radius_bohr": rad, "element_density": float((au != 0).mean()),
                     "block_density_32mo": float(blk),
                     "contract_fp32_ms": prof["contract_fp32"][1] / steps,
                     "gauss_jordan_ms": prof["gauss_jordan"][1] / steps})
    S.close()
    return {"workload": f"sparse-A-{config}-W{W}-fp32-forward", "rows": rows,
            "note": "radius None: dense A; the products skip MFMA groups whose 32-MO block has no non-zero "
                    "coefficient on the group's eight slots"}


def roofline_of(kernels, kinds, workload):
    """The dominant kernel's roofline entry (algorithmic work over its
    average launch time, against its peak)."""
    dom = max((k for k in kernels if k in kinds), key=lambda k: kernels[k]["ms_per_step"])
    d = kernels[dom]
    r = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
         "frac": d["frac"], "traffic": measured_traffic(workload, dom)}
    if dom == "contract_fp32" and d["peak"] == PEAK["bf16x3"][1]:
        # FP32 products run as six bf16 MFMA products: the same algorithmic
        # rate against the FP32 MFMA peak, for comparison with the FP32 tiles
        r.update(mfma_dtype="bf16 (FP32 operands split into three bf16, six products per FP32 product)",
                 fp32_equivalent_frac=d["achieved"] / PEAK["fp32"][1])
    return r


def outputs_of(wl):
    """Forward outputs, dR and dA of the first system of a workload."""
    r = dict(wl.out)
    r.update(dR=wl.dR, dA_up=wl.dA[0], dA_dn=wl.dA[1])
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="fp32", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--config", default="434e")
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true", help="skip the companion runs")
    ap.add_argument("--no-forms", action="store_true", help="skip timing the other launch forms of the tuning")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after timing, run one plain copy kernel over MIB MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the walker batch of one "
              "GPU is the unit of work; the design notes describe how walkers shard across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import qsl_synth as q
    torch.cuda.set_device(0)

    cfg = q.CONFIGS[args.config]
    W = args.walkers or cfg["W"]
    mode = args.mode
    wname = f"{args.config}-W{W}-{mode}-fwd+adjoint"
    log(f"workload {args.config} W={W} mode={mode}: generating inputs")
    main_wl = Workload(args.config, W, mode)
    log(f"timing {args.steps} graph replays after {args.warmup} warm-up")
    ms, ms_eager, prof = main_wl.time(args.steps, args.warmup)
    value = W / (ms * 1e-3)
    log(f"{ms:.3f} ms/step (eager {ms_eager:.3f}), {value:.1f} walkers/s; kernels {prof}")
    forms = {f"tile{t}-{'persistent' if p_ else 'per-item'}": dict(contract_tile=t, persistent=p_)
             for t in (0, 1, 2) for p_ in (0, 1)}
    forms["det_dA"] = dict(det_dA=1)
    by_form = None
    if not args.no_forms:
        log("launch forms")
        by_form = main_wl.time_tunings(forms, max(3, args.steps // 2))
        log(f"launch forms: {by_form}")
    sysm = main_wl.sysm
    kinds = main_wl.work()
    nnz = main_wl.items[0]["nnz"]
    kernels = kernel_table(prof, args.steps, kinds)
    roofline = roofline_of(kernels, kinds, wname)
    if args.copy_calibration > 0:
        # a plain copy of known size: reads and writes MIB MiB once (its HBM
        # counter readings scale the other kernels' readings)
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    st = main_wl.out["status"].cpu().numpy()
    res = {
        "metric": METRIC, "value": value, "unit": "walker Slater-builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": main_wl.dtype(), "data": "synthetic",
        "config": {"workload": wname, "electrons": sysm.n_elec,
                   "n_basis": sysm.n_basis, "walkers": W, "mode": mode, "survivors_per_electron": round(nnz, 1),
                   "singular_walkers": int(((st & 1) != 0).sum()), "timed": "HIP graph replays of the plan",
                   "eager_ms_per_step": ms_eager, "ms_per_step_by_launch_form": by_form},
        "roofline": roofline,
        "kernels": kernels,
    }

    also = []

    def companion(name, Wx, m, steps2, more=(), autotune=False, label=None):
        log(f"companion {label or name} W={Wx} mode={m}")
        wl = Workload(name, Wx, m, more=more, autotune=autotune)
        msx, _, prx = wl.time(steps2, 2)
        lab = label or f"{name}-W{Wx}-{m}-fwd+adjoint"
        wk = wl.work()
        ktab = kernel_table(prx, steps2, wk)
        Wtot = sum(it["W"] for it in wl.items)
        entry = {"workload": lab, "value": Wtot / (msx * 1e-3), "unit": "walker Slater-builds/s",
                 "ms_per_step": msx, "steps": steps2, "dtype": wl.dtype(),
                 "roofline": roofline_of(ktab, wk, lab),
                 "kernels_ms_per_step": {k: round(v["ms_per_step"], 3) for k, v in ktab.items()},
                 "kernel_frac": {k: round(v["frac"], 4) for k, v in ktab.items() if "frac" in v}}
        if wl.tuning is not None:
            entry["tuning"] = wl.tuning
        also.append(entry)
        return wl, entry

    if not args.no_also:
        steps2 = max(3, args.steps // 2)
        # the same workload in the other two modes; errors against FP64
        others = [m for m in ("bf16x3", "fp32") if m != mode]
        ref_wl, _ = (main_wl, None) if mode == "fp64" else companion(args.config, W, "fp64", steps2)
        if mode != "fp64":
            res["config"]["err_vs_fp64"] = err_vs_fp64(outputs_of(main_wl), outputs_of(ref_wl))
        for m in others:
            wl, entry = companion(args.config, W, m, steps2)
            entry["err_vs_fp64"] = err_vs_fp64(outputs_of(wl), outputs_of(ref_wl))
            wl.close()
            del wl
            torch.cuda.empty_cache()
        if ref_wl is not main_wl:
            ref_wl.close()
        del ref_wl
        torch.cuda.empty_cache()
        # 1731 electrons, FP32 and FP64
        W5 = q.CONFIGS["1731e"]["W"]
        wl32, e32 = companion("1731e", W5, "fp32", steps2)
        wl64, _ = companion("1731e", W5, "fp64", steps2)
        e32["err_vs_fp64"] = err_vs_fp64(outputs_of(wl32), outputs_of(wl64))
        wl32.close()
        wl64.close()
        del wl32, wl64
        torch.cuda.empty_cache()
        # the uneven batch: 512 walkers each of 44e, 158e, 434e, one autotuned FP32 plan
        wlb, eb = companion("44e", 512, "fp32", steps2, more=(("158e", 512), ("434e", 512)), autotune=True,
                            label="batch-44e+158e+434e-W512x3-fp32-fwd+adjoint")
        # the launch forms around the tuned choice: one workgroup per item or
        # persistent, both contraction tiles, atomic or deterministic dA
        forms = {f"tile{t}-{'persistent' if p_ else 'per-item'}": dict(contract_tile=t, persistent=p_)
                 for t in (0, 1, 2) for p_ in (0, 1)}
        forms["det_dA"] = dict(det_dA=1)
        eb["ms_per_step_by_launch_form"] = wlb.time_tunings(forms, steps2)
        wlb.close()
        del wlb
        torch.cuda.empty_cache()
        # dense versus localised (block-sparse) MO coefficients
        log("sparse A sweep")
        also.append(sparse_a_line("1731e", q.CONFIGS["1731e"]["W"], (25.0, 15.0, 10.0)))
        also.append(sparse_a_line(args.config, W, (15.0, 10.0)))
        torch.cuda.empty_cache()
        # one fixed-node DMC step around the builder, the whole population
        log(f"dmc step {args.config} W={W} mode={mode}")
        also.append(dmc_line(args.config, W, mode, steps2))
        torch.cuda.empty_cache()
    res["also"] = also
    main_wl.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        sysm_b, A_up, A_dn, R_b = q.make_config(args.config, W=W)
        res["cpu_baseline"] = cpu_baseline(sysm_b, A_up, A_dn, R_b, args.config)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
