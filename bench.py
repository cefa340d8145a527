#!/usr/bin/env python3
"""Benchmark: walker Slater-builds per second, forward + adjoint, on one GPU.

A step is one pass of the whole hot path over one batch of walkers:
screening, fused AO evaluation + AO->MO products (split BF16 on MFMA with
FP32 accumulation), FP64 Gauss-Jordan log|det| / sign / inverse, drift and
Laplacian, then the adjoint (AO recomputation, dA and dR).  The workload is
the synthetic 434-electron peptide-shaped system (134 atoms, 1270 AOs,
217 x 1270 MO coefficients per spin) with 4096 walkers.  Inputs are resident
in HBM before the timed region.

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
PEAK_FP64_VALU = 78.6
PEAK_FP32_VALU = 157.3
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def survivors_per_electron(sysm, R, max_walkers=64):
    """Mean surviving AOs per electron (cost model for the flop counts):
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


def cpu_baseline(sysm, A_up, A_dn, R, target_s=12.0):
    """The FP64 oracle, forward + adjoint, on a bounded sample of walkers."""
    import oracle
    oracle.load()
    nthr = oracle.max_threads()
    W = R.shape[0]

    def run(ws):
        t0 = time.perf_counter()
        out = oracle.forward(sysm, A_up, A_dn, R[:ws])
        g = np.ones((ws, 2))
        oracle.backward(sysm, A_up, A_dn, R[:ws], out["Dinv_up"], out["Dinv_dn"], g)
        return time.perf_counter() - t0

    cal = max(1, min(W, nthr))
    t = run(cal)
    n = int(min(W, max(cal, round(cal * target_s / max(t, 1e-3)))))
    n = max(cal, (n // cal) * cal)
    log(f"cpu baseline: calibration {cal} walkers {t:.2f}s -> sample {n} walkers")
    t = run(n)
    return {"value": n / t, "unit": "walker Slater-builds/s", "cores": nthr, "kind": "oracle",
            "sample": f"{n} of the {W} walkers of the 434e workload, FP64 forward + adjoint, "
                      f"OpenMP over walkers on {nthr} threads, {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="bf16x3", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--config", default="434e")
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the walker batch of one "
              "GPU is the unit of work; see the design notes for how walkers shard across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import qsl_synth as q
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import System

    cfg = q.CONFIGS[args.config]
    W = args.walkers or cfg["W"]
    mode = args.mode
    log(f"workload {args.config} W={W} mode={mode}: generating inputs")
    sysm, A_up, A_dn, R_np = q.make_config(args.config, W=W)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = System.from_synth(sysm)
    S.set_mo(0, A_up)
    S.set_mo(1, A_dn)
    R = torch.from_numpy(R_np).to(dev)
    out = S.alloc_outputs(W, mode)
    g = torch.ones((W, 2), dtype=torch.float64, device=dev)
    N, nb = sysm.n_elec, sysm.n_basis
    dR = torch.empty((W, N, 3), dtype=torch.float64, device=dev)
    dA = (torch.empty((sysm.n_up, nb), dtype=torch.float64, device=dev),
          torch.empty((sysm.n_dn, nb), dtype=torch.float64, device=dev))
    torch.cuda.synchronize()

    def step():
        S.forward(R, mode, out=out)
        S.backward(R, out["Dinv_up"], out["Dinv_dn"], g, mode, dR=dR, dA=dA)

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    n_sing = int(((st & 1) != 0).sum())
    _lib.profile_enable(True)
    _lib.profile_read(reset=True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = _lib.profile_read(reset=True)
    _lib.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    value = W / (ms * 1e-3)
    log(f"{ms:.3f} ms/step, {value:.1f} walkers/s; kernels {prof}")

    # algorithmic work per launch (one launch = one spin over all W walkers)
    nnz = survivors_per_electron(sysm, R_np)
    ns = [sysm.n_up, sysm.n_dn]
    contract_flops = [10.0 * n * n * nnz * W for n in ns]          # 5 products x 2 flops x MOs x survivors
    gj_flops = [2.0 * n ** 3 * W for n in ns]                        # 2 n^3 per matrix
    adjoint_flops = [2.0 * n * n * nnz * W for n in ns]              # H or dA: 2 flops per (electron, survivor, MO)
    cbytes = 8 if mode == "fp64" else 4
    epi_bytes = [(8.0 * n * n + 4 * cbytes * n * n + 32.0 * n) * W for n in ns]
    kinds = {
        f"contract_{mode}": (sum(contract_flops), PEAK[mode][0], PEAK[mode][1], "TFLOP/s"),
        "gauss_jordan": (sum(gj_flops), "alu", PEAK_FP64_VALU, "TFLOP/s"),
        "adjoint_h": (sum(adjoint_flops), PEAK[mode][0], PEAK[mode][1], "TFLOP/s"),
        "adjoint_dA": (sum(adjoint_flops), PEAK[mode][0], PEAK[mode][1], "TFLOP/s"),
        "drift_lap": (sum(epi_bytes), "hbm", HBM_PEAK, "GB/s"),
    }
    kernels = {}
    for name, (launches, tot) in prof.items():
        per_launch_ms = tot / max(launches, 1)
        entry = {"launches": launches, "avg_ms": per_launch_ms, "ms_per_step": tot / args.steps}
        if name in kinds:
            work, bound, peak, unit = kinds[name]
            per_step_work = work  # summed over both spins = the launches of one step
            achieved = per_step_work / (tot / args.steps * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
            entry.update(bound=bound, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak)
        kernels[name] = entry
    dom = max((k for k in kernels if k in kinds), key=lambda k: kernels[k]["ms_per_step"])
    d = kernels[dom]
    roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                "unit": d["unit"], "frac": d["frac"], "traffic": None}

    res = {
        "metric": METRIC, "value": value, "unit": "walker Slater-builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3+f32acc/f64", "fp32": "f32/f64", "fp64": "f64"}[mode],
        "data": "synthetic",
        "config": {"workload": f"{args.config}-W{W}-{mode}-fwd+adjoint", "electrons": N, "n_basis": nb,
                   "walkers": W, "mode": mode, "survivors_per_electron": round(nnz, 1),
                   "singular_walkers": n_sing},
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(sysm, A_up, A_dn, R_np)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
