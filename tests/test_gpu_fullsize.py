"""The HIP path against the FP64 oracle at the batch sizes the benchmark runs:
the adjoint of the 434-electron plan over 1024 walkers (FP32 dA by electron
in one group of 1024 walkers or eight of 128, by 32-electron range with the
deterministic reduction, split BF16; FP32 atomics across groups), the
1731-electron plan over its 512
walkers (forward on sampled walkers, dA over 64 of them), the FP64 adjoint
through the oracle's own inverse (the whole chain), and the screening's
survivor sets compared bit for bit.

Bounds (u32 = 2^-24; bA, bR are the oracle's sums of absolute values of
every term of dA and dR, oracle.backward(..., want_abs=True)):
  dA   FP32 / BF16X3: (64 + 1 + m) u32 bA  [+ 3 * 2^-16 bA in BF16X3]
       (tests/gpu_common.py dA_tol) with m the longest chain of FP32
       additions into one dA element: by electron (FP32), m = gw +
       ceil(W / gw) n (the group's walkers in one MFMA accumulator, then one
       atomic add per (electron, walker group)); by 32-electron range,
       m = 3 gw 32 + ceil(W / gw) ceil(n / 32) (gw walkers of 32 electrons,
       at most three split products per term, then one atomic add per
       (walker group, electron range)); 64 u32 covers the FP32 AO value,
       1 u32 the FP32 rounding of G = g D^-1, 3 * 2^-16 the split-BF16
       products (hi*hi + hi*lo + lo*hi: the dropped lo*lo and the bf16
       rounding of both lo parts).
  dR   (the plan takes dR = g * drift, the drift from the forward's C):
       tol_C bR + 1e-12 bR, the forward's product bound carried through the
       drift sum, plus its FP64 rounding.
These are worst-case bounds; beside them a structural check compares the
Frobenius norm of the dA difference with the smallest contribution of one
walker group (a dropped or doubled group, electron range or window block
would exceed it).
"""
import math

import numpy as np
import pytest

import oracle
import qsl_synth as q
from tests.gpu_common import U32, compare_forward, dA_tol, default_dA_group, max_survivors, tol_C

pytestmark = pytest.mark.gpu

TE = 32


def _plan_run(sysm, A_up, A_dn, R, mode, g, keep_walkers=None, tuning=None):
    """Forward + adjoint of one system through an eager plan with the default
    tuning (as the benchmark's plan) or `tuning`.  Returns numpy copies of log|det|,
    sign, status, drift, dR and dA, and of D^-1 and C for keep_walkers
    (all walkers when None)."""
    import torch
    from paper_1209_6630_amd.api import Plan, System
    S = System.from_synth(sysm)
    S.set_mo(0, A_up)
    S.set_mo(1, A_dn)
    W = R.shape[0]
    Rt = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    out = S.alloc_outputs(W, mode)
    gt = torch.from_numpy(np.ascontiguousarray(g)).cuda()
    dR = torch.empty((W, S.n_elec, 3), dtype=torch.float64, device="cuda")
    dA = (torch.empty((S.n_up, S.n_basis), dtype=torch.float64, device="cuda"),
          torch.empty((S.n_dn, S.n_basis), dtype=torch.float64, device="cuda"))
    P = Plan([S], [W], mode, graph=False)
    P.bind(0, Rt, out, g=gt, dR=dR, dA=dA)
    if tuning is not None:
        P.tuning = tuning
    P.launch()
    torch.cuda.synchronize()
    idx = torch.arange(W, device="cuda") if keep_walkers is None else torch.as_tensor(keep_walkers, device="cuda")
    res = {k: out[k].cpu().numpy() for k in ("logdet", "sign", "status", "drift", "lap")}
    for k in ("Dinv_up", "Dinv_dn", "C_up", "C_dn"):
        res[k] = out[k].index_select(0, idx).cpu().numpy()
    res["dR"] = dR.cpu().numpy()
    res["dA_up"], res["dA_dn"] = dA[0].cpu().numpy(), dA[1].cpu().numpy()
    t = P.tuning
    res["det"] = bool(t["det_dA"])
    res["gw"] = t["adj_group"] or default_dA_group(mode, W, res["det"])
    P.close()
    S.close()
    del out, Rt, dR, dA
    torch.cuda.empty_cache()
    return res


def _check_adjoint(sysm, A_up, A_dn, R, mode, g, res, gw, nnz, W_plan, group_of=None):
    """dA and dR of the GPU against the oracle adjoint on the GPU's own
    D^-1, within the bounds of the module docstring (W_plan: the walkers of
    the plan, which set the chain length), plus the structural Frobenius
    check against the smallest walker-group contribution."""
    W = W_plan
    Du = np.nan_to_num(res["Dinv_up"])
    Dd = np.nan_to_num(res["Dinv_dn"])
    rdR, rdAu, rdAd, (bR, bAu, bAd) = oracle.backward(sysm, A_up, A_dn, R, Du, Dd, g, want_abs=True)
    for s, (got, want, b) in enumerate([(res["dA_up"], rdAu, bAu), (res["dA_dn"], rdAd, bAd)]):
        n = sysm.n_dn if s else sysm.n_up
        tol = dA_tol(mode, W, n, gw, det=res.get("det", False))
        err = np.abs(got - want)
        assert np.all(err <= tol * b + 1e-300), (s, float((err / (b + 1e-300)).max()), tol)
        print(f"  dA spin {s}: max |err| / bA = {float((err / (b + 1e-300)).max()):.3e} (bound {tol:.3e}), "
              f"|err|_F / |dA|_F = {np.linalg.norm(err) / np.linalg.norm(want):.3e}", flush=True)
    tR = tol_C(mode, nnz) + 1e-12
    errR = np.abs(res["dR"] - rdR)
    assert np.all(errR <= tR * bR + 1e-300), float((errR / (bR + 1e-300)).max())
    # structural: no walker group, electron range or window block dropped or doubled
    if group_of is not None:
        groups = sorted(set(group_of.tolist()))
        contrib = []
        for gi in groups:
            m = group_of == gi
            _, cu, cd = oracle.backward(sysm, A_up, A_dn, R[m], Du[m], Dd[m], g[m])
            contrib.append(min(np.linalg.norm(cu), np.linalg.norm(cd)))
        smallest = min(contrib)
        for got, want in [(res["dA_up"], rdAu), (res["dA_dn"], rdAd)]:
            assert np.linalg.norm(got - want) <= 0.01 * smallest, (np.linalg.norm(got - want), smallest)


@pytest.mark.parametrize("mode,tuning", [("fp32", None), ("fp32", dict(adj_group=128)),
                                         ("fp32", dict(det_dA=1)), ("fp32", dict(contract_tile=0)),
                                         ("bf16x3", None)])
def test_adjoint_434e_plan_1024_walkers(mode, tuning):
    """dA over 1024 walkers and dR of every walker against the oracle,
    through the benchmark's plan: FP32 by electron (one group of 1024, or
    eight of 128), FP32 by 32-electron range with the deterministic
    reduction (eight groups of 128), split BF16 (eight groups of 128, seven
    electron ranges per spin); FP32 atomics across groups and ranges. The
    default FP32 tile takes split-bf16 products in the forward and the dA;
    tile 0 takes the FP32 MFMA kernels of both."""
    W = 1024
    print(f"[case] adjoint 434e plan W={W} mode={mode} tuning={tuning}", flush=True)
    sysm, A_up, A_dn, R = q.make_config("434e", W=W)
    g = np.random.default_rng(11).normal(size=(W, 2))
    res = _plan_run(sysm, A_up, A_dn, R, mode, g, tuning=tuning)
    sing = (res["status"] & 1) != 0
    assert not sing.any()
    gw = res["gw"]
    one_group = mode == "fp32" and not (tuning or {}).get("adj_group") and not (tuning or {}).get("det_dA")
    assert math.ceil(W / gw) >= (1 if one_group else 8)
    nnz = max_survivors(sysm, R[:2])
    _check_adjoint(sysm, A_up, A_dn, R, mode, g, res, gw, nnz, W, group_of=np.arange(W) // gw)


@pytest.mark.parametrize("name,W", [("158e", 64), ("434e", 64)])
def test_fp64_adjoint_whole_chain(name, W):
    """FP64 forward + adjoint on the GPU against the oracle's forward and
    adjoint (the oracle's own D^-1): the whole chain.

    Both inverses come from backward-stable eliminations (Gauss-Jordan here,
    LU in the oracle, the same pivots), so per walker and spin they differ by
    eps_w |D^-1|_F with eps_w of order cond(D) n 2^-53; eps_w is measured and
    checked against 4 cond(D) n 2^-53.  Walkers with cond(D) >= 1e8 get g = 0:
    there the inverses themselves are uncertain beyond what the adjoint test
    is about.  The effect of eps_w on dA and dR is bounded by the oracle's
    absolute sums with D^-1 replaced by eps_w |D^-1|_F everywhere and g by
    |g|; the adjoint arithmetic itself by 1e-10 of the plain absolute sums."""
    print(f"[case] fp64 whole-chain adjoint {name} W={W}", flush=True)
    sysm, A_up, A_dn, R = q.make_config(name, W=W)
    ref = oracle.forward(sysm, A_up, A_dn, R)
    g = np.random.default_rng(5).normal(size=(W, 2))
    cond = np.zeros((W, 2))
    for s, Ck in enumerate(("C_up", "C_dn")):
        for w in range(W):
            cond[w, s] = np.linalg.cond(ref[Ck][w][0].T)
    g[cond >= 1e8] = 0.0
    assert (g != 0).sum() >= W  # most walkers take part
    res = _plan_run(sysm, A_up, A_dn, R, "fp64", g)
    np.testing.assert_allclose(res["logdet"], ref["logdet"], rtol=1e-10, atol=1e-10)
    rdR, rdAu, rdAd, (bR, bAu, bAd) = oracle.backward(sysm, A_up, A_dn, R, ref["Dinv_up"], ref["Dinv_dn"], g,
                                                      want_abs=True)
    scaled = []
    for s, (Dk, n) in enumerate([("Dinv_up", sysm.n_up), ("Dinv_dn", sysm.n_dn)]):
        nrm = np.linalg.norm(ref[Dk], axis=(1, 2))
        eps = np.linalg.norm(res[Dk] - ref[Dk], axis=(1, 2)) / nrm
        ok = g[:, s] != 0
        assert np.all(eps[ok] <= 4 * cond[ok, s] * n * 2.0 ** -53), float((eps[ok] / cond[ok, s]).max())
        scaled.append((eps * nrm)[:, None, None] * np.ones_like(ref[Dk]))
    _, _, _, (cR, cAu, cAd) = oracle.backward(sysm, A_up, A_dn, R, scaled[0], scaled[1], np.abs(g), want_abs=True)
    for got, want, b, c in [(res["dA_up"], rdAu, bAu, cAu), (res["dA_dn"], rdAd, bAd, cAd)]:
        assert np.all(np.abs(got - want) <= 1e-10 * b + c + 1e-300), float(np.abs(got - want).max())
    assert np.all(np.abs(res["dR"] - rdR) <= 1e-10 * bR + cR + 1e-300)


def test_forward_1731e_plan_512_walkers_sampled():
    """The 1731-electron FP32 plan over its full 512 walkers (blocked
    inversion over 1024 matrices): every forward output of walkers spread
    over the batch (first, last, tile edges) against the oracle."""
    W = 512
    print(f"[case] forward 1731e plan W={W} fp32 sampled", flush=True)
    sysm, A_up, A_dn, R = q.make_config("1731e", W=W)
    keep = [0, 31, 32, 300, 511]
    g = np.zeros((W, 2))
    res = _plan_run(sysm, A_up, A_dn, R, "fp32", g, keep_walkers=keep)
    gpu = {k: res[k] for k in ("C_up", "C_dn", "Dinv_up", "Dinv_dn")}
    for k in ("logdet", "sign", "status", "drift", "lap"):
        gpu[k] = res[k][keep]
    compare_forward(sysm, A_up, A_dn, R[keep], gpu, "fp32")


def test_adjoint_1731e_plan_512_walkers():
    """dA of the 1731-electron FP32 plan with W = 512 (four walker groups),
    g non-zero on 64 walkers spread over all groups, against the oracle
    adjoint over those 64; dR of the same walkers."""
    W = 512
    print(f"[case] adjoint 1731e plan W={W} fp32 (64 weighted walkers)", flush=True)
    sysm, A_up, A_dn, R = q.make_config("1731e", W=W)
    sel = np.arange(3, W, 8)
    g = np.zeros((W, 2))
    g[sel] = np.random.default_rng(17).normal(size=(sel.size, 2))
    res = _plan_run(sysm, A_up, A_dn, R, "fp32", g, keep_walkers=sel)
    assert not ((res["status"][sel] & 1) != 0).any()
    gw = res["gw"]
    nnz = max_survivors(sysm, R[sel[:1]])
    sub = {"Dinv_up": res["Dinv_up"], "Dinv_dn": res["Dinv_dn"], "dR": res["dR"][sel],
           "dA_up": res["dA_up"], "dA_dn": res["dA_dn"]}
    # the chain bound counts every walker of a group, weighted or not
    _check_adjoint(sysm, A_up, A_dn, R[sel], "fp32", g[sel], sub, gw, nnz, W, group_of=sel // gw)


# ------------------------------------------------------------ screening

def _unit_mo_chunks(sysm):
    """MO matrices whose rows are unit vectors: chunk k maps MO i of spin s
    to AO k n_s + i (zero rows past N_b), so C_1[e][i] = chi_(k n_s + i)(r_e)
    and its non-zero pattern is the survivor set."""
    nb = sysm.n_basis
    nch = math.ceil(nb / max(1, sysm.n_dn))
    chunks = []
    for k in range(nch):
        mats = []
        for n in (sysm.n_up, sysm.n_dn):
            A = np.zeros((n, nb))
            for i in range(n):
                if k * n + i < nb:
                    A[i, k * n + i] = 1.0
            mats.append(A)
        chunks.append(mats)
    return chunks


def _gpu_survivors(sysm, R, walkers, mode):
    """{(w, e): sorted AO indices with C_1 != 0} over all unit-MO chunks."""
    import torch
    from paper_1209_6630_amd.api import System
    S = System.from_synth(sysm)
    Rt = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    out = S.alloc_outputs(R.shape[0], mode, drift=False)
    idx = torch.as_tensor(walkers, device="cuda")
    surv = {(w, e): [] for w in walkers for e in range(sysm.n_up + sysm.n_dn)}
    for k, (Au, Ad) in enumerate(_unit_mo_chunks(sysm)):
        S.set_mo(0, Au)
        S.set_mo(1, Ad)
        S.forward(Rt, mode, out=out, drift=False)
        torch.cuda.synchronize()
        for s, (Ck, n) in enumerate([("C_up", sysm.n_up), ("C_dn", sysm.n_dn)]):
            C1 = out[Ck].index_select(0, idx)[:, 0].cpu().numpy()  # [w][e][i]
            e0 = sysm.n_up if s else 0
            for a, w in enumerate(walkers):
                for e in range(n):
                    nz = np.nonzero(C1[a, e])[0]
                    surv[(w, e0 + e)].extend((k * n + nz[k * n + nz < sysm.n_basis]).tolist())
    S.close()
    del out, Rt
    torch.cuda.empty_cache()
    return {key: sorted(v) for key, v in surv.items()}


def _check_survivors(sysm, R, walkers, modes):
    want = {(w, e): oracle.ao_eval(sysm, R[w, e])[0].tolist()
            for w in walkers for e in range(sysm.n_up + sysm.n_dn)}
    for mode in modes:
        got = _gpu_survivors(sysm, R, walkers, mode)
        bad = [key for key in want if got[key] != want[key]]
        assert not bad, (mode, bad[:5], [(got[k][:8], want[k][:8]) for k in bad[:2]])


@pytest.mark.parametrize("name,W,walkers", [("434e", 4096, [0, 31, 32, 2047, 4095]),
                                            ("1731e", 512, [0, 255, 511])])
def test_survivor_sets_exact_full_batch(name, W, walkers):
    """Screening and compaction, bit for bit: with unit-vector MO rows the
    non-zero pattern of C_1 is the set of surviving AOs, which must equal the
    oracle's for every electron of walkers sampled from the full batch, in
    all three modes (the decision is FP64 in every mode)."""
    print(f"[case] exact survivors {name} W={W}", flush=True)
    sysm, _, _, R = q.make_config(name, W=W)
    _check_survivors(sysm, R, walkers, ("fp64", "fp32", "bf16x3"))


def _tie_position(Q, u, gamma, T, keep):
    """A point Q + s u with gamma r^2 within a few ulp of T, computed with
    the screening's own FP64 expression: the largest s found with
    gamma r^2 <= T (keep) or the next one up (> T)."""
    def t_of(s):
        p = Q + s * u
        d = p - Q
        r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        return gamma * r2, p
    s0 = math.sqrt(T / gamma)
    lo, hi = 0.9 * s0, 1.1 * s0
    assert t_of(lo)[0] <= T < t_of(hi)[0]
    while np.nextafter(lo, hi) < hi:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if t_of(mid)[0] <= T:
            lo = mid
        else:
            hi = mid
    t, p = t_of(lo if keep else hi)
    assert (t <= T) == keep and abs(t - T) <= 1e-13 * T
    return p


def test_survivor_sets_exact_near_ties():
    """Electrons placed so that gamma r^2 of some primitive lies within a few
    ulp of T on either side (the atom's most diffuse primitive, which
    decides the atomic radius, and other primitives): the GPU's survivor sets
    equal the oracle's exactly in all three modes."""
    print("[case] exact survivors near ties 434e", flush=True)
    sysm, _, _, R = q.make_config("434e", W=64)
    R = R.copy()
    rng = np.random.default_rng(23)
    N = sysm.n_up + sysm.n_dn
    off = np.concatenate([[0], np.cumsum(sysm.shell_nprim)])
    placed = 0
    for w in range(R.shape[0]):
        for e in rng.choice(N, size=8, replace=False):
            a = int(np.argmin(((sysm.atom_xyz - R[w, e]) ** 2).sum(1)))
            shells = np.nonzero(sysm.shell_atom == a)[0]
            exps = np.concatenate([sysm.prim_exp[off[s_]:off[s_ + 1]] for s_ in shells])
            gamma = exps.min() if placed % 2 == 0 else rng.choice(exps)
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            R[w, e] = _tie_position(sysm.atom_xyz[a], u, float(gamma), sysm.screen_T, keep=(placed // 2) % 2 == 0)
            placed += 1
    _check_survivors(sysm, R, list(range(0, 64, 3)), ("fp64", "fp32", "bf16x3"))
