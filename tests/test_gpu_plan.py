"""Uneven batches (plans): batched launches equal per-system launches bit for
bit, graph replays equal eager launches, every tuning (launch form, group
size, Gauss-Jordan block, FP32 contraction tile, persistent launch,
deterministic dA) agrees with the default, the deterministic dA repeats
bit for bit, the autotuner's choice and cache, and the 512 x (44e, 158e,
434e) FP32 batch against the FP64 oracle on sampled walkers."""
import json
import os

import numpy as np
import pytest

import oracle
import qsl_synth as q
from tests.gpu_common import U32, compare_forward, make_gpu_system, max_survivors
from tests.systems import random_tiny, walkers_near

pytestmark = pytest.mark.gpu

FWD_KEYS = ("C_up", "C_dn", "logdet", "sign", "Dinv_up", "Dinv_dn", "drift", "lap", "status")


def _batch(spec, seed=0):
    """spec: list of (config name or ('tiny', n_up, n_dn), W)."""
    import torch
    items = []
    for k, (name, W) in enumerate(spec):
        if isinstance(name, tuple):
            _, nu, nd = name
            sysm, A_up, A_dn = random_tiny(n_atoms=max(3, (nu + nd) // 6 + 1), n_up=nu, n_dn=nd, seed=40 + k)
            R = walkers_near(sysm, W, seed=k)
        else:
            sysm, A_up, A_dn, R = q.make_config(name, W=W)
        S = make_gpu_system(sysm, A_up, A_dn)
        g = np.random.default_rng(seed + k).normal(size=(W, 2))
        items.append(dict(sysm=sysm, A_up=A_up, A_dn=A_dn, R=R, S=S,
                          Rt=torch.from_numpy(np.ascontiguousarray(R)).cuda(),
                          gt=torch.from_numpy(g).cuda(), g=g))
    return items


def _per_system(it, mode):
    import torch
    S = it["S"]
    out = S.forward(it["Rt"], mode)
    # the plan's adjoint takes dR from the forward's drift
    dR, dAu, dAd = S.backward(it["Rt"], out["Dinv_up"], out["Dinv_dn"], it["gt"], mode, drift=out["drift"])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res.update(dR=dR.cpu().numpy(), dA_up=dAu.cpu().numpy(), dA_dn=dAd.cpu().numpy())
    return res


def _plan(items, mode, graph, tuning=None):
    import torch
    from paper_1209_6630_amd.api import Plan
    P = Plan([it["S"] for it in items], [it["R"].shape[0] for it in items], mode, graph=graph)
    bufs = []
    for i, it in enumerate(items):
        S, W = it["S"], it["R"].shape[0]
        out = S.alloc_outputs(W, mode)
        dR = torch.empty((W, S.n_elec, 3), dtype=torch.float64, device="cuda")
        dA = (torch.empty((S.n_up, S.n_basis), dtype=torch.float64, device="cuda"),
              torch.empty((S.n_dn, S.n_basis), dtype=torch.float64, device="cuda"))
        P.bind(i, it["Rt"], out, g=it["gt"], dR=dR, dA=dA)
        bufs.append((out, dR, dA))
    if tuning is not None:
        P.tuning = tuning
    return P, bufs


def _read(bufs):
    import torch
    torch.cuda.synchronize()
    res = []
    for out, dR, dA in bufs:
        r = {k: v.cpu().numpy() for k, v in out.items()}
        r.update(dR=dR.cpu().numpy(), dA_up=dA[0].cpu().numpy(), dA_dn=dA[1].cpu().numpy())
        res.append(r)
    return res


def _dA_close(a, b, mode):
    # the same terms summed in another order (atomics over walker groups)
    rel = 1e-12 if mode == "fp64" else 1e-4
    m = max(np.abs(a).max(initial=0.0), 1e-300)
    assert np.all(np.abs(a - b) <= rel * m), float(np.abs(a - b).max() / m)


def _same(ref, got, mode, exact=True):
    for k in FWD_KEYS + ("dR",):
        if exact:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        else:
            x, y = ref[k].astype(np.float64), got[k].astype(np.float64)
            m = np.nanmax(np.abs(x), initial=0.0)
            assert np.allclose(x, y, rtol=0, atol=1e-9 * max(m, 1e-300), equal_nan=True), k
    _dA_close(ref["dA_up"], got["dA_up"], mode)
    _dA_close(ref["dA_dn"], got["dA_dn"], mode)


SPEC = [("44e", 12), ("158e", 5), ("434e", 3), (("tiny", 3, 0), 4), (("tiny", 2, 1), 0)]


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("graph", [False, True])
def test_plan_equals_per_system_calls(mode, graph):
    print(f"[case] plan vs per-system mode={mode} graph={graph}", flush=True)
    items = _batch(SPEC)
    ref = [_per_system(it, mode) for it in items]
    P, bufs = _plan(items, mode, graph)
    P.launch()
    got = _read(bufs)
    for r, g_ in zip(ref, got):
        _same(r, g_, mode)
    P.close()


@pytest.mark.parametrize("mode", ["bf16x3", "fp32"])
@pytest.mark.parametrize("graph", [False, True])
def test_plan_without_drift_splits_g_itself(graph, mode):
    """A plan bound without drift and Laplacian outputs: dR comes from
    recomputed AO gradients and the dA adjoint's G (split BF16, or FP32 for
    the dA by electron) from its own pre-pass (no epilogue to write it);
    equal to the per-system calls."""
    import torch
    from paper_1209_6630_amd.api import Plan
    print(f"[case] plan without drift graph={graph} mode={mode}", flush=True)
    items = _batch([("44e", 6), ("158e", 3)])
    P = Plan([it["S"] for it in items], [it["R"].shape[0] for it in items], mode, graph=graph)
    bufs = []
    for i, it in enumerate(items):
        S, W = it["S"], it["R"].shape[0]
        out = S.alloc_outputs(W, mode, drift=False)
        dR = torch.empty((W, S.n_elec, 3), dtype=torch.float64, device="cuda")
        dA = (torch.empty((S.n_up, S.n_basis), dtype=torch.float64, device="cuda"),
              torch.empty((S.n_dn, S.n_basis), dtype=torch.float64, device="cuda"))
        P.bind(i, it["Rt"], out, g=it["gt"], dR=dR, dA=dA)
        bufs.append((out, dR, dA))
    P.launch()
    got = _read(bufs)
    for it, g_ in zip(items, got):
        S = it["S"]
        out = S.forward(it["Rt"], mode)
        dR, dAu, dAd = S.backward(it["Rt"], out["Dinv_up"], out["Dinv_dn"], it["gt"], mode)
        torch.cuda.synchronize()
        for k in ("logdet", "sign", "Dinv_up", "Dinv_dn", "C_up", "C_dn"):
            np.testing.assert_array_equal(g_[k], out[k].cpu().numpy(), err_msg=k)
        np.testing.assert_array_equal(g_["dR"], dR.cpu().numpy())
        _dA_close(dAu.cpu().numpy(), g_["dA_up"], mode)
        _dA_close(dAd.cpu().numpy(), g_["dA_dn"], mode)
    P.close()


def test_graph_replays_follow_new_coordinates():
    """Replays of one captured graph, with eager work and new walker
    coordinates copied into the bound R between them, each equal the eager
    (uncaptured) plan on the same coordinates."""
    print("[case] graph replays", flush=True)
    import torch
    mode = "fp32"
    items = _batch([("44e", 16), ("158e", 4), (("tiny", 3, 0), 4)])
    Pg, bg = _plan(items, mode, graph=True)
    Pe, be = _plan(items, mode, graph=False)
    rng = np.random.default_rng(7)
    for rep in range(3):
        if rep:
            for it in items:
                it["Rt"].add_(torch.from_numpy(rng.normal(scale=0.05, size=it["R"].shape)).cuda())
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()   # unrelated eager work and a synchronisation
        Pg.launch()
        torch.cuda.synchronize()
        got = _read(bg)
        Pe.launch()
        ref = _read(be)
        for r, g_ in zip(ref, got):
            _same(r, g_, mode)
    Pg.close()
    Pe.close()


TUNINGS = [dict(batched=0, adj_group=16, gj_bias=0),
           dict(batched=1, adj_group=32, gj_bias=1),
           dict(batched=1, adj_group=256, gj_bias=1),
           dict(batched=1, adj_group=0, gj_bias=0, contract_tile=1),
           dict(batched=1, adj_group=0, gj_bias=0, persistent=1),
           dict(batched=1, adj_group=64, gj_bias=0, contract_tile=1, persistent=1),
           dict(batched=1, adj_group=16, gj_bias=0, det_dA=1),
           dict(batched=0, adj_group=0, gj_bias=0, contract_tile=1, det_dA=1),
           dict(batched=1, adj_group=0, gj_bias=0, contract_tile=2),
           dict(batched=1, adj_group=32, gj_bias=0, contract_tile=2, persistent=1)]


@pytest.mark.parametrize("mode", ["fp32", "fp64", "bf16x3"])
@pytest.mark.parametrize("tuning", TUNINGS)
def test_tunings_agree(tuning, mode):
    if mode != "fp32" and (tuning.get("contract_tile") or tuning["gj_bias"]):
        pytest.skip("the contraction tile is an FP32 choice; block shapes are covered in FP32")
    print(f"[case] tuning {tuning} mode={mode}", flush=True)
    items = _batch([("44e", 40), ("158e", 6), (("tiny", 70, 60), 3)])
    # the reference: the default tuning with the same FP32 tile family (tiles
    # 0 and 1 round alike, the split-bf16 tile 2 otherwise; each against the
    # oracle in test_contract_tiles_against_oracle)
    ref_tile = 2 if tuning.get("contract_tile", 2) == 2 else 0
    P0, b0 = _plan(items, mode, graph=False, tuning=dict(contract_tile=ref_tile))
    P0.launch()
    ref = _read(b0)
    P1, b1 = _plan(items, mode, graph=True, tuning=tuning)
    assert {k: P1.tuning[k] for k in tuning} == tuning
    P1.launch()
    got = _read(b1)
    for r, g_ in zip(ref, got):
        # another Gauss-Jordan block shape may break pivot ties differently;
        # tiles of one family and the persistent launch change no sum
        _same(r, g_, mode, exact=tuning["gj_bias"] == 0)
    P0.close()
    P1.close()


@pytest.mark.parametrize("mode", ["fp32", "fp64", "bf16x3"])
def test_deterministic_dA_repeats_bit_for_bit(mode):
    """With det_dA the adjoint's dA is the same on every launch, in a plan
    and in a second plan of the same tuning, and accumulates onto what the
    buffer holds; the atomic dA agrees with it to rounding."""
    print(f"[case] deterministic dA mode={mode}", flush=True)
    import torch
    from paper_1209_6630_amd.api import Plan
    items = _batch([("44e", 96), ("158e", 20), (("tiny", 40, 33), 7)])
    det = dict(batched=1, adj_group=16, gj_bias=0, det_dA=1)
    P1, b1 = _plan(items, mode, graph=True, tuning=det)
    P2, b2 = _plan(items, mode, graph=False, tuning=det)
    P1.launch()
    first = _read(b1)
    P1.launch()
    P2.launch()
    second, other = _read(b1), _read(b2)
    for a, b, c in zip(first, second, other):
        for k in ("dA_up", "dA_dn"):
            np.testing.assert_array_equal(a[k], b[k])
            np.testing.assert_array_equal(a[k], c[k])
    P0, b0 = _plan(items, mode, graph=False, tuning=dict(det, det_dA=0))
    P0.launch()
    for r, g_ in zip(_read(b0), first):
        _same(r, g_, mode)
    # accumulate: the partial sums are added to the buffer's contents
    P3 = Plan([it["S"] for it in items], [it["R"].shape[0] for it in items], mode, graph=True)
    P3.tuning = det
    acc = []
    for i, it in enumerate(items):
        S, W = it["S"], it["R"].shape[0]
        out = S.alloc_outputs(W, mode)
        dR = torch.empty((W, S.n_elec, 3), dtype=torch.float64, device="cuda")
        dA = (torch.full((S.n_up, S.n_basis), 3.0, dtype=torch.float64, device="cuda"),
              torch.full((S.n_dn, S.n_basis), 3.0, dtype=torch.float64, device="cuda"))
        P3.bind(i, it["Rt"], out, g=it["gt"], dR=dR, dA=dA, accumulate=True)
        acc.append((out, dR, dA))
    P3.launch()
    for r, g_ in zip(first, _read(acc)):
        for k in ("dA_up", "dA_dn"):
            # (3 + p_0) + p_1 + ... against 3 + (p_0 + p_1 + ...): rounding only
            np.testing.assert_allclose(g_[k], r[k] + 3.0, rtol=0, atol=1e-12 * max(3.0, np.abs(r[k]).max()))
    for p_ in (P0, P1, P2, P3):
        p_.close()


@pytest.mark.parametrize("tile,persistent", [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (2, 1)])
def test_contract_tiles_against_oracle(tile, persistent):
    """Each FP32 contraction tile, in one launch per item or persistent,
    on the 434- and 44-electron systems against the FP64 oracle on sampled
    walkers (the forward bounds of the per-system tests)."""
    print(f"[case] contraction tile={tile} persistent={persistent}", flush=True)
    mode = "fp32"
    items = _batch([("434e", 64), ("44e", 100)])
    P, bufs = _plan(items, mode, graph=False,
                    tuning=dict(batched=1, adj_group=0, gj_bias=0, contract_tile=tile, persistent=persistent))
    P.launch()
    got = _read(bufs)
    for it, g_ in zip(items, got):
        sysm, A_up, A_dn, R = it["sysm"], it["A_up"], it["A_dn"], it["R"]
        sample = [0, 13, R.shape[0] - 1]
        gs = {k: v[sample] for k, v in g_.items() if k in FWD_KEYS}
        compare_forward(sysm, A_up, A_dn, R[sample], gs, mode)
    P.close()


def test_autotune_and_cache(tmp_path):
    print("[case] autotune", flush=True)
    import torch
    mode = "fp32"
    spec = [("44e", 64), ("158e", 16)]
    items = _batch(spec)
    cache = str(tmp_path / "tune.json")
    P, bufs = _plan(items, mode, graph=True)
    t = P.autotune(cache)
    assert P.tuning == t
    doc = json.load(open(cache))
    entries = doc["qslater_autotune"]
    assert len(entries) == 1 and entries[0]["batched"] == t["batched"]
    assert all(entries[0][k] == t[k] for k in t)
    P.launch()
    tuned = _read(bufs)
    P0, b0 = _plan(items, mode, graph=False)
    P0.launch()
    ref = _read(b0)
    for r, g_ in zip(ref, tuned):
        _same(r, g_, mode, exact=t["gj_bias"] == 0)
    # a cache hit sets the tuning without launching anything
    P2, b2 = _plan(items, mode, graph=True)
    for out, dR, dA in b2:
        out["logdet"].fill_(12345.0)
    t2 = P2.autotune(cache)
    assert t2 == t and P2.tuning == t
    torch.cuda.synchronize()
    assert all(np.all(out["logdet"].cpu().numpy() == 12345.0) for out, _, _ in b2)
    # another batch shape appends a second entry
    items3 = _batch([("44e", 8)])
    P3, _ = _plan(items3, mode, graph=False)
    P3.autotune(cache)
    assert len(json.load(open(cache))["qslater_autotune"]) == 2
    # the caller's choice of the deterministic dA is kept
    P4, _ = _plan(items3, mode, graph=False, tuning=dict(batched=1, adj_group=0, gj_bias=0, det_dA=1))
    assert P4.autotune(None)["det_dA"] == 1
    for p_ in (P, P0, P2, P3, P4):
        p_.close()


def test_uneven_batch_512_each_fp32_against_oracle():
    """512 walkers each of the 44-, 158- and 434-electron systems in one
    FP32 plan (autotuned, graph): forward outputs and dR of sampled walkers
    against the FP64 oracle, dA against the per-system calls."""
    print("[case] uneven batch 3 x 512 fp32", flush=True)
    mode = "fp32"
    items = _batch([("44e", 512), ("158e", 512), ("434e", 512)])
    P, bufs = _plan(items, mode, graph=True)
    P.autotune(None)
    P.launch()
    got = _read(bufs)
    for it, g_ in zip(items, got):
        sysm, A_up, A_dn, R = it["sysm"], it["A_up"], it["A_dn"], it["R"]
        sample = [0, 1, 257, 511]
        Rs = R[sample]
        ref = oracle.forward(sysm, A_up, A_dn, Rs, want_abs=True)
        gs = {k: v[sample] for k, v in g_.items() if k in FWD_KEYS}
        compare_forward(sysm, A_up, A_dn, Rs, gs, mode, ref=ref)
        # dR of the sampled walkers: the oracle adjoint from the GPU's inverse
        from tests.test_gpu_adjoint import _abs_bounds
        Di = {"Dinv_up": gs["Dinv_up"], "Dinv_dn": gs["Dinv_dn"]}
        gsm = it["g"][sample]
        rdR, _, _ = oracle.backward(sysm, A_up, A_dn, Rs, Di["Dinv_up"], Di["Dinv_dn"], gsm)
        _, bR = _abs_bounds(sysm, A_up, A_dn, Rs, Di, gsm)
        nnz = max_survivors(sysm, Rs[:1])
        tol = (64 + 64 + 2 * nnz) * U32
        assert np.all(np.abs(g_["dR"][sample] - rdR) <= tol * bR + 1e-300)
        ps = _per_system(it, mode)
        _dA_close(ps["dA_up"], g_["dA_up"], mode)
        _dA_close(ps["dA_dn"], g_["dA_dn"], mode)
    P.close()


def test_autotune_with_accumulated_dA():
    """Autotuning a plan bound with accumulate_dA: the tuning runs overwrite
    dA (all candidates pass the self-check), the caller's flag applies again
    afterwards, and a launch then adds the new dA to what the buffer holds."""
    print("[case] autotune with accumulate", flush=True)
    import torch
    from paper_1209_6630_amd.api import Plan
    mode = "fp32"
    items = _batch([("44e", 32), ("158e", 8)])
    P = Plan([it["S"] for it in items], [it["R"].shape[0] for it in items], mode, graph=True)
    bufs = []
    for i, it in enumerate(items):
        S, W = it["S"], it["R"].shape[0]
        out = S.alloc_outputs(W, mode)
        dR = torch.empty((W, S.n_elec, 3), dtype=torch.float64, device="cuda")
        dA = (torch.zeros((S.n_up, S.n_basis), dtype=torch.float64, device="cuda"),
              torch.zeros((S.n_dn, S.n_basis), dtype=torch.float64, device="cuda"))
        P.bind(i, it["Rt"], out, g=it["gt"], dR=dR, dA=dA, accumulate=True)
        bufs.append((out, dR, dA))
    t = P.autotune(None)
    assert P.tuning == t
    for _, _, dA in bufs:
        for a in dA:
            a.fill_(3.0)
    P.launch()
    got = _read(bufs)
    for it, g_ in zip(items, got):
        ps = _per_system(it, mode)
        _dA_close(ps["dA_up"] + 3.0, g_["dA_up"], mode)
        _dA_close(ps["dA_dn"] + 3.0, g_["dA_dn"], mode)
    P.close()
