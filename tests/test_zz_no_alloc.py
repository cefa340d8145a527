"""The allocation-free forward (qsl_forward_noalloc, workspace in the
library's static device array) against qsl_forward with a caller workspace:
bit-identical outputs on two calls in a row, the second with fewer walkers,
and a clear WORKSPACE error when the static array is too small."""
import ctypes as ct

import numpy as np
import pytest

import qsl_synth as q
from tests.gpu_common import make_gpu_system
from tests.systems import random_tiny, walkers_near

pytestmark = pytest.mark.gpu

KEYS = ("C_up", "C_dn", "logdet", "sign", "Dinv_up", "Dinv_dn", "drift", "lap", "status")


def _call(S, R, mode, noalloc):
    import torch
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import _fwd_args
    Rt = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    out = S.alloc_outputs(R.shape[0], mode)
    for v in out.values():
        v.fill_(7) if v.dtype in (torch.int8, torch.int32) else v.fill_(float("nan"))
    a = _fwd_args(S, Rt, mode, out)
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        _lib.check(_lib.lib().qsl_forward_noalloc(S._h, ct.byref(a), stream))
    else:
        ws = S.workspace(R.shape[0], mode, backward=False)
        a.ws, a.ws_bytes = ws.data_ptr(), ws.numel()
        _lib.check(_lib.lib().qsl_forward(S._h, ct.byref(a), stream))
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


def _same(a, b):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("case", ["44e-fp64", "158e-fp32", "434e-bf16x3", "blocked-fp32"])
def test_noalloc_forward_equals_forward(case):
    """Two calls in a row (the second with fewer walkers, so the array
    still holds the first call's lists) equal qsl_forward bit for bit."""
    print(f"[case] noalloc forward {case}", flush=True)
    if case == "blocked-fp32":
        sysm, A_up, A_dn = random_tiny(n_atoms=45, n_up=240, n_dn=236, seed=31)
        Rs = [walkers_near(sysm, 3, seed=1), walkers_near(sysm, 2, seed=2)]
        mode = "fp32"
    else:
        name, mode = case.split("-")
        sysm, A_up, A_dn, R = q.make_config(name, W=96)
        Rs = [R, R[:33] + 0.01]
    S = make_gpu_system(sysm, A_up, A_dn)
    for R in Rs:
        _same(_call(S, R, mode, noalloc=True), _call(S, R, mode, noalloc=False))


def test_noalloc_rejects_more_than_the_static_scratch():
    print("[case] noalloc size limit", flush=True)
    import torch
    from paper_1209_6630_amd import _lib
    from paper_1209_6630_amd.api import _fwd_args
    sysm, A_up, A_dn, R = q.make_config("434e", W=1)
    S = make_gpu_system(sysm, A_up, A_dn)
    W = 8192
    n = ct.c_size_t()
    _lib.check(_lib.lib().qsl_workspace_size(S._h, W, 1, _lib.WS_FORWARD, ct.byref(n)))
    assert n.value > _lib.NOALLOC_SCRATCH_BYTES
    # the size check comes before any launch: small placeholders suffice
    Rt = torch.zeros((1, S.n_elec, 3), dtype=torch.float64, device="cuda")
    out = S.alloc_outputs(1, "fp32")
    a = _fwd_args(S, Rt, "fp32", out)
    a.W = W
    assert _lib.lib().qsl_forward_noalloc(S._h, ct.byref(a), None) == 4
    assert b"static scratch" in _lib.lib().qsl_last_error()
