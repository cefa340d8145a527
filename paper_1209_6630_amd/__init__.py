"""MI355X (gfx950) Slater-matrix builder for quantum Monte Carlo walkers.

Screened contracted-Gaussian AO evaluation, the AO->MO products on MFMA,
FP64 log|det| / inverse and a hand-written adjoint, behind the C ABI of
include/qslater.h.  The binding loads the in-tree libqslater.so and never
falls back to CPU code.
"""
from ._lib import MODES, QslError, lib  # noqa: F401


def __getattr__(name):
    # torch-dependent parts are imported lazily
    if name in ("System", "Plan", "SlaterLogDet", "slater_logdet", "mode_id"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
