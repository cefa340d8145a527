"""FP64 CPU oracle for the Slater-matrix build (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this package.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    build, load, OracleSystem, n_basis, normalize, cart_factor, ao_eval,
    lu_inverse, forward, backward, max_threads,
    jastrow_potential, local_energy, drift_diffuse, branch_weights, reconfigure, multidet,
)
