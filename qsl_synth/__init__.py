"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This package only draws random numbers and lays them out; it contains none
of the method's arithmetic (no normalisation, no screening, no AO values, no
products, no determinants).
"""
from .gen import (CONFIGS, dmc_randoms, localize_mos, make_config, make_mos, make_system, make_walkers,  # noqa: F401
                  nuclear_charges)
