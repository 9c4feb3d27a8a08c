"""MI355X-native DG solver for the rain-augmented shallow water equations.

The compute path is the HIP library ``libdgswe.so`` (C ABI in
``include/dgswe.h``); this package only marshals arguments to it.
"""
from .solver import Solver, Batch, params_from_dict  # noqa: F401
from .serve import Server, Request, latency_summary  # noqa: F401
