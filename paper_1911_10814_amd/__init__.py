"""MI355X (gfx950) nested block solver for the Newton-step linear system of
the VMS / generalized-alpha incompressible Navier-Stokes discretisation.

The computation lives in the HIP library ``libns_hip.so`` (C ABI in
``include/ns_api.h``); this package only marshals arguments and uses PyTorch
for device memory and streams.
"""
from .solver import NestedSolveFn, NsContext, SolveOptions, context_for, gen_alpha, stream_bench  # noqa: F401
from ._lib import NsError, load  # noqa: F401
