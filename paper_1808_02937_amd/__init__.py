"""MI355X (gfx950) fast solver for the SEM discretisation of the 1-D two-sided
Riemann-Liouville fractional diffusion equation with an H-LU preconditioner.

All numerical work runs in the HIP library libfde.so (C ABI in include/fde.h);
this package only marshals arguments and owns device buffers through PyTorch.
"""
from ._abi import FDEError, load  # noqa: F401
from .fde import (Context, HLU, HMatrix, Operator, Server, factor_batched, gauss_jacobi,  # noqa: F401
                  plan_hlu, sigma_estimate, solve, solve_batched)
