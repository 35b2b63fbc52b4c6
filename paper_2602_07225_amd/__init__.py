"""MI355X (gfx950) solver for the linearized pseudo-4D DFN battery Jacobian
(arXiv 2602.07225): FGMRES with a block preconditioner built from exact
per-node particle eliminations, a surface Schur coupling and geometric
multigrid V-cycles for the electrode-level fields; block Jacobi and block
Gauss-Seidel preconditioners, a Krylov space reduced to the Schur complement
of the particle blocks, batched cells, and Newton steps of the physical cell
around the linear solve.

All numerical work runs in the HIP library ``libp4d.so``; this package only
marshals torch tensors to its C ABI (``include/p4d.h``)."""
from . import _lib
from ._lib import (P4D_FP32, P4D_FP64, P4D_PC_BGS, P4D_PC_BJ, P4D_PC_SCHUR, P4DError, default_opts,
                   desc_from)
from .solver import P4DBatch, P4DSolver, PhysCell
from .autograd import P4DSolve, solve

__all__ = ["_lib", "P4DSolver", "P4DBatch", "PhysCell", "P4DSolve", "solve", "P4DError", "default_opts",
           "desc_from", "P4D_PC_SCHUR", "P4D_PC_BJ", "P4D_PC_BGS", "P4D_FP64", "P4D_FP32"]
