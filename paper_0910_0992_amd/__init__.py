"""Temporally preconditioned anisotropic Wilson / SW fermion solver for MI355X.

A thin Python layer over the C ABI of libtprec.so (include/tprec.h): it only
marshals torch tensors (device memory) and the current HIP stream into the
library's entry points.  Every step of the operator and the solver runs in the
hand-written HIP kernels; there is no CPU fallback.

    op = Operator(links, m0=-0.05, gamma_f=3.0, c_s=1.6/3, c_t=1.0, bc_t=-1)
    x, info = op.solve(eta, scheme="TEMPORAL_SCHUR", prec="F32")

Fields are torch complex128 CUDA tensors in the canonical layout:
spinors [Lt][Lz][Ly][Lx][4][3] (Dirac-Pauli basis), links [4][Lt][Lz][Ly][Lx][3][3]
with direction 0=x, 1=y, 2=z, 3=t.
"""
from .api import Field, Operator, SolveFn, solve
from ._lib import TprecError, SCHEMES, SOLVERS, PRECS

__all__ = ["Field", "Operator", "SolveFn", "solve", "TprecError", "SCHEMES", "SOLVERS", "PRECS"]
