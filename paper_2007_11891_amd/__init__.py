"""MI355X (gfx950) library for the matrix-free statically condensed HDG
operator of Huismann, Stiller & Froehlich (arXiv:2007.11891) and the
preconditioned CG solve around it.

The computation lives in the HIP library ``libhdg.so`` (C ABI in
``include/hdg.h``); this package holds its ctypes binding, a
``torch.autograd.Function`` for the adjoint, and the build script.
"""
from .hdg import (  # noqa: F401
    HdgBatch, HdgContext, HdgError, SolveOpts, default_opts, layout, load_library, tables, LIB_PATH,
    EXPORTS,
    TO_EIGEN_UNKNOWN, TO_EIGEN_RESIDUAL, TO_NODAL_UNKNOWN, TO_NODAL_RESIDUAL,
    PRECOND_NONE, PRECOND_EIGEN_JACOBI, PRECOND_NODAL_DIAG, PRECOND_NODAL_BLOCK,
)
