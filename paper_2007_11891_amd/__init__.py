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
    TIME_ELEM_APPLY_F64, TIME_ELEM_APPLY_F32, TIME_CG2_ITER_F64, TIME_CG2_ITER_F32,
    TIME_CG2_APPLY_F64, TIME_CG2_UPDATE_F64, TIME_CG2_APPLY_F32, TIME_CG2_UPDATE_F32, TIME_COPY_F64,
    TIME_CG1_ITER_F64, TIME_CG1_ITER_F32, TIME_CG1_GRAPH_F64, TIME_CG1_GRAPH_F32,
    TIME_NODAL_UNPREC_F64, TIME_NODAL_DIAG_F64, TIME_NODAL_BLOCK_F64, TIME_APPLY_F64, TIME_APPLY_F32,
    TIME_PENCIL_ITER_F64, TIME_PENCIL_ITER_F32,
)
