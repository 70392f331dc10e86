"""CPU oracle for the statically condensed HDG operator (Huismann, Stiller,
Froehlich, arXiv:2007.11891), in plain numpy/scipy, FP64.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The GPU library never does, and this package shares no code with
it: the oracle assembles the dense element LDG system (paper, equation
(ldg_element_operator_threed) with Table 1), forms the trace Schur complement
explicitly (equation (hdg_operator)), and solves the condensed system with a
dense or sparse direct solver.

Modules:
  basis     - GLL points, Lagrange basis, 1D standard matrices
  layout    - canonical trace / volume numbering and node coordinates
  element   - dense element system and K_e (F_e and recovery: system)
  system    - global assembly, Dirichlet elimination, solve, adjoint
  fastdiag  - the paper's factorised operator, used only to pin its claims
  pcg       - the paper's nodal-basis CG solvers (no, diagonal, block
              preconditioner) by definition, for the solver comparison

Every function is pinned by tests in ``tests/test_oracle_*.py`` against closed
forms, invariants and exactness properties of the discretisation.
"""
from .basis import gll_nodes_weights, standard_matrices  # noqa: F401
from .layout import Layout  # noqa: F401
from .element import element_operator, ElementSystem  # noqa: F401
from .system import HdgOracle  # noqa: F401
