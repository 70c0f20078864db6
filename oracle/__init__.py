"""Plain FP64 CPU oracle for multigrid-preconditioned SQMR on the 3D MAC Stokes system.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path never does.  It shares no code with the GPU library.

Paper: Tao & Sifakis, "A Symmetric Multigrid-Preconditioned Krylov Subspace
Solver for Stokes Equations" (arXiv 2312.10615).  Each function cites the
section, equation or algorithm it follows.  Readings taken where the paper
is silent or ambiguous are marked "Reading:" in the docstrings.

Representation: a state is a tuple (ux, uy, uz, p) of float64 arrays indexed
[i, j, k] (i along x).  ux has shape (nx+1, ny, nz) with ux[i] on the face
x = i*h (faces 0 and nx are walls, always zero); uy, uz analogous; p has shape
(nx, ny, nz) at cell centres.  Entries that are not unknowns are zero.

Parity status: every function here is pinned by a `-m "not gpu"` test
(tests/test_oracle_*.py) except the iteration counts and residual histories of
complete solves, which the paper only shows in figures that are absent from
its text ("parity unpinned" for those two quantities; the iterates themselves
are pinned by the dense-solve and symmetry tests).
"""

from .domain import Domain, box_labels, coarsen_labels, classify, dof_counts  # noqa: F401
from .operator import apply_operator, residual, assemble, to_vector, from_vector, zeros_like_state  # noqa: F401
from .transfer import prolong, restrict  # noqa: F401
from .smoother import (dgs_forward, dgs_reverse, dgs_symmetric, vanka_color, vanka_symmetric,  # noqa: F401
                       smooth, vanka_local_matrix)
from .multigrid import Hierarchy, vcycle  # noqa: F401
from .sqmr import sqmr, mg_sqmr  # noqa: F401
