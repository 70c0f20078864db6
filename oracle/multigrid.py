"""Recursive V-cycle (paper Alg. 1) used as the preconditioner W of Section 4.

The V-cycle runs on the penalised matrix L~ at every level, with operators
re-discretised on the coarsened domain (Section 2; label coarsening of
Section 5) and an exact solve at the coarsest level.  As a preconditioner it
is called with a zero initial guess, which makes t = V-CYCLE(L~, s, 0, n)
linear in s (Section 3).

Reading (smoothing counts): the pre- and post-smoothing steps are `nu`
applications of Alg. 3 each; the default nu = 1 holds one symmetric DGS
(a forward and a reverse sweep) per smoothing step, as in Section 6 where the
interior DGS is applied once per V-cycle phase.
Reading (levels): with levels = 0 the hierarchy halves every axis while all
axes are even and every halved axis keeps at least 4 cells; an explicit
level count may go down to 2 cells per axis.
"""
from __future__ import annotations

import numpy as np

from .domain import Domain, box_labels
from .operator import apply_operator, assemble, from_vector, residual, to_vector, zeros_like_state
from .smoother import dgs_diagonals, smooth
from .transfer import prolong, restrict


def auto_levels(dims, min_cells: int = 4) -> int:
    levels, d = 1, list(dims)
    while all(n % 2 == 0 and n // 2 >= min_cells for n in d):
        d = [n // 2 for n in d]
        levels += 1
    return levels


def max_levels(dims) -> int:
    """Deepest hierarchy allowed when levels are given explicitly: every
    coarsening needs even axes and leaves at least 2 cells per axis."""
    return auto_levels(dims, 2)


class Hierarchy:
    """Levels 0 (finest) .. levels-1 (coarsest) of a box domain."""

    def __init__(self, dims, h, eta=1.0, gamma=1e-3, levels=0, nu=1, n_boundary=1):
        if levels == 0:
            levels = auto_levels(dims)
        if levels < 1 or levels > max_levels(dims):
            raise ValueError("too many levels for these dimensions")
        self.nu, self.n_boundary = nu, n_boundary
        self.doms = [Domain(box_labels(dims), h, eta, gamma)]
        for _ in range(levels - 1):
            self.doms.append(self.doms[-1].coarsen())
        self.diags = [dgs_diagonals(d) for d in self.doms[:-1]]
        self.coarse_matrix = assemble(self.doms[-1], self.doms[-1].gamma, dense=True)

    @property
    def levels(self):
        return len(self.doms)

    def coarse_solve(self, b):
        """Exact solve at the coarsest level (Alg. 1, n = 1): LAPACK LU."""
        dom = self.doms[-1]
        return from_vector(dom, np.linalg.solve(self.coarse_matrix, to_vector(dom, b)))


def vcycle(H: Hierarchy, b, level: int = 0):
    """t = V-CYCLE(L~, b, 0, levels - level) of Alg. 1."""
    if level == H.levels - 1:
        return H.coarse_solve(b)
    dom, coarse = H.doms[level], H.doms[level + 1]
    x = zeros_like_state(dom)
    for _ in range(H.nu):
        x = smooth(dom, x, b, H.n_boundary, H.diags[level])
    r = residual(dom, x, b, dom.gamma)
    e = vcycle(H, restrict(dom, coarse, r), level + 1)
    x = tuple(v + dv for v, dv in zip(x, prolong(dom, coarse, e)))
    for _ in range(H.nu):
        x = smooth(dom, x, b, H.n_boundary, H.diags[level])
    return x


def apply_L(H: Hierarchy, x):
    """The system matrix L of Eq. 2 (no penalty) on the finest level."""
    return apply_operator(H.doms[0], x, 0.0)
