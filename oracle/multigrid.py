"""Recursive V-cycle (paper Alg. 1) used as the preconditioner W of Section 4.

The V-cycle runs on the penalised matrix L~ at every level, with operators
re-discretised on the coarsened domain (Section 2; label coarsening of
Section 5) and an exact solve at the coarsest level.  As a preconditioner it
is called with a zero initial guess, which makes t = V-CYCLE(L~, s, 0, n)
linear in s (Section 3).

Smoothing schedules.  `nu` counts DGS sweeps per smoothing phase (a
"sweep" is one directional pass, Section 3.1), so nu = 2 is "2 pre / 2 post".
  * "symmetric" (default) - the paper's choice (Section 3): the same
    symmetric smoother in both phases, Alg. 3 applied nu/2 times, each with
    one symmetric DGS (forward sweep on L M, Eq. dist, then reverse sweep on
    M^T L, Eq. ldist).
  * "split" - the other arrangement Section 3 allows: different smoothers in
    the two phases whose matrices are transposes of each other.  Pre-smoothing
    is Alg. 3 with nu reverse sweeps on V2, post-smoothing Alg. 3 with nu
    forward sweeps; the reverse sweep's error propagator is the L~-adjoint of
    the forward sweep's, symmetric Vanka is L~-self-adjoint, so the pair meets
    the transpose condition and W stays symmetric.
`order` is the DGS pressure traversal (smoother.pressure_classes): the eight
colour classes by default; with red/black pressures the "symmetric" schedule
loses its grid independence (a forward-then-reverse pair amplifies smooth
interior pressure modes) and only "split" converges well.
Reading (levels): with levels = 0 the hierarchy halves every axis while all
axes are even and every halved axis keeps at least 4 cells; an explicit
level count may go down to 2 cells per axis.

Variants.  `vanka` picks the V1 smoother (smoother.vanka_apply: the paper's
8-colour symmetric multiplicative Vanka, a 27-colour one, or additive Vanka,
Eq. av).  `cycle` = 2 makes the W-cycle the paper mentions (Section 2,
compared with the V-cycle in the appendix experiments): the coarse
correction of every non-coarsest level is two cycles on the next level, the
second starting from the first's result.
"""
from __future__ import annotations

import numpy as np

from .domain import Domain, box_labels
from .operator import apply_operator, assemble, from_vector, residual, to_vector, zeros_like_state
from .smoother import PRESSURE_ORDERS, dgs_diagonals, dgs_forward, dgs_reverse, smooth
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

    def __init__(self, dims, h, eta=1.0, gamma=1e-3, levels=0, nu=2, n_boundary=1, schedule="symmetric",
                 vanka="mult8", cycle=1, order="c8", labels=None):
        """`labels`: optional (nx+2, ny+2, nz+2) cell labels of Section 5 (a box
        padded by Dirichlet cells when None); `dims` must match them."""
        if labels is not None and tuple(s - 2 for s in labels.shape) != tuple(dims):
            raise ValueError("labels do not match dims")
        if levels == 0:
            levels = auto_levels(dims)
        if levels < 1 or levels > max_levels(dims):
            raise ValueError("too many levels for these dimensions")
        if schedule not in ("split", "symmetric") or nu < 1 or (schedule == "symmetric" and nu % 2):
            raise ValueError("bad smoothing schedule")
        if vanka not in ("mult8", "mult27", "additive") or cycle not in (1, 2):
            raise ValueError("bad smoother variant or cycle")
        if order not in PRESSURE_ORDERS:
            raise ValueError("bad DGS pressure order")
        self.nu, self.n_boundary, self.schedule, self.order = nu, n_boundary, schedule, order
        self.vanka, self.cycle = vanka, cycle
        self.doms = [Domain(box_labels(dims) if labels is None else np.asarray(labels, dtype=np.int8), h, eta, gamma)]
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


def vcycle(H: Hierarchy, b, level: int = 0, x=None):
    """t = V-CYCLE(L~, b, x, levels - level) of Alg. 1 (x = 0 unless given);
    a W-cycle when H.cycle = 2."""
    if level == H.levels - 1:
        return H.coarse_solve(b)
    dom, coarse = H.doms[level], H.doms[level + 1]
    x = zeros_like_state(dom) if x is None else x
    x = presmooth(H, level, x, b)
    r = residual(dom, x, b, dom.gamma)
    bc = restrict(dom, coarse, r)
    e = None
    for _ in range(H.cycle):
        e = vcycle(H, bc, level + 1, e)
    x = tuple(v + dv for v, dv in zip(x, prolong(dom, coarse, e)))
    return postsmooth(H, level, x, b)


def _sweeps(sweep, k, order):
    def interior(dom, x, b, diags):
        for _ in range(k):
            x = sweep(dom, x, b, diags, order)
        return x
    return interior


def presmooth(H: Hierarchy, level: int, x, b):
    dom, diags = H.doms[level], H.diags[level]
    if H.schedule == "symmetric":
        for _ in range(H.nu // 2):
            x = smooth(dom, x, b, H.n_boundary, diags, vanka=H.vanka, order=H.order)
        return x
    return smooth(dom, x, b, H.n_boundary, diags, _sweeps(dgs_reverse, H.nu, H.order), vanka=H.vanka)


def postsmooth(H: Hierarchy, level: int, x, b):
    dom, diags = H.doms[level], H.diags[level]
    if H.schedule == "symmetric":
        for _ in range(H.nu // 2):
            x = smooth(dom, x, b, H.n_boundary, diags, vanka=H.vanka, order=H.order)
        return x
    return smooth(dom, x, b, H.n_boundary, diags, _sweeps(dgs_forward, H.nu, H.order), vanka=H.vanka)


def apply_L(H: Hierarchy, x):
    """The system matrix L of Eq. 2 (no penalty) on the finest level."""
    return apply_operator(H.doms[0], x, 0.0)
