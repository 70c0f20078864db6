"""The discrete Stokes operator on the MAC grid (paper Section 2, Eq. 2) and the
penalised preconditioner matrix of Section 4.

    L  = [[A, B^T], [B, 0]],      L~ = [[A, B^T], [B, -gamma I]]

A is -eta times the 7-point Laplacian on each velocity lattice, B^T is the
central-difference gradient of the pressure onto faces and B is minus the
central-difference divergence of the velocity onto cells.

Reading (scaling): the physical scaling is used, A = (eta/h^2) * (6 u -
sum of the six lattice neighbours), (B^T p)_face = (p_plus - p_minus)/h,
(B u)_cell = -(1/h) * sum over axes of (u_plus_face - u_minus_face).  With it
the restriction R = P^T/8 of Section 2 gives coarse equations that agree with
the re-discretised coarse operator.  Neighbours that are not unknowns
(Dirichlet faces, including the tangential ghost at the face centre of a
Dirichlet cell) hold zero and are simply dropped, so the diagonal stays
6 eta/h^2.  Homogeneous Dirichlet data only; non-zero data belongs in b.
Next to exterior cells (Section 5's Neumann faces) the pressure of an
exterior cell is zero and a velocity neighbour on the exterior side is
dropped from the diagonal as well (zero normal derivative, Domain.ndiag).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .domain import Domain


def zeros_like_state(dom: Domain):
    return tuple(np.zeros(s) for s in dom.shapes)


def masked(dom: Domain, x):
    """Zero every entry of x that is not an unknown."""
    return tuple(np.where(m, v, 0.0) for m, v in zip(dom.active, x))


def grad(dom: Domain, p: np.ndarray):
    """B^T p: (p[cell on + side] - p[cell on - side]) / h at active faces."""
    h = dom.h
    out = []
    for a in range(3):
        pad = [(0, 0)] * 3
        pad[a] = (1, 1)
        pp = np.pad(p, pad)
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[a] = slice(1, None)
        lo[a] = slice(0, -1)
        g = (pp[tuple(hi)] - pp[tuple(lo)]) / h
        out.append(np.where(dom.active[a], g, 0.0))
    return out


def neg_div(dom: Domain, u):
    """B u: -(1/h) * sum_a (u_a[face a+1] - u_a[face a]) at active cells."""
    h = dom.h
    acc = np.zeros(dom.shapes[3])
    for a in range(3):
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[a] = slice(1, None)
        lo[a] = slice(0, -1)
        acc += u[a][tuple(hi)] - u[a][tuple(lo)]
    return np.where(dom.active[3], -acc / h, 0.0)


def viscous(dom: Domain, u_a: np.ndarray, a: int):
    """A on one velocity component: (eta/h^2)(n_f u - sum of the lattice
    neighbours), n_f = 6 except next to exterior cells (Domain.ndiag)."""
    c = dom.eta / dom.h ** 2
    up = np.pad(np.where(dom.active[a], u_a, 0.0), 1)
    core = up[1:-1, 1:-1, 1:-1]
    nb = (up[2:, 1:-1, 1:-1] + up[:-2, 1:-1, 1:-1] + up[1:-1, 2:, 1:-1]
          + up[1:-1, :-2, 1:-1] + up[1:-1, 1:-1, 2:] + up[1:-1, 1:-1, :-2])
    return np.where(dom.active[a], c * (dom.ndiag[a] * core - nb), 0.0)


def apply_operator(dom: Domain, x, gamma: float = 0.0):
    """y = L x (gamma = 0) or y = L~ x (gamma = the penalty), Eq. 2 / Section 4."""
    x = masked(dom, x)
    g = grad(dom, x[3])
    y = [viscous(dom, x[a], a) + g[a] for a in range(3)]
    y.append(neg_div(dom, x[:3]) - np.where(dom.active[3], gamma * x[3], 0.0))
    return tuple(y)


def residual(dom: Domain, x, b, gamma: float):
    y = apply_operator(dom, x, gamma)
    return tuple(np.where(m, bb - yy, 0.0) for m, bb, yy in zip(dom.active, b, y))


def continuity_residual(dom: Domain, x, b, gamma: float):
    """The pressure rows of `residual` alone: b_p - (B u - gamma p)."""
    x = masked(dom, x)
    y = neg_div(dom, x[:3]) - np.where(dom.active[3], gamma * x[3], 0.0)
    return np.where(dom.active[3], b[3] - y, 0.0)


def to_vector(dom: Domain, x) -> np.ndarray:
    """Active entries of (ux, uy, uz, p), each in C order, concatenated."""
    return np.concatenate([v[m] for m, v in zip(dom.active, x)])


def from_vector(dom: Domain, v: np.ndarray):
    out, pos = [], 0
    for m, s in zip(dom.active, dom.shapes):
        a = np.zeros(s)
        cnt = int(m.sum())
        a[m] = v[pos:pos + cnt]
        pos += cnt
        out.append(a)
    return tuple(out)


def assemble(dom: Domain, gamma: float = 0.0, dense: bool = False):
    """Matrix of L (or L~) in the `to_vector` ordering, built column by column
    from the matrix-free operator (small grids only)."""
    n = dom.n_dofs()
    cols = []
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        cols.append(to_vector(dom, apply_operator(dom, from_vector(dom, e), gamma)))
        e[j] = 0.0
    m = np.stack(cols, axis=1)
    return m if dense else sp.csr_matrix(m)


def lid_lift(dom: Domain, velocity: float):
    """Right-hand side of a lid: the top wall (the plus-z side) moves along x
    with `velocity`, every other wall is at rest (the driven cavity of
    Section 6).  The paper moves Dirichlet values to the right-hand side
    (Section 5); with the tangential ghost value at the Dirichlet cell's face
    centre (first order), the u_x faces of the top cell row have the lid's
    u_x as their +z lattice neighbour, so each of their rows gains
    (eta / h^2) * velocity.  Returns the state to add to b (zero elsewhere)."""
    nx, ny, nz = dom.dims
    bx = np.zeros(dom.shapes[0])
    bx[:, :, nz - 1] = dom.eta / dom.h ** 2 * velocity
    bx = np.where(dom.active[0], bx, 0.0)
    return bx, np.zeros(dom.shapes[1]), np.zeros(dom.shapes[2]), np.zeros(dom.shapes[3])
