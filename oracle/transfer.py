"""Grid transfer operators (paper Section 2).

Prolongation P: bilinear (in 3D, trilinear) interpolation of each velocity
component on its own staggered lattice, and constant per-cell interpolation
of the pressure.  Restriction R = P^T / c with c = 8 in 3D, which makes both
operators a partition of unity away from walls.

Reading (the stencil figure is missing): on the lattice of u_a,
  * along axis a (face lattice), a fine face that coincides with a coarse face
    takes weight 1 from it, a fine face midway between two coarse faces takes
    1/2 from each;
  * along each other axis (cell-centre lattice), a fine cell row takes 3/4 from
    the coarse row that contains it and 1/4 from the next coarse row on its
    side (the one whose centre is 3h/2 away);
  * coarse values outside the coarse unknowns (walls, Dirichlet ghosts) are
    zero for a correction, so their weights are dropped.
The 3D weights are products of the 1D weights.
"""
from __future__ import annotations

import numpy as np

from .domain import Domain


def _face_lattice_1d(n_fine: int) -> np.ndarray:
    """1D interpolation matrix for face positions 0..n_fine from 0..n_fine/2."""
    nc = n_fine // 2
    m = np.zeros((n_fine + 1, nc + 1))
    for i in range(n_fine + 1):
        if i % 2 == 0:
            m[i, i // 2] = 1.0
        else:
            m[i, i // 2] = 0.5
            m[i, i // 2 + 1] = 0.5
    return m


def _cell_lattice_1d(n_fine: int) -> np.ndarray:
    """1D interpolation matrix for cell centres 0..n_fine-1 from 0..n_fine/2-1."""
    nc = n_fine // 2
    m = np.zeros((n_fine, nc))
    for j in range(n_fine):
        near = j // 2
        far = near - 1 if j % 2 == 0 else near + 1
        m[j, near] = 0.75
        if 0 <= far < nc:
            m[j, far] = 0.25
    return m


def _constant_1d(n_fine: int) -> np.ndarray:
    nc = n_fine // 2
    m = np.zeros((n_fine, nc))
    for j in range(n_fine):
        m[j, j // 2] = 1.0
    return m


def _matrices(fine: Domain, field_index: int):
    dims = fine.dims
    if field_index == 3:
        return [_constant_1d(n) for n in dims]
    return [_face_lattice_1d(n) if a == field_index else _cell_lattice_1d(n) for a, n in enumerate(dims)]


def prolong(fine: Domain, coarse: Domain, e):
    """e_fine = P e_coarse."""
    out = []
    for f in range(4):
        mx, my, mz = _matrices(fine, f)
        ec = np.where(coarse.active[f], e[f], 0.0)
        ef = np.einsum("ia,abc->ibc", mx, ec)
        ef = np.einsum("jb,ibc->ijc", my, ef)
        ef = np.einsum("kc,ijc->ijk", mz, ef)
        out.append(np.where(fine.active[f], ef, 0.0))
    return tuple(out)


def restrict(fine: Domain, coarse: Domain, r):
    """r_coarse = R r_fine = P^T r_fine / 8."""
    out = []
    for f in range(4):
        mx, my, mz = _matrices(fine, f)
        rf = np.where(fine.active[f], r[f], 0.0)
        rc = np.einsum("ia,ijk->ajk", mx, rf)
        rc = np.einsum("jb,ajk->abk", my, rc)
        rc = np.einsum("kc,abk->abc", mz, rc) / 8.0
        out.append(np.where(coarse.active[f], rc, 0.0))
    return tuple(out)
