"""Discrete domain description (paper Section 5, "Discrete Domain Design").

Every cell carries a label: interior, Dirichlet or exterior.  From the labels
the paper derives which variables are unknowns:
  * a velocity on a face of a Dirichlet cell is a Dirichlet value (not solved);
  * a velocity on the face between two interior cells is active;
  * a velocity on the face between an interior and an exterior cell carries a
    Neumann condition; reading: it is an unknown too (its momentum row sees
    zero pressure in the exterior cell and zero-Neumann velocity stencils);
  * faces with no interior cell and no Dirichlet cell are outside the solve;
  * a pressure at an interior cell centre is active.
Coarse labels: a coarse cell is Dirichlet if it encloses any fine Dirichlet
cell, otherwise interior if it encloses any fine interior cell, otherwise
exterior.  The boundary set V1 holds all degrees of freedom of the cells that
are proximal to a Dirichlet or exterior cell; V2 holds the rest.

Readings, both pinned by Table 1: the rows of the 2D cylinder channel (no-slip
walls and obstacle, an outflow of exterior cells) come out exactly, total and
boundary DOFs at all four resolutions, when (a) interior-exterior faces are
unknowns, and (b) "proximal" means within one cell (sharing a face, edge or
corner) of a Dirichlet cell or within two cells of an exterior cell.  For a
box padded by Dirichlet cells (b) is the face-sharing rule, which reproduces
the driven-cavity rows.

The labelled arrays are padded: padded index = cell index + 1, so a box of n
cells per axis has label arrays of n+2 per axis whose outer layer is
Dirichlet.  Classification is written for any dimension d (2 or 3) so that
both the 2D and 3D rows of Table 1 can be checked.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INTERIOR, DIRICHLET, EXTERIOR = 0, 1, 2


def box_labels(dims) -> np.ndarray:
    """Labels of a box of `dims` interior cells padded by one Dirichlet layer."""
    lab = np.full(tuple(n + 2 for n in dims), DIRICHLET, dtype=np.int8)
    lab[tuple(slice(1, n + 1) for n in dims)] = INTERIOR
    return lab


def coarsen_labels(lab: np.ndarray) -> np.ndarray:
    """Label coarsening of Section 5.

    Coarse cell I covers fine cells 2I and 2I+1 (cell indices).  In padded
    indices this means coarse padded index c covers fine padded 2c-1 and 2c;
    an extra layer repeating the outer layer stands in for the fine cells
    beyond the padding (a padding of exterior cells stays exterior).
    """
    d = lab.ndim
    dims = [s - 2 for s in lab.shape]
    if any(n % 2 for n in dims):
        raise ValueError("label coarsening needs an even number of cells per axis")
    ext = np.pad(lab, 1, mode="edge")  # ext index = padded + 1
    cdims = [n // 2 for n in dims]
    # fine padded indices 2c-1, 2c  ->  ext indices 2c, 2c+1, for c = 0 .. n/2+1
    blocks = ext.reshape(tuple(x for n in cdims for x in (n + 2, 2)))
    axes = tuple(2 * a + 1 for a in range(d))
    any_dir = (blocks == DIRICHLET).any(axis=axes)
    any_int = (blocks == INTERIOR).any(axis=axes)
    out = np.where(any_dir, DIRICHLET, np.where(any_int, INTERIOR, EXTERIOR)).astype(np.int8)
    return out


def _dilate(mask: np.ndarray, reach: int) -> np.ndarray:
    """Cells within `reach` steps of `mask`, a step reaching all 3^d - 1 cells
    that share a face, edge or corner (no wrap-around at the array ends)."""
    d = mask.ndim
    out = mask.copy()
    for _ in range(reach):
        pad = np.pad(out, 1, constant_values=False)
        nxt = out.copy()
        for off in np.ndindex(*(3,) * d):
            nxt |= pad[tuple(slice(o, o + n) for o, n in zip(off, out.shape))]
        out = nxt
    return out


def classify(lab: np.ndarray):
    """Active masks and V1 masks for every velocity component and the pressure.

    Returns (active, v1) where each is a list of d boolean arrays for the face
    fields (face field for axis a has n_a+1 entries along a) followed by one
    boolean array for the pressure (cell field).  V2 = active & ~v1.
    """
    d = lab.ndim
    dims = [s - 2 for s in lab.shape]
    inner = tuple(slice(1, n + 1) for n in dims)
    interior = lab == INTERIOR
    dirichlet = lab == DIRICHLET
    cell_active = interior[inner]

    prox = (_dilate(dirichlet, 1) | _dilate(lab == EXTERIOR, 2)) & interior
    cell_v1 = prox[inner]

    face_active, face_v1 = [], []
    for a in range(d):
        # face f (0..n_a) along axis a separates cells f-1 and f -> padded f and f+1
        lo = [slice(1, n + 1) for n in dims]
        hi = [slice(1, n + 1) for n in dims]
        lo[a] = slice(0, dims[a] + 1)
        hi[a] = slice(1, dims[a] + 2)
        lo, hi = tuple(lo), tuple(hi)
        act = (interior[lo] | interior[hi]) & ~dirichlet[lo] & ~dirichlet[hi]
        face_active.append(act)
        face_v1.append(act & (prox[lo] | prox[hi]))
    return face_active + [cell_active], face_v1 + [cell_v1]


def viscous_diagonals(lab: np.ndarray):
    """For each velocity component, the count n_f of lattice neighbours that
    enter the diagonal of A at face f: A u_f = (eta/h^2)(n_f u_f - sum of the
    neighbours that are unknowns).

    Reading (zero Neumann): a lattice neighbour that is an unknown or a
    Dirichlet value counts (a Dirichlet value sits in the right-hand side); a
    neighbour with no interior and no Dirichlet cell beside it lies on the
    exterior side of a Neumann boundary, and the zero normal derivative there
    sets it equal to u_f, which removes it from both sides of the stencil.
    Inside a Dirichlet box every n_f is 6.  Labels beyond the array repeat its
    outer layer."""
    if lab.ndim != 3:
        raise ValueError("3D labels only")
    dims = [s - 2 for s in lab.shape]
    ext = np.pad(lab, 1, mode="edge")          # ext index = padded index + 1 = cell index + 2
    out = []
    for a in range(3):
        # kinds of the lattice positions of u_a for face index -1..n_a+1 and cell index -1..n
        lo = [slice(1, n + 3) for n in dims]
        hi = [slice(1, n + 3) for n in dims]
        lo[a] = slice(0, dims[a] + 3)
        hi[a] = slice(1, dims[a] + 4)
        L, H = ext[tuple(lo)], ext[tuple(hi)]
        counts = ((L == DIRICHLET) | (H == DIRICHLET) | (L == INTERIOR) | (H == INTERIOR)).astype(np.int64)
        n = np.zeros(tuple(dims[b] + (1 if b == a else 0) for b in range(3)), dtype=np.int64)
        core = tuple(slice(1, m - 1) for m in counts.shape)
        for b in range(3):
            for sgn in (-1, 1):
                sl = list(core)
                sl[b] = slice(1 + sgn, counts.shape[b] - 1 + sgn)
                n += counts[tuple(sl)]
        out.append(n)
    return out


def dof_counts(lab: np.ndarray):
    """(#active DOFs, #V1 DOFs) - the two integer columns of Table 1."""
    active, v1 = classify(lab)
    return int(sum(m.sum() for m in active)), int(sum(m.sum() for m in v1))


@dataclass
class Domain:
    """One level of the hierarchy: a labelled 3D grid of spacing h.

    Holds the constants of the discrete Stokes operator (Eq. 2): viscosity
    eta and the penalty gamma of the preconditioner matrix (Section 4).  The
    outer layer of the labels must hold no interior cell.
    """
    labels: np.ndarray
    h: float
    eta: float = 1.0
    gamma: float = 1e-3
    active: list = field(init=False)
    v1: list = field(init=False)
    v2: list = field(init=False)
    ndiag: list = field(init=False)

    def __post_init__(self):
        if self.labels.ndim != 3:
            raise ValueError("the oracle's Stokes operator is 3D")
        inner = self.labels[1:-1, 1:-1, 1:-1]
        if (self.labels == INTERIOR).sum() != (inner == INTERIOR).sum():
            raise ValueError("the outer layer of the labels must hold no interior cell")
        self.active, self.v1 = classify(self.labels)
        self.v2 = [a & ~v for a, v in zip(self.active, self.v1)]
        self.ndiag = viscous_diagonals(self.labels)

    @property
    def has_neumann(self):
        """True when some unknown face borders an exterior cell (the pressure is
        then unique: exterior pressures are zero)."""
        ext = self.labels == EXTERIOR
        inter = self.labels == INTERIOR
        for a in range(3):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[a] = slice(0, -1)
            hi[a] = slice(1, None)
            if ((ext[tuple(lo)] & inter[tuple(hi)]) | (inter[tuple(lo)] & ext[tuple(hi)])).any():
                return True
        return False

    @property
    def dims(self):
        return tuple(s - 2 for s in self.labels.shape)

    @property
    def shapes(self):
        nx, ny, nz = self.dims
        return [(nx + 1, ny, nz), (nx, ny + 1, nz), (nx, ny, nz + 1), (nx, ny, nz)]

    def n_dofs(self):
        return int(sum(m.sum() for m in self.active))

    def coarsen(self):
        return Domain(coarsen_labels(self.labels), 2.0 * self.h, self.eta, self.gamma)

    def parity(self, field_index: int) -> np.ndarray:
        """Red (0) / black (1) colour of every entry of a field: (i+j+k) mod 2
        in the field's own index (face number along its normal axis, cell
        numbers along the others)."""
        shp = self.shapes[field_index]
        i, j, k = np.ogrid[0:shp[0], 0:shp[1], 0:shp[2]]
        return ((i + j + k) & 1).astype(np.int8)

    def vanka_colour(self, period: int = 2) -> np.ndarray:
        """Colour class of every cell: (i mod q) + q (j mod q) + q^2 (k mod q).
        q = 2 is the paper's 8-colour scheme (Section 6); with q = 3 (27
        classes) same-class cells are three apart and share no stencil entry."""
        nx, ny, nz = self.dims
        i, j, k = np.ogrid[0:nx, 0:ny, 0:nz]
        q = period
        return ((i % q) + q * (j % q) + q * q * (k % q)).astype(np.int16)
