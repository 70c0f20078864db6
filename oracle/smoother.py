"""Smoothers of paper Section 3: symmetric distributive Gauss-Seidel on the
interior set V2, symmetric multiplicative Vanka on the boundary set V1, and
their symmetric composition (Alg. 3).  All of them act on the penalised matrix
L~ of Section 4 (the V-cycle only ever sees L~).

Every smoother is written as the relaxation x <- x + S (b - L~ x) of Eq.
relaxation, one colour class at a time, with the residual recomputed before
each class (in full for DGS; for Vanka its rows at the class's local
unknowns, pinned against the full residual).  Inside one colour class the updates do not influence each
other's residuals (checked by a test that runs the literal one-unknown-at-a-
time loop of Alg. 2), so applying a class at once equals visiting its members
in any order.
"""
from __future__ import annotations

import numpy as np

from .domain import Domain
from .operator import apply_operator, continuity_residual, grad, neg_div, residual


# ---------------------------------------------------------------------------
# Distribution matrix (Eq. dist): M = [[I, -B^T], [0, eta B B^T]].
#
# Reading: DGS on V2 is Alg. 2 with the loop over the V2 unknowns only; each
# update moves x along the full column m_j of the global M.  For a V2 cell
# that column is the interior stencil (all six faces and six neighbours are
# unknowns), which is where L M has the block-triangular form of Eq. disc -
# the reason Section 3.1 keeps DGS away from the boundary.  A pressure update
# therefore also moves the faces it shares with V1 cells and the pressures of
# V1 neighbours.  Symmetry is unaffected: Appendix A's argument holds for the
# rectangular M of the V2 columns, and every stage of Alg. 3 keeps an
# L~-self-adjoint error propagator.
# ---------------------------------------------------------------------------

def distribute(dom: Domain, delta: np.ndarray):
    """M applied to a pressure-cell vector delta supported on the V2 cells."""
    g = grad(dom, np.where(dom.v2[3], delta, 0.0))
    dp = np.where(dom.active[3], dom.eta * neg_div(dom, g), 0.0)
    return (-g[0], -g[1], -g[2], dp)


def collect(dom: Domain, r):
    """Pressure rows of M^T r at the V2 cells: -B r_u + eta B B^T r_p (Eq. ldist)."""
    g = grad(dom, np.where(dom.active[3], r[3], 0.0))
    out = -neg_div(dom, list(r[:3])) + dom.eta * neg_div(dom, g)
    return np.where(dom.v2[3], out, 0.0)


def dgs_diagonals(dom: Domain):
    """d_j = L~_{j,:} M_{:,j} (Alg. 2), for every V2 unknown.

    Returns (d_u, d_p): d_u is a list of three face arrays, d_p a cell array;
    entries outside V2 are zero.  Evaluated for a whole colour class at once:
    members of one class do not couple, so (L~ M 1_class)_j = (L~ M)_jj.
    """
    gam = dom.gamma
    d_u = [np.zeros(s) for s in dom.shapes[:3]]
    d_p = np.zeros(dom.shapes[3])
    for colour in (0, 1):
        ind = tuple(np.where(dom.v2[a] & (dom.parity(a) == colour), 1.0, 0.0) for a in range(3))
        y = apply_operator(dom, ind + (np.zeros(dom.shapes[3]),), gam)
        for a in range(3):
            d_u[a] += np.where(ind[a] > 0, y[a], 0.0)
        sel = dom.v2[3] & (dom.parity(3) == colour)
        y = apply_operator(dom, distribute(dom, np.where(sel, 1.0, 0.0)), gam)
        d_p += np.where(sel, y[3], 0.0)
    return d_u, d_p


PRESSURE_ORDERS = ("c8", "rb")


def pressure_classes(dom: Domain, order: str = "c8"):
    """The V2 pressure cells in forward traversal order, as a list of masks.

    Reading (traversal order): the paper leaves the order in which Alg. 2
    visits the unknowns open (the reverse sweep only has to run it
    backwards).  Velocities go red,
    black by lattice parity.  Pressures go by the 8 colour classes of the
    paper's parallel Vanka scheme (Section 6), class (i&1) + 2(j&1) + 4(k&1),
    taken 0..7 ("c8").  Cells of one class are never face neighbours, so a
    class updates at once.  Red/black pressures ("rb") are kept as the
    alternative: with them the forward-then-reverse pair of the symmetric
    smoother amplifies smooth interior pressure modes, while with the eight
    classes (as with a lexicographic order) it does not.
    """
    if order == "c8":
        col = dom.vanka_colour(2)
        return [dom.v2[3] & (col == k) for k in range(8)]
    if order == "rb":
        par = dom.parity(3)
        return [dom.v2[3] & (par == k) for k in range(2)]
    raise ValueError(order)


def _velocity_class(dom: Domain, x, b, colour, d_u):
    r = residual(dom, x, b, dom.gamma)
    return tuple(np.where(dom.v2[a] & (dom.parity(a) == colour), x[a] + r[a] / np.where(d_u[a] != 0, d_u[a], 1.0), x[a])
                 for a in range(3)) + (x[3],)


def dgs_forward(dom: Domain, x, b, diags=None, order: str = "c8"):
    """One DGS sweep over the V2 unknowns (Alg. 2 with the right preconditioning of Eq. dist).

    Reading (order): L M is block lower triangular (Eq. disc), so the sweep is
    a block forward substitution: all velocities first (red, then black),
    then all pressures (classes of `pressure_classes` in order).  A velocity
    update is the plain Gauss-Seidel step (velocity columns of M are unit
    vectors); a pressure update moves x along the column m_j of M.
    """
    d_u, d_p = diags if diags is not None else dgs_diagonals(dom)
    x = tuple(v.copy() for v in x)
    for colour in (0, 1):
        x = _velocity_class(dom, x, b, colour, d_u)
    for cls in pressure_classes(dom, order):
        r3 = continuity_residual(dom, x, b, dom.gamma)
        sel = cls & (d_p != 0)
        delta = np.where(sel, r3 / np.where(d_p != 0, d_p, 1.0), 0.0)
        dx = distribute(dom, delta)
        x = tuple(v + dv for v, dv in zip(x, dx))
    return x


def dgs_reverse(dom: Domain, x, b, diags=None, order: str = "c8"):
    """Gauss-Seidel on the left-preconditioned system M^T L~ (Eq. ldist), rows of V2, in
    exactly the reverse order of `dgs_forward`: pressure classes last to
    first, then velocities black, red.  Each step updates its own unknown by
    (M^T r)_j / d_j; for velocities (M^T)_j = e_j^T."""
    d_u, d_p = diags if diags is not None else dgs_diagonals(dom)
    x = tuple(v.copy() for v in x)
    for cls in reversed(pressure_classes(dom, order)):
        r = residual(dom, x, b, dom.gamma)
        rt = collect(dom, r)
        sel = cls & (d_p != 0)
        x = x[:3] + (x[3] + np.where(sel, rt / np.where(d_p != 0, d_p, 1.0), 0.0),)
    for colour in (1, 0):
        x = _velocity_class(dom, x, b, colour, d_u)
    return x


def dgs_symmetric(dom: Domain, x, b, diags=None, order: str = "c8"):
    """Symmetric DGS (Section 3.1, Appendix A): forward sweep, then reverse."""
    diags = diags if diags is not None else dgs_diagonals(dom)
    return dgs_reverse(dom, dgs_forward(dom, x, b, diags, order), b, diags, order)


# ---------------------------------------------------------------------------
# Vanka (Eq. mv, Section 3.2, Appendix C)
# ---------------------------------------------------------------------------

# Local unknowns of the subdomain of cell (i, j, k), in this order:
#   0: u_x[i]   1: u_x[i+1]   2: u_y[j]   3: u_y[j+1]   4: u_z[k]   5: u_z[k+1]   6: p
_SLOT_FIELD = (0, 0, 1, 1, 2, 2, 3)
_SLOT_SHIFT = (0, 1, 0, 1, 0, 1, 0)


def vanka_slots(dom: Domain, cells: np.ndarray):
    """Index tuples of the 7 local unknowns of each cell, and their activity."""
    idx, act = [], []
    for s in range(7):
        f = _SLOT_FIELD[s]
        ii = [cells[:, 0].copy(), cells[:, 1].copy(), cells[:, 2].copy()]
        if f < 3:
            ii[f] += _SLOT_SHIFT[s]
        ii = tuple(ii)
        idx.append(ii)
        act.append(dom.active[f][ii])
    return idx, np.stack(act, axis=1)


def vanka_diagonals(dom: Domain, idx):
    """n_f of the six local faces of each subdomain (Domain.ndiag)."""
    return np.stack([dom.ndiag[_SLOT_FIELD[s]][idx[s]].astype(float) for s in range(6)], axis=1)


def vanka_local_matrix(eta: float, h: float, gamma: float, act: np.ndarray, nd=None) -> np.ndarray:
    """K_i = C_i L~ C_i^T for each subdomain (Eq. mv), written out.

    Reading (subdomain): one V1 cell - its pressure and its active faces, at
    most 7 unknowns, matching the prefactorised 3^6 local problems keyed on
    the six neighbour labels (Section 6).  Entries: n_f eta/h^2 on velocity
    diagonals (n_f = nd[:, slot], 6 unless an exterior cell is near:
    Domain.ndiag), -eta/h^2 between the two faces of one axis (lattice
    neighbours), +1/h (minus face) and -1/h (plus face) between a face and the
    pressure, -gamma on the pressure diagonal.  Slots that are not unknowns
    get an identity row and column, so their update is zero.
    """
    n = act.shape[0]
    nd = np.full((n, 6), 6.0) if nd is None else nd
    K = np.zeros((n, 7, 7))
    c = eta / h ** 2
    for a in range(3):
        lo, hi = 2 * a, 2 * a + 1
        K[:, lo, lo] = nd[:, lo] * c
        K[:, hi, hi] = nd[:, hi] * c
        both = act[:, lo] & act[:, hi]
        K[:, lo, hi] = np.where(both, -c, 0.0)
        K[:, hi, lo] = K[:, lo, hi]
        K[:, lo, 6] = K[:, 6, lo] = np.where(act[:, lo], 1.0 / h, 0.0)
        K[:, hi, 6] = K[:, 6, hi] = np.where(act[:, hi], -1.0 / h, 0.0)
    K[:, 6, 6] = -gamma
    for s in range(7):
        off = ~act[:, s]
        K[off, s, :] = 0.0
        K[off, :, s] = 0.0
        K[off, s, s] = 1.0
    return K


def local_residual(dom: Domain, x, b, idx, act):
    """C_i (b - L~ x) for a set of subdomains: the rows of the residual at
    their local unknowns (slot s of cell c is row idx[s][c]), each row written
    from Eq. 2 / Section 4 with the neighbours that are not unknowns taken as
    zero - the same rows `residual` evaluates over the whole grid.  Rows of
    slots that are not unknowns are 0."""
    c = dom.eta / dom.h ** 2
    up = [np.pad(np.where(dom.active[a], x[a], 0.0), 1) for a in range(3)]
    pp = np.pad(np.where(dom.active[3], x[3], 0.0), 1)
    rows = []
    for s in range(7):
        f = _SLOT_FIELD[s]
        i, j, k = (t + 1 for t in idx[s])   # padded indices
        if f < 3:
            u = up[f]
            nb = u[i - 1, j, k] + u[i + 1, j, k] + u[i, j - 1, k] + u[i, j + 1, k] + u[i, j, k - 1] + u[i, j, k + 1]
            m = [i, j, k]
            m[f] = m[f] - 1                 # the cell on the minus side of the face
            n_f = dom.ndiag[f][idx[s]]
            row = c * (n_f * u[i, j, k] - nb) + (pp[i, j, k] - pp[tuple(m)]) / dom.h
        else:
            div = ((up[0][i + 1, j, k] - up[0][i, j, k]) + (up[1][i, j + 1, k] - up[1][i, j, k]) +
                   (up[2][i, j, k + 1] - up[2][i, j, k]))
            row = -div / dom.h - dom.gamma * pp[i, j, k]
        rows.append(np.where(act[:, s], b[f][idx[s]] - row, 0.0))
    return np.stack(rows, axis=1)


def _vanka_cells_into(dom: Domain, x: list, b, cells: np.ndarray):
    """The class step of `vanka_cells_step`, updating the list x in place."""
    if cells.shape[0] == 0:
        return
    idx, act = vanka_slots(dom, cells)
    rloc = local_residual(dom, x, b, idx, act)
    K = vanka_local_matrix(dom.eta, dom.h, dom.gamma, act, vanka_diagonals(dom, idx))
    delta = np.linalg.solve(K, rloc[:, :, None])[:, :, 0]
    for s in range(7):
        f = _SLOT_FIELD[s]
        np.add.at(x[f], idx[s], np.where(act[:, s], delta[:, s], 0.0))


def vanka_cells_step(dom: Domain, x, b, cells: np.ndarray):
    """x <- x + sum_i C_i^T K_i^{-1} C_i (b - L~ x) over the given V1 cells, every
    local residual taken from the same state; corrections of subdomains that
    share an unknown add up (Eq. av when the cells are all of V1)."""
    x = [v.copy() for v in x]
    _vanka_cells_into(dom, x, b, cells)
    return tuple(x)


def vanka_color(dom: Domain, x, b, colour: int, period: int = 2):
    """One colour class of multiplicative Vanka on V1.

    Reading (intra-colour semantics): all subdomains of one class take their
    local residual from the state at the start of the class and then apply
    their corrections, i.e. x <- x + sum_i C_i^T K_i^{-1} C_i (b - L~ x) over
    the class.  Same-class subdomains share no unknown (cells two apart), so
    the corrections never overlap.  With period 3 (27 classes) they do not
    even share a stencil entry, so the class step equals the one-subdomain-
    at-a-time sequence of Eq. mv in any order inside the class.
    """
    cells = np.argwhere(dom.v1[3] & (dom.vanka_colour(period) == colour))
    return vanka_cells_step(dom, x, b, cells)


# Forward order of the 8 classes.  Section 3.2 takes the subdomains in one
# order and then in its reverse, and Section 6 colours them with 8 classes
# without fixing an order of the classes.  Reading: each class is followed by
# its complement (the class whose parity bits all differ), 0 7 1 6 2 5 3 4.
VANKA_ORDER8 = (0, 7, 1, 6, 2, 5, 3, 4)


def vanka_class_order(period: int = 2) -> list:
    """Forward order of the colour classes: VANKA_ORDER8 for 8 classes,
    0..26 for 27."""
    return list(VANKA_ORDER8) if period == 2 else list(range(period ** 3))


def vanka_symmetric(dom: Domain, x, b, period: int = 2):
    """Symmetric multiplicative Vanka (Section 3.2): the classes in the order
    of `vanka_class_order`, then in the reverse order, each one step of
    `vanka_color`."""
    n = period ** 3
    col = dom.vanka_colour(period)
    cells = [np.argwhere(dom.v1[3] & (col == k)) for k in range(n)]
    x = [v.copy() for v in x]
    order = vanka_class_order(period)
    for colour in order + order[::-1]:
        _vanka_cells_into(dom, x, b, cells[colour])
    return tuple(x)


def vanka_additive(dom: Domain, x, b):
    """Additive Vanka (Eq. av): every V1 subdomain solves from the same
    residual and the corrections are summed, x <- x + S_AV (b - L~ x)."""
    return vanka_cells_step(dom, x, b, np.argwhere(dom.v1[3]))


VANKA_KINDS = ("mult8", "mult27", "additive")


def vanka_apply(dom: Domain, x, b, kind: str = "mult8"):
    """One application of the chosen V1 smoother: symmetric multiplicative with
    8 or 27 colour classes, or additive (symmetric by itself, App. B)."""
    if kind == "mult8":
        return vanka_symmetric(dom, x, b, 2)
    if kind == "mult27":
        return vanka_symmetric(dom, x, b, 3)
    if kind == "additive":
        return vanka_additive(dom, x, b)
    raise ValueError(kind)


def smooth(dom: Domain, x, b, n_boundary: int = 1, diags=None, interior=None, vanka: str = "mult8", order: str = "c8"):
    """Alg. 3: symmetric Vanka on V1, an interior smoother on V2, symmetric
    Vanka on V1.  The interior smoother defaults to the symmetric DGS of
    Section 3.1; `interior(dom, x, b, diags)` replaces it.

    Reading: the three calls are chained (each starts from the previous
    output), as in the symmetry proof of Appendix D; `n_boundary` symmetric
    Vanka applications fill each Vanka slot.
    """
    for _ in range(n_boundary):
        x = vanka_apply(dom, x, b, vanka)
    if interior is None:
        x = dgs_symmetric(dom, x, b, diags, order)
    else:
        x = interior(dom, x, b, diags)
    for _ in range(n_boundary):
        x = vanka_apply(dom, x, b, vanka)
    return x
