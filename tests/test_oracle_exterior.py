"""Exterior cells and Neumann faces (paper Section 5) in the oracle: the DOF
rule and the boundary set pinned by Table 1's 2D cylinder rows, the zero-
Neumann velocity stencil, symmetry, null vectors, label coarsening, and the
multigrid-preconditioned solve against a dense solve on a small domain with
an obstacle and an outflow."""
import json
import os

import numpy as np
import pytest

from oracle.domain import DIRICHLET, EXTERIOR, INTERIOR, Domain, coarsen_labels, dof_counts
from oracle.multigrid import Hierarchy, vcycle
from oracle.operator import apply_operator, assemble, to_vector
from oracle.sqmr import mg_sqmr
from paper_2312_10615_amd.workloads import random_state, sinusoid_forcing

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def channel_2d(nx, ny):
    """The 2D cylinder channel of the golden fixture (labels with padding)."""
    h = 2.2 / nx
    lab = np.full((nx + 2, ny + 2), DIRICHLET, np.int8)
    lab[1:-1, 1:-1] = INTERIOR
    lab[-1, 1:-1] = EXTERIOR
    xc = (np.arange(nx) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    inside = (xc[:, None] - 0.2) ** 2 + (yc[None, :] - 0.2) ** 2 < 0.05 ** 2
    lab[1:-1, 1:-1][inside] = DIRICHLET
    return lab


def test_table1_cylinder_rows_exact():
    rows = json.load(open(os.path.join(GOLDEN, "table1_cylinder_dofs.json")))["rows"]
    for r in rows:
        total, boundary = dof_counts(channel_2d(*r["dims"]))
        assert (total, boundary) == (r["total"], r["boundary"]), r["name"]


def obstacle_outflow(n, m=None):
    """A 3D channel n x m x m: Dirichlet walls and inflow side, a block
    obstacle of Dirichlet cells inside, one exterior layer on the +x side."""
    m = m or n
    lab = np.full((n + 2, m + 2, m + 2), DIRICHLET, np.int8)
    lab[1:-1, 1:-1, 1:-1] = INTERIOR
    lab[-1, 1:-1, 1:-1] = EXTERIOR
    q = max(1, n // 4)
    lab[q + 1:2 * q + 1, m // 4 + 1:m // 2 + 1, m // 4 + 1:m // 2 + 1] = DIRICHLET
    return lab


def closed_obstacle(n):
    lab = obstacle_outflow(n)
    lab[-1, 1:-1, 1:-1] = DIRICHLET
    return lab


def rand_state(dom, seed):
    x = random_state(*dom.dims, seed=seed)
    return tuple(np.where(mk, v, 0.0) for mk, v in zip(dom.active, x))


def test_interior_exterior_faces_are_unknowns_and_v1_reaches_two_cells():
    lab = obstacle_outflow(8)
    dom = Domain(lab, 1 / 8)
    # the outflow faces between the last interior cells and the exterior layer
    assert dom.active[0][8, 2, 2] and dom.v1[0][8, 2, 2]
    # cells one and two away from the exterior layer are V1, three away are not
    # (away from the walls and the obstacle)
    assert dom.v1[3][7, 6, 6] and dom.v1[3][6, 6, 6] and not dom.v1[3][5, 6, 6]
    assert not (lab == INTERIOR)[0].any()


def test_zero_neumann_stencil_annihilates_constants_and_counts_neighbours():
    """With no Dirichlet cell at all (exterior outer layer) A has zero row
    sums: a velocity component that is constant over its unknowns is in the
    kernel of A (zero normal derivative on every boundary).  The diagonal
    counts: 6 in the interior, 5 for an outflow face (its neighbour on the
    exterior side is dropped), 6 next to a Dirichlet wall."""
    n = 6
    lab = np.full((n + 2,) * 3, EXTERIOR, np.int8)
    lab[1:-1, 1:-1, 1:-1] = INTERIOR
    dom = Domain(lab, 1 / n)
    for a in range(3):
        x = [np.zeros(s) for s in dom.shapes]
        x[a] = np.where(dom.active[a], 1.0, 0.0)
        y = apply_operator(dom, tuple(x), 0.0)
        assert np.abs(y[a]).max() <= 1e-12 / dom.h ** 2
    ch = Domain(obstacle_outflow(8), 1 / 8)
    assert ch.ndiag[0][4, 6, 6] == 6      # interior face
    assert ch.ndiag[0][8, 6, 6] == 5      # outflow face: its +x neighbour is on the exterior side
    assert ch.ndiag[1][7, 6, 6] == 5      # a u_y face of the last cell: its +x neighbour lies in the exterior
    assert ch.ndiag[0][4, 0, 6] == 6      # next to a no-slip wall: the ghost is a Dirichlet value


@pytest.mark.parametrize("maker", [obstacle_outflow, closed_obstacle])
def test_operator_symmetry_and_null_space(maker):
    n = 6
    dom = Domain(maker(n), 1 / n)
    L = assemble(dom, 0.0, dense=True)
    assert np.abs(L - L.T).max() == 0.0
    ones_p = to_vector(dom, tuple(np.zeros(s) for s in dom.shapes[:3]) + (np.ones(dom.shapes[3]),))
    sv = np.linalg.svd(L, compute_uv=False)
    if maker is closed_obstacle:
        # closed domain: constant pressure is the one null vector
        assert np.abs(L @ ones_p).max() == 0.0 and not dom.has_neumann
        assert sv[-1] <= 1e-12 * sv[0] and sv[-2] >= 1e-8 * sv[0]
    else:
        # an outflow fixes the pressure level (exterior pressures are zero)
        assert np.abs(L @ ones_p).max() > 0 and dom.has_neumann
        assert sv[-1] >= 1e-8 * sv[0]


def test_label_coarsening_with_exterior_cells_matches_a_cell_loop():
    """Section 5's rule, cell by cell; the exterior outflow layer stays an
    exterior layer on the coarse grid."""
    lab = obstacle_outflow(8)
    lab[5, 3, 3] = EXTERIOR
    got = coarsen_labels(lab)
    n = 8
    want = np.full((n // 2 + 2,) * 3, DIRICHLET, np.int8)
    for I in range(n // 2 + 2):
        for J in range(n // 2 + 2):
            for K in range(n // 2 + 2):
                kids = []
                for di in (0, 1):
                    for dj in (0, 1):
                        for dk in (0, 1):
                            # beyond the array the outer layer repeats
                            i, j, k = (min(max(t, 0), n + 1) for t in (2 * I - 1 + di, 2 * J - 1 + dj, 2 * K - 1 + dk))
                            kids.append(lab[i, j, k])
                kids = np.array(kids)
                want[I, J, K] = DIRICHLET if (kids == DIRICHLET).any() else (
                    INTERIOR if (kids == INTERIOR).any() else EXTERIOR)
    assert np.array_equal(got, want)
    assert (got[-1, 1:-1, 1:-1] == EXTERIOR).all()


def test_vcycle_symmetric_on_a_labelled_domain():
    n = 16
    H = Hierarchy((n, n, n), 1 / n, labels=obstacle_outflow(n), levels=3)
    dom = H.doms[0]
    x, y = rand_state(dom, 1), rand_state(dom, 2)
    a = sum(float(np.sum(u * v)) for u, v in zip(x, vcycle(H, y)))
    b = sum(float(np.sum(u * v)) for u, v in zip(vcycle(H, x), y))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_mg_sqmr_reaches_the_dense_solution_with_an_obstacle_and_an_outflow():
    n = 8
    H = Hierarchy((n, n, n), 1 / n, labels=obstacle_outflow(n), levels=2)
    dom = H.doms[0]
    f = sinusoid_forcing(n, n, n, 1 / n, seed=3)
    b = tuple(np.where(dom.active[a], f[a], 0.0) for a in range(3)) + (np.zeros((n, n, n)),)
    x, info = mg_sqmr(H, b, rtol=1e-12, maxit=200)
    assert info["status"] == "converged", info
    L = assemble(dom, 0.0, dense=True)
    want = np.linalg.solve(L, to_vector(dom, b))
    got = to_vector(dom, x)
    assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want)


def test_mg_sqmr_iterations_with_an_obstacle_and_an_outflow():
    """The block obstacle and outflow channel at 16^3 and 32^3 (3 and 4
    levels, seed 0 forcing): 9 and 11 iterations to 1e-8."""
    its = []
    for n in (16, 32):
        H = Hierarchy((n, n, n), 1 / n, labels=obstacle_outflow(n))
        dom = H.doms[0]
        f = sinusoid_forcing(n, n, n, 1 / n, seed=0)
        b = tuple(np.where(dom.active[a], f[a], 0.0) for a in range(3)) + (np.zeros((n, n, n)),)
        _, info = mg_sqmr(H, b, rtol=1e-8, maxit=60)
        assert info["status"] == "converged"
        its.append(info["iters"])
    assert its[0] <= 10 and its[1] <= 12
