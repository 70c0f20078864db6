"""Pins of the oracle's domain, operator and grid transfers against facts the
paper and the mathematics fix (not against the oracle itself)."""
import json
import os

import numpy as np
import pytest

from oracle.domain import (DIRICHLET, EXTERIOR, INTERIOR, Domain, box_labels, classify,
                           coarsen_labels, dof_counts)
from oracle.multigrid import auto_levels
from oracle.operator import (apply_operator, assemble, from_vector, grad, neg_div, to_vector,
                             viscous)
from oracle.transfer import prolong, restrict
from paper_2312_10615_amd.workloads import random_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dom_of(dims, h=None, eta=1.0, gamma=1e-3):
    return Domain(box_labels(dims), h if h is not None else 1.0 / max(dims), eta, gamma)


def rand_state(dom, seed):
    x = random_state(*dom.dims, seed=seed)
    return tuple(np.where(m, v, 0.0) for m, v in zip(dom.active, x))


def vdot(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


# --- Table 1: DOF classification (Section 5) --------------------------------

def test_table1_cavity_rows_exact():
    rows = json.load(open(os.path.join(GOLDEN, "table1_cavity_dofs.json")))["rows"]
    for row in rows:
        total, boundary = dof_counts(box_labels(tuple(row["dims"])))
        assert (total, boundary) == (row["total"], row["boundary"]), row["name"]


def test_dof_count_closed_form_small_boxes():
    # n = 3(N-1)N^2 + N^3 on a cube; V1 = ring cells and all their faces
    for n in (3, 4, 7, 10):
        tot, v1 = dof_counts(box_labels((n, n, n)))
        assert tot == 3 * (n - 1) * n * n + n ** 3
        ring = n ** 3 - (n - 2) ** 3
        faces_v2 = max(n - 3, 0) * (n - 2) ** 2
        assert v1 == ring + 3 * ((n - 1) * n * n - faces_v2)


def _coarsen_brute(lab):
    """Per-cell loop of the Section 5 rule, with missing fine cells Dirichlet."""
    dims = [s - 2 for s in lab.shape]
    out = np.zeros([n // 2 + 2 for n in dims], dtype=np.int8)
    for c in np.ndindex(*out.shape):
        kids = []
        for off in np.ndindex(*([2] * lab.ndim)):
            f = tuple(2 * ci - 1 + o for ci, o in zip(c, off))
            ok = all(0 <= fi < s for fi, s in zip(f, lab.shape))
            kids.append(lab[f] if ok else DIRICHLET)
        kids = np.array(kids)
        out[c] = DIRICHLET if (kids == DIRICHLET).any() else (INTERIOR if (kids == INTERIOR).any() else EXTERIOR)
    return out


def test_label_coarsening_matches_cellwise_rule():
    rng = np.random.default_rng(3)
    lab = box_labels((8, 6, 4))
    inner = lab[1:-1, 1:-1, 1:-1]
    inner[...] = rng.choice([INTERIOR, INTERIOR, INTERIOR, DIRICHLET, EXTERIOR], size=inner.shape)
    assert np.array_equal(coarsen_labels(lab), _coarsen_brute(lab))
    # a padded box coarsens to a padded box of half the size
    assert np.array_equal(coarsen_labels(box_labels((8, 12, 4))), box_labels((4, 6, 2)))


def test_auto_levels():
    assert auto_levels((32, 32, 32)) == 4
    assert auto_levels((256, 256, 256)) == 7
    assert auto_levels((384, 384, 384)) == 7
    assert auto_levels((48, 48, 48)) == 4
    assert auto_levels((32, 48, 128)) == 4


# --- Operator (Eq. 2, Section 4) --------------------------------------------

@pytest.mark.parametrize("gamma", [0.0, 1e-3])
def test_operator_symmetric(gamma):
    dom = dom_of((6, 8, 10))
    x, y = rand_state(dom, 1), rand_state(dom, 2)
    a = vdot(x, apply_operator(dom, y, gamma))
    b = vdot(apply_operator(dom, x, gamma), y)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_pressure_constant_is_the_null_vector():
    dom = dom_of((4, 6, 4))
    one = tuple(np.zeros(s) for s in dom.shapes[:3]) + (np.ones(dom.shapes[3]),)
    y = apply_operator(dom, one, 0.0)
    assert all(np.all(v == 0.0) for v in y)
    L = assemble(dom, 0.0, dense=True)
    assert np.linalg.matrix_rank(L) == dom.n_dofs() - 1
    Lt = assemble(dom, 1e-3, dense=True)
    assert np.linalg.matrix_rank(Lt) == dom.n_dofs()
    assert np.allclose(L, L.T, rtol=0, atol=1e-12 * np.abs(L).max())


def test_operator_on_polynomials():
    """Central differences are exact on quadratics: -eta*Lap(x^2) = -2 eta,
    grad(x) = 1, and B = -div gives -1 for u_x = x, away from the walls."""
    n, eta = 8, 0.7
    h = 1.0 / n
    dom = Domain(box_labels((n, n, n)), h, eta, 0.0)
    xf = (np.arange(n + 1) * h)[:, None, None] * np.ones((1, n, n))
    a = viscous(dom, xf ** 2, 0)
    assert np.allclose(a[2:-2, 1:-1, 1:-1], -2.0 * eta, rtol=0, atol=1e-9)
    xc = ((np.arange(n) + 0.5) * h)[:, None, None] * np.ones((1, n, n))
    g = grad(dom, xc)
    assert np.allclose(g[0][1:-1], 1.0, atol=1e-12) and np.all(g[1] == 0) and np.all(g[2] == 0)
    u = [np.where(dom.active[0], xf, 0.0), np.zeros(dom.shapes[1]), np.zeros(dom.shapes[2])]
    d = neg_div(dom, u)
    assert np.allclose(d[1:-1], -1.0, atol=1e-12)


def test_eq_disc_top_right_block_vanishes_in_interior():
    """L M = [[-eta Lap, 0], [-div, Lap]] in the interior (Eq. disc):
    A(-B^T p) + B^T(eta B B^T p) = 0 and -B B^T p = Lap_h p, for p supported
    two or more cells from the walls."""
    n = 10
    dom = dom_of((n, n, n), eta=1.3)
    rng = np.random.default_rng(5)
    p = np.zeros((n, n, n))
    p[3:-3, 3:-3, 3:-3] = rng.standard_normal((n - 6,) * 3)
    g = grad(dom, p)
    bbt = neg_div(dom, g)
    top = [viscous(dom, -g[a], a) + grad(dom, dom.eta * bbt)[a] for a in range(3)]
    assert max(np.abs(t).max() for t in top) <= 1e-9 * np.abs(g[0]).max() / dom.h
    pp = np.pad(p, 1)
    lap = (pp[2:, 1:-1, 1:-1] + pp[:-2, 1:-1, 1:-1] + pp[1:-1, 2:, 1:-1] + pp[1:-1, :-2, 1:-1]
           + pp[1:-1, 1:-1, 2:] + pp[1:-1, 1:-1, :-2] - 6 * p) / dom.h ** 2
    assert np.allclose(-bbt, lap, rtol=0, atol=1e-9 * np.abs(lap).max())


def test_vector_roundtrip_and_order():
    dom = dom_of((4, 6, 2))
    x = rand_state(dom, 4)
    v = to_vector(dom, x)
    assert v.size == dom.n_dofs()
    y = from_vector(dom, v)
    assert all(np.array_equal(a, b) for a, b in zip(x, y))


# --- Grid transfers (Section 2) ---------------------------------------------

def _pair(dims):
    f = dom_of(dims)
    return f, f.coarsen()


def test_prolongation_reproduces_linear_fields_away_from_walls():
    fine, coarse = _pair((16, 12, 8))
    H = fine.h
    rng = np.random.default_rng(0)
    for f in range(3):
        c = rng.standard_normal(4)
        # coarse face/cell-centre coordinates of field f
        def coords(dims, h):
            out = []
            for a, n in enumerate(dims):
                if a == f:
                    v = np.arange(n + 1) * h
                else:
                    v = (np.arange(n) + 0.5) * h
                shp = [1, 1, 1]
                shp[a] = v.size
                out.append(v.reshape(shp))
            return out
        X, Y, Z = coords(coarse.dims, 2 * H)
        lin_c = c[0] + c[1] * X + c[2] * Y + c[3] * Z
        e = [np.zeros(s) for s in coarse.shapes]
        e[f] = np.where(coarse.active[f], lin_c, 0.0)
        out = prolong(fine, coarse, tuple(e))[f]
        Xf, Yf, Zf = coords(fine.dims, H)
        lin_f = np.broadcast_to(c[0] + c[1] * Xf + c[2] * Yf + c[3] * Zf, out.shape)
        sl = [slice(3, -3)] * 3
        assert np.allclose(out[tuple(sl)], lin_f[tuple(sl)], rtol=0, atol=1e-12)


def test_prolongation_pressure_is_piecewise_constant():
    fine, coarse = _pair((8, 4, 6))
    rng = np.random.default_rng(1)
    pc = rng.standard_normal(coarse.shapes[3])
    e = tuple(np.zeros(s) for s in coarse.shapes[:3]) + (pc,)
    pf = prolong(fine, coarse, e)[3]
    assert np.array_equal(pf, np.repeat(np.repeat(np.repeat(pc, 2, 0), 2, 1), 2, 2))


def test_restriction_is_a_partition_of_unity_in_the_interior():
    fine, coarse = _pair((16, 16, 16))
    ones = tuple(np.where(m, 1.0, 0.0) for m in fine.active)
    rc = restrict(fine, coarse, ones)
    for f in range(4):
        assert np.allclose(rc[f][2:-2, 2:-2, 2:-2], 1.0, rtol=0, atol=1e-15)
    # prolongation also reproduces constants in the interior (partition of unity)
    onec = tuple(np.where(m, 1.0, 0.0) for m in coarse.active)
    pf = prolong(fine, coarse, onec)
    for f in range(4):
        assert np.allclose(pf[f][3:-3, 3:-3, 3:-3], 1.0, rtol=0, atol=1e-15)


def test_restriction_is_transposed_prolongation_over_eight():
    fine, coarse = _pair((8, 12, 4))
    r = rand_state(fine, 7)
    e = rand_state(coarse, 8)
    lhs = vdot(restrict(fine, coarse, r), e)
    rhs = vdot(r, prolong(fine, coarse, e)) / 8.0
    assert abs(lhs - rhs) <= 1e-14 * abs(rhs) * 10


def test_classify_masks_are_consistent():
    lab = box_labels((5, 4, 6))
    act, v1 = classify(lab)
    for a, v in zip(act, v1):
        assert not np.any(v & ~a)
    # every face of a V1 cell is V1; V2 faces have two V2 cells on their sides
    dom = Domain(lab, 0.2)
    ring = dom.v1[3]
    for a in range(3):
        lo = [slice(None)] * 3
        lo[a] = slice(0, -1)
        hi = [slice(None)] * 3
        hi[a] = slice(1, None)
        minus_cell = np.pad(ring, [(1, 0) if b == a else (0, 0) for b in range(3)])
        plus_cell = np.pad(ring, [(0, 1) if b == a else (0, 0) for b in range(3)])
        assert np.array_equal(dom.v1[a], dom.active[a] & (minus_cell | plus_cell))
