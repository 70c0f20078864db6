"""Pins of the oracle's variants (additive and 27-colour Vanka, W-cycle, the
lid-driven cavity's boundary lift) against definitions they do not use:
dense matrix algebra, literal one-subdomain-at-a-time loops, the symmetry
theorems, and the reflection symmetries of the cavity problem."""
import numpy as np
import pytest

from oracle.domain import Domain, box_labels
from oracle.multigrid import Hierarchy, vcycle
from oracle.operator import apply_operator, assemble, from_vector, lid_lift, to_vector, zeros_like_state
from oracle.smoother import _SLOT_FIELD, vanka_additive, vanka_slots, vanka_symmetric


def _dense_step(dom, step):
    """Matrix of x = step(0, b) over the unknowns, column by column."""
    n = to_vector(dom, zeros_like_state(dom)).size
    S = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        S[:, j] = to_vector(dom, step(dom, zeros_like_state(dom), from_vector(dom, e)))
    return S


def _subdomain_dofs(dom, cells):
    """Positions (in the to_vector order) of each V1 cell's active local unknowns."""
    n = to_vector(dom, zeros_like_state(dom)).size
    pos = from_vector(dom, np.arange(n, dtype=np.float64))
    idx, act = vanka_slots(dom, cells)
    out = []
    for c in range(cells.shape[0]):
        out.append([int(pos[_SLOT_FIELD[s]][tuple(i[c] for i in idx[s])]) for s in range(7) if act[c, s]])
    return out


def test_additive_vanka_is_the_sum_of_local_solves_and_symmetric():
    dom = Domain(box_labels((4, 4, 4)), 0.25)
    S = _dense_step(dom, vanka_additive)
    Lt = assemble(dom, dom.gamma, dense=True)
    want = np.zeros_like(S)
    for d in _subdomain_dofs(dom, np.argwhere(dom.v1[3])):
        want[np.ix_(d, d)] += np.linalg.inv(Lt[np.ix_(d, d)])
    assert np.allclose(S, want, rtol=0, atol=1e-12 * np.abs(want).max())
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())   # App. B


def test_27_colour_vanka_equals_sequential_subdomain_solves():
    dom = Domain(box_labels((6, 6, 6)), 1.0 / 6)
    rng = np.random.default_rng(0)
    b = tuple(np.where(m, rng.standard_normal(m.shape), 0.0) for m in dom.active)
    got = to_vector(dom, vanka_symmetric(dom, zeros_like_state(dom), b, period=3))
    # literal Eq. mv: one subdomain at a time, cells in colour order then reversed
    Lt = assemble(dom, dom.gamma, dense=True)
    bv = to_vector(dom, b)
    colour = dom.vanka_colour(3)
    cells = np.argwhere(dom.v1[3])
    order = sorted(range(len(cells)), key=lambda c: colour[tuple(cells[c])])
    dofs = _subdomain_dofs(dom, cells)
    x = np.zeros_like(bv)
    for c in order + order[::-1]:
        d = dofs[c]
        x[d] += np.linalg.solve(Lt[np.ix_(d, d)], (bv - Lt @ x)[d])
    assert np.allclose(got, x, rtol=0, atol=1e-12 * np.abs(x).max())


def test_w_cycle_two_levels_is_the_v_cycle_and_is_symmetric():
    rng = np.random.default_rng(1)
    dims, h = (8, 8, 8), 1.0 / 8
    Hv = Hierarchy(dims, h, levels=2)
    Hw = Hierarchy(dims, h, levels=2, cycle=2)
    dom = Hv.doms[0]
    b = tuple(np.where(m, rng.standard_normal(m.shape), 0.0) for m in dom.active)
    # with an exact coarse solve, a second coarse visit changes nothing
    assert np.allclose(to_vector(dom, vcycle(Hw, b)), to_vector(dom, vcycle(Hv, b)), rtol=0, atol=1e-12)
    H3 = Hierarchy(dims, h, levels=3, cycle=2)
    x = tuple(np.where(m, rng.standard_normal(m.shape), 0.0) for m in dom.active)
    y = tuple(np.where(m, rng.standard_normal(m.shape), 0.0) for m in dom.active)
    wx, wy = to_vector(dom, vcycle(H3, x)), to_vector(dom, vcycle(H3, y))
    lhs, rhs = to_vector(dom, x) @ wy, wx @ to_vector(dom, y)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.slow
def test_w_cycle_contracts_faster_than_the_v_cycle():
    dims, h = (16, 16, 16), 1.0 / 16
    rng = np.random.default_rng(2)
    rates = {}
    for cyc in (1, 2):
        H = Hierarchy(dims, h, levels=3, cycle=cyc)
        dom = H.doms[0]
        b = tuple(np.zeros(s) for s in dom.shapes)
        x = tuple(np.where(m, rng.standard_normal(m.shape), 0.0) for m in dom.active)
        norms = []
        for _ in range(4):   # stationary multigrid on L~ x = 0: x <- x + W(0 - L~ x)
            r = tuple(-v for v in apply_operator(dom, x, dom.gamma))
            e = vcycle(H, r)
            x = tuple(a + c for a, c in zip(x, e))
            norms.append(np.linalg.norm(to_vector(dom, x)))
        rates[cyc] = (norms[-1] / norms[0]) ** (1 / 3)
    assert rates[2] < rates[1] < 1.0, rates


def _cavity_solution(n):
    dom = Domain(box_labels((n, n, n)), 1.0 / n)
    b = lid_lift(dom, 1.0)
    L = assemble(dom, 0.0, dense=True)
    ones = to_vector(dom, tuple(np.zeros(s) for s in dom.shapes[:3]) + (np.ones(dom.shapes[3]),))
    K = np.block([[L, ones[:, None]], [ones[None, :], np.zeros((1, 1))]])
    x = np.linalg.solve(K, np.concatenate([to_vector(dom, b), [0.0]]))[:-1]
    return dom, b, from_vector(dom, x)


def test_lid_cavity_solution_has_the_reflection_symmetries():
    dom, b, (ux, uy, uz, p) = _cavity_solution(6)
    s = np.abs(ux).max()
    tol = 1e-10 * s
    # the lid moves along x: the problem is symmetric under y -> 1 - y
    assert np.allclose(ux, ux[:, ::-1, :], atol=tol) and np.allclose(uz, uz[:, ::-1, :], atol=tol)
    assert np.allclose(uy, -uy[:, ::-1, :], atol=tol) and np.allclose(p, p[:, ::-1, :], atol=tol)
    # x -> 1 - x maps the lid velocity to its negative; Stokes is linear, so the
    # solution is mapped to minus itself: u_x even, u_y, u_z, p odd
    assert np.allclose(ux, ux[::-1], atol=tol) and np.allclose(uy, -uy[::-1], atol=tol)
    assert np.allclose(uz, -uz[::-1], atol=tol) and np.allclose(p, -p[::-1], atol=10 * tol / dom.h)
    # the flow follows the lid near the top and returns below it
    assert ux[3, 3, -1] > 0 and ux[3, 3, 1] < 0
    # discrete incompressibility of the lifted problem's solution
    div = apply_operator(dom, (ux, uy, uz, p), 0.0)[3]
    assert np.abs(div).max() <= 1e-9 * s / dom.h


def test_lid_lift_enters_only_the_top_row_of_x_velocities():
    dom = Domain(box_labels((4, 5, 6)), 0.25)
    bx, by, bz, bp = lid_lift(dom, 2.0)
    assert not by.any() and not bz.any() and not bp.any()
    c = dom.eta / dom.h ** 2
    assert np.array_equal(bx[1:4, :, 5], np.full((3, 5), 2.0 * c))
    assert bx.sum() == pytest.approx(3 * 5 * 2.0 * c)
