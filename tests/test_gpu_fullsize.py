"""Full-size (256^3, 7 levels) checks of the GPU path, in the launch
configuration bench.py times.  The oracle cannot iterate at this size within a
test, so the checks are (a) the operator element by element against the
oracle's, (b) the converged solution's residual recomputed by the oracle's
operator on the host, (c) symmetry of the V-cycle, and (d) the manufactured
solution's O(h^2) error between 128^3 and 256^3."""
import numpy as np
import pytest

from oracle.domain import Domain, box_labels
from oracle.operator import apply_operator
from oracle.sqmr import remove_pressure_mean
from paper_2312_10615_amd.stokes import StokesSolver
from paper_2312_10615_amd.workloads import mms_fields
from tests.gpu_helpers import announce, cuda, forcing_rhs, max_rel, random_fields

pytestmark = pytest.mark.gpu

N = 256


@pytest.fixture(scope="module")
def big():
    cuda()
    sol = StokesSolver(N, N, N, h=1.0 / N)
    dom = Domain(box_labels((N, N, N)), 1.0 / N)
    return sol, dom


def test_256_solve_reaches_tolerance_checked_by_the_oracle_operator(big):
    torch = cuda()
    sol, dom = big
    announce("256^3 seed 0 solve")
    b = forcing_rhs(dom.active, (N, N, N), 1.0 / N, 0)
    x, info = sol.solve(sol.pack(b), rtol=1e-8, maxit=300)
    torch.cuda.synchronize()
    assert info["status"] == "ok" and info["relres"] <= 1e-8
    assert sol.layout.levels == 7
    xs = sol.unpack(x)
    r = apply_operator(dom, xs, 0.0)
    num = np.sqrt(sum(float(np.sum((np.where(m, bb - rr, 0.0)) ** 2)) for m, bb, rr in zip(dom.active, b, r)))
    den = np.sqrt(sum(float(np.sum(np.where(m, bb, 0.0) ** 2)) for m, bb in zip(dom.active, b)))
    assert num / den <= 1.0001e-8
    assert abs(num / den - info["relres"]) <= 1e-3 * info["relres"]
    assert abs(float(np.mean(xs[3]))) <= 1e-12 * float(np.abs(xs[3]).max())


@pytest.mark.parametrize("penalized", [0, 1])
def test_256_operator_matches_oracle(big, penalized):
    torch = cuda()
    sol, dom = big
    announce(f"256^3 apply penalized={penalized}")
    x = random_fields(dom.active, (N, N, N), seed=11)
    y = sol.apply(sol.pack(x), penalized=bool(penalized))
    torch.cuda.synchronize()
    assert max_rel(sol.unpack(y), apply_operator(dom, x, 1e-3 if penalized else 0.0)) <= 1e-14


def test_256_vcycle_is_symmetric(big):
    torch = cuda()
    sol, dom = big
    announce("256^3 vcycle symmetry")
    x = sol.pack(random_fields(dom.active, (N, N, N), seed=1))
    y = sol.pack(random_fields(dom.active, (N, N, N), seed=2))
    a = float(torch.dot(x, sol.vcycle(y)))
    b = float(torch.dot(sol.vcycle(x), y))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_manufactured_solution_second_order_at_128_and_256():
    torch = cuda()
    errs = []
    for n in (128, 256):
        announce(f"mms {n}^3")
        sol = StokesSolver(n, n, n, h=1.0 / n)
        m = mms_fields(n, eta=1.0)
        x, info = sol.solve(sol.pack(m["f"] + (np.zeros((n, n, n)),)), rtol=1e-11, maxit=400)
        torch.cuda.synchronize()
        assert info["status"] == "ok"
        ux, uy, uz, p = sol.unpack(x)
        dom = Domain(box_labels((n, n, n)), 1.0 / n)
        eu = np.sqrt(sum(float(np.sum(np.where(dom.active[a], v - m["u"][a], 0.0) ** 2))
                         for a, v in enumerate((ux, uy, uz))) / dom.n_dofs())
        ep = np.sqrt(float(np.mean((p - np.mean(p) - m["p"]) ** 2)))
        errs.append((eu, ep))
        announce(f"  n={n} iters={info['iters']} e_u={eu:.3e} e_p={ep:.3e}")
        del sol
    assert np.log2(errs[0][0] / errs[1][0]) >= 1.8
    assert np.log2(errs[0][1] / errs[1][1]) >= 1.5
