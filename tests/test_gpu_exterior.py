"""Labelled domains (Section 5: interior, Dirichlet and exterior cells) on
the GPU against the oracle: the operator, one V-cycle (both schedules, FP64
and FP32), and MG-SQMR solves, on a channel with a block obstacle and an
outflow layer of exterior cells, on a closed box with an obstacle, and on a
ragged box with an exterior pocket beside interior cells (Neumann faces
inside the domain)."""
import numpy as np
import pytest

from oracle.domain import DIRICHLET, EXTERIOR, Domain
from oracle.multigrid import Hierarchy, vcycle
from oracle.operator import apply_operator
from oracle.sqmr import mg_sqmr, remove_pressure_mean
from paper_2312_10615_amd.workloads import random_state, sinusoid_forcing
from tests.gpu_helpers import announce, cuda, max_rel, rel_err
from tests.test_oracle_exterior import closed_obstacle, obstacle_outflow

pytestmark = pytest.mark.gpu


def pocket(nx, ny, nz):
    """A ragged box: Dirichlet walls, an exterior outflow on the -y side, a
    Dirichlet block, and a block of exterior cells inside the domain."""
    lab = np.full((nx + 2, ny + 2, nz + 2), DIRICHLET, np.int8)
    lab[1:-1, 1:-1, 1:-1] = 0
    lab[1:-1, 0, 1:-1] = EXTERIOR
    lab[nx // 2 + 1:nx // 2 + 4, ny // 2 + 1:ny // 2 + 3, 2:5] = DIRICHLET
    lab[3:6, ny - 3:ny - 1, nz // 2:nz // 2 + 3] = EXTERIOR
    return lab


CASES = {"outflow16": ((16, 16, 16), lambda: obstacle_outflow(16)),
         "closed16": ((16, 16, 16), lambda: closed_obstacle(16)),
         "pocket24": ((24, 16, 20), lambda: pocket(24, 16, 20)),
         "outflow32": ((32, 32, 32), lambda: obstacle_outflow(32))}


def _setup(name, **kw):
    dims, make = CASES[name]
    lab = make()
    h = 1.0 / max(dims)
    return dims, lab, h


def _rand(dom, seed):
    x = random_state(*dom.dims, seed=seed)
    return tuple(np.where(m, v, 0.0) for m, v in zip(dom.active, x))


@pytest.mark.parametrize("name", ["outflow16", "closed16", "pocket24"])
def test_labelled_operator_matches_oracle(name):
    torch = cuda()
    from paper_2312_10615_amd.stokes import StokesSolver
    dims, lab, h = _setup(name)
    announce(f"labelled apply {name}")
    dom = Domain(lab, h)
    sol = StokesSolver(*dims, h=h, labels=lab)
    assert sol.layout.n_dofs == dom.n_dofs()
    x = _rand(dom, 3)
    for pen in (0, 1):
        y = sol.apply(sol.pack(x), penalized=bool(pen))
        torch.cuda.synchronize()
        assert max_rel(sol.unpack(y), apply_operator(dom, x, dom.gamma if pen else 0.0)) <= 1e-14


@pytest.mark.parametrize("name,sched,prec", [("outflow16", "symmetric", 64), ("closed16", "symmetric", 64),
                                             ("pocket24", "symmetric", 64), ("pocket24", "split", 64),
                                             ("outflow32", "symmetric", 64), ("outflow16", "symmetric", 32),
                                             ("pocket24", "symmetric", 32)])
def test_labelled_vcycle_matches_oracle(name, sched, prec):
    torch = cuda()
    from paper_2312_10615_amd.stokes import StokesSolver
    dims, lab, h = _setup(name)
    announce(f"labelled vcycle {name} {sched} FP{prec}")
    sol = StokesSolver(*dims, h=h, labels=lab, schedule=sched, precision=prec)
    H = Hierarchy(dims, h, labels=lab, schedule=sched)
    assert sol.layout.levels == H.levels
    s = _rand(H.doms[0], 7)
    t = sol.vcycle(sol.pack(s))
    torch.cuda.synchronize()
    err = max_rel(sol.unpack(t), vcycle(H, s))
    announce(f"  levels {H.levels}: max-rel difference {err:.2e}")
    assert err <= (1e-12 if prec == 64 else 2e-5)


@pytest.mark.parametrize("name", ["outflow16", "closed16", "pocket24", "outflow32"])
def test_labelled_solve_matches_oracle(name):
    torch = cuda()
    from paper_2312_10615_amd.stokes import StokesSolver
    dims, lab, h = _setup(name)
    announce(f"labelled solve {name}")
    H = Hierarchy(dims, h, labels=lab)
    dom = H.doms[0]
    f = sinusoid_forcing(*dims, h, seed=2)
    b = tuple(np.where(dom.active[a], f[a], 0.0) for a in range(3)) + (np.zeros(dims),)
    xo, io = mg_sqmr(H, b, rtol=1e-8, maxit=100)
    assert io["status"] == "converged"
    sol = StokesSolver(*dims, h=h, labels=lab)
    x, info = sol.solve(sol.pack(b), rtol=1e-8, maxit=100)
    torch.cuda.synchronize()
    # the pressure mean is removed only in a closed domain (an outflow fixes the pressure)
    want = remove_pressure_mean(dom, xo) if not dom.has_neumann else xo
    e = rel_err(sol.unpack(x), want)
    announce(f"  iterations gpu {info['iters']} oracle {io['iters']}; relative difference {e:.2e}")
    assert info["status"] == "ok" and info["iters"] == io["iters"]
    assert e <= 1e-10
