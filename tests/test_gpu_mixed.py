"""FP32 V-cycle inside FP64 SQMR (mixed precision) against the FP64 oracle.

The oracle computes in FP64; the FP32 V-cycle differs from it by FP32
rounding, so the bars here are derived from FP32's unit roundoff (6e-8)
times the growth through one V-cycle (measured ~1e-6 at 32^3), not the FP64
bars.  The solve itself is held to the same 1e-8 FP64 true residual.
"""
import numpy as np
import pytest

from oracle.domain import Domain, box_labels
from oracle.multigrid import Hierarchy, vcycle
from oracle.operator import apply_operator
from paper_2312_10615_amd.stokes import StokesSolver
from tests.gpu_helpers import announce, cuda, forcing_rhs, max_rel, random_fields, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,sched", [((32, 32, 32), "symmetric"), ((16, 24, 8), "symmetric"),
                                        ((32, 32, 32), "split")])
def test_fp32_vcycle_matches_fp64_oracle_to_fp32_accuracy(dims, sched):
    torch = cuda()
    h = 1.0 / max(dims)
    sol = StokesSolver(*dims, h=h, precision=32, schedule=sched)
    H = Hierarchy(dims, h, schedule=sched)
    s = random_fields(H.doms[0].active, dims, seed=7)
    t = sol.vcycle(sol.pack(s))
    torch.cuda.synchronize()
    err = max_rel(sol.unpack(t), vcycle(H, s))
    announce(f"fp32 vcycle dims={dims} schedule={sched}: max-rel error vs FP64 oracle {err:.2e}")
    assert err <= 2e-5


def test_fp32_vcycle_asymmetry_is_at_fp32_level():
    torch = cuda()
    n = 64
    sol = StokesSolver(n, n, n, precision=32)
    dom = Domain(box_labels((n, n, n)), 1.0 / n)
    x = sol.pack(random_fields(dom.active, (n, n, n), seed=1))
    y = sol.pack(random_fields(dom.active, (n, n, n), seed=2))
    a = float(torch.dot(x, sol.vcycle(y)))
    b = float(torch.dot(sol.vcycle(x), y))
    asym = abs(a - b) / abs(a)
    announce(f"fp32 V-cycle asymmetry at 64^3: {asym:.2e}")
    assert asym <= 1e-5


@pytest.mark.parametrize("n", [32, 256])
def test_mixed_precision_solve_reaches_fp64_tolerance(n):
    torch = cuda()
    h = 1.0 / n
    dom = Domain(box_labels((n, n, n)), h)
    b = forcing_rhs(dom.active, (n, n, n), h, 0)
    s64 = StokesSolver(n, n, n, h=h)
    s32 = StokesSolver(n, n, n, h=h, precision=32)
    x64, i64 = s64.solve(s64.pack(b), rtol=1e-8, maxit=300)
    x32, i32 = s32.solve(s32.pack(b), rtol=1e-8, maxit=300)
    torch.cuda.synchronize()
    assert i32["status"] == "ok" and i32["relres"] <= 1e-8
    # the residual, recomputed by the oracle's FP64 operator on the host
    got = s32.unpack(x32)
    r = apply_operator(dom, got, 0.0)
    num = np.sqrt(sum(float(np.sum(np.where(m, bb - rr, 0.0) ** 2)) for m, bb, rr in zip(dom.active, b, r)))
    den = np.sqrt(sum(float(np.sum(np.where(m, bb, 0.0) ** 2)) for m, bb in zip(dom.active, b)))
    assert num / den <= 1.0001e-8
    diff = rel_err(got, s64.unpack(x64))
    announce(f"mixed n={n}: iters fp64={i64['iters']} fp32-vcycle={i32['iters']}, "
             f"|x32 - x64|/|x64| = {diff:.2e}")
    assert i32["iters"] <= i64["iters"] + 2
    assert diff <= 1e-6
