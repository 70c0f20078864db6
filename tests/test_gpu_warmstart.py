"""The trained warm-start network (paper_2312_10615_amd/weights) against the
method without it: same solver, same tolerance, zero initial guess vs the
network's guess, on held-out seeds (never used in training)."""
import numpy as np
import pytest

from tests.gpu_helpers import announce, cuda

pytestmark = pytest.mark.gpu


def _setup(n, coarse_net):
    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.warmstart import WEIGHTS_FILE, load_weights
    params, sigma, record = load_weights(WEIGHTS_FILE)
    sol = StokesSolver(n, n, n, h=1.0 / n)
    lay = sol.level_layout(1) if coarse_net else sol.layout
    net = U.WarmStartNet(lay.nx, lay.ny, lay.nz, params=params, sigma=sigma)
    return sol, lay, net


def test_guess_beats_the_zero_guess_in_error_at_128():
    torch = cuda()
    from paper_2312_10615_amd.warmstart import EVAL_SEED0, _forcing_state
    announce("warm start 128^3: error of the network guess")
    sol, lay, net = _setup(128, False)
    for s in (EVAL_SEED0, EVAL_SEED0 + 1):
        b = _forcing_state(sol, 128, s, "cuda")
        xs, info = sol.solve(b, rtol=1e-10, maxit=200)
        x0 = net.initial_guess(b, lay, sol.new_state())
        xw, iw = sol.solve(b, x0=x0, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        # velocity error (pressure is defined up to a constant): guess vs zero
        nu = lay.off[3]
        err = float(torch.linalg.vector_norm((x0 - xs)[:nu]) / torch.linalg.vector_norm(xs[:nu]))
        announce(f"  seed {s}: |u0 - u| / |u| = {err:.3f}, warm solve iters {iw['iters']} status {iw['status']}")
        assert iw["status"] == "ok" and iw["relres"] <= 1e-8
        assert err < 0.6


def _iterations(n, coarse_net, seeds):
    torch = cuda()
    import time
    from paper_2312_10615_amd.warmstart import EVAL_SEED0, _forcing_state
    sol, lay, net = _setup(n, coarse_net)
    xc = torch.zeros(lay.total, dtype=torch.float64, device="cuda") if coarse_net else sol.new_state()
    zero, warm, tz, tw = [], [], 0.0, 0.0
    for s in range(EVAL_SEED0, EVAL_SEED0 + seeds):
        b = _forcing_state(sol, n, s, "cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0 = sol.solve(b, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if coarse_net:
            net.initial_guess(sol.restrict(b), lay, xc)
            x0 = sol.prolong(xc)
        else:
            x0 = net.initial_guess(b, lay, xc)
        _, i1 = sol.solve(b, x0=x0, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        assert i0["status"] == "ok" and i1["status"] == "ok"
        zero.append(i0["iters"])
        warm.append(i1["iters"])
        tz += t1 - t0
        tw += t2 - t1
    announce(f"  iterations zero guess {zero}, network guess {warm}; time to 1e-8 {1e3 * tz / seeds:.1f} ms "
             f"vs {1e3 * tw / seeds:.1f} ms with the guess")
    return zero, warm


# Over 200 held-out seeds (profiles/warmstart_eval.md) the guess saves 0.86
# iterations on average at 128^3, and is one iteration worse on 7 seeds of
# 200; at 256^3, from the 128^3 level, 0.94, never worse.  The seeds are fixed
# and the solver deterministic, so these are regression bars on the first
# eight held-out seeds (observed: 6 iterations fewer at 128^3, 5 at 256^3).
def test_fewer_iterations_at_128_with_the_guess():
    announce("warm start 128^3: iterations and time vs zero guess")
    zero, warm = _iterations(128, False, 8)
    assert all(w <= z + 1 for z, w in zip(zero, warm))
    assert sum(zero) - sum(warm) >= 4


def test_fewer_iterations_at_256_with_the_guess_from_128():
    announce("warm start 256^3 (network on the 128^3 level): iterations and time vs zero guess")
    zero, warm = _iterations(256, True, 8)
    assert all(w <= z for z, w in zip(zero, warm))
    assert sum(zero) - sum(warm) >= 3
