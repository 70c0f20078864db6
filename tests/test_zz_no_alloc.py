"""stokes_solve_static (the entry point for callers that cannot allocate)
against stokes_solve on the same inputs: two calls in a row on the shared
static scratch, the second on a smaller box, each compared element by
element with a solve through a caller-owned workspace."""
import numpy as np
import pytest

from tests.gpu_helpers import announce, cuda

pytestmark = pytest.mark.gpu


def _rhs(dims, h, seed):
    from oracle.domain import Domain, box_labels
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    dom = Domain(box_labels(dims), h)
    f = sinusoid_forcing(*dims, h, seed=seed)
    return tuple(np.where(dom.active[a], f[a], 0.0) for a in range(3)) + (np.zeros(dims),)


@pytest.mark.parametrize("cases", [[((32, 32, 32), 64, 0), ((16, 24, 8), 32, 1)],
                                   [((64, 48, 32), 64, 2), ((24, 16, 16), 64, 3)]])
def test_static_solve_matches_the_workspace_solve(cases):
    torch = cuda()
    from paper_2312_10615_amd import stokes as S
    for dims, prec, seed in cases:
        announce(f"static solve {dims} FP{prec} seed {seed}")
        h = 1.0 / max(dims)
        ref = S.StokesSolver(*dims, h=h, precision=prec)
        b = ref.pack(_rhs(dims, h, seed))
        x_ref, info_ref = ref.solve(b, rtol=1e-8, maxit=100)
        x = torch.zeros_like(x_ref)
        stream = torch.cuda.current_stream()
        code, info, hist = S.stokes_solve_static(ref.params, b.data_ptr(), x.data_ptr(), 1e-8, 100,
                                                 stream.cuda_stream)
        torch.cuda.synchronize()
        assert code == S.STOKES_OK, S.stokes_strerror(code)
        assert info.iters == info_ref["iters"]
        err = float((x - x_ref).abs().max()) / float(x_ref.abs().max())
        announce(f"  iters {info.iters}, max rel diff vs workspace solve {err:.2e}")
        assert err <= 1e-12
        assert np.allclose(hist, info_ref["history"], rtol=1e-10, atol=0)
        ref.close()
