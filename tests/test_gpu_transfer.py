"""stokes_restrict / stokes_prolong (the V-cycle's R and P between the finest
level and the next) against the oracle's transfer operators."""
import numpy as np
import pytest

from tests.gpu_helpers import announce, cuda, random_fields, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [(16, 8, 12), (32, 32, 32), (10, 8, 8)])  # (10, 8, 8): odd coarse nx
def test_restrict_and_prolong_match_oracle(dims):
    cuda()
    from oracle.domain import Domain, box_labels
    from oracle.transfer import prolong, restrict
    from paper_2312_10615_amd.stokes import StokesSolver
    nx, ny, nz = dims
    announce(f"stokes restrict/prolong {dims}")
    h = 1.0 / nx
    sol = StokesSolver(nx, ny, nz, h=h)
    csol = StokesSolver(nx // 2, ny // 2, nz // 2, h=2 * h)
    lay1, lay_c = sol.level_layout(1), csol.layout
    # a box of half the cells at level 0 has the layout of level 1
    assert (lay1.nx, lay1.sy, lay1.sz, lay1.field, lay1.total) == (lay_c.nx, lay_c.sy, lay_c.sz, lay_c.field,
                                                                    lay_c.total)
    fine = Domain(box_labels(dims), h)
    coarse = fine.coarsen()
    r = random_fields(fine.active, dims, seed=3)
    got = csol.unpack(sol.restrict(sol.pack(r)))
    assert rel_err(got, restrict(fine, coarse, r)) <= 1e-14
    cdims = (nx // 2, ny // 2, nz // 2)
    e = random_fields(coarse.active, cdims, seed=4)
    x = sol.new_state().fill_(5.0)  # overwritten
    got = sol.unpack(sol.prolong(csol.pack(e), out=x))
    assert rel_err(got, prolong(fine, coarse, e)) <= 1e-14
    # slots that are not unknowns come back as zero
    assert float(x.abs().sum()) == pytest.approx(sum(float(np.abs(a).sum()) for a in got), rel=1e-12)
