"""The host set-up of a labelled domain (csrc/host_tables.hpp: label
coarsening, flag words, Vanka local inverses), built with g++ and run on the
CPU, against the oracle on the same labels: coarse labels, unknowns, V1/V2,
the diagonals n_f of A, and for every V1 cell the local inverse its type
points at against the inverse of the oracle's local matrix."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.domain import Domain
from oracle.multigrid import Hierarchy
from oracle.smoother import vanka_diagonals, vanka_local_matrix, vanka_slots

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def tool(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = tmp_path_factory.mktemp("lt") / "label_tables_dump"
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(HERE, "label_tables_dump.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _cases():
    from tests.test_gpu_exterior import pocket
    from tests.test_oracle_exterior import closed_obstacle, obstacle_outflow
    return {"outflow16": obstacle_outflow(16), "closed16": closed_obstacle(16), "pocket24": pocket(24, 16, 20)}


@pytest.mark.parametrize("name", ["outflow16", "closed16", "pocket24"])
def test_host_label_tables_match_the_oracle(tool, tmp_path, name):
    lab = _cases()[name]
    dims = tuple(s - 2 for s in lab.shape)
    H = Hierarchy(dims, 1.0 / max(dims), labels=lab)
    src = tmp_path / "labels.bin"
    src.write_bytes(np.ascontiguousarray(lab.transpose(2, 1, 0), dtype=np.uint8).tobytes())
    prefix = str(tmp_path / "out")
    r = subprocess.run([str(tool), *map(str, dims), str(H.levels), str(src), prefix], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    for l, dom in enumerate(H.doms):
        shp = tuple(s + 2 for s in dom.dims)
        got_lab = np.fromfile(f"{prefix}_labels{l}.bin", dtype=np.uint8).reshape(shp[::-1]).transpose(2, 1, 0)
        assert np.array_equal(got_lab, dom.labels), f"labels of level {l}"
        w = np.fromfile(f"{prefix}_flags{l}.bin", dtype=np.uint32).reshape(shp[::-1]).transpose(2, 1, 0)
        nx, ny, nz = dom.dims
        for a in range(3):
            # face f of axis a (0..n_a) is the minus face of padded cell f+1
            sl = [slice(1, nx + 1), slice(1, ny + 1), slice(1, nz + 1)]
            sl[a] = slice(1, dom.dims[a] + 2)
            wa = w[tuple(sl)]
            assert np.array_equal((wa >> a) & 1 == 1, dom.active[a]), f"active u{a} level {l}"
            assert np.array_equal((wa >> (4 + a)) & 1 == 1, dom.v2[a]), f"V2 u{a} level {l}"
            nd = (wa >> (8 + 3 * a)) & 7
            assert np.array_equal(np.where(dom.active[a], nd, 0), np.where(dom.active[a], dom.ndiag[a], 0)), \
                f"n_f u{a} level {l}"
        wp = w[1:nx + 1, 1:ny + 1, 1:nz + 1]
        assert np.array_equal((wp >> 3) & 1 == 1, dom.active[3]) and np.array_equal((wp >> 7) & 1 == 1, dom.v2[3])
        if l == H.levels - 1:
            continue
        kinv = np.fromfile(f"{prefix}_kinv{l}.bin", dtype=np.float64).reshape(-1, 8, 8)
        cells = np.argwhere(dom.v1[3])
        idx, act = vanka_slots(dom, cells)
        K = vanka_local_matrix(dom.eta, dom.h, dom.gamma, act, vanka_diagonals(dom, idx))
        types = (wp[tuple(cells.T)] >> 17) & 1023
        for c in range(cells.shape[0]):
            live = [s for s in range(7) if act[c, s]]
            want = np.linalg.inv(K[c][np.ix_(live, live)])
            got = kinv[types[c]][np.ix_(live, live)]
            assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max()), (l, cells[c])
