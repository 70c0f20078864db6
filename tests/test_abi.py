"""The C-ABI library loads without a GPU and exports every symbol the header
declares; host-side validation works without a device."""
import os
import re

import pytest

from paper_2312_10615_amd import stokes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokes_mgsqmr.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(stokes_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("stokes_setup", "stokes_vcycle", "stokes_solve", "stokes_apply", "stokes_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = S.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(S.EXPORTS) == declared_functions()


def test_defaults_and_workspace_sizes():
    p = S.stokes_default_params(32, 32, 32, 1 / 32)
    assert (p.eta, p.gamma, p.levels, p.nu, p.n_boundary, p.vcycle_precision, p.smoother) == \
        (1.0, 1e-3, 0, 2, 1, 64, S.SMOOTHERS["symmetric"])
    small = S.stokes_workspace_bytes(p)
    big = S.stokes_workspace_bytes(S.stokes_default_params(64, 64, 64, 1 / 64))
    assert 0 < small < big
    # four SQMR vectors of (N+2)^3-ish float64 slots at least
    assert small >= 4 * 4 * 34 ** 3 * 8
    p.vcycle_precision = 32
    mixed = S.stokes_workspace_bytes(p)
    # FP32 level buffers (plus the level-0 copies) are smaller than FP64 ones
    assert 0 < mixed < small * 1.1


@pytest.mark.parametrize("field,value", [("nx", 1), ("h", 0.0), ("eta", -1.0), ("gamma", 0.0), ("gamma", -1e-3),
                                         ("nu", 0), ("n_boundary", 0),
                                         ("vcycle_precision", 16), ("vcycle_precision", 33), ("levels", 6), ("levels", -1), ("smoother", 7),
                                         ("vanka", 3), ("cycle", 3), ("cycle", 0),
                                         ("symmetric-odd-nu", 3)])
def test_invalid_parameters_are_rejected_on_the_host(field, value):
    p = S.stokes_default_params(32, 32, 32, 1 / 32)
    if field == "symmetric-odd-nu":
        p.smoother, p.nu = S.SMOOTHERS["symmetric"], value
    else:
        setattr(p, field, value)
    with pytest.raises(S.StokesError) as e:
        S.stokes_workspace_bytes(p)
    assert e.value.code == S.STOKES_EINVAL


def test_levels_rule_matches_auto_choice():
    # 48 -> 24 -> 12 -> 6 (auto: 4 levels); explicit 5 reaches 3 cells (allowed as
    # the coarsest); a sixth level would need to halve an odd axis
    p = S.stokes_default_params(48, 48, 48, 1 / 48)
    S.stokes_workspace_bytes(p)
    p.levels = 5
    S.stokes_workspace_bytes(p)
    p.levels = 6
    with pytest.raises(S.StokesError):
        S.stokes_workspace_bytes(p)


def test_setup_rejects_null_workspace_without_touching_a_device():
    p = S.stokes_default_params(8, 8, 8, 1 / 8)
    with pytest.raises(S.StokesError) as e:
        S.stokes_setup(p, 0, 0, 0)
    assert e.value.code == S.STOKES_EINVAL


def test_strerror_names_every_status():
    for code in range(7):
        assert S.stokes_strerror(code) != "unknown status"


def test_static_solve_rejects_oversized_and_null_inputs_on_the_host():
    """stokes_solve_static checks the problem against its static scratch
    (64 MiB) and its pointers before any GPU work."""
    p = S.stokes_default_params(64, 64, 64, 1 / 64)
    assert S.stokes_workspace_bytes(p) <= S.STOKES_STATIC_BYTES
    big = S.stokes_default_params(128, 128, 128, 1 / 128)
    assert S.stokes_workspace_bytes(big) > S.STOKES_STATIC_BYTES
    code, _, _ = S.stokes_solve_static(big, 0, 0, 1e-8, 10, 0)
    assert code == S.STOKES_ETOOLARGE
    code, _, _ = S.stokes_solve_static(S.stokes_default_params(16, 16, 16, 1 / 16), 0, 0, 1e-8, 10, 0)
    assert code == S.STOKES_EINVAL


@pytest.mark.parametrize("dims", [(4, 4, 4), (5, 6, 7), (16, 9, 3)])
def test_red_black_field_index_is_a_bijection_split_by_colour(dims):
    """Host view of the state layout: odd pitches make the slot parity the
    cell colour (I + J + K) & 1, and each field stores colour 0 in its first
    half and colour 1 in its second, every slot at its own element."""
    import types

    import torch
    nx, ny, nz = dims
    sy = (nx + 2) | 1
    sz = (sy * (ny + 2)) | 1
    slots = sz * (nz + 2)
    lay = types.SimpleNamespace(nx=nx, ny=ny, nz=nz, sy=sy, sz=sz, field=(slots + 15) // 8 * 8)
    e = S.field_index(lay, "cpu")
    assert e.shape == (nz + 2, ny + 2, sy)
    flat = e.flatten()
    assert flat.unique().numel() == flat.numel() and int(flat.min()) >= 0 and int(flat.max()) < lay.field
    K, J, I = torch.meshgrid(torch.arange(nz + 2), torch.arange(ny + 2), torch.arange(sy), indexing="ij")
    colour = (I + J + K) & 1
    assert bool(((e >= lay.field // 2) == (colour == 1)).all())
    # along a row, same-colour cells are neighbours in memory
    assert bool((e[1, 1, 3::2][:-1] + 1 == e[1, 1, 3::2][1:]).all())


def test_labels_are_validated_on_the_host():
    """Labelled domains: a valid label array is sized like the box; a label
    value above 2, an interior cell on the outer layer, or labels passed to the
    batch calls are rejected without a device."""
    import ctypes

    import numpy as np
    n = 8
    lab = np.ones((n + 2,) * 3, dtype=np.uint8)
    lab[1:-1, 1:-1, 1:-1] = 0
    lab[-1, 1:-1, 1:-1] = 2
    p = S.stokes_default_params(n, n, n, 1 / n)
    box = S.stokes_workspace_bytes(p)
    p.labels = lab.ctypes.data
    assert S.stokes_workspace_bytes(p) > box     # the flag words
    bad = lab.copy()
    bad[0, 3, 3] = 0
    p.labels = bad.ctypes.data
    with pytest.raises(S.StokesError):
        S.stokes_workspace_bytes(p)
    bad = lab.copy()
    bad[4, 4, 4] = 3
    p.labels = bad.ctypes.data
    with pytest.raises(S.StokesError):
        S.stokes_workspace_bytes(p)
    p.labels = lab.ctypes.data
    arr = (S.StokesParams * 1)(p)
    nbytes = ctypes.c_size_t(0)
    assert S.load_library().stokes_batch_workspace_bytes(1, arr, ctypes.byref(nbytes)) == S.STOKES_EINVAL
