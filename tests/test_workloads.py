"""Pins of the seeded input generators (they hold no solver arithmetic)."""
import math

import numpy as np
import sympy as sym

from paper_2312_10615_amd import workloads as W


def test_mms_force_is_the_continuous_stokes_residual():
    x, y, z, eta = sym.symbols("x y z eta")
    psi = (sym.sin(sym.pi * x) * sym.sin(sym.pi * y) * sym.sin(sym.pi * z)) ** 3
    g = [sym.diff(psi, v) for v in (x, y, z)]
    u = [g[1] - g[2], g[2] - g[0], g[0] - g[1]]
    p = sym.cos(sym.pi * x) * sym.cos(sym.pi * y) * sym.cos(sym.pi * z)
    lap = lambda f: sum(sym.diff(f, v, 2) for v in (x, y, z))
    f = [-eta * lap(u[a]) + sym.diff(p, v) for a, v in enumerate((x, y, z))]
    div = sum(sym.diff(u[a], v) for a, v in enumerate((x, y, z)))
    rng = np.random.default_rng(0)
    for _ in range(5):
        pt = rng.uniform(0, 1, 3)
        subs = {x: pt[0], y: pt[1], z: pt[2], eta: 0.7}
        X, Y, Z = (np.array(v) for v in pt)
        for a in range(3):
            assert math.isclose(float(f[a].evalf(subs=subs)), float(W.mms_force(a, X, Y, Z, 0.7)), rel_tol=1e-11, abs_tol=1e-11)
            assert math.isclose(float(u[a].evalf(subs=subs)), float(W.mms_velocity(a, X, Y, Z)), rel_tol=1e-12, abs_tol=1e-13)
        assert abs(float(div.evalf(subs=subs))) < 1e-10
    # no-slip: velocity vanishes on the walls
    for a in range(3):
        assert abs(W.mms_velocity(a, np.array(0.0), np.array(0.3), np.array(0.6))) < 1e-14


def test_forcing_is_seeded_and_sized():
    f1 = W.sinusoid_forcing(8, 6, 4, 0.125, seed=3)
    f2 = W.sinusoid_forcing(8, 6, 4, 0.125, seed=3)
    f3 = W.sinusoid_forcing(8, 6, 4, 0.125, seed=4)
    assert [a.shape for a in f1] == [(9, 6, 4), (8, 7, 4), (8, 6, 5)]
    assert all(np.array_equal(a, b) for a, b in zip(f1, f2))
    assert not np.array_equal(f1[0], f3[0])


def test_device_forcing_generator_agrees_with_numpy():
    import torch
    from paper_2312_10615_amd.workloads import sinusoid_forcing, sinusoid_forcing_device
    a = sinusoid_forcing(12, 8, 10, 1 / 12, seed=5)
    b = sinusoid_forcing_device(12, 8, 10, 1 / 12, seed=5, device="cpu")
    for x, y in zip(a, b):
        assert isinstance(y, torch.Tensor) and tuple(y.shape) == x.shape
        assert np.allclose(y.numpy(), x, rtol=0, atol=1e-12)
