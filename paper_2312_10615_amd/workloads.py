"""Seeded synthetic inputs for the 3D MAC Stokes problem.

This module only samples analytic functions and draws random numbers.  It
holds none of the solver's arithmetic (no stencil, no transfer operator, no
smoother), so both the CPU oracle and the GPU path can take their inputs from
it without sharing any part of the method.

Geometry convention (the paper's staggered MAC grid, Section 2 / Eq. 2):
  * a box of nx*ny*nz cells of edge h, occupying [0, nx*h] x [0, ny*h] x [0, nz*h];
  * u_x lives at x-face centres (i*h, (j+1/2)h, (k+1/2)h), i = 0..nx, array shape
    (nx+1, ny, nz); u_y and u_z are analogous; p lives at cell centres
    ((i+1/2)h, (j+1/2)h, (k+1/2)h), shape (nx, ny, nz).
  * Faces i = 0 and i = nx of u_x lie on the walls.  Generators return values
    there too; consumers ignore them (they are not unknowns).

Every array is float64 and indexed [i, j, k] with i along x.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "face_centres",
    "cell_centres",
    "sinusoid_forcing",
    "sinusoid_forcing_device",
    "batch_dims",
    "mms_fields",
    "random_state",
]


def face_centres(nx: int, ny: int, nz: int, h: float, axis: int):
    """Coordinates (X, Y, Z) of the face centres normal to `axis`, broadcastable."""
    dims = [nx, ny, nz]
    coords = []
    for a in range(3):
        if a == axis:
            c = np.arange(dims[a] + 1, dtype=np.float64) * h
        else:
            c = (np.arange(dims[a], dtype=np.float64) + 0.5) * h
        shape = [1, 1, 1]
        shape[a] = c.size
        coords.append(c.reshape(shape))
    return coords


def cell_centres(nx: int, ny: int, nz: int, h: float):
    coords = []
    for a, n in enumerate((nx, ny, nz)):
        c = (np.arange(n, dtype=np.float64) + 0.5) * h
        shape = [1, 1, 1]
        shape[a] = n
        coords.append(c.reshape(shape))
    return coords


def sinusoid_forcing(nx: int, ny: int, nz: int, h: float, seed: int, n_modes: int = 8):
    """Body force as a seeded sum of random-phase sinusoids, one sum per component.

    For each component c in (x, y, z) and each mode m < n_modes, in that order,
    the PCG64 stream `numpy.random.default_rng(seed)` gives an integer wave
    vector k in {1..4}^3, an amplitude A ~ N(0, 1) and a phase phi ~ U(0, 2pi);
    f_c = sum_m A sin(2 pi k . x + phi) evaluated at the c-face centres.
    The continuity right-hand side is zero.  Returns (fx, fy, fz).
    """
    rng = np.random.default_rng(seed)
    out = []
    for axis in range(3):
        X, Y, Z = face_centres(nx, ny, nz, h, axis)
        f = np.zeros(np.broadcast_shapes(X.shape, Y.shape, Z.shape), dtype=np.float64)
        for _ in range(n_modes):
            k = rng.integers(1, 5, size=3)
            amp = rng.standard_normal()
            phase = rng.uniform(0.0, 2.0 * math.pi)
            f += amp * np.sin(2.0 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + phase)
        out.append(f)
    return tuple(out)


# ---------------------------------------------------------------------------
# Manufactured solution on the unit cube.
#
# Potential psi = s(x) s(y) s(z) with s(t) = sin^3(pi t); velocity
# u = curl(psi, psi, psi) = (d_y psi - d_z psi, d_z psi - d_x psi, d_x psi - d_y psi),
# which is divergence free and vanishes, with its first derivatives, on every
# wall of [0,1]^3 (s and s' are zero at t = 0 and t = 1).  Pressure
# p = cos(pi x) cos(pi y) cos(pi z) has zero mean over any symmetric set of
# cell centres.  The body force is the continuous Stokes residual
# f = -eta * Laplacian(u) + grad(p), written out in closed form below.
# ---------------------------------------------------------------------------

def _s(t):
    return np.sin(math.pi * t) ** 3


def _s1(t):
    return 3.0 * math.pi * np.sin(math.pi * t) ** 2 * np.cos(math.pi * t)


def _s2(t):
    sn = np.sin(math.pi * t)
    return 3.0 * math.pi ** 2 * sn * (2.0 - 3.0 * sn * sn)


def _s3(t):
    sn = np.sin(math.pi * t)
    return 3.0 * math.pi ** 3 * np.cos(math.pi * t) * (2.0 - 9.0 * sn * sn)


def _grad_psi(X, Y, Z):
    return (_s1(X) * _s(Y) * _s(Z), _s(X) * _s1(Y) * _s(Z), _s(X) * _s(Y) * _s1(Z))


def _grad_lap_psi(X, Y, Z):
    """Gradient of Laplacian(psi)."""
    gx = _s3(X) * _s(Y) * _s(Z) + _s1(X) * _s2(Y) * _s(Z) + _s1(X) * _s(Y) * _s2(Z)
    gy = _s2(X) * _s1(Y) * _s(Z) + _s(X) * _s3(Y) * _s(Z) + _s(X) * _s1(Y) * _s2(Z)
    gz = _s2(X) * _s(Y) * _s1(Z) + _s(X) * _s2(Y) * _s1(Z) + _s(X) * _s(Y) * _s3(Z)
    return gx, gy, gz


def mms_velocity(axis: int, X, Y, Z):
    g = _grad_psi(X, Y, Z)
    a, b = (axis + 1) % 3, (axis + 2) % 3
    return g[a] - g[b]


def mms_pressure(X, Y, Z):
    return np.cos(math.pi * X) * np.cos(math.pi * Y) * np.cos(math.pi * Z)


def mms_force(axis: int, X, Y, Z, eta: float):
    gl = _grad_lap_psi(X, Y, Z)
    a, b = (axis + 1) % 3, (axis + 2) % 3
    lap_u = gl[a] - gl[b]
    cx, cy, cz = (np.cos(math.pi * X), np.cos(math.pi * Y), np.cos(math.pi * Z))
    sx, sy, sz = (np.sin(math.pi * X), np.sin(math.pi * Y), np.sin(math.pi * Z))
    grad_p = (-math.pi * sx * cy * cz, -math.pi * cx * sy * cz, -math.pi * cx * cy * sz)[axis]
    return -eta * lap_u + grad_p


def sinusoid_forcing_device(nx: int, ny: int, nz: int, h: float, seed: int, device, n_modes: int = 8):
    """`sinusoid_forcing` evaluated with torch on `device` (float64): the same
    draws from the same PCG64 stream in the same order, so the two agree to the
    rounding of the sine.  For generating many large right-hand sides quickly.
    Returns torch tensors (fx, fy, fz) indexed [i, j, k]."""
    import torch
    rng = np.random.default_rng(seed)
    dims = (nx, ny, nz)
    out = []
    for axis in range(3):
        coords = []
        for a in range(3):
            n = dims[a] + 1 if a == axis else dims[a]
            c = torch.arange(n, dtype=torch.float64, device=device) * h
            if a != axis:
                c = c + 0.5 * h
            shape = [1, 1, 1]
            shape[a] = n
            coords.append(c.reshape(shape))
        X, Y, Z = coords
        f = torch.zeros((X.shape[0], Y.shape[1], Z.shape[2]), dtype=torch.float64, device=device)
        for _ in range(n_modes):
            k = rng.integers(1, 5, size=3)
            amp = rng.standard_normal()
            phase = rng.uniform(0.0, 2.0 * math.pi)
            f += amp * torch.sin(2.0 * math.pi * (int(k[0]) * X + int(k[1]) * Y + int(k[2]) * Z) + phase)
        out.append(f)
    return tuple(out)


def batch_dims(n_domains: int = 48, choices=(32, 48, 64, 96, 128), seed: int = 0):
    """Box sizes of a batched workload: each of nx, ny, nz drawn uniformly from
    `choices` (PCG64 stream `numpy.random.default_rng(seed)`, domain by domain,
    x then y then z).  Returns a list of (nx, ny, nz)."""
    rng = np.random.default_rng(seed)
    return [tuple(int(choices[i]) for i in rng.integers(0, len(choices), size=3)) for _ in range(n_domains)]


def mms_fields(n: int, eta: float = 1.0):
    """Manufactured solution sampled on the n^3 MAC grid of the unit cube (h = 1/n).

    Returns dict with 'f' = (fx, fy, fz) at face centres, 'u' = (ux, uy, uz)
    exact velocity at face centres, 'p' exact pressure at cell centres.
    """
    h = 1.0 / n
    f, u = [], []
    for axis in range(3):
        X, Y, Z = face_centres(n, n, n, h, axis)
        f.append(np.broadcast_to(mms_force(axis, X, Y, Z, eta), (n + (axis == 0), n + (axis == 1), n + (axis == 2))).copy())
        u.append(np.broadcast_to(mms_velocity(axis, X, Y, Z), f[-1].shape).copy())
    X, Y, Z = cell_centres(n, n, n, h)
    p = np.broadcast_to(mms_pressure(X, Y, Z), (n, n, n)).copy()
    return {"f": tuple(f), "u": tuple(u), "p": p}


def random_state(nx: int, ny: int, nz: int, seed: int):
    """Standard-normal values at every face and cell position (walls included;
    consumers zero what is not an unknown).  Returns (ux, uy, uz, p)."""
    rng = np.random.default_rng(seed)
    ux = rng.standard_normal((nx + 1, ny, nz))
    uy = rng.standard_normal((nx, ny + 1, nz))
    uz = rng.standard_normal((nx, ny, nz + 1))
    p = rng.standard_normal((nx, ny, nz))
    return ux, uy, uz, p
