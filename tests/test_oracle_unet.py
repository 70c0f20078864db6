"""Pins of the warm-start network oracle against definitions it does not use
itself: brute-force loops, adjoint identities, finite differences, a library
bfloat16 conversion and closed forms of Adam's first step."""
import numpy as np
import pytest
import torch

from oracle import unet as U


def brute_conv3(x, w, b):
    D, H, W, cin = x.shape
    cout = w.shape[2]
    y = np.zeros((D, H, W, cout))
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for co in range(cout):
                    s = b[co]
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, y2, x2 = z + dz, yy + dy, xx + dx
                                if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    for ci in range(cin):
                                        s += x[zz, y2, x2, ci] * w[t, ci, co]
                    y[z, yy, xx, co] = s
    return y


def test_conv3_matches_loops_on_non_cubic_grid():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    assert np.allclose(U.conv3(x, w, b), brute_conv3(x, w, b), rtol=0, atol=1e-12)


def test_conv3_centre_tap_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 4, 8))
    w = np.zeros((27, 8, 8))
    w[13] = np.eye(8)
    assert np.array_equal(U.conv3(x, w, np.zeros(8)), x)


def test_conv3_gradients_are_adjoint_of_forward():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 5, 3))
    w = rng.standard_normal((27, 3, 2))
    dz = rng.standard_normal((4, 6, 5, 2))
    y = U.conv3(x, w, np.zeros(2))
    lhs = np.sum(y * dz)
    assert np.isclose(np.sum(x * U.conv3_grad_input(dz, w)), lhs, rtol=1e-12)
    dw, db = U.conv3_grad_weight(x, dz)
    assert np.isclose(np.sum(w * dw), lhs, rtol=1e-12)
    assert np.allclose(db, dz.sum(axis=(0, 1, 2)))


def test_pool_up_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(U.pool(x) * y), np.sum(x * U.pool_grad(y)), rtol=1e-12)
    assert np.isclose(np.sum(U.up(y) * x), np.sum(y * U.up_grad(x)), rtol=1e-12)
    assert np.allclose(U.pool(U.up(y)), y, rtol=1e-15, atol=0)
    # a brute-force check of the pooling definition at one coarse voxel
    assert np.isclose(U.pool(x)[1, 2, 3, 1], x[2:4, 4:6, 6:8, 1].mean())


def test_round_bf16_matches_library_conversion():
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, 3.0]])
    # torch converts float32 to bfloat16 with round-to-nearest-even; use inputs
    # exactly representable in float32 so no double rounding is involved
    a = a.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(a).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.round_bf16(a), ref)
    assert U.round_bf16(1.0 + 2.0 ** -8) == 1.0                # tie to even
    assert U.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def _tiny_problem(n=8, seed=5):
    rng = np.random.default_rng(seed)
    params = U.init_params(seed)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape) * 0.1
    x = np.zeros((n, n, n, U.IN_CHANNELS))
    x[..., :3] = rng.standard_normal((n, n, n, 3))
    target = rng.standard_normal((n, n, n, U.HEAD_OUT))
    mask = U.unknown_mask(n, n, n)
    return params, x, target, mask


def test_network_gradient_matches_finite_differences():
    params, x, target, mask = _tiny_problem()
    out, cache = U.forward(params, x, rounding=False)
    g = U.backward(params, cache, U.loss_grad(out, target, mask), rounding=False)
    rng = np.random.default_rng(6)
    for k in list(params):
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in params[k].shape)
            eps = 1e-6 * max(1.0, abs(params[k][idx]))
            vals = []
            for sgn in (1, -1):
                p2 = {kk: vv.copy() for kk, vv in params.items()}
                p2[k][idx] += sgn * eps
                vals.append(U.loss(U.forward(p2, x, rounding=False)[0], target, mask))
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, idx, fd, g[k][idx])


def test_rounded_network_stays_near_exact_network():
    params, x, target, mask = _tiny_problem()
    o1, c1 = U.forward(params, x, rounding=True)
    o0, c0 = U.forward(params, x, rounding=False)
    assert np.linalg.norm(o1 - o0) <= 0.05 * np.linalg.norm(o0)
    g1 = U.backward(params, c1, U.loss_grad(o1, target, mask), rounding=True)
    g0 = U.backward(params, c0, U.loss_grad(o0, target, mask), rounding=False)
    # bfloat16 activation gradients lose 2^-9 per rounding and flip ReLU masks at
    # this tiny size; through ten layers the parameter gradients stay within 25%
    for k in g0:
        assert np.linalg.norm(g1[k] - g0[k]) <= 0.25 * np.linalg.norm(g0[k]) + 1e-12, k


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(7)
    p = {"w": rng.standard_normal((3, 4))}
    g = {"w": rng.standard_normal((3, 4))}
    w0 = p["w"].copy()
    st = {}
    U.adam_step(p, g, st, step=1, lr=1e-2)
    # bias correction makes the first moment g and the second g^2 exactly
    assert np.allclose(p["w"], w0 - 1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=0, atol=1e-15)
    # with the same gradient again, the bias-corrected moments are again g and
    # g^2 (the (1 - beta^2) factors cancel), so the step is the same
    w1 = p["w"].copy()
    U.adam_step(p, g, st, step=2, lr=1e-2)
    assert np.allclose(p["w"] - w1, -1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("dims", [(4, 5, 6), (8, 8, 8)])
def test_voxel_layout_round_trip_and_unknown_count(dims):
    nx, ny, nz = dims
    rng = np.random.default_rng(8)
    ux = rng.standard_normal((nx + 1, ny, nz))
    uy = rng.standard_normal((nx, ny + 1, nz))
    uz = rng.standard_normal((nx, ny, nz + 1))
    p = rng.standard_normal((nx, ny, nz))
    for a, ax in ((ux, 0), (uy, 1), (uz, 2)):
        sl = [slice(None)] * 3
        sl[ax] = 0
        a[tuple(sl)] = 0.0
        sl[ax] = -1
        a[tuple(sl)] = 0.0
    v = U.to_voxels(ux, uy, uz, p, channels=4)
    back = U.from_voxels(v)
    for a, b in zip((ux, uy, uz, p), back):
        assert np.array_equal(a, b)
    # unknowns of the 4-channel state: 3 velocity lattices with one wall-normal
    # face pair removed each, plus every cell (the count behind Table 1)
    n_u = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert U.unknown_mask(nx, ny, nz).sum() == n_u + nx * ny * nz
    assert v[2, 3, 1, 0] == ux[1, 3, 2] and v[2, 3, 1, 3] == p[1, 3, 2]
