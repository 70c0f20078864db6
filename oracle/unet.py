"""Learned warm start: the 3D U-Net whose output is SQMR's initial guess (oracle).

TEST INFRASTRUCTURE ONLY.  Plain float64 NumPy, written for clarity, never for
speed.  Only tests, the smoke check and the benchmark's CPU baseline use it.

Alg. 4 (SQMR) starts from an arbitrary x0; the method itself is unchanged by
where x0 comes from.  This module defines the network that proposes x0 from
the forcing and computes, layer by layer:
  * the forward pass (`forward`),
  * the gradients of the training loss by the chain rule written out per layer
    (`backward`),
  * one Adam step (`adam_step`, Kingma & Ba 2015, Algorithm 1).

Network (a 3-level U-Net, channels 16/32/64, 3x3x3 convolutions with zero
padding, ReLU after every convolution, 2x2x2 average pooling down, nearest
neighbour upsampling up, skip tensors concatenated after the upsampled one):

  c0a: in(8)            -> 16      c0b: 16 -> 16          = e0   (N^3)
  c1a: pool(e0) 16      -> 32      c1b: 32 -> 32          = e1   ((N/2)^3)
  c2a: pool(e1) 32      -> 64      c2b: 64 -> 64          = e2   ((N/4)^3)
  c1c: [up(e2), e1] 96  -> 32      c1d: 32 -> 32          = d1   ((N/2)^3)
  c0c: [up(d1), e0] 48  -> 16      c0d: 16 -> 16          = d0   (N^3)
  head: 1x1x1 16 -> 4, no activation, float output.

Voxel tensors are [z, y, x, channel] (x fastest, channel innermost).  The
staggered state maps onto N^3 voxels by giving voxel (i, j, k) the u_x of its
minus-x face (face index i), likewise u_y and u_z, and its cell-centre p.  The
plus-side wall faces are dropped (always zero); the minus-side wall faces
(index 0) are kept as zero entries that the loss ignores.

Precision model (mirrors the GPU kernels): weights and activations are bfloat16
(round to nearest even), sums are exact here (float32 on the GPU), biases and
the head output are not rounded.  `rounding=False` turns every rounding off,
which makes the network a smooth function for finite-difference checks.
"""
from __future__ import annotations

import numpy as np

# (name, input spec, cin, cout).  Input spec: "in" (the forcing), a layer name,
# ("pool", name) or ("cat", ("up", coarse name), skip name).
LAYERS = (
    ("c0a", "in", 8, 16),
    ("c0b", "c0a", 16, 16),
    ("c1a", ("pool", "c0b"), 16, 32),
    ("c1b", "c1a", 32, 32),
    ("c2a", ("pool", "c1b"), 32, 64),
    ("c2b", "c2a", 64, 64),
    ("c1c", ("cat", ("up", "c2b"), "c1b"), 96, 32),
    ("c1d", "c1c", 32, 32),
    ("c0c", ("cat", ("up", "c1d"), "c0b"), 48, 16),
    ("c0d", "c0c", 16, 16),
)
HEAD_IN, HEAD_OUT = 16, 4
IN_CHANNELS = 8      # forcing (3) padded with zero channels to a multiple of 8
TAPS = tuple((dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))


def round_bf16(a):
    """Round float64 values to the nearest bfloat16 (8 significant bits), ties to even."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                     # a = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def _r(a, rounding):
    return round_bf16(a) if rounding else a


# ---------------------------------------------------------------- layers ---

def conv3(x, w, b):
    """3x3x3 convolution (cross-correlation) with zero padding:
    y[v] = b + sum_t x[v + tap_t] @ w[t];  x [D,H,W,Cin], w [27,Cin,Cout]."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, W, w.shape[2]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] @ w[t]
    return y + b


def conv3_grad_input(dz, w):
    """d/dx of sum(dz * conv3(x, w, b)): dx[v] = sum_t dz[v - tap_t] @ w[t]^T."""
    D, H, W, _ = dz.shape
    dp = np.pad(dz, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((D, H, W, w.shape[1]))
    for t, (oz, oy, ox) in enumerate(TAPS):
        dx += dp[1 - oz:1 - oz + D, 1 - oy:1 - oy + H, 1 - ox:1 - ox + W, :] @ w[t].T
    return dx


def conv3_grad_weight(x, dz):
    """d/dw of sum(dz * conv3(x, w, b)): dw[t] = sum_v x[v + tap_t]^T dz[v]; and db."""
    D, H, W, cin = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((27, cin, dz.shape[3]))
    for t, (oz, oy, ox) in enumerate(TAPS):
        xs = xp[1 + oz:1 + oz + D, 1 + oy:1 + oy + H, 1 + ox:1 + ox + W, :]
        dw[t] = xs.reshape(-1, cin).T @ dz.reshape(-1, dz.shape[3])
    return dw, dz.sum(axis=(0, 1, 2))


def pool(x):
    """2x2x2 average: y[v] = mean of the 8 children of v."""
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_grad(dy):
    """Adjoint of `pool`: each child receives dy/8."""
    return up(dy) / 8.0


def up(x):
    """Nearest-neighbour doubling: every child copies its parent."""
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up_grad(dy):
    """Adjoint of `up`: each parent receives the sum over its 8 children."""
    D, H, W, C = dy.shape
    return dy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


# ---------------------------------------------------------------- network ---

def init_params(seed=0):
    """He-style initialisation of every layer (float32 master values stored as float64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, _, cin, cout in LAYERS:
        fan_in = 27 * cin
        p[name + ".w"] = (rng.standard_normal((27, cin, cout)) * np.sqrt(2.0 / fan_in)).astype(np.float32).astype(
            np.float64)
        p[name + ".b"] = np.zeros(cout)
    p["head.w"] = (rng.standard_normal((HEAD_IN, HEAD_OUT)) * np.sqrt(1.0 / HEAD_IN)).astype(np.float32).astype(
        np.float64)
    p["head.b"] = np.zeros(HEAD_OUT)
    return p


def _layer_input(spec, acts, x_in, rounding):
    if spec == "in":
        return x_in
    if isinstance(spec, str):
        return acts[spec]
    if spec[0] == "pool":
        return _r(pool(acts[spec[1]]), rounding)
    if spec[0] == "cat":
        return np.concatenate([up(acts[spec[1][1]]), acts[spec[2]]], axis=3)
    raise ValueError(spec)


def forward(params, x_in, rounding=True):
    """Network output (head values, float) for an input [N,N,N,8]; returns (out, cache)."""
    x_in = _r(x_in, rounding)
    acts, inputs, pre = {}, {}, {}
    for name, spec, cin, cout in LAYERS:
        xi = _layer_input(spec, acts, x_in, rounding)
        assert xi.shape[3] == cin, (name, xi.shape)
        z = conv3(xi, _r(params[name + ".w"], rounding), params[name + ".b"])
        inputs[name] = xi
        pre[name] = z
        acts[name] = _r(np.maximum(z, 0.0), rounding)
    out = acts["c0d"] @ _r(params["head.w"], rounding) + params["head.b"]
    return out, {"acts": acts, "inputs": inputs, "pre": pre, "x_in": x_in}


def loss(out, target, mask):
    """Mean squared error over the entries where mask is 1: sum(mask (o - t)^2) / sum(mask)."""
    n = mask.sum()
    return float((mask * (out - target) ** 2).sum() / n)


def loss_grad(out, target, mask):
    return 2.0 * mask * (out - target) / mask.sum()


def backward(params, cache, dout, rounding=True):
    """Gradients of a scalar loss with d loss / d out = dout, for every parameter.

    Activation gradients are bfloat16 where the GPU stores them: each layer's
    input gradient is rounded as it is produced, and a tensor read by two
    layers (a skip) sums both contributions exactly and rounds the sum once,
    when its own layer's backward step starts.  Weight and bias gradients are
    not rounded."""
    acts, inputs = cache["acts"], cache["inputs"]
    g = {}
    hw = _r(params["head.w"], rounding)
    g["head.w"] = acts["c0d"].reshape(-1, HEAD_IN).T @ dout.reshape(-1, HEAD_OUT)
    g["head.b"] = dout.sum(axis=(0, 1, 2))
    dact = {"c0d": dout @ hw.T}
    for name, spec, cin, cout in reversed(LAYERS):
        dy = _r(dact.pop(name), rounding)   # every consumer of this tensor has run
        dz = dy * (acts[name] > 0)
        w = _r(params[name + ".w"], rounding)
        g[name + ".w"], g[name + ".b"] = conv3_grad_weight(inputs[name], dz)
        if spec == "in":
            continue
        dx = _r(conv3_grad_input(dz, w), rounding)
        if isinstance(spec, str):
            contrib = {spec: dx}
        elif spec[0] == "pool":
            contrib = {spec[1]: pool_grad(dx)}
        else:
            cc = acts[spec[1][1]].shape[3]
            contrib = {spec[1][1]: up_grad(dx[..., :cc]), spec[2]: dx[..., cc:]}
        for k, v in contrib.items():
            dact[k] = dact[k] + v if k in dact else v
    return g


def adam_step(params, grads, state, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) of every parameter, in place.
    `step` counts from 1.  state holds the first and second moment per parameter."""
    for k in params:
        m = state.setdefault(k + ".m", np.zeros_like(params[k]))
        v = state.setdefault(k + ".v", np.zeros_like(params[k]))
        m[...] = beta1 * m + (1.0 - beta1) * grads[k]
        v[...] = beta2 * v + (1.0 - beta2) * grads[k] ** 2
        mhat = m / (1.0 - beta1 ** step)
        vhat = v / (1.0 - beta2 ** step)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params


# ------------------------------------------------------ staggered <-> voxel ---

def to_voxels(ux, uy, uz, p=None, channels=IN_CHANNELS):
    """Natural staggered arrays ([i,j,k], u_x of shape (nx+1,ny,nz), ...) to a
    voxel tensor [k,j,i,c]: channels u_x(minus face), u_y, u_z, then p (or 0)."""
    nx, ny, nz = ux.shape[0] - 1, uy.shape[1] - 1, uz.shape[2] - 1
    v = np.zeros((nz, ny, nx, channels))
    v[..., 0] = ux[:nx].transpose(2, 1, 0)
    v[..., 1] = uy[:, :ny].transpose(2, 1, 0)
    v[..., 2] = uz[:, :, :nz].transpose(2, 1, 0)
    if p is not None:
        v[..., 3] = p.transpose(2, 1, 0)
    return v


def from_voxels(v):
    """Inverse of `to_voxels` for a 4-channel output; wall faces come back as 0."""
    nz, ny, nx, _ = v.shape
    ux = np.zeros((nx + 1, ny, nz))
    uy = np.zeros((nx, ny + 1, nz))
    uz = np.zeros((nx, ny, nz + 1))
    ux[1:nx] = v[:, :, 1:, 0].transpose(2, 1, 0)
    uy[:, 1:ny] = v[:, 1:, :, 1].transpose(2, 1, 0)
    uz[:, :, 1:nz] = v[1:, :, :, 2].transpose(2, 1, 0)
    p = v[..., 3].transpose(2, 1, 0).copy()
    return ux, uy, uz, p


def unknown_mask(nx, ny, nz):
    """1 where a voxel channel holds an unknown of the 4-channel state, else 0."""
    m = np.ones((nz, ny, nx, HEAD_OUT))
    m[:, :, 0, 0] = 0.0
    m[:, 0, :, 1] = 0.0
    m[0, :, :, 2] = 0.0
    return m
