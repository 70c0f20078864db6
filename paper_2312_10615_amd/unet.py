"""Learned warm start: the 3D U-Net that proposes SQMR's initial guess.

Thin binding of libstokes_unet.so (include/stokes_unet.h) plus the layer
schedule of the network.  Every arithmetic step runs in the library's HIP
kernels; PyTorch only provides device memory.  Alg. 4 of the paper accepts
any x0; `WarmStartNet.initial_guess` supplies one from the forcing, and the
solve that follows is the unchanged MG-SQMR.

Network (3 levels, 16/32/64 channels, 3x3x3 convolutions + ReLU, 2x2x2
average pooling down, nearest upsampling + skip concatenation up, 1x1x1 head
to (u_x, u_y, u_z, p) in float).  Input: the forcing of the voxel's minus faces
divided by its RMS; output: the state divided by (RMS * sigma_c).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstokes_unet.so")
_lib = None

UNET_OK, UNET_EINVAL, UNET_EDEVICE = 0, 1, 5
SRC_DIRECT, SRC_POOL, SRC_CAT_UP, SRC_MASKED = 0, 1, 2, 3

# (name, input spec, cin, cout); spec: "in", a layer, ("pool", layer) or ("cat", coarse layer, skip layer)
LAYERS = (
    ("c0a", "in", 8, 16),
    ("c0b", "c0a", 16, 16),
    ("c1a", ("pool", "c0b"), 16, 32),
    ("c1b", "c1a", 32, 32),
    ("c2a", ("pool", "c1b"), 32, 64),
    ("c2b", "c2a", 64, 64),
    ("c1c", ("cat", "c2b", "c1b"), 96, 32),
    ("c1d", "c1c", 32, 32),
    ("c0c", ("cat", "c1d", "c0b"), 48, 16),
    ("c0d", "c0c", 16, 16),
)
LEVEL = {"c0a": 0, "c0b": 0, "c1a": 1, "c1b": 1, "c2a": 2, "c2b": 2, "c1c": 1, "c1d": 1, "c0c": 0, "c0d": 0}
HEAD_IN, HEAD_OUT, IN_CH = 16, 4, 8

EXPORTS = ("unet_packed_elems", "unet_pack_weights", "unet_conv3", "unet_wgrad_workspace_bytes", "unet_conv3_wgrad",
           "unet_up_grad", "unet_skip_grad", "unet_head_forward", "unet_head_workspace_bytes", "unet_head_backward",
           "unet_mse_workspace_bytes", "unet_mse", "unet_adam", "unet_reduce_workspace_bytes", "unet_state_scale",
           "unet_state_to_input", "unet_state_to_target", "unet_output_to_state", "unet_channel_sumsq")


class UnetError(RuntimeError):
    pass


class Source(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("nz", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("c_first", ctypes.c_int32), ("src0", ctypes.c_void_p),
                ("src1", ctypes.c_void_p)]


class StateLayout(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("sy", ctypes.c_int64),
                ("sz", ctypes.c_int64), ("off", ctypes.c_int64 * 4), ("half", ctypes.c_int64)]


def load_library():
    """Load libstokes_unet.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise UnetError(f"{_LIB_PATH} is missing: build it with paper_2312_10615_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, SZ, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
    SRC = ctypes.POINTER(Source)
    LAY = ctypes.POINTER(StateLayout)
    sig = {
        "unet_packed_elems": (SZ, [I32, I32, I32]),
        "unet_pack_weights": (I32, [P, I32, I32, I32, P, P]),
        "unet_conv3": (I32, [SRC, I32, P, P, I32, I32, P, P]),
        "unet_wgrad_workspace_bytes": (SZ, [SRC, I32]),
        "unet_conv3_wgrad": (I32, [SRC, SRC, I32, P, SZ, P, P, P]),
        "unet_up_grad": (I32, [P, I32, I32, I32, I32, I32, I32, P, P]),
        "unet_skip_grad": (I32, [P, I32, I32, P, I32, I32, I32, I32, P, P]),
        "unet_head_forward": (I32, [P, P, P, P, I64, P]),
        "unet_head_workspace_bytes": (SZ, [I64]),
        "unet_head_backward": (I32, [P, P, P, P, P, SZ, P, P, I64, P]),
        "unet_mse_workspace_bytes": (SZ, [I64]),
        "unet_mse": (I32, [P, P, I32, I32, I32, P, P, SZ, P, P]),
        "unet_adam": (I32, [P, P, P, P, I64, F, F, F, F, I32, P]),
        "unet_reduce_workspace_bytes": (SZ, [LAY]),
        "unet_state_scale": (I32, [P, LAY, P, SZ, P, P]),
        "unet_state_to_input": (I32, [P, LAY, P, P, P]),
        "unet_state_to_target": (I32, [P, LAY, P, P, P, P]),
        "unet_output_to_state": (I32, [P, LAY, P, P, P, P]),
        "unet_channel_sumsq": (I32, [P, I64, P, SZ, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(rc, what):
    if rc != UNET_OK:
        raise UnetError(f"{what} failed with status {rc}")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------ C-named calls

def unet_packed_elems(cin, cout, transpose):
    return load_library().unet_packed_elems(cin, cout, 1 if transpose else 0)


def unet_pack_weights(w, cin, cout, transpose, frag):
    _check(load_library().unet_pack_weights(_ptr(w), cin, cout, 1 if transpose else 0, _ptr(frag), _stream()),
           "unet_pack_weights")


def source(mode, dims, channels, src0, src1=None, c_first=0):
    """unet_source over device tensors; the struct keeps them alive while it is in use."""
    nz, ny, nx = dims
    s = Source(mode, nz, ny, nx, channels, c_first, src0.data_ptr(), 0 if src1 is None else src1.data_ptr())
    s._keep = (src0, src1)
    return s


def unet_conv3(src, cout, frag, bias, relu, out_f32, out):
    _check(load_library().unet_conv3(ctypes.byref(src), cout, _ptr(frag), _ptr(bias), int(relu), int(out_f32),
                                     _ptr(out), _stream()), "unet_conv3")


def unet_wgrad_workspace_bytes(x, cout):
    return load_library().unet_wgrad_workspace_bytes(ctypes.byref(x), cout)


def unet_conv3_wgrad(x, dz, cout, workspace, dw, db):
    _check(load_library().unet_conv3_wgrad(ctypes.byref(x), ctypes.byref(dz), cout, _ptr(workspace),
                                           workspace.numel() * workspace.element_size(), _ptr(dw), _ptr(db),
                                           _stream()), "unet_conv3_wgrad")


def unet_up_grad(fine, cf, coff, c, coarse_dims, coarse):
    nz, ny, nx = coarse_dims
    _check(load_library().unet_up_grad(_ptr(fine), cf, coff, c, nz, ny, nx, _ptr(coarse), _stream()), "unet_up_grad")


def unet_skip_grad(fine, cf, coff, pooled, c, dims, out):
    nz, ny, nx = dims
    _check(load_library().unet_skip_grad(_ptr(fine), cf, coff, _ptr(pooled), c, nz, ny, nx, _ptr(out), _stream()),
           "unet_skip_grad")


def unet_head_forward(d, hw, hb, out):
    _check(load_library().unet_head_forward(_ptr(d), _ptr(hw), _ptr(hb), _ptr(out), d.numel() // HEAD_IN,
                                            _stream()), "unet_head_forward")


def unet_head_workspace_bytes(nvox):
    return load_library().unet_head_workspace_bytes(nvox)


def unet_head_backward(d, dout, hw, dd, workspace, dhw, dhb):
    _check(load_library().unet_head_backward(_ptr(d), _ptr(dout), _ptr(hw), _ptr(dd), _ptr(workspace),
                                             workspace.numel() * workspace.element_size(), _ptr(dhw), _ptr(dhb),
                                             d.numel() // HEAD_IN, _stream()), "unet_head_backward")


def unet_mse_workspace_bytes(nvox):
    return load_library().unet_mse_workspace_bytes(nvox)


def unet_mse(out, target, dims, dout, workspace, loss):
    nz, ny, nx = dims
    _check(load_library().unet_mse(_ptr(out), _ptr(target), nz, ny, nx, _ptr(dout), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _ptr(loss), _stream()), "unet_mse")


def unet_adam(p, g, m, v, lr, beta1, beta2, eps, step):
    _check(load_library().unet_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), lr, beta1, beta2, eps, step,
                                    _stream()), "unet_adam")


def state_layout(lay):
    """unet_state_layout from a stokes layout (paper_2312_10615_amd.stokes.Layout)."""
    L = StateLayout()
    L.nx, L.ny, L.nz = lay.nx, lay.ny, lay.nz
    L.sy, L.sz = lay.sy, lay.sz
    for f in range(4):
        L.off[f] = lay.off[f]
    L.half = lay.field // 2
    return L


def unet_reduce_workspace_bytes(L):
    return load_library().unet_reduce_workspace_bytes(ctypes.byref(L))


def unet_state_scale(b, L, workspace, scale):
    _check(load_library().unet_state_scale(_ptr(b), ctypes.byref(L), _ptr(workspace),
                                           workspace.numel() * workspace.element_size(), _ptr(scale), _stream()),
           "unet_state_scale")


def unet_state_to_input(b, L, scale, inp):
    _check(load_library().unet_state_to_input(_ptr(b), ctypes.byref(L), _ptr(scale), _ptr(inp), _stream()),
           "unet_state_to_input")


def unet_state_to_target(x, L, scale, sigma, target):
    _check(load_library().unet_state_to_target(_ptr(x), ctypes.byref(L), _ptr(scale), _ptr(sigma), _ptr(target),
                                               _stream()), "unet_state_to_target")


def unet_output_to_state(out, L, scale, sigma, x):
    _check(load_library().unet_output_to_state(_ptr(out), ctypes.byref(L), _ptr(scale), _ptr(sigma), _ptr(x),
                                               _stream()), "unet_output_to_state")


def unet_channel_sumsq(t, workspace, sumsq):
    _check(load_library().unet_channel_sumsq(_ptr(t), t.numel() // 4, _ptr(workspace),
                                             workspace.numel() * workspace.element_size(), _ptr(sumsq), _stream()),
           "unet_channel_sumsq")


# ------------------------------------------------------------------ network

def param_shapes():
    shapes = []
    for name, _, cin, cout in LAYERS:
        shapes.append((name + ".w", (27, cin, cout)))
        shapes.append((name + ".b", (cout,)))
    shapes.append(("head.w", (HEAD_IN, HEAD_OUT)))
    shapes.append(("head.b", (HEAD_OUT,)))
    return shapes


def init_params(seed=0):
    """He-style random initial parameters (float32 numpy): N(0, 2 / fan_in) for the
    ReLU convolutions, N(0, 1 / fan_in) for the head, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, _, cin, cout in LAYERS:
        p[name + ".w"] = (rng.standard_normal((27, cin, cout)) * math.sqrt(2.0 / (27 * cin))).astype(np.float32)
        p[name + ".b"] = np.zeros(cout, np.float32)
    p["head.w"] = (rng.standard_normal((HEAD_IN, HEAD_OUT)) * math.sqrt(1.0 / HEAD_IN)).astype(np.float32)
    p["head.b"] = np.zeros(HEAD_OUT, np.float32)
    return p


class WarmStartNet:
    """Parameters, activations and gradients of the U-Net on one GPU, for one
    grid of nx x ny x nz voxels (each divisible by 4).  All buffers are
    allocated once here; forward/backward/step only launch kernels."""

    def __init__(self, nx, ny, nz, params=None, sigma=(1.0, 1.0, 1.0, 1.0), device="cuda"):
        import torch
        if nx % 4 or ny % 4 or nz % 4:
            raise ValueError("grid dimensions must be divisible by 4 (two poolings)")
        load_library()
        self.dims = {0: (nz, ny, nx), 1: (nz // 2, ny // 2, nx // 2), 2: (nz // 4, ny // 4, nx // 4)}
        self.nvox = nx * ny * nz
        self.device = device
        shapes = param_shapes()
        self.n_params = sum(int(np.prod(s)) for _, s in shapes)
        f32 = dict(dtype=torch.float32, device=device)
        bf = dict(dtype=torch.bfloat16, device=device)
        self.flat = torch.zeros(self.n_params, **f32)
        self.grad = torch.zeros(self.n_params, **f32)
        self.m = torch.zeros(self.n_params, **f32)
        self.v = torch.zeros(self.n_params, **f32)
        self.p, self.g = {}, {}
        o = 0
        for k, s in shapes:
            n = int(np.prod(s))
            self.p[k] = self.flat[o:o + n].view(s)
            self.g[k] = self.grad[o:o + n].view(s)
            o += n
        self.load_params(params if params is not None else init_params(0))
        self.sigma = torch.tensor(sigma, **f32)
        self.frag, self.fragT = {}, {}
        for name, _, cin, cout in LAYERS:
            self.frag[name] = torch.zeros(unet_packed_elems(cin, cout, False), **bf)
            if name != "c0a":
                self.fragT[name] = torch.zeros(unet_packed_elems(cin, cout, True), **bf)
        self.inp = torch.zeros(self.dims[0] + (IN_CH,), **bf)
        self.act, self.dact, self.dx = {}, {}, {}
        for name, _, cin, cout in LAYERS:
            d = self.dims[LEVEL[name]]
            self.act[name] = torch.zeros(d + (cout,), **bf)
            self.dact[name] = torch.zeros(d + (cout,), **bf)
            if name != "c0a":
                self.dx[name] = torch.zeros(d + (cin,), **bf)
        # a tensor read only by the next layer takes that layer's input gradient as is
        for name, spec, cin, cout in LAYERS:
            if isinstance(spec, str) and spec != "in":
                self.dact[spec] = self.dx[name]
        self.out = torch.zeros(self.dims[0] + (HEAD_OUT,), **f32)
        self.dout = torch.zeros_like(self.out)
        self.target = torch.zeros_like(self.out)
        ws = max(unet_wgrad_workspace_bytes(self._src(name, spec, cin), cout) for name, spec, cin, cout in LAYERS)
        ws = max(ws, unet_head_workspace_bytes(self.nvox), unet_mse_workspace_bytes(self.nvox), 8 * 4 * 1024)
        self.ws = torch.zeros((ws + 15) // 16 * 4, **f32)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=device)
        self.scale = torch.zeros(1, dtype=torch.float64, device=device)
        self.sumsq = torch.zeros(4, dtype=torch.float64, device=device)
        self.step_count = 0
        self.pack()

    # ---- parameters
    def load_params(self, params):
        import torch
        for k, t in self.p.items():
            t.copy_(torch.as_tensor(np.asarray(params[k], dtype=np.float32).reshape(t.shape)))

    def params_numpy(self):
        return {k: t.detach().cpu().numpy().copy() for k, t in self.p.items()}

    def pack(self):
        for name, _, cin, cout in LAYERS:
            unet_pack_weights(self.p[name + ".w"], cin, cout, False, self.frag[name])
            if name != "c0a":
                unet_pack_weights(self.p[name + ".w"], cin, cout, True, self.fragT[name])

    # ---- sources
    def _src(self, name, spec, cin):
        d = self.dims[LEVEL[name]]
        if spec == "in":
            return source(SRC_DIRECT, d, cin, self.inp)
        if isinstance(spec, str):
            return source(SRC_DIRECT, d, cin, self.act[spec])
        if spec[0] == "pool":
            return source(SRC_POOL, d, cin, self.act[spec[1]])
        coarse, skip = spec[1], spec[2]
        return source(SRC_CAT_UP, d, cin, self.act[coarse], self.act[skip], c_first=self.act[coarse].shape[3])

    # ---- passes
    def forward(self):
        """out = network(inp)."""
        for name, spec, cin, cout in LAYERS:
            unet_conv3(self._src(name, spec, cin), cout, self.frag[name], self.p[name + ".b"], 1, 0, self.act[name])
        unet_head_forward(self.act["c0d"], self.p["head.w"], self.p["head.b"], self.out)
        return self.out

    def backward(self):
        """Parameter gradients into self.grad for d loss / d out = self.dout."""
        unet_head_backward(self.act["c0d"], self.dout, self.p["head.w"], self.dact["c0d"], self.ws, self.g["head.w"],
                           self.g["head.b"])
        for name, spec, cin, cout in reversed(LAYERS):
            d = self.dims[LEVEL[name]]
            dz = source(SRC_MASKED, d, cout, self.dact[name], self.act[name])
            unet_conv3_wgrad(self._src(name, spec, cin), dz, cout, self.ws, self.g[name + ".w"], self.g[name + ".b"])
            if spec == "in":
                continue
            dx = self.dx[name]
            unet_conv3(dz, cin, self.fragT[name], None, 0, 0, dx)
            if isinstance(spec, str):
                pass  # self.dact[spec] is dx itself
            elif spec[0] == "pool":
                # the pooled tensor is also the skip input of the concatenating layer seen earlier
                src = spec[1]
                cat_name, cc = self._skip_reader(src)
                unet_skip_grad(self.dx[cat_name], self.dx[cat_name].shape[3], cc, dx, dx.shape[3],
                               self.dims[LEVEL[src]], self.dact[src])
            else:
                coarse = spec[1]
                cc = self.act[coarse].shape[3]
                unet_up_grad(dx, cin, 0, cc, self.dims[LEVEL[coarse]], self.dact[coarse])

    def _skip_reader(self, tensor):
        for name, spec, cin, cout in LAYERS:
            if isinstance(spec, tuple) and spec[0] == "cat" and spec[2] == tensor:
                return name, self.act[spec[1]].shape[3]
        raise KeyError(tensor)

    def loss_and_grad(self):
        unet_mse(self.out, self.target, self.dims[0], self.dout, self.ws, self.loss_dev)
        return self.loss_dev

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        unet_adam(self.flat, self.grad, self.m, self.v, lr, beta1, beta2, eps, self.step_count)
        self.pack()

    def train_step(self, lr):
        """One step on the pair (self.inp, self.target); returns the loss (device tensor) before the update."""
        self.forward()
        loss = self.loss_and_grad()
        self.backward()
        self.adam(lr)
        return loss

    # ---- Stokes state vectors
    def set_input_from_state(self, b, layout):
        L = state_layout(layout)
        unet_state_scale(b, L, self.ws, self.scale)
        unet_state_to_input(b, L, self.scale, self.inp)

    def set_target_from_state(self, x, layout):
        unet_state_to_target(x, state_layout(layout), self.scale, self.sigma, self.target)

    def initial_guess(self, b, layout, x0):
        """x0 (state vector, overwritten) = the network's guess for L x = b."""
        self.set_input_from_state(b, layout)
        self.forward()
        unet_output_to_state(self.out, state_layout(layout), self.scale, self.sigma, x0)
        return x0
