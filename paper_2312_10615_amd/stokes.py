"""Python binding of the gfx950 MG-SQMR Stokes library (include/stokes_mgsqmr.h).

Functions with the C names marshal arguments only; every step of the solve
runs in the HIP library.  `StokesSolver` adds the torch plumbing: device
workspace, state vectors, and packing between the natural MAC arrays and the
library's padded layout.  There is no CPU fallback: if the shared library is
missing this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libstokes_mgsqmr.so")

STOKES_OK, STOKES_EINVAL, STOKES_ENOCONV, STOKES_EBREAKDOWN, STOKES_ENONFINITE, STOKES_EDEVICE, STOKES_ETOOLARGE = range(7)
STOKES_STATIC_BYTES = 64 << 20
STOKES_FLAG_REMOVE_MEAN = 1
STOKES_FLAG_NO_GRAPH = 2
SMOOTHERS = {"split": 0, "symmetric": 1}
VANKA = {"mult8": 0, "mult27": 1, "additive": 2}
STATUS_NAMES = {0: "ok", 1: "einval", 2: "enoconv", 3: "ebreakdown", 4: "enonfinite", 5: "edevice", 6: "etoolarge"}


class StokesParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("eta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("levels", ctypes.c_int32), ("nu", ctypes.c_int32), ("n_boundary", ctypes.c_int32),
                ("vcycle_precision", ctypes.c_int32), ("smoother", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("vanka", ctypes.c_int32), ("cycle", ctypes.c_int32), ("labels", ctypes.c_void_p)]


class StokesLayout(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("sy", ctypes.c_int64), ("sz", ctypes.c_int64), ("off", ctypes.c_int64 * 4),
                ("field", ctypes.c_int64), ("total", ctypes.c_int64), ("n_dofs", ctypes.c_int64),
                ("levels", ctypes.c_int32)]


class StokesInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double))]


EXPORTS = ("stokes_default_params", "stokes_workspace_bytes", "stokes_setup", "stokes_layout", "stokes_level_layout",
           "stokes_restrict", "stokes_prolong", "stokes_lift", "stokes_apply", "stokes_vcycle", "stokes_solve", "stokes_solve_static", "stokes_profile",
           "stokes_profile_read", "stokes_destroy", "stokes_strerror", "stokes_batch_workspace_bytes",
           "stokes_batch_setup", "stokes_batch_layout", "stokes_batch_size", "stokes_batch_autotune",
           "stokes_batch_set_chunks", "stokes_batch_solve", "stokes_batch_destroy")

# kernel classes of stokes_profile()
KC = {"apply": 0, "dgs_u": 1, "dgs_pf_own": 2, "dgs_pf_nbr": 3, "dgs_pr": 4, "vanka_delta": 5, "vanka_apply": 6,
      "restrict": 7, "prolong": 8, "coarse": 9, "blas": 10}
KC_ALL, KC_OFF = -1, -2

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the shared library (no GPU needed) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with `python -m paper_2312_10615_amd.build`")
    lib = ctypes.CDLL(path)
    P, vp, i32, f64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.stokes_default_params.argtypes = [i32, i32, i32, f64, P(StokesParams)]
    lib.stokes_workspace_bytes.argtypes = [P(StokesParams), P(ctypes.c_size_t)]
    lib.stokes_setup.argtypes = [P(StokesParams), vp, ctypes.c_size_t, vp, P(vp)]
    lib.stokes_layout.argtypes = [vp, P(StokesLayout)]
    lib.stokes_level_layout.argtypes = [vp, i32, P(StokesLayout)]
    lib.stokes_restrict.argtypes = [vp, vp, vp]
    lib.stokes_lift.argtypes = [vp, vp, vp, vp]
    lib.stokes_prolong.argtypes = [vp, vp, vp]
    lib.stokes_apply.argtypes = [vp, vp, vp, i32]
    lib.stokes_vcycle.argtypes = [vp, vp, vp]
    lib.stokes_solve.argtypes = [vp, vp, vp, f64, i32, P(StokesInfo)]
    lib.stokes_solve_static.argtypes = [P(StokesParams), vp, vp, f64, i32, P(StokesInfo), vp]
    lib.stokes_profile.argtypes = [vp, i32, i32]
    lib.stokes_profile_read.argtypes = [vp, i32, i32, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.stokes_destroy.argtypes = [vp]
    lib.stokes_destroy.restype = None
    lib.stokes_batch_workspace_bytes.argtypes = [i32, P(StokesParams), P(ctypes.c_size_t)]
    lib.stokes_batch_setup.argtypes = [i32, P(StokesParams), vp, ctypes.c_size_t, vp, P(vp)]
    lib.stokes_batch_layout.argtypes = [vp, i32, P(ctypes.c_int64), P(StokesLayout)]
    lib.stokes_batch_size.argtypes = [vp, P(ctypes.c_int64)]
    lib.stokes_batch_autotune.argtypes = [vp, P(i32)]
    lib.stokes_batch_set_chunks.argtypes = [vp, i32, i32]
    lib.stokes_batch_solve.argtypes = [vp, vp, vp, f64, i32, P(StokesInfo)]
    lib.stokes_batch_destroy.argtypes = [vp]
    lib.stokes_batch_destroy.restype = None
    lib.stokes_strerror.argtypes = [ctypes.c_int]
    lib.stokes_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("stokes_destroy", "stokes_strerror", "stokes_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class StokesError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {stokes_strerror(code)} (status {code})")
        self.code = code


def _check(code, where):
    if code != STOKES_OK:
        raise StokesError(code, where)


# --- C-named wrappers ---------------------------------------------------------

def stokes_default_params(nx, ny, nz, h) -> StokesParams:
    p = StokesParams()
    _check(load_library().stokes_default_params(nx, ny, nz, h, ctypes.byref(p)), "stokes_default_params")
    return p


def stokes_workspace_bytes(params: StokesParams) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().stokes_workspace_bytes(ctypes.byref(params), ctypes.byref(n)), "stokes_workspace_bytes")
    return int(n.value)


def stokes_setup(params: StokesParams, workspace_ptr: int, nbytes: int, stream_ptr: int):
    ctx = ctypes.c_void_p()
    _check(load_library().stokes_setup(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), nbytes,
                                       ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)), "stokes_setup")
    return ctx


def stokes_layout(ctx) -> StokesLayout:
    lay = StokesLayout()
    _check(load_library().stokes_layout(ctx, ctypes.byref(lay)), "stokes_layout")
    return lay


def stokes_level_layout(ctx, level: int) -> StokesLayout:
    lay = StokesLayout()
    _check(load_library().stokes_level_layout(ctx, level, ctypes.byref(lay)), "stokes_level_layout")
    return lay


def stokes_restrict(ctx, fine_ptr: int, coarse_ptr: int) -> int:
    return load_library().stokes_restrict(ctx, ctypes.c_void_p(fine_ptr), ctypes.c_void_p(coarse_ptr))


def stokes_prolong(ctx, coarse_ptr: int, fine_ptr: int) -> int:
    return load_library().stokes_prolong(ctx, ctypes.c_void_p(coarse_ptr), ctypes.c_void_p(fine_ptr))


def stokes_apply(ctx, x_ptr: int, y_ptr: int, penalized: int = 0) -> int:
    return load_library().stokes_apply(ctx, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), int(penalized))


def stokes_vcycle(ctx, s_ptr: int, t_ptr: int) -> int:
    return load_library().stokes_vcycle(ctx, ctypes.c_void_p(s_ptr), ctypes.c_void_p(t_ptr))


def stokes_solve(ctx, b_ptr: int, x_ptr: int, rtol: float, maxit: int, record_history: bool = True):
    info = StokesInfo()
    hist = None
    if record_history:
        hist = (ctypes.c_double * (maxit + 1))()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    code = load_library().stokes_solve(ctx, ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr), float(rtol),
                                       int(maxit), ctypes.byref(info))
    history = [hist[i] for i in range(info.iters + 1)] if hist is not None and code != STOKES_EINVAL else None
    return code, info, history


def stokes_solve_static(params: StokesParams, b_ptr: int, x_ptr: int, rtol: float, maxit: int, stream_ptr: int,
                        record_history: bool = True):
    """stokes_solve on the library's static scratch (no context, no workspace):
    returns (status, info, history) like `stokes_solve`."""
    info = StokesInfo()
    hist = None
    if record_history:
        hist = (ctypes.c_double * (maxit + 1))()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    code = load_library().stokes_solve_static(ctypes.byref(params), ctypes.c_void_p(b_ptr), ctypes.c_void_p(x_ptr),
                                              float(rtol), int(maxit), ctypes.byref(info),
                                              ctypes.c_void_p(stream_ptr))
    ok = hist is not None and code not in (STOKES_EINVAL, STOKES_ETOOLARGE, STOKES_EDEVICE)
    history = [hist[i] for i in range(info.iters + 1)] if ok else None
    return code, info, history


def stokes_profile(ctx, kernel_class: int, level: int = -1) -> None:
    _check(load_library().stokes_profile(ctx, int(kernel_class), int(level)), "stokes_profile")


def stokes_profile_read(ctx, kernel_class: int, level: int = -1):
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(load_library().stokes_profile_read(ctx, int(kernel_class), int(level), ctypes.byref(ms), ctypes.byref(n)),
           "stokes_profile_read")
    return float(ms.value), int(n.value)


def stokes_destroy(ctx) -> None:
    load_library().stokes_destroy(ctx)


def stokes_strerror(code: int) -> str:
    return load_library().stokes_strerror(code).decode()


# --- torch plumbing -------------------------------------------------------------

def field_index(layout, device):
    """[K, J, I] -> element of padded cell (I, J, K) inside a field: its slot
    s = I + sy J + sz K is stored at (s & 1) * field/2 + (s >> 1) (red and
    black slots apart)."""
    import torch
    L = layout
    K = torch.arange(L.nz + 2, dtype=torch.int64, device=device).view(-1, 1, 1)
    J = torch.arange(L.ny + 2, dtype=torch.int64, device=device).view(1, -1, 1)
    I = torch.arange(L.sy, dtype=torch.int64, device=device).view(1, 1, -1)
    s = I + L.sy * J + L.sz * K
    return (s & 1) * (L.field // 2) + (s >> 1)


def unknown_masks(labels):
    """The unknowns of a labelled domain (the rule of stokes_params.labels) as
    boolean arrays of the natural shapes: ux (nx+1, ny, nz), uy, uz, p.
    `labels` is indexed [i, j, k] over the padded box."""
    lab = np.asarray(labels)
    inter, dirc = lab == 0, lab == 1
    out = []
    for a in range(3):
        lo = [slice(1, -1)] * 3
        hi = [slice(1, -1)] * 3
        lo[a], hi[a] = slice(0, -1), slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        out.append((inter[lo] | inter[hi]) & ~dirc[lo] & ~dirc[hi])
    out.append(inter[1:-1, 1:-1, 1:-1].copy())
    return out


def pack_fields(layout, fields, out, device, masks=None):
    """Natural arrays (ux (nx+1,ny,nz), uy, uz, p), numpy or torch, indexed
    [i,j,k] -> the padded state `out`; only unknowns are copied (the box's, or
    those of `masks` for a labelled domain), every other slot is 0."""
    import torch
    L = layout
    nx, ny, nz = L.nx, L.ny, L.nz
    st = out.zero_()
    e = field_index(L, st.device)
    t = [torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
                         dtype=torch.float64).to(device) for a in fields]
    if masks is not None:
        t = [v * torch.as_tensor(m, device=v.device) for v, m in zip(t, masks)]
        st[L.off[0] + e[1:nz + 1, 1:ny + 1, 1:nx + 2]] = t[0].permute(2, 1, 0)
        st[L.off[1] + e[1:nz + 1, 1:ny + 2, 1:nx + 1]] = t[1].permute(2, 1, 0)
        st[L.off[2] + e[1:nz + 2, 1:ny + 1, 1:nx + 1]] = t[2].permute(2, 1, 0)
        st[L.off[3] + e[1:nz + 1, 1:ny + 1, 1:nx + 1]] = t[3].permute(2, 1, 0)
        return st
    st[L.off[0] + e[1:nz + 1, 1:ny + 1, 2:nx + 1]] = t[0][1:nx].permute(2, 1, 0)
    st[L.off[1] + e[1:nz + 1, 2:ny + 1, 1:nx + 1]] = t[1][:, 1:ny].permute(2, 1, 0)
    st[L.off[2] + e[2:nz + 1, 1:ny + 1, 1:nx + 1]] = t[2][:, :, 1:nz].permute(2, 1, 0)
    st[L.off[3] + e[1:nz + 1, 1:ny + 1, 1:nx + 1]] = t[3].permute(2, 1, 0)
    return st


def unpack_fields(layout, state, masks=None):
    """Padded state -> natural numpy arrays (walls included, zero; for a
    labelled domain every slot that is not an unknown of `masks` is zero)."""
    L = layout
    nx, ny, nz = L.nx, L.ny, L.nz
    e = field_index(L, state.device)
    ux = state[L.off[0] + e[1:nz + 1, 1:ny + 1, 1:nx + 2]].permute(2, 1, 0).cpu().numpy().copy()
    uy = state[L.off[1] + e[1:nz + 1, 1:ny + 2, 1:nx + 1]].permute(2, 1, 0).cpu().numpy().copy()
    uz = state[L.off[2] + e[1:nz + 2, 1:ny + 1, 1:nx + 1]].permute(2, 1, 0).cpu().numpy().copy()
    p = state[L.off[3] + e[1:nz + 1, 1:ny + 1, 1:nx + 1]].permute(2, 1, 0).cpu().numpy().copy()
    if masks is not None:
        return tuple(np.where(m, v, 0.0) for m, v in zip(masks, (ux, uy, uz, p)))
    ux[0] = ux[-1] = 0.0
    uy[:, 0] = uy[:, -1] = 0.0
    uz[:, :, 0] = uz[:, :, -1] = 0.0
    return ux, uy, uz, p


class StokesSolver:
    """Device workspace + context for one box.  State vectors are float64
    torch tensors of `layout.total` elements on the context's device."""

    def __init__(self, nx, ny, nz, h=None, *, eta=1.0, gamma=1e-3, levels=0, nu=2, n_boundary=1,
                 schedule="symmetric", precision=64, remove_mean=True, graphs=True, vanka="mult8",
                 cycle=1, labels=None, device=None, stream=None):
        """`labels`: optional cell labels of Section 5 indexed [i, j, k] over the
        padded box ((nx+2, ny+2, nz+2); 0 interior, 1 Dirichlet, 2 exterior)."""
        import torch
        self.torch = torch
        h = 1.0 / max(nx, ny, nz) if h is None else h
        p = stokes_default_params(nx, ny, nz, h)
        self.masks = None
        lab_c = None
        if labels is not None:
            labels = np.asarray(labels)
            if labels.shape != (nx + 2, ny + 2, nz + 2):
                raise ValueError("labels must have shape (nx+2, ny+2, nz+2)")
            lab_c = np.ascontiguousarray(labels.transpose(2, 1, 0), dtype=np.uint8)   # x fastest
            p.labels = lab_c.ctypes.data
            self.masks = unknown_masks(labels)
        p.eta, p.gamma, p.levels, p.nu, p.n_boundary = eta, gamma, levels, nu, n_boundary
        p.smoother = SMOOTHERS[schedule]
        p.vcycle_precision = precision
        p.vanka, p.cycle = VANKA[vanka], int(cycle)
        p.flags = (STOKES_FLAG_REMOVE_MEAN if remove_mean else 0) | (0 if graphs else STOKES_FLAG_NO_GRAPH)
        self.params = p
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = stokes_workspace_bytes(p)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr, self._ws_bytes = base + off, nbytes
        with torch.cuda.device(self.device):
            self.ctx = stokes_setup(p, self._ws_ptr, nbytes, self.stream.cuda_stream)
        p.labels = None   # read during set-up only
        del lab_c
        self.layout = stokes_layout(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            stokes_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # layout helpers
    def new_state(self):
        return self.torch.zeros(self.layout.total, dtype=self.torch.float64, device=self.device)

    def pack(self, fields, out=None):
        """Natural arrays (ux (nx+1,ny,nz), uy, uz, p), numpy or torch, indexed
        [i,j,k] -> padded state; only unknowns are copied, every other slot is 0."""
        return pack_fields(self.layout, fields, self.new_state() if out is None else out, self.device, self.masks)

    def unpack(self, state):
        """Padded state -> natural numpy arrays (walls included, zero)."""
        return unpack_fields(self.layout, state, self.masks)

    # operations
    def apply(self, x, penalized=False, out=None):
        y = self.new_state() if out is None else out
        _check(stokes_apply(self.ctx, x.data_ptr(), y.data_ptr(), int(penalized)), "stokes_apply")
        return y

    def level_layout(self, level):
        return stokes_level_layout(self.ctx, level)

    def restrict(self, fine, out=None):
        """coarse = R fine (level 0 -> level 1 layout)."""
        lay = self.level_layout(1)
        c = out if out is not None else self.torch.zeros(lay.total, dtype=self.torch.float64, device=self.device)
        _check(stokes_restrict(self.ctx, fine.data_ptr(), c.data_ptr()), "stokes_restrict")
        return c

    def prolong(self, coarse, out=None):
        """fine = P coarse (level 1 -> level 0 layout)."""
        f = out if out is not None else self.new_state()
        _check(stokes_prolong(self.ctx, coarse.data_ptr(), f.data_ptr()), "stokes_prolong")
        return f

    def lift(self, g, b, out=None):
        """out = b - L g at the unknowns: boundary values held in g's non-unknown slots
        moved to the right-hand side."""
        o = out if out is not None else self.new_state()
        _check(load_library().stokes_lift(self.ctx, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                          ctypes.c_void_p(o.data_ptr())), "stokes_lift")
        return o

    def lid_boundary(self, velocity):
        """State vector holding a lid on the plus-z wall moving along x with
        `velocity`: the u_x ghost slots above the top cell row, zero elsewhere."""
        L = self.layout
        g = self.new_state()
        e = field_index(L, g.device)
        g[L.off[0] + e[L.nz + 1, 1:L.ny + 1, 2:L.nx + 1]] = velocity
        return g

    def vcycle(self, s, out=None):
        t = self.new_state() if out is None else out
        _check(stokes_vcycle(self.ctx, s.data_ptr(), t.data_ptr()), "stokes_vcycle")
        return t

    def profile(self, kernel_class, level=-1):
        """Select kernels to time with HIP events (name from KC, 'all' or 'off')."""
        k = {"all": KC_ALL, "off": KC_OFF}.get(kernel_class, KC.get(kernel_class, kernel_class))
        stokes_profile(self.ctx, k, level)

    def profile_read(self, kernel_class, level=-1):
        """(total milliseconds, launches) accumulated since profile()."""
        return stokes_profile_read(self.ctx, KC.get(kernel_class, kernel_class), level)

    def solve(self, b, x0=None, rtol=1e-8, maxit=200):
        x = self.new_state() if x0 is None else x0.clone()
        code, info, hist = stokes_solve(self.ctx, b.data_ptr(), x.data_ptr(), rtol, maxit)
        if code in (STOKES_EINVAL, STOKES_EDEVICE):
            _check(code, "stokes_solve")
        return x, {"iters": info.iters, "status": STATUS_NAMES.get(code, str(code)), "relres": info.relres,
                   "bnorm": info.bnorm, "history": hist}


class StokesBatch:
    """Many boxes solved together (stokes_batch_*).  `dims` is a list of
    (nx, ny, nz); every box gets spacing h (default 1 / 128) and the same
    schedule and V-cycle precision.  Batch vectors are float64 tensors of
    `size` elements; box d's state is `vector[offset[d] : offset[d] + total]`."""

    def __init__(self, dims, h=1.0 / 128, *, eta=1.0, gamma=1e-3, nu=2, n_boundary=1, schedule="symmetric",
                 precision=32, remove_mean=True, levels=None, device=None, stream=None):
        import torch
        self.torch = torch
        n = len(dims)
        arr = (StokesParams * n)()
        for i, (nx, ny, nz) in enumerate(dims):
            p = stokes_default_params(nx, ny, nz, h)
            p.eta, p.gamma, p.nu, p.n_boundary = eta, gamma, nu, n_boundary
            p.levels = 0 if levels is None else int(levels[i])
            p.smoother = SMOOTHERS[schedule]
            p.vcycle_precision = precision
            p.flags = STOKES_FLAG_REMOVE_MEAN if remove_mean else 0
            arr[i] = p
        self.params, self.n = arr, n
        lib = load_library()
        nbytes = ctypes.c_size_t(0)
        _check(lib.stokes_batch_workspace_bytes(n, arr, ctypes.byref(nbytes)), "stokes_batch_workspace_bytes")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        ptr = base + (-base) % 256
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.stokes_batch_setup(n, arr, ctypes.c_void_p(ptr), nbytes.value,
                                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
                   "stokes_batch_setup")
        self.ctx = ctx
        self.offset, self.layouts = [], []
        for d in range(n):
            off = ctypes.c_int64(0)
            lay = StokesLayout()
            _check(lib.stokes_batch_layout(ctx, d, ctypes.byref(off), ctypes.byref(lay)), "stokes_batch_layout")
            self.offset.append(int(off.value))
            self.layouts.append(lay)
        tot = ctypes.c_int64(0)
        _check(lib.stokes_batch_size(ctx, ctypes.byref(tot)), "stokes_batch_size")
        self.size = int(tot.value)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            load_library().stokes_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_vector(self):
        return self.torch.zeros(self.size, dtype=self.torch.float64, device=self.device)

    def part(self, vec, d):
        return vec[self.offset[d]:self.offset[d] + self.layouts[d].total]

    def pack(self, fields_per_box, out=None):
        v = self.new_vector() if out is None else out.zero_()
        for d, f in enumerate(fields_per_box):
            pack_fields(self.layouts[d], f, self.part(v, d), self.device)
        return v

    def unpack(self, vec, d):
        return unpack_fields(self.layouts[d], self.part(vec, d))

    def autotune(self):
        """Pick the tile shape of every stencil kernel class on every level; returns
        {class: [x-extent per level]}."""
        ch = (ctypes.c_int32 * (8 * 16))()
        _check(load_library().stokes_batch_autotune(self.ctx, ch), "stokes_batch_autotune")
        names = ("apply", "resid", "dgs_u", "dgs_pf_own", "dgs_pf_nbr", "dgs_pr", "restrict", "prolong")
        return {nm: [int(ch[k * 16 + l]) for l in range(16)] for k, nm in enumerate(names)}

    def set_chunks(self, first, later):
        _check(load_library().stokes_batch_set_chunks(self.ctx, int(first), int(later)), "stokes_batch_set_chunks")

    def solve(self, b, x0=None, rtol=1e-8, maxit=200):
        x = self.new_vector() if x0 is None else x0.clone()
        infos = (StokesInfo * self.n)()
        code = load_library().stokes_batch_solve(self.ctx, ctypes.c_void_p(b.data_ptr()),
                                                 ctypes.c_void_p(x.data_ptr()), rtol, maxit, infos)
        if code in (STOKES_EINVAL, STOKES_EDEVICE):
            _check(code, "stokes_batch_solve")
        return x, [{"iters": i.iters, "status": STATUS_NAMES.get(i.status, str(i.status)), "relres": i.relres,
                    "bnorm": i.bnorm} for i in infos]
