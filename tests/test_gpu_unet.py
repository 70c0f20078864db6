"""Parity of the warm-start network kernels (libstokes_unet.so, gfx950 MFMA)
with the float64 oracle (oracle/unet.py).

Inputs and weights are bfloat16-exact, so the only differences are float32
accumulation on the GPU against exact sums in the oracle:
  * float outputs: |gpu - oracle| <= 4e-5 * S, S = the same sum over |terms|
    (a dropped or doubled term of a K-term sum is >= S / K >= 3.8e-4 S);
  * bfloat16 outputs: additionally one rounding step, 2^-7 |value|.
Whole-network comparisons use the oracle's rounding model and bound the
relative L2 difference (float32 sums flip an occasional bfloat16 rounding).
"""
import numpy as np
import pytest

from tests.gpu_helpers import announce, cuda
from oracle import unet as O

pytestmark = pytest.mark.gpu


def bf16_exact(rng, shape, scale=1.0):
    return O.round_bf16(rng.standard_normal(shape) * scale)


def to_dev(a, dtype):
    torch = cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def packed(w, transpose=False):
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    cin, cout = w.shape[1], w.shape[2]
    wd = to_dev(w, torch.float32)
    frag = torch.zeros(U.unet_packed_elems(cin, cout, transpose), dtype=torch.bfloat16, device="cuda")
    U.unet_pack_weights(wd, cin, cout, transpose, frag)
    return frag


def within(got, want, S, rel=4e-5, bf16=False, what=""):
    tol = rel * S + 1e-30
    if bf16:
        tol = tol + 2.0 ** -7 * np.abs(want)
    bad = np.abs(got - want) > tol
    assert not bad.any(), (what, int(bad.sum()), float(np.abs(got - want).max()), float(S.max()))


CONV_SHAPES = [(8, 16), (16, 16), (16, 32), (32, 64), (64, 64), (64, 16), (96, 32), (48, 16)]


@pytest.mark.parametrize("cin,cout", CONV_SHAPES)
def test_conv3_forward_direct(cin, cout):
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    dims = (6, 9, 20)  # ragged against the 16 x 4 x 4 tile in every axis
    announce(f"unet conv3 direct {cin}->{cout} {dims}")
    rng = np.random.default_rng(cin * 100 + cout)
    x = bf16_exact(rng, dims + (cin,))
    w = rng.standard_normal((27, cin, cout)).astype(np.float32).astype(np.float64) * 0.2
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    wr = O.round_bf16(w)
    ref = O.conv3(x, wr, b)
    S = O.conv3(np.abs(x), np.abs(wr), np.abs(b))
    xd = to_dev(x, torch.bfloat16)
    frag = packed(w)
    bd = to_dev(b, torch.float32)
    out32 = torch.zeros(dims + (cout,), dtype=torch.float32, device="cuda")
    U.unet_conv3(U.source(U.SRC_DIRECT, dims, cin, xd), cout, frag, bd, 0, 1, out32)
    out16 = torch.zeros(dims + (cout,), dtype=torch.bfloat16, device="cuda")
    U.unet_conv3(U.source(U.SRC_DIRECT, dims, cin, xd), cout, frag, bd, 1, 0, out16)
    torch.cuda.synchronize()
    within(out32.double().cpu().numpy(), ref, S, what="f32")
    within(out16.double().cpu().numpy(), O.round_bf16(np.maximum(ref, 0.0)), S, bf16=True, what="bf16 relu")


def test_conv3_forward_pooled_and_concatenated_inputs():
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    rng = np.random.default_rng(11)
    announce("unet conv3 pool 16->32 and cat 64+32->32")
    # pooled input: fine (12, 18, 40) -> conv on (6, 9, 20)
    fine = bf16_exact(rng, (12, 18, 40, 16))
    w = rng.standard_normal((27, 16, 32)) * 0.2
    xin = O.round_bf16(O.pool(fine))
    wr = O.round_bf16(w)
    ref, S = O.conv3(xin, wr, np.zeros(32)), O.conv3(np.abs(xin), np.abs(wr), np.zeros(32))
    out = torch.zeros((6, 9, 20, 32), dtype=torch.float32, device="cuda")
    U.unet_conv3(U.source(U.SRC_POOL, (6, 9, 20), 16, to_dev(fine, torch.bfloat16)), 32, packed(w), None, 0, 1, out)
    torch.cuda.synchronize()
    within(out.double().cpu().numpy(), ref, S, what="pool")
    # concatenation of an upsampled coarse tensor (64 ch) and a skip tensor (32 ch)
    coarse = bf16_exact(rng, (3, 5, 10, 64))
    skip = bf16_exact(rng, (6, 10, 20, 32))
    w = rng.standard_normal((27, 96, 32)) * 0.1
    xin = np.concatenate([O.up(coarse), skip], axis=3)
    wr = O.round_bf16(w)
    ref, S = O.conv3(xin, wr, np.zeros(32)), O.conv3(np.abs(xin), np.abs(wr), np.zeros(32))
    out = torch.zeros((6, 10, 20, 32), dtype=torch.float32, device="cuda")
    src = U.source(U.SRC_CAT_UP, (6, 10, 20), 96, to_dev(coarse, torch.bfloat16), to_dev(skip, torch.bfloat16),
                   c_first=64)
    U.unet_conv3(src, 32, packed(w), None, 0, 1, out)
    torch.cuda.synchronize()
    within(out.double().cpu().numpy(), ref, S, what="cat")


@pytest.mark.parametrize("cin,cout", [(16, 16), (48, 16), (32, 32), (96, 32), (64, 64), (32, 64), (16, 32)])
def test_conv3_input_gradient(cin, cout):
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    dims = (6, 10, 20)
    announce(f"unet conv3 input gradient {cin}->{cout} {dims}")
    rng = np.random.default_rng(1000 + cin * 10 + cout)
    dy = bf16_exact(rng, dims + (cout,))
    y = bf16_exact(rng, dims + (cout,))  # about half of the gate is <= 0
    y[0, 0, 0, :4] = 0.0  # the gate is strict: y = 0 blocks the gradient
    w = rng.standard_normal((27, cin, cout)) * 0.2
    dz = dy * (y > 0)
    wr = O.round_bf16(w)
    ref = O.conv3_grad_input(dz, wr)
    S = O.conv3_grad_input(np.abs(dz), np.abs(wr))
    out = torch.zeros(dims + (cin,), dtype=torch.float32, device="cuda")
    src = U.source(U.SRC_MASKED, dims, cout, to_dev(dy, torch.bfloat16), to_dev(y, torch.bfloat16))
    U.unet_conv3(src, cin, packed(w, transpose=True), None, 0, 1, out)
    torch.cuda.synchronize()
    within(out.double().cpu().numpy(), ref, S, what="dgrad")


@pytest.mark.parametrize("mode,cin,cout", [("direct", 8, 16), ("direct", 16, 16), ("direct", 32, 32),
                                           ("direct", 64, 64), ("pool", 16, 32), ("pool", 32, 64),
                                           ("cat", 96, 32), ("cat", 48, 16)])
def test_conv3_weight_gradient(mode, cin, cout):
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    dims = (6, 10, 20)
    announce(f"unet conv3 weight gradient {mode} {cin}->{cout} {dims}")
    rng = np.random.default_rng(2000 + cin * 10 + cout)
    nz, ny, nx = dims
    if mode == "direct":
        x = bf16_exact(rng, dims + (cin,))
        xin, src = x, U.source(U.SRC_DIRECT, dims, cin, to_dev(x, torch.bfloat16))
    elif mode == "pool":
        fine = bf16_exact(rng, (2 * nz, 2 * ny, 2 * nx, cin))
        xin = O.round_bf16(O.pool(fine))
        src = U.source(U.SRC_POOL, dims, cin, to_dev(fine, torch.bfloat16))
    else:
        c0 = cin * 2 // 3
        coarse = bf16_exact(rng, (nz // 2, ny // 2, nx // 2, c0))
        skip = bf16_exact(rng, dims + (cin - c0,))
        xin = np.concatenate([O.up(coarse), skip], axis=3)
        src = U.source(U.SRC_CAT_UP, dims, cin, to_dev(coarse, torch.bfloat16), to_dev(skip, torch.bfloat16),
                       c_first=c0)
    dy = bf16_exact(rng, dims + (cout,))
    y = bf16_exact(rng, dims + (cout,))
    dz = dy * (y > 0)
    rdw, rdb = O.conv3_grad_weight(xin, dz)
    Sw, Sb = O.conv3_grad_weight(np.abs(xin), np.abs(dz))
    dzs = U.source(U.SRC_MASKED, dims, cout, to_dev(dy, torch.bfloat16), to_dev(y, torch.bfloat16))
    ws = torch.zeros(U.unet_wgrad_workspace_bytes(src, cout) // 4 + 4, dtype=torch.float32, device="cuda")
    dw = torch.zeros((27, cin, cout), dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    U.unet_conv3_wgrad(src, dzs, cout, ws, dw, db)
    torch.cuda.synchronize()
    within(dw.double().cpu().numpy(), rdw, Sw, rel=1e-4, what="dw")
    within(db.double().cpu().numpy(), rdb, Sb, rel=1e-4, what="db")
    # a second call gives the same bits (fixed summation order)
    dw2 = torch.zeros_like(dw)
    U.unet_conv3_wgrad(src, dzs, cout, ws, dw2, db)
    torch.cuda.synchronize()
    assert torch.equal(dw, dw2)


def test_head_loss_adam_and_skip_kernels():
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    announce("unet head / mse / adam / skip kernels")
    rng = np.random.default_rng(3)
    dims = (4, 6, 8)
    nvox = 4 * 6 * 8
    d = O.round_bf16(np.abs(rng.standard_normal(dims + (16,))))
    hw = rng.standard_normal((16, 4)).astype(np.float32).astype(np.float64)
    hb = rng.standard_normal(4).astype(np.float32).astype(np.float64)
    hwr = O.round_bf16(hw)
    out_ref = d @ hwr + hb
    dd_ = to_dev(d, torch.bfloat16)
    hwd, hbd = to_dev(hw, torch.float32), to_dev(hb, torch.float32)
    out = torch.zeros(dims + (4,), dtype=torch.float32, device="cuda")
    U.unet_head_forward(dd_, hwd, hbd, out)
    torch.cuda.synchronize()
    S = np.abs(d) @ np.abs(hwr) + np.abs(hb)
    within(out.double().cpu().numpy(), out_ref, S, what="head fwd")
    # loss and its gradient
    tgt = rng.standard_normal(dims + (4,)).astype(np.float32).astype(np.float64)
    mask = O.unknown_mask(8, 6, 4)
    o64 = out.double().cpu().numpy()
    ws = torch.zeros(1 << 16, dtype=torch.float32, device="cuda")
    dout = torch.zeros_like(out)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    U.unet_mse(out, to_dev(tgt, torch.float32), dims, dout, ws, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - O.loss(o64, tgt, mask)) <= 1e-12 * max(1.0, O.loss(o64, tgt, mask))
    g_ref = O.loss_grad(o64, tgt, mask)
    assert np.allclose(dout.double().cpu().numpy(), g_ref, rtol=1e-6, atol=1e-12)
    # head backward
    gd = dout.double().cpu().numpy()
    dd = torch.zeros(dims + (16,), dtype=torch.bfloat16, device="cuda")
    dhw = torch.zeros((16, 4), dtype=torch.float32, device="cuda")
    dhb = torch.zeros(4, dtype=torch.float32, device="cuda")
    U.unet_head_backward(dd_, dout, hwd, dd, ws, dhw, dhb)
    torch.cuda.synchronize()
    ref_dd = O.round_bf16(gd @ hwr.T)
    within(dd.double().cpu().numpy(), ref_dd, np.abs(gd) @ np.abs(hwr.T), bf16=True, what="head dd")
    within(dhw.double().cpu().numpy(), d.reshape(-1, 16).T @ gd.reshape(-1, 4),
           np.abs(d).reshape(-1, 16).T @ np.abs(gd).reshape(-1, 4), rel=1e-5, what="dhw")
    within(dhb.double().cpu().numpy(), gd.sum(axis=(0, 1, 2)), np.abs(gd).sum(axis=(0, 1, 2)), rel=1e-5, what="dhb")
    # Adam: two steps against the oracle's update
    p = rng.standard_normal(1000).astype(np.float32).astype(np.float64)
    g = rng.standard_normal(1000).astype(np.float32).astype(np.float64)
    pd, gdv = to_dev(p, torch.float32), to_dev(g, torch.float32)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    params, st = {"p": p.copy()}, {}
    for step in (1, 2):
        U.unet_adam(pd, gdv, md, vd, 1e-3, 0.9, 0.999, 1e-8, step)
        O.adam_step(params, {"p": g}, st, step, 1e-3)
    torch.cuda.synchronize()
    assert np.allclose(pd.double().cpu().numpy(), params["p"], rtol=0, atol=1e-6)
    # gradient at a skip link: bf16(fine[..., coff:] + pooled / 8) and the upsampling adjoint
    fine = bf16_exact(rng, (4, 6, 8, 48))
    pooled = bf16_exact(rng, (2, 3, 4, 16))
    out = torch.zeros((4, 6, 8, 16), dtype=torch.bfloat16, device="cuda")
    U.unet_skip_grad(to_dev(fine, torch.bfloat16), 48, 32, to_dev(pooled, torch.bfloat16), 16, (4, 6, 8), out)
    coarse = torch.zeros((2, 3, 4, 32), dtype=torch.bfloat16, device="cuda")
    U.unet_up_grad(to_dev(fine, torch.bfloat16), 48, 0, 32, (2, 3, 4), coarse)
    torch.cuda.synchronize()
    assert np.array_equal(out.double().cpu().numpy(), O.round_bf16(fine[..., 32:] + O.pool_grad(pooled)))
    assert np.array_equal(coarse.double().cpu().numpy(), O.round_bf16(O.up_grad(fine[..., :32])))


def test_state_vector_conversions():
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    nx, ny, nz = 16, 8, 12
    announce(f"unet state conversions {nx}x{ny}x{nz}")
    h = 1.0 / 16
    sol = StokesSolver(nx, ny, nz, h=h)
    f = sinusoid_forcing(nx, ny, nz, h, seed=4)
    fields = [f[0].copy(), f[1].copy(), f[2].copy()]
    fields[0][[0, -1]] = 0.0
    fields[1][:, [0, -1]] = 0.0
    fields[2][:, :, [0, -1]] = 0.0
    b = sol.pack(tuple(fields) + (np.zeros((nx, ny, nz)),))
    L = U.state_layout(sol.layout)
    ws = torch.zeros(U.unet_reduce_workspace_bytes(L) // 4 + 4, dtype=torch.float32, device="cuda")
    scale = torch.zeros(1, dtype=torch.float64, device="cuda")
    U.unet_state_scale(b, L, ws, scale)
    inp = torch.zeros((nz, ny, nx, 8), dtype=torch.bfloat16, device="cuda")
    U.unet_state_to_input(b, L, scale, inp)
    torch.cuda.synchronize()
    n_u = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    s_ref = np.sqrt(sum(float(np.sum(a ** 2)) for a in fields) / n_u)
    assert abs(scale.item() - s_ref) <= 1e-14 * s_ref
    want = O.round_bf16(O.to_voxels(*fields) / s_ref)
    assert np.array_equal(inp.double().cpu().numpy(), want)
    # output -> state and state -> target are inverse on the unknowns
    rng = np.random.default_rng(5)
    outv = rng.standard_normal((nz, ny, nx, 4)).astype(np.float32)
    sigma = torch.tensor([0.5, 2.0, 1.0, 4.0], dtype=torch.float32, device="cuda")
    x = torch.full_like(b, 7.0)  # every slot is overwritten
    U.unet_output_to_state(to_dev(outv, torch.float32), L, scale, sigma, x)
    tgt = torch.zeros((nz, ny, nx, 4), dtype=torch.float32, device="cuda")
    U.unet_state_to_target(x, L, scale, sigma, tgt)
    torch.cuda.synchronize()
    got = sol.unpack(x)
    sig = np.array([0.5, 2.0, 1.0, 4.0])
    ref = O.from_voxels(outv.astype(np.float64) * s_ref * sig)
    for g_, r_ in zip(got, ref):
        assert np.allclose(g_, r_, rtol=1e-7, atol=0)
    mask = O.unknown_mask(nx, ny, nz)
    assert np.allclose(tgt.double().cpu().numpy(), outv * mask, rtol=1e-6, atol=0)
    # slots that are not unknowns are zero in the state vector
    assert float(x.abs().sum()) == pytest.approx(sum(float(np.abs(a).sum()) for a in got), rel=1e-12)


def _oracle_pass(params, x, target, mask, perturb_seed=None):
    """Oracle forward + backward; with a seed, every convolution result is
    multiplied by (1 + 8 * 2^-24 * N(0, 1)) before rounding: the size of the
    float32 accumulation error of the GPU kernels."""
    conv, gin = O.conv3, O.conv3_grad_input
    if perturb_seed is not None:
        r = np.random.default_rng(perturb_seed)

        def wrap(f):
            return lambda *a: (lambda y: y * (1 + 8 * 2.0 ** -24 * r.standard_normal(y.shape)))(f(*a))
        O.conv3, O.conv3_grad_input = wrap(conv), wrap(gin)
    try:
        out, cache = O.forward(params, x, rounding=True)
        g = O.backward(params, cache, O.loss_grad(out, target, mask), rounding=True)
    finally:
        O.conv3, O.conv3_grad_input = conv, gin
    return out, g


@pytest.mark.parametrize("dims", [(16, 16, 16), (8, 12, 16)])
def test_network_forward_and_backward_match_oracle(dims):
    """The bfloat16 network amplifies float32-sized differences (ReLU gates and
    rounding ties flip), so the bound is the oracle's own spread under
    perturbations of that size, per output and per parameter gradient."""
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    nz, ny, nx = dims
    announce(f"unet network fwd+bwd {dims}")
    params = O.init_params(7)
    rng = np.random.default_rng(8)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.standard_normal(params[k].shape).astype(np.float32).astype(np.float64) * 0.1
    x = np.zeros(dims + (8,))
    x[..., :3] = O.round_bf16(rng.standard_normal(dims + (3,)))
    target = rng.standard_normal(dims + (4,)).astype(np.float32).astype(np.float64)
    mask = O.unknown_mask(nx, ny, nz)
    out_ref, g_ref = _oracle_pass(params, x, target, mask)
    env_out, env_g = 0.0, {k: 0.0 for k in g_ref}
    for seed in (1, 2):
        o_p, g_p = _oracle_pass(params, x, target, mask, perturb_seed=seed)
        env_out = max(env_out, np.linalg.norm(o_p - out_ref) / np.linalg.norm(out_ref))
        for k in g_ref:
            env_g[k] = max(env_g[k], np.linalg.norm(g_p[k] - g_ref[k]) / max(np.linalg.norm(g_ref[k]), 1e-30))
    net = U.WarmStartNet(nx, ny, nz, params={k: v.astype(np.float32) for k, v in params.items()})
    net.inp.copy_(to_dev(x, torch.bfloat16))
    net.target.copy_(to_dev(target, torch.float32))
    net.forward()
    loss = net.loss_and_grad()
    net.backward()
    torch.cuda.synchronize()
    out = net.out.double().cpu().numpy()
    e_out = np.linalg.norm(out - out_ref) / np.linalg.norm(out_ref)
    announce(f"  out rel err {e_out:.2e} (oracle spread {env_out:.2e})")
    assert e_out <= 3 * env_out + 1e-6, (e_out, env_out)
    lref = O.loss(out_ref, target, mask)
    assert abs(loss.item() - lref) <= (2 * e_out + 1e-6) * lref
    for k, t in net.g.items():
        gk = t.double().cpu().numpy()
        e = np.linalg.norm(gk - g_ref[k]) / max(np.linalg.norm(g_ref[k]), 1e-30)
        announce(f"  grad {k}: rel err {e:.2e} (oracle spread {env_g[k]:.2e})")
        assert e <= 3 * env_g[k] + 1e-4, (k, e, env_g[k])


def test_training_steps_reduce_the_loss_on_a_solver_pair():
    torch = cuda()
    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    n = 16
    announce("unet training steps on a 16^3 solver pair")
    h = 1.0 / n
    sol = StokesSolver(n, n, n, h=h)
    f = sinusoid_forcing(n, n, n, h, seed=1)
    fl = [f[0].copy(), f[1].copy(), f[2].copy()]
    fl[0][[0, -1]] = 0.0
    fl[1][:, [0, -1]] = 0.0
    fl[2][:, :, [0, -1]] = 0.0
    b = sol.pack(tuple(fl) + (np.zeros((n, n, n)),))
    xs, info = sol.solve(b, rtol=1e-8, maxit=100)
    assert info["status"] == "ok"
    net = U.WarmStartNet(n, n, n)
    net.set_input_from_state(b, sol.layout)
    net.sigma.fill_(1.0)
    net.set_target_from_state(xs, sol.layout)
    # per-channel scale of the target so that every output is O(1)
    U.unet_channel_sumsq(net.target, net.ws, net.sumsq)
    torch.cuda.synchronize()
    rms = np.sqrt(net.sumsq.cpu().numpy() / n ** 3)
    net.sigma.copy_(torch.tensor(rms, dtype=torch.float32))
    net.set_target_from_state(xs, sol.layout)
    losses = [float(net.train_step(1e-3).item()) for _ in range(60)]
    announce(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses[::10]
