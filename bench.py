#!/usr/bin/env python3
"""Benchmark: time for MG-SQMR to reach relative residual 1e-8 on the 256^3
MAC Stokes problem (FP64, 7-level V-cycle), on one MI355X.

One step = one complete solve from x0 = 0 (all hot-path kernels: operator,
V-cycle smoothers and transfers, coarse solve, SQMR recurrences).  The input
(seeded sinusoid forcing) is resident in HBM before timing starts.  Prints
one JSON line.

Roofline: the dominant kernel is timed live with HIP events (recorded by the
library on its stream) during the timed steps; `achieved` = its algorithmic
bytes per launch / its average launch duration.  `traffic` comes from the
rocprofv3 counter summary under profiles/ when that summary was taken on the
current kernel source, else null.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak of MI355X
WEIGHTS = os.path.join(ROOT, "paper_2312_10615_amd", "weights", "warmstart_128.npz")
S = 8  # bytes per FP64 value


def dof_counts(n):
    nu = 3 * (n - 1) * n * n
    return nu, n ** 3


def algorithmic_bytes(kernel, n):
    """Compulsory bytes of one launch at level 0 (each operand streamed once).
    dgs_pr: one colour's worth of the reverse pressure step (the stage
    launches of one sweep split it unevenly)."""
    nu, npr = dof_counts(n)
    return {
        "dgs_u": (2 * nu + npr) * S,            # read u, p, b_u(colour); write u(colour)
        "dgs_pr": (nu + 2.5 * npr) * S,         # read b_u, b_p, p; write p(colour)
        "apply": 3 * (nu + npr) * S,            # residual: read x, b; write r
        "restrict": 1.125 * (nu + npr) * S,
        "prolong": 2.125 * (nu + npr) * S,
    }[kernel]


def kernel_source_hash():
    from paper_2312_10615_amd.profiling import kernel_source_hash as h
    return h()


def counter_traffic(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on this kernel source and workload."""
    path = os.path.join(ROOT, "profiles", "counters_fp64_256.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n") != n:
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    if not d.get("fetch_scale") or not d.get("write_scale"):
        return None
    return round((k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0)


def vcycle_model_bytes(n, s=S, levels=7):
    """Compulsory HBM bytes of one V-cycle on an n^3 box (per-sweep traffic
    model: each dependent colour half-sweep streams its operands once).  Per
    level: two symmetric DGS (forward + reverse sweep, (16 n_u + 14 n_p) s
    each), four symmetric Vanka steps (~114 values per V1 cell each: 16 class
    steps, run as 8 passes of two classes, x 1/8 of the cells x ~57 values),
    residual + restriction and prolongation + correction ((2 n + n/8) s
    each); the coarsest level's dense
    solve reads its inverse once (8-byte values).  With 4-byte level values
    (the FP32 V-cycle) the conversions of s to FP32 and of the result back to
    FP64 add (8 + 4) bytes per unknown each."""
    nu0, np0 = dof_counts(n)
    total = 0.0 if s == 8 else 24.0 * (nu0 + np0)
    m = n
    for lev in range(levels):
        nu, npr = dof_counts(m)
        if lev == levels - 1:
            total += (nu + npr) ** 2 * 8
            break
        v1_cells = m ** 3 - (m - 2) ** 3
        total += 2 * (16 * nu + 14 * npr) * s + 4 * 114 * v1_cells * s + 2 * (2 + 1 / 8) * (nu + npr) * s
        m //= 2
    return total


def cpu_baseline(iters, n_full, seed, gpu_small):
    """The oracle timed on the host, one thread.
    Measured: the complete oracle MG-SQMR solve of the 32^3 workload (4 levels,
    seed 0, rtol 1e-8), median of 3, beside the GPU's time for the same solve.
    Extrapolated to the headline 256^3 solve (labelled as such): one oracle
    V-cycle, two operator applications and SQMR's vector passes of one
    iteration at 128^3, scaled by 8 (work linear in the unknowns) and by the
    number of V-cycles of the GPU solve (iterations + 1)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.multigrid import Hierarchy, vcycle
    from oracle.operator import apply_operator, to_vector
    from oracle.sqmr import mg_sqmr
    from paper_2312_10615_amd.workloads import sinusoid_forcing

    def rhs(H, m):
        dom = H.doms[0]
        f = sinusoid_forcing(m, m, m, 1.0 / m, seed=seed)
        return tuple(np.where(dom.active[a], f[a], 0.0) for a in range(3)) + (np.zeros((m, m, m)),)

    with threadpool_limits(limits=1):
        m = 32
        H = Hierarchy((m, m, m), 1.0 / m)
        b = rhs(H, m)
        runs, it_small = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            _, inf = mg_sqmr(H, b, rtol=1e-8, maxit=200)
            runs.append(time.perf_counter() - t0)
            it_small = inf["iters"]
        t_small = float(np.median(runs))
        n = n_full // 2
        H = Hierarchy((n, n, n), 1.0 / n)
        b = rhs(H, n)
        bv = to_vector(H.doms[0], b)
        t0 = time.perf_counter()
        vcycle(H, b)
        apply_operator(H.doms[0], b, 0.0)
        apply_operator(H.doms[0], b, 0.0)
        q, t, d, x, r = bv.copy(), bv.copy(), bv.copy(), bv.copy(), bv.copy()
        for _ in range(3):   # dots (sigma, ||t||, rho, ||r||) and updates (s, d, x, q): ~16 vector passes
            r = r - 0.5 * t
            d = 0.3 * d + 0.2 * q
            x = x + d
            q = t + 0.7 * q
            float(np.dot(q, t))
        t1 = time.perf_counter()
    per_iter = (t1 - t0) * (n_full / n) ** 3
    return {"value": round(per_iter * (iters + 1), 1), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"extrapolated: one oracle V-cycle, two operator applications and one iteration's SQMR "
                      f"vector passes at {n}^3 (seed {seed}, 1 thread) took {t1 - t0:.1f} s, scaled x"
                      f"{(n_full // n) ** 3} to {n_full}^3 and x{iters + 1} V-cycles of the GPU solve",
            "measured_32": {"oracle_s": round(t_small, 3), "oracle_iterations": it_small,
                            "gpu_s": gpu_small["s"], "gpu_iterations": gpu_small["iters"],
                            "ratio": round(t_small / gpu_small["s"], 1),
                            "what": "complete MG-SQMR solve of the 32^3 workload (4 levels, seed 0, rtol 1e-8); "
                                    "oracle median of 3 on 1 thread, GPU median of 5"},
            "host_cpus": os.cpu_count()}


def gpu_small_solve(seed, rtol):
    """The 32^3 workload on the GPU (the size the oracle finishes in seconds)."""
    import numpy as np
    import torch

    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    m = 32
    sol = StokesSolver(m, m, m, h=1.0 / m)
    f = sinusoid_forcing(m, m, m, 1.0 / m, seed=seed)
    b = sol.pack((f[0], f[1], f[2], np.zeros((m, m, m))))
    sol.solve(b, rtol=rtol, maxit=200)
    ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = sol.solve(b, rtol=rtol, maxit=200)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    sol.close()
    return {"s": round(float(np.median(ts)), 5), "iters": info["iters"]}


def channel_labels(n):
    """A 256^3-style channel of Section 5 labels: Dirichlet walls and inflow
    side, a Dirichlet block obstacle, one layer of exterior cells on the +x
    (outflow) side.  Indexed [i, j, k] over the padded box."""
    import numpy as np
    lab = np.ones((n + 2,) * 3, dtype=np.uint8)
    lab[1:-1, 1:-1, 1:-1] = 0
    lab[-1, 1:-1, 1:-1] = 2
    q = n // 4
    lab[q + 1:2 * q + 1, q + 1:2 * q + 1, q + 1:2 * q + 1] = 1
    return lab


def labelled_leg(n, steps, rtol, seed):
    """The same solve on a labelled domain (obstacle + outflow, Section 5):
    time, iterations and V-cycle time, FP64."""
    import numpy as np
    import torch

    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    lab = channel_labels(n)
    sol = StokesSolver(n, n, n, h=1.0 / n, labels=lab)
    f = sinusoid_forcing(n, n, n, 1.0 / n, seed=seed)
    b = sol.pack((f[0], f[1], f[2], np.zeros((n, n, n))))
    del f
    x, info = sol.solve(b, rtol=rtol, maxit=500)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info = sol.solve(b, rtol=rtol, maxit=500)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / steps
    t = sol.new_state()
    sol.vcycle(b, out=t)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        sol.vcycle(b, out=t)
    e1.record()
    torch.cuda.synchronize()
    out = {"value": round(ts, 6), "unit": "s", "iterations": info["iters"], "final_relres": info["relres"],
           "status": info["status"], "vcycle_ms": round(e0.elapsed_time(e1) / 5, 3), "unknowns": int(sol.layout.n_dofs),
           "domain": f"{n}^3 labelled channel: no-slip walls and inflow side, a {n // 4}^3 Dirichlet block obstacle, "
                     f"an exterior (outflow, Neumann) layer on the +x side"}
    sol.close()
    print(f"[bench] labelled {n}^3: {ts * 1e3:.1f} ms, iters={info['iters']}", file=sys.stderr, flush=True)
    return out


def mixed_384_leg(steps, rtol, seed):
    """FP32 V-cycle at 384^3 (7 levels down to 6^3, 756 coarsest unknowns)
    against the FP64 GPU solve of the same problem (the error reference)."""
    import numpy as np
    import torch

    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing_device
    n = 384
    h = 1.0 / n
    out = {}
    x64 = None
    for prec in (64, 32):
        sol = StokesSolver(n, n, n, h=h, precision=prec)
        f = sinusoid_forcing_device(n, n, n, h, seed, sol.device)
        b = sol.pack(f + (torch.zeros((n, n, n), dtype=torch.float64, device=sol.device),))
        del f
        x, info = sol.solve(b, rtol=rtol, maxit=500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = steps if prec == 32 else 1
        for _ in range(k):
            x, info = sol.solve(b, rtol=rtol, maxit=500)
        torch.cuda.synchronize()
        out[prec] = {"s": (time.perf_counter() - t0) / k, "iters": info["iters"], "relres": info["relres"],
                     "status": info["status"], "levels": sol.layout.levels}
        if prec == 64:
            x64 = x
        else:
            out["err"] = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
            g = torch.Generator(device=sol.device).manual_seed(5)
            shapes = [(n + 1, n, n), (n, n + 1, n), (n, n, n + 1), (n, n, n)]
            xa = sol.pack(tuple(torch.randn(sh, generator=g, dtype=torch.float64, device=sol.device) for sh in shapes))
            ya = sol.pack(tuple(torch.randn(sh, generator=g, dtype=torch.float64, device=sol.device) for sh in shapes))
            wa, wb = float(torch.dot(xa, sol.vcycle(ya))), float(torch.dot(sol.vcycle(xa), ya))
            out["asym"] = abs(wa - wb) / abs(wa)
            del xa, ya
        sol.close()
        del sol, b, x
        torch.cuda.empty_cache()
    print(f"[bench] 384^3: fp64 {out[64]['s'] * 1e3:.1f} ms ({out[64]['iters']} it), fp32 V-cycle "
          f"{out[32]['s'] * 1e3:.1f} ms ({out[32]['iters']} it), err {out['err']:.2e}", file=sys.stderr, flush=True)
    return {"value": round(out[32]["s"], 6), "unit": "s", "n": n, "levels": out[32]["levels"],
            "iterations": out[32]["iters"], "final_relres": out[32]["relres"], "status": out[32]["status"],
            "fp64_s": round(out[64]["s"], 6), "fp64_iterations": out[64]["iters"],
            "speedup_vs_fp64": round(out[64]["s"] / out[32]["s"], 3),
            "rel_err_vs_fp64_solution": out["err"], "vcycle_asymmetry": out["asym"],
            "error_reference": "the FP64 GPU solve of the same problem (the oracle at 384^3 needs ~40 GB and hours)"}


def batched_leg(steps, rtol, seed):
    """48 boxes with sizes drawn from {32,48,64,96,128} per axis, each with its
    own seeded forcing, solved together (FP32 V-cycle, FP64 SQMR); also the
    same boxes one after another with the single-box solver."""
    import torch

    from paper_2312_10615_amd.stokes import StokesBatch, StokesSolver
    from paper_2312_10615_amd.workloads import batch_dims, sinusoid_forcing_device

    dims = batch_dims(48, seed=seed)
    h = 1.0 / 128
    t0 = time.perf_counter()
    bt = StokesBatch(dims, h=h, precision=32)
    setup = time.perf_counter() - t0
    fields = []
    for d, (nx, ny, nz) in enumerate(dims):
        f = sinusoid_forcing_device(nx, ny, nz, h, 1000 + d, bt.device)
        fields.append(f + (torch.zeros((nx, ny, nz), dtype=torch.float64, device=bt.device),))
    b = bt.pack(fields)
    del fields
    t0 = time.perf_counter()
    tiles = bt.autotune()
    tune_s = time.perf_counter() - t0
    x, infos = bt.solve(b, rtol=rtol, maxit=200)  # warm-up (captures the graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, infos = bt.solve(b, rtol=rtol, maxit=200)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    assert all(i["status"] == "ok" for i in infos), infos
    # the same boxes one by one (single-box solver, graph V-cycle, FP32 form)
    t_seq = 0.0
    seq_iters = []
    for d, dm in enumerate(dims):
        sol = StokesSolver(*dm, h=h, precision=32, levels=bt.layouts[d].levels)
        bd = bt.part(b, d).clone()
        sol.solve(bd, rtol=rtol, maxit=200)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, inf = sol.solve(bd, rtol=rtol, maxit=200)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - ts
        seq_iters.append(inf["iters"])
        del sol
    unknowns = int(sum(l.n_dofs for l in bt.layouts))
    print(f"[bench] batched: {t_batch * 1e3:.1f} ms per batch, sequential {t_seq * 1e3:.1f} ms", file=sys.stderr,
          flush=True)
    return {"value": round(len(dims) / t_batch, 3), "unit": "solves/s", "boxes": len(dims),
            "ms_per_batch": round(t_batch * 1e3, 3), "unknowns": unknowns,
            "iterations": [i["iters"] for i in infos], "levels": [l.levels for l in bt.layouts],
            "dims": [list(dm) for dm in dims], "final_relres_max": max(i["relres"] for i in infos),
            "sequential_ms": round(t_seq * 1e3, 3), "sequential_iterations": seq_iters,
            "speedup_vs_sequential": round(t_seq / t_batch, 3), "setup_s": round(setup, 3),
            "autotune_s": round(tune_s, 3), "tile_x_extent": {k: v[:max(bt.layouts[i].levels for i in range(len(dims)))]
                                                              for k, v in tiles.items()},
            "form": "FP32 V-cycle, FP64 SQMR; h = 1/128; one graph replay for the set-up and first 10 iterations, "
                    "then 2 iterations per replay"}


def warm_start_leg(sol, b, steps, rtol, zero_ms, zero_iters, held_out=16):
    """The learned warm start at 256^3: the network runs on the 128^3 level
    (R b there), its guess is prolonged with P and SQMR starts from it.  Time
    includes the guess.  Also the network forward's matrix-core throughput,
    and zero guess vs network guess on the first `held_out` held-out seeds at
    128^3 and 256^3 (iterations and time to the tolerance, means)."""
    import torch

    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.warmstart import load_weights

    params, sigma, record = load_weights(WEIGHTS)
    lay1 = sol.level_layout(1)
    net = U.WarmStartNet(lay1.nx, lay1.ny, lay1.nz, params=params, sigma=sigma)
    xc = torch.zeros(lay1.total, dtype=torch.float64, device=sol.device)
    x0 = sol.new_state()

    def guess():
        net.initial_guess(sol.restrict(b), lay1, xc)
        sol.prolong(xc, out=x0)

    guess()
    x, info = sol.solve(b, x0=x0, rtol=rtol, maxit=500)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        guess()
        x, info = sol.solve(b, x0=x0, rtol=rtol, maxit=500)
    torch.cuda.synchronize()
    t_warm = (time.perf_counter() - t0) / steps
    r0 = info["history"][0]
    # network forward alone, HIP events around the 10 convolutions and the head
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nf = 10
    ev0.record()
    for _ in range(nf):
        net.forward()
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / nf
    flops = 0
    bound_s = 0.0  # per layer, the larger of its matrix-core time and its HBM time (bf16 in and out once)
    chans = {name: cout for name, _, _, cout in U.LAYERS}
    for name, spec, cin, cout in U.LAYERS:
        dz, dy, dx = net.dims[U.LEVEL[name]]
        vox = dz * dy * dx
        f = 2 * 27 * cin * cout * vox
        if isinstance(spec, tuple) and spec[0] == "pool":
            elems_in = 8 * vox * cin
        elif isinstance(spec, tuple) and spec[0] == "cat":
            elems_in = vox // 8 * chans[spec[1]] + vox * (cin - chans[spec[1]])
        else:
            elems_in = vox * cin
        flops += f
        bound_s += max(f / (BF16_PEAK_TFLOPS * 1e12), 2 * (elems_in + vox * cout) / (HBM_PEAK_GBPS * 1e9))
    vox0 = net.dims[0][0] * net.dims[0][1] * net.dims[0][2]
    bound_s += (2 * U.HEAD_IN + 4 * U.HEAD_OUT) * vox0 / (HBM_PEAK_GBPS * 1e9)  # head: bf16 in, float out
    tf = flops / (fwd_ms * 1e-3) / 1e12
    print(f"[bench] warm start: {t_warm * 1e3:.1f} ms, iters {info['iters']} (zero guess {zero_iters})",
          file=sys.stderr, flush=True)
    held = {}
    if held_out > 0:
        from paper_2312_10615_amd.warmstart import evaluate
        for n, coarse in ((128, False), (sol.layout.nx, True)):
            summ, _ = evaluate(WEIGHTS, n=n, seeds=held_out, rtol=rtol, coarse_net=coarse, log=lambda m: None)
            held[f"{n}^3"] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in summ.items()
                              if k in ("seeds", "iters_zero_mean", "iters_warm_mean", "time_zero_mean_s",
                                       "time_warm_mean_s", "speedup", "guess_rel_residual_median", "all_converged")}
            print(f"[bench] warm start, {held_out} held-out seeds at {n}^3: iterations {summ['iters_zero_mean']:.2f} -> "
                  f"{summ['iters_warm_mean']:.2f}, {summ['speedup']:.3f}x", file=sys.stderr, flush=True)
        held["note"] = "means over the first held-out seeds; 200 seeds: profiles/warmstart_eval.md"
        torch.cuda.empty_cache()
    return {"value": round(t_warm, 6), "unit": "s", "iterations": info["iters"], "zero_guess_iterations": zero_iters,
            "final_relres": info["relres"], "status": info["status"],
            "speedup_vs_fp64": round(zero_ms / 1000.0 / t_warm, 3), "guess_relres": r0, "held_out": held,
            "network": f"3-level U-Net 16/32/64 channels on the {lay1.nx}^3 level, bf16 on matrix cores",
            "training": {k: record.get(k) for k in ("n", "pairs", "epochs", "lr", "train_seconds", "sigma")}
            | {"final_loss": record.get("loss_history", [[0, None]])[-1][1]},
            "roofline": {"bound": "mfma", "kernel": "k_conv3 (10 layers) + head, 128^3 forward",
                         "achieved": round(tf, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / BF16_PEAK_TFLOPS, 4), "traffic": None, "forward_ms": round(fwd_ms, 4),
                         "algorithmic_flops_per_forward": flops,
                         "layer_bound_ms": round(bound_s * 1e3, 4),
                         "frac_of_layer_bound": round(bound_s * 1e3 / fwd_ms, 4)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--kernel", default="dgs_u", help="dominant kernel class timed for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-V-cycle (mixed precision) leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-box batched leg")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-384", action="store_true", help="skip the 384^3 FP32-V-cycle leg")
    ap.add_argument("--no-split", action="store_true", help="skip the split-schedule leg")
    ap.add_argument("--no-labelled", action="store_true", help="skip the labelled-domain (obstacle + outflow) leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference dispatch for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the solve does not shard "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_10615_amd.stokes import StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing

    n = args.n
    h = 1.0 / n
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    sol = StokesSolver(n, n, n, h=h)
    t_setup = time.perf_counter() - t_setup
    layout_levels = sol.layout.levels
    n_dofs = int(sol.layout.n_dofs)
    f = sinusoid_forcing(n, n, n, h, seed=args.seed)
    b = sol.pack((f[0], f[1], f[2], np.zeros((n, n, n))))
    del f
    torch.cuda.synchronize()
    print(f"[bench] setup {t_setup:.2f}s, levels={sol.layout.levels}, unknowns={sol.layout.n_dofs}", file=sys.stderr,
          flush=True)

    info = None
    for w in range(args.warmup):
        x, info = sol.solve(b, rtol=args.rtol, maxit=500)
        print(f"[bench] warmup {w}: iters={info['iters']} relres={info['relres']:.3e} {info['status']}",
              file=sys.stderr, flush=True)

    sol.profile(args.kernel, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, info = sol.solve(b, rtol=args.rtol, maxit=500)
        print(f"[bench] step {k}: iters={info['iters']} relres={info['relres']:.3e} {info['status']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, klaunch = sol.profile_read(args.kernel, 0)
    sol.profile("off")
    assert info["status"] == "ok", info
    ms_per_step = (t1 - t0) * 1000.0 / args.steps

    # V-cycle time alone (outside the timed region)
    s = b.clone()
    t = sol.new_state()
    sol.vcycle(s, out=t)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    nvc = 5
    for _ in range(nvc):
        sol.vcycle(s, out=t)
    ev1.record()
    torch.cuda.synchronize()
    vcycle_ms = ev0.elapsed_time(ev1) / nvc

    split = None
    if not args.no_split:
        # the other arrangement Section 3 allows: reverse sweeps before, forward sweeps after
        ssp = StokesSolver(n, n, n, h=h, schedule="split")
        xs, isp = ssp.solve(b, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for _ in range(args.steps):
            xs, isp = ssp.solve(b, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        tsp = (time.perf_counter() - tm0) / args.steps
        ev0.record()
        for _ in range(nvc):
            ssp.vcycle(s, out=t)
        ev1.record()
        torch.cuda.synchronize()
        split = {"value": round(tsp, 6), "unit": "s", "iterations": isp["iters"], "final_relres": isp["relres"],
                 "status": isp["status"], "vcycle_ms": round(ev0.elapsed_time(ev1) / nvc, 3),
                 "rel_diff_vs_default_solution": float(torch.linalg.vector_norm(xs - x) / torch.linalg.vector_norm(x)),
                 "form": "pre-smoothing: Vanka, 2 reverse DGS sweeps, Vanka; post-smoothing: Vanka, 2 forward "
                         "sweeps, Vanka (Section 3's transposed pair)"}
        ssp.close()
        del ssp, xs
        print(f"[bench] split schedule: {tsp * 1e3:.1f} ms, iters={isp['iters']}", file=sys.stderr, flush=True)

    warm = None
    if not args.no_warm_start and os.path.exists(WEIGHTS):
        warm = warm_start_leg(sol, b, args.steps, args.rtol, ms_per_step, info["iters"])

    mixed = None
    if not args.no_mixed:
        # Mixed precision: FP32 V-cycle inside FP64 SQMR, same input and tolerance.
        s32 = StokesSolver(n, n, n, h=h, precision=32)
        b32 = b  # same layout (the layout does not depend on the V-cycle precision)
        x32, i32 = s32.solve(b32, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for _ in range(args.steps):
            x32, i32 = s32.solve(b32, rtol=args.rtol, maxit=500)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - tm0) / args.steps
        err = float(torch.linalg.vector_norm(x32 - x) / torch.linalg.vector_norm(x))
        xa = s32.pack(tuple(np.random.default_rng(1).standard_normal(a.shape) for a in sol.unpack(b)))
        ya = s32.pack(tuple(np.random.default_rng(2).standard_normal(a.shape) for a in sol.unpack(b)))
        wa, wb = float(torch.dot(xa, s32.vcycle(ya))), float(torch.dot(s32.vcycle(xa), ya))
        ev0.record()
        for _ in range(nvc):
            s32.vcycle(s, out=t)
        ev1.record()
        torch.cuda.synchronize()
        mixed = {"value": round(t32, 6), "unit": "s", "iterations": i32["iters"], "final_relres": i32["relres"],
                 "status": i32["status"], "speedup_vs_fp64": round(ms_per_step / 1000.0 / t32, 3),
                 "rel_err_vs_fp64_solution": err, "vcycle_asymmetry": abs(wa - wb) / abs(wa),
                 "vcycle_ms": round(ev0.elapsed_time(ev1) / nvc, 3),
                 "form": "FP32 V-cycle (level vectors, smoothers, transfers, stencils), FP64 SQMR, dots, "
                         "true residual and coarsest solve"}
        del s32, x32, xa, ya
        print(f"[bench] mixed: {t32 * 1e3:.1f} ms, iters={i32['iters']}, err={err:.2e}", file=sys.stderr,
              flush=True)

    batched = None
    if not args.no_batched:
        batched = batched_leg(args.steps, args.rtol, args.seed)

    m384 = None
    labelled = None
    if (not args.no_384 and n == 256) or not args.no_labelled:
        sol.close()
        del sol, x, s, t, b
        torch.cuda.empty_cache()
    if not args.no_labelled:
        labelled = labelled_leg(n, args.steps, args.rtol, args.seed)
        torch.cuda.empty_cache()
    if not args.no_384 and n == 256:
        m384 = mixed_384_leg(args.steps, args.rtol, args.seed)

    gsmall = None
    if not args.no_cpu_baseline:
        gsmall = gpu_small_solve(args.seed, args.rtol)

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    levels = layout_levels
    vbytes = vcycle_model_bytes(n, S, levels)
    avg_ms = kms / max(klaunch, 1)
    abytes = algorithmic_bytes(args.kernel, n)
    achieved = abytes / (avg_ms * 1e-3) / 1e9
    traffic = counter_traffic(args.kernel, n)
    line = {
        "metric": "time to 1e-8 rel. residual, 256^3 Stokes; V-cycle HBM GB/s vs plain FP64",
        "value": round(ms_per_step / 1000.0, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 8-mode sinusoid forcing per component, zero divergence RHS)",
        "config": {"workload": f"3D MAC Stokes {n}^3 cells unit cube, no-slip box, eta=1, gamma=1e-3, "
                               f"{layout_levels}-level V-cycle (the same Alg. 3 smoother before and after the coarse correction: symmetric Vanka, one symmetric DGS, symmetric Vanka; n_b=1), "
                               f"MG-SQMR to rtol {args.rtol:g}",
                   "unknowns": n_dofs, "seed": args.seed, "precision": "fp64 throughout"},
        "iterations": info["iters"],
        "final_relres": info["relres"],
        "vcycle_ms": round(vcycle_ms, 3),
        "vcycle_model_bytes": round(vbytes),
        "vcycle_gbps": round(vbytes / (vcycle_ms * 1e-3) / 1e9, 1),
        "vcycle_frac": round(vbytes / (vcycle_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "setup_s": round(t_setup, 3),
        "roofline": {"bound": "hbm", "scope": "dominant kernel of the V-cycle (per kernel; the whole V-cycle "
                     "is vcycle_gbps / vcycle_frac)", "kernel": f"k_{args.kernel} (level 0)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "avg_launch_ms": round(avg_ms, 4), "launches": klaunch,
                     "algorithmic_bytes_per_launch": abytes},
    }
    if split is not None:
        line["split_schedule"] = split
    if mixed is not None:
        vb32 = vcycle_model_bytes(n, 4, levels)
        mixed["vcycle_model_bytes"] = round(vb32)
        mixed["vcycle_gbps"] = round(vb32 / (mixed["vcycle_ms"] * 1e-3) / 1e9, 1)
        mixed["vcycle_frac"] = round(vb32 / (mixed["vcycle_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        line["mixed_precision"] = mixed
    if m384 is not None:
        line["mixed_precision_384"] = m384
    if labelled is not None:
        line["labelled_domain"] = labelled
    if batched is not None:
        line["batched"] = batched
    if warm is not None:
        line["warm_start"] = warm
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(info["iters"], n, args.seed, gsmall)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
