"""Training and evaluation of the warm-start network on solver-generated pairs.

Data: for each seed, the seeded sinusoid forcing b = (f, 0) on an n^3 box and
the MG-SQMR solution x of L x = b (the solver itself generates the targets).
Pairs live in device memory: the network input (bfloat16, 8 channels) and the
target x / (scale * sigma_c) (float, 4 channels) per voxel.

Training: Adam on the mean squared error of the normalised state, one pair
per step, cosine learning-rate decay, all in the library's kernels
(paper_2312_10615_amd.unet).  Evaluation: SQMR iterations and time to the
tolerance from the zero guess and from the network's guess, on held-out seeds;
a larger box takes the guess computed on its next-coarser level (R b on the
coarse grid, the network there, P back to the fine grid).

Usage:
  python -m paper_2312_10615_amd.warmstart train --n 128 --pairs 2000 --epochs 4 --out W.npz
  python -m paper_2312_10615_amd.warmstart eval --weights W.npz --n 128 --seeds 200
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

TRAIN_SEED0 = 1000      # training seeds: TRAIN_SEED0 .. TRAIN_SEED0 + pairs - 1
EVAL_SEED0 = 100000     # held-out seeds
# weights trained by `train --n 128 --pairs 2000 --epochs 4` (record inside the file)
WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_128.npz")


def _forcing_state(sol, n, seed, device):
    from paper_2312_10615_amd.workloads import sinusoid_forcing_device
    import torch
    fx, fy, fz = sinusoid_forcing_device(n, n, n, 1.0 / n, seed, device)
    return sol.pack((fx, fy, fz, torch.zeros((n, n, n), dtype=torch.float64, device=device)))


def make_pairs(n, seeds, sigma=None, precision=32, rtol=1e-6, log=print):
    """Solve for every seed; returns (inputs, targets, sigma, solve stats)."""
    import torch
    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.stokes import StokesSolver
    dev = "cuda"
    sol = StokesSolver(n, n, n, h=1.0 / n, precision=precision)
    L = U.state_layout(sol.layout)
    ws = torch.zeros(U.unet_reduce_workspace_bytes(L) // 4 + 64, dtype=torch.float32, device=dev)
    scale = torch.zeros(1, dtype=torch.float64, device=dev)
    if sigma is None:
        # channel RMS of x / scale over the first pairs
        ones = torch.ones(4, dtype=torch.float32, device=dev)
        tmp = torch.zeros((n, n, n, 4), dtype=torch.float32, device=dev)
        sumsq = torch.zeros(4, dtype=torch.float64, device=dev)
        acc = np.zeros(4)
        for s in seeds[:8]:
            b = _forcing_state(sol, n, s, dev)
            x, info = sol.solve(b, rtol=rtol, maxit=200)
            U.unet_state_scale(b, L, ws, scale)
            U.unet_state_to_target(x, L, scale, ones, tmp)
            U.unet_channel_sumsq(tmp, ws, sumsq)
            acc += sumsq.cpu().numpy()
        sigma = np.sqrt(acc / (8 * n ** 3)).astype(np.float32)
    sig = torch.tensor(sigma, dtype=torch.float32, device=dev)
    N = len(seeds)
    inputs = torch.zeros((N, n, n, n, U.IN_CH), dtype=torch.bfloat16, device=dev)
    targets = torch.zeros((N, n, n, n, 4), dtype=torch.float32, device=dev)
    iters = []
    t0 = time.perf_counter()
    for i, s in enumerate(seeds):
        b = _forcing_state(sol, n, s, dev)
        x, info = sol.solve(b, rtol=rtol, maxit=200)
        if info["status"] != "ok":
            raise RuntimeError(f"solve for seed {s} ended with {info['status']}")
        iters.append(info["iters"])
        U.unet_state_scale(b, L, ws, scale)
        U.unet_state_to_input(b, L, scale, inputs[i])
        U.unet_state_to_target(x, L, scale, sig, targets[i])
        if (i + 1) % 200 == 0 or i + 1 == N:
            log(f"[pairs] {i + 1}/{N} solved, {time.perf_counter() - t0:.1f} s, mean iters {np.mean(iters):.2f}")
    return inputs, targets, sigma, {"solve_iters_mean": float(np.mean(iters)), "rtol": rtol,
                                    "seconds": time.perf_counter() - t0}


def train(n=128, pairs=2000, epochs=4, lr=2e-3, lr_min=2e-5, warmup=100, seed=0, log=print):
    """Generate pairs, train from a seeded initialisation; returns (net, record)."""
    import torch
    from paper_2312_10615_amd import unet as U
    seeds = list(range(TRAIN_SEED0, TRAIN_SEED0 + pairs))
    inputs, targets, sigma, gen = make_pairs(n, seeds, log=log)
    net = U.WarmStartNet(n, n, n, params=U.init_params(seed), sigma=tuple(float(s) for s in sigma))
    steps = epochs * pairs
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    step = 0
    loss_acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    for ep in range(epochs):
        for i in rng.permutation(pairs):
            frac = step / max(steps - 1, 1)
            a = lr * min(1.0, (step + 1) / warmup) if step < warmup else \
                lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * frac))
            net.inp, net.target = inputs[int(i)], targets[int(i)]
            loss_acc += net.train_step(a)
            step += 1
            if step % 250 == 0 or step == steps:
                m = float(loss_acc.item()) / (250 if step % 250 == 0 else step % 250)
                loss_acc.zero_()
                hist.append((step, m))
                log(f"[train] epoch {ep} step {step}/{steps} lr {a:.2e} mean loss {m:.4e} "
                    f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    record = {"n": n, "pairs": pairs, "epochs": epochs, "lr": lr, "lr_min": lr_min, "warmup": warmup,
              "init_seed": seed, "train_seeds": [seeds[0], seeds[-1]], "loss_history": hist,
              "train_seconds": time.perf_counter() - t0, "pair_generation": gen,
              "sigma": [float(s) for s in sigma]}
    del inputs, targets
    return net, record


def save_weights(path, net, record):
    params = net.params_numpy()
    np.savez(path, sigma=net.sigma.cpu().numpy(), record=np.array(json.dumps(record)),
             **{k.replace(".", "__"): v for k, v in params.items()})


def load_weights(path):
    """(params dict, sigma, record) from a file written by save_weights (no pickles)."""
    d = np.load(path, allow_pickle=False)
    params = {k.replace("__", "."): d[k] for k in d.files if k not in ("sigma", "record")}
    return params, tuple(float(s) for s in d["sigma"]), json.loads(str(d["record"]))


def evaluate(weights, n=128, seeds=200, rtol=1e-8, precision=64, coarse_net=False, log=print):
    """Zero guess vs network guess on held-out seeds at n^3.  coarse_net: the
    network runs on the next-coarser level (n/2)^3 and its guess is prolonged."""
    import torch
    from paper_2312_10615_amd import unet as U
    from paper_2312_10615_amd.stokes import StokesSolver
    params, sigma, _ = load_weights(weights)
    sol = StokesSolver(n, n, n, h=1.0 / n, precision=precision)
    nn_ = n // 2 if coarse_net else n
    net = U.WarmStartNet(nn_, nn_, nn_, params=params, sigma=sigma)
    net_layout = sol.level_layout(1) if coarse_net else sol.layout
    x0 = sol.new_state()
    x0c = torch.zeros(net_layout.total, dtype=torch.float64, device="cuda") if coarse_net else None
    rows = []
    for k in range(seeds):
        s = EVAL_SEED0 + k
        b = _forcing_state(sol, n, s, "cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0 = sol.solve(b, rtol=rtol, maxit=500)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if coarse_net:
            bc = sol.restrict(b)
            net.initial_guess(bc, net_layout, x0c)
            sol.prolong(x0c, out=x0)
        else:
            net.initial_guess(b, net_layout, x0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, i1 = sol.solve(b, x0=x0, rtol=rtol, maxit=500)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rows.append({"seed": s, "iters_zero": i0["iters"], "iters_warm": i1["iters"], "t_zero": t1 - t0,
                     "t_guess": t2 - t1, "t_warm_solve": t3 - t2, "r0_warm": i1["history"][0],
                     "status": [i0["status"], i1["status"]]})
        if (k + 1) % 50 == 0 or k + 1 == seeds:
            r = rows
            log(f"[eval n={n}{' coarse-net' if coarse_net else ''}] {k + 1}/{seeds}: iters zero "
                f"{np.mean([q['iters_zero'] for q in r]):.2f} warm {np.mean([q['iters_warm'] for q in r]):.2f}, "
                f"initial rel. residual of the guess {np.median([q['r0_warm'] for q in r]):.3e}")
    summary = {
        "n": n, "seeds": [EVAL_SEED0, EVAL_SEED0 + seeds - 1], "rtol": rtol, "precision": precision,
        "network_grid": nn_, "iters_zero_mean": float(np.mean([q["iters_zero"] for q in rows])),
        "iters_warm_mean": float(np.mean([q["iters_warm"] for q in rows])),
        "time_zero_mean_s": float(np.mean([q["t_zero"] for q in rows[1:]] or [rows[0]["t_zero"]])),
        "time_warm_mean_s": float(np.mean([q["t_guess"] + q["t_warm_solve"] for q in rows[1:]] or
                                          [rows[0]["t_guess"] + rows[0]["t_warm_solve"]])),
        "guess_time_mean_s": float(np.mean([q["t_guess"] for q in rows[1:]] or [rows[0]["t_guess"]])),
        "guess_rel_residual_median": float(np.median([q["r0_warm"] for q in rows])),
        "all_converged": all(q["status"] == ["ok", "ok"] for q in rows),
    }
    summary["speedup"] = summary["time_zero_mean_s"] / summary["time_warm_mean_s"]
    return summary, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n", type=int, default=128)
    t.add_argument("--pairs", type=int, default=2000)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--n", type=int, default=128)
    e.add_argument("--seeds", type=int, default=200)
    e.add_argument("--coarse-net", action="store_true")
    e.add_argument("--precision", type=int, default=64)
    e.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if a.cmd == "train":
        net, rec = train(n=a.n, pairs=a.pairs, epochs=a.epochs, lr=a.lr, seed=a.seed, log=log)
        save_weights(a.out, net, rec)
        log(json.dumps({k: v for k, v in rec.items() if k != "loss_history"}))
    else:
        summary, rows = evaluate(a.weights, n=a.n, seeds=a.seeds, precision=a.precision,
                                 coarse_net=a.coarse_net, log=log)
        log(json.dumps(summary))
        if a.out:
            json.dump({"summary": summary, "rows": rows}, open(a.out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
