"""Summaries of rocprofv3 output for the committed profiles.

`summarize_counters` turns the per-dispatch FETCH_SIZE / WRITE_SIZE CSVs of
two `rocprofv3 --pmc` runs of bench.py (run with --copy-calibration) into the
JSON that bench.py reads for `roofline.traffic`:
  * for each kernel, the counters of its largest dispatches (the finest level);
  * fetch/write scale factors from the plain 1 GiB device copy in the same run
    (bytes copied / counter reading), which absorb the counters' request-size
    accounting on this GPU.

`level_times` times one V-cycle per level and kernel class with the
library's own event timing (diagnostics; needs a GPU).

Usage:
  python -m paper_2312_10615_amd.profiling counters FETCH.csv WRITE.csv out.json --n 256
  python -m paper_2312_10615_amd.profiling levels --n 256 --precision 64
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def code_lines(text):
    """Source text without // comments, trailing blanks and empty lines: what
    the counters depend on."""
    out = []
    for line in text.splitlines():
        i = line.find("//")
        if i >= 0:
            line = line[:i]
        line = line.rstrip()
        if line:
            out.append(line)
    return "\n".join(out)


def kernel_source_hash(read=None):
    """Hash of the level-0 kernels' code (comments excluded); `read(name)`
    returns a source file's text (default: the files in this tree)."""
    if read is None:
        def read(f):
            return open(os.path.join(ROOT, "paper_2312_10615_amd", "csrc", f)).read()
    h = hashlib.sha256()
    for f in ("geom.hpp", "kernels.hpp", "packed_kernels.hpp"):
        h.update(code_lines(read(f)).encode())
    return h.hexdigest()[:16]


def _largest_dispatches(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    best = {}
    for r in rows:
        name = r["Kernel_Name"]
        grid = int(r["Grid_Size"])
        val = float(r["Counter_Value"])
        cur = best.get(name)
        if cur is None or grid > cur[0]:
            best[name] = (grid, [val])
        elif grid == cur[0]:
            cur[1].append(val)
    return best


SHORT = {"k_dgs_u_v<": "dgs_u", "k_dgs_pr_v<": "dgs_pr", "k_dgs_pf_v<": "dgs_pf",
         "k_apply_v<1,": "apply", "k_restrict<": "restrict", "k_prolong_pairs<": "prolong",
         "k_resid_restrict_xy<": "resid_restrict_xy", "k_restrict_z<": "restrict_z",
         "k_vanka_delta8_xs<": "vanka_delta8_xs", "k_vanka_apply_xs<": "vanka_apply_xs",
         "k_xslab_copy<": "xslab_copy", "k_vanka_pp8<": "vanka_pp8"}


def summarize_counters(fetch_csv, write_csv, n, copy_bytes=1 << 30):
    f = _largest_dispatches(fetch_csv, "FETCH_SIZE")
    w = _largest_dispatches(write_csv, "WRITE_SIZE")
    # the calibration copy is the dispatch whose WRITE_SIZE equals the copied bytes
    copy_kib = copy_bytes / 1024.0
    fetch_scale = write_scale = None
    for name, (grid, vals) in w.items():
        if ("copy" in name.lower()) and abs(max(vals) - copy_kib) / copy_kib < 0.01:
            write_scale = copy_kib / max(vals)
            if name in f:
                fetch_scale = copy_kib / max(f[name][1])
    out = {"n": n, "kernel_source_hash": kernel_source_hash(), "fetch_scale": fetch_scale, "write_scale": write_scale,
           "kernels": {}}
    for name, (grid, vals) in f.items():
        for key, short in SHORT.items():
            if key in name and "double" in name:
                wv = w.get(name, (0, [0.0]))[1]
                out["kernels"][short] = {"grid": grid, "fetch_kib": sum(vals) / len(vals),
                                         "write_kib": sum(wv) / len(wv), "dispatches": len(vals)}
    return out


def level_times(n, precision, vcycles=3):
    """Per level and kernel class of one V-cycle at n^3 (sinusoid forcing, seed 0):
    (milliseconds, launches), from the library's own event timing (which adds
    about 2 us per launch), plus the graph-replayed V-cycle time in ms."""
    import numpy as np
    import torch

    from paper_2312_10615_amd.stokes import KC, StokesSolver
    from paper_2312_10615_amd.workloads import sinusoid_forcing
    sol = StokesSolver(n, n, n, precision=precision)
    f = sinusoid_forcing(n, n, n, 1.0 / n, seed=0)
    b = sol.pack((f[0], f[1], f[2], np.zeros((n, n, n))))
    t = sol.new_state()
    rows = []
    for lv in range(sol.layout.levels):
        sol.profile("all", lv)
        for _ in range(vcycles):
            sol.vcycle(b, out=t)
        parts = {}
        for name in KC:
            ms, cnt = sol.profile_read(name, lv)
            if cnt:
                parts[name] = (ms / vcycles, cnt // vcycles)
        rows.append(parts)
    sol.profile("off")
    sol.vcycle(b, out=t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        sol.vcycle(b, out=t)
    e1.record()
    torch.cuda.synchronize()
    return rows, e0.elapsed_time(e1) / 5


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd")
    c = sub.add_parser("counters", help="summarise FETCH_SIZE / WRITE_SIZE runs")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("out")
    c.add_argument("--n", type=int, default=256)
    lv = sub.add_parser("levels", help="time one V-cycle per level and kernel class (GPU)")
    lv.add_argument("--n", type=int, default=256)
    lv.add_argument("--precision", type=int, default=64, choices=(32, 64))
    a = ap.parse_args()
    if a.cmd == "levels":
        rows, vc_ms = level_times(a.n, a.precision)
        for i, parts in enumerate(rows):
            tot = sum(ms for ms, _ in parts.values())
            print(f"FP{a.precision} level {i}: {tot:.3f} ms  " +
                  " ".join(f"{k}={ms:.3f}ms/{cnt}" for k, (ms, cnt) in parts.items()), flush=True)
        print(f"FP{a.precision} V-cycle replayed from its graph: {vc_ms:.3f} ms", flush=True)
        return
    if a.cmd != "counters":
        ap.error("choose a subcommand: counters or levels")
    d = summarize_counters(a.fetch_csv, a.write_csv, a.n)
    json.dump(d, open(a.out, "w"), indent=1)
    print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
