"""Summaries of rocprofv3 output for the committed profiles.

`summarize_counters` turns the per-dispatch FETCH_SIZE / WRITE_SIZE CSVs of
two `rocprofv3 --pmc` runs of bench.py (run with --copy-calibration) into the
JSON that bench.py reads for `roofline.traffic`:
  * for each kernel, the counters of its largest dispatches (the finest level);
  * fetch/write scale factors from the plain 1 GiB device copy in the same run
    (bytes copied / counter reading), which absorb the counters' request-size
    accounting on this GPU.

Usage:
  python -m paper_2312_10615_amd.profiling FETCH.csv WRITE.csv out.json --n 256
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("geom.hpp", "kernels.hpp", "packed_kernels.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2312_10615_amd", "csrc", f), "rb").read())
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


SHORT = {"k_dgs_u_v<": "dgs_u", "k_dgs_pr<": "dgs_pr", "k_dgs_pf_own_v<": "dgs_pf_own", "k_dgs_pf_nbr_v<": "dgs_pf_nbr",
         "k_apply_v<1,": "apply", "k_restrict<": "restrict", "k_prolong_children<": "prolong"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("out")
    ap.add_argument("--n", type=int, default=256)
    a = ap.parse_args()
    d = summarize_counters(a.fetch_csv, a.write_csv, a.n)
    json.dump(d, open(a.out, "w"), indent=1)
    print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
