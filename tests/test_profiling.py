"""The measurement plumbing behind bench.py's roofline.traffic (CPU only):
the counter summary of two rocprofv3 --pmc runs, its key on the kernel code,
and the bytes per launch the bench derives from it."""
import csv
import json

from paper_2312_10615_amd import profiling


def _write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_code_hash_ignores_comments_and_blank_lines():
    src = {"geom.hpp": "int a;  // x\n\n// only a comment\nint b;\n",
           "kernels.hpp": "k();\n", "packed_kernels.hpp": "p();\n"}
    edited = dict(src, **{"geom.hpp": "int a;   // another comment\n// more\nint b;   \n\n"})
    changed = dict(src, **{"geom.hpp": "int a;\nint c;\n"})
    h = profiling.kernel_source_hash(src.__getitem__)
    assert profiling.kernel_source_hash(edited.__getitem__) == h
    assert profiling.kernel_source_hash(changed.__getitem__) != h
    assert profiling.code_lines("x = 1;  // c\n  \n// d\ny;") == "x = 1;\ny;"


def test_counter_summary_takes_the_largest_dispatches_and_the_copy_scale(tmp_path):
    kib = (1 << 30) / 1024.0
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # two finest-level dispatches (largest grid) and a coarse one per kernel; the copy's
    # counters read half (fetch) and all (write) of the 1 GiB it moves
    _write_csv(fetch, "FETCH_SIZE", [("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 4096, 100.0),
                                     ("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 4096, 300.0),
                                     ("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 64, 7.0),
                                     ("sg::k_dgs_u_v<float, float, 4>(Geom, ...)", 8192, 9.0),
                                     ("__amd_rocclr_copyBuffer", 1 << 20, kib / 2)])
    _write_csv(write, "WRITE_SIZE", [("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 4096, 50.0),
                                     ("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 4096, 70.0),
                                     ("sg::k_dgs_u_v<double, double, 2>(Geom, ...)", 64, 1.0),
                                     ("__amd_rocclr_copyBuffer", 1 << 20, kib)])
    d = profiling.summarize_counters(str(fetch), str(write), 256)
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    k = d["kernels"]["dgs_u"]  # the FP64 kernel only, its two largest dispatches averaged
    assert k["grid"] == 4096 and k["dispatches"] == 2
    assert k["fetch_kib"] == 200.0 and k["write_kib"] == 60.0
    assert d["kernel_source_hash"] == profiling.kernel_source_hash()


def test_bench_traffic_needs_the_current_kernel_code(tmp_path, monkeypatch):
    import bench
    summary = {"n": 256, "kernel_source_hash": profiling.kernel_source_hash(), "fetch_scale": 2.0,
               "write_scale": 1.0, "kernels": {"dgs_u": {"grid": 1, "fetch_kib": 10.0, "write_kib": 4.0,
                                                         "dispatches": 1}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "counters_fp64_256.json").write_text(json.dumps(summary))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("dgs_u", 256) == (10.0 * 2.0 + 4.0) * 1024
    assert bench.counter_traffic("dgs_u", 128) is None       # another workload
    assert bench.counter_traffic("restrict", 256) is None    # not summarised
    summary["kernel_source_hash"] = "0" * 16                  # taken on other kernel code
    (prof / "counters_fp64_256.json").write_text(json.dumps(summary))
    assert bench.counter_traffic("dgs_u", 256) is None
