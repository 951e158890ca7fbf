"""CPU tests of the rocprofv3 summariser (synthetic profiler CSVs): the copy
calibration factors, per-launch-shape trace averages and the JSON block that
bench.py reads."""
import csv
import json
import re

from paper_1807_08271_amd import profsum

K0 = "void rgbid::(anonymous namespace)::k_reduce<false, 0, true>(rgbid::IterLaunch)"
K2 = "void rgbid::(anonymous namespace)::k_warp<false, 2>(rgbid::IterLaunch)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summary_tables_and_json(tmp_path):
    d = tmp_path
    _write(d / "stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [[K0, 3, 300000, 100000], [K2, 1, 50000, 50000]])
    # two whole-batch launches (140 and 138 us) and one small one of the same kernel
    _write(d / "trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X",
                             "Grid_Size_Y", "Grid_Size_Z"],
           [[K0, 1000, 141000, 1228800, 1, 1], [K0, 200000, 338000, 1228800, 1, 1],
            [K0, 400000, 420000, 38400, 1, 1], [K2, 500000, 550000, 1228800, 1, 1]])
    _write(d / "pmc1.csv", ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
           [[K0, 1228800, "FETCH_SIZE", 1000.0], [K0, 1228800, "FETCH_SIZE", 1200.0],
            [K0, 38400, "FETCH_SIZE", 10.0], [K2, 1228800, "FETCH_SIZE", 500.0]])
    _write(d / "pmc2.csv", ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
           [[K0, 1228800, "WRITE_SIZE", 40.0], [K2, 1228800, "WRITE_SIZE", 8.0]])
    # a 1 MiB copy reading 512 KiB of FETCH_SIZE and 1024 KiB of WRITE_SIZE
    _write(d / "cpy1.csv", ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
           [[COPY, 4096, "FETCH_SIZE", 512.0]])
    _write(d / "cpy2.csv", ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
           [[COPY, 4096, "WRITE_SIZE", 1024.0]])
    out = d / "o.md"
    profsum.main(["--stats", str(d / "stats.csv"), "--trace", str(d / "trace.csv"),
                  "--pmc", str(d / "pmc1.csv"), str(d / "pmc2.csv"),
                  "--copy", str(d / "cpy1.csv"), str(d / "cpy2.csv"),
                  "--copy-bytes", str(1 << 20), "--cmd", "cmd", "--workload", "w",
                  "--out", str(out)])
    text = out.read_text()
    blob = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    assert blob["fetch_factor"] == 2.0 and blob["write_factor"] == 1.0
    r0 = blob["kernels"]["reduce_l0"]
    # the largest dispatch of the kernel is kept; counters averaged over its dispatches
    assert r0["grid"] == 1228800
    assert r0["fetch_kib"] == 1100.0 and r0["write_kib"] == 40.0
    assert r0["hbm_bytes_per_launch"] == round((1100.0 * 2.0 + 40.0) * 1024.0)
    # trace average of the whole-batch launches only (140 and 138 us)
    assert r0["trace_avg_us"] == 139.0 and r0["trace_calls"] == 2
    assert blob["kernels"]["warp_l2"]["trace_avg_us"] == 50.0
    assert "| k_reduce | false, 0, true | 38400 | 1 | 20.00 |" in text


def test_kernel_key_levels():
    assert profsum.kernel_key(K0) == ("reduce", 0, "false, 0, true")
    assert profsum.kernel_key(K2) == ("warp", 2, "false, 2")
    assert profsum.kernel_key("void rgbid::(anonymous namespace)::k_scale<19>(rgbid::IterLaunch)") \
        == ("scale", None, "19")
