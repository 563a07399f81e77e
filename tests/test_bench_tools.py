"""The helpers bench.py uses to turn raw rocprofv3 output into the summaries under
profiles/ and to key measured figures to the device code, on synthetic files: the
mean per dispatch of each counter, the timed-region average of a kernel trace, and
the hash of the stage kernels' machine code."""
import csv
import os
import re

import pytest

import bench


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_pmc_means_per_dispatch_and_kernel(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(str(tmp_path / "host" / "1" / "p_counter_collection.csv"), hdr, [
        [1, "void k_stage<double, 1>(x)", "SQ_WAVES", 10],
        [2, "void k_stage<double, 1>(x)", "SQ_WAVES", 30],
        [1, "void k_stage<double, 1>(x)", "SQ_INSTS_VALU", 5],
        [3, "void k_alpha<double>(x)", "SQ_WAVES", 7],
    ])
    # a second process's file is merged in
    _write_csv(str(tmp_path / "host" / "2" / "p_counter_collection.csv"), hdr, [
        [4, "void k_stage<double, 1>(x)", "SQ_INSTS_VALU", 15],
    ])
    out = bench.summarize_pmc(str(tmp_path))
    lines = out.splitlines()
    assert lines[0] == "| kernel | dispatches | SQ_WAVES | SQ_INSTS_VALU |"
    row = [ln for ln in lines if ln.startswith("| void k_stage")][0].split("|")
    assert [c.strip() for c in row[2:5]] == ["2", "20", "10"]
    alpha = [ln for ln in lines if ln.startswith("| void k_alpha")][0].split("|")
    assert [c.strip() for c in alpha[2:5]] == ["1", "7", ""]
    only = bench.summarize_pmc(str(tmp_path), match="k_alpha")
    assert "k_stage" not in only and "k_alpha" in only


def test_summarize_trace_averages_the_last_matching_dispatches(tmp_path):
    d = tmp_path / "h" / "9"
    _write_csv(str(d / "t_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"],
               [["void k_stage<float, 1>(x)", 3, 600, 200.0, 95.5, 100, 300, 1.0]])
    hdr = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size",
           "Scratch_Size", "VGPR_Count", "Workgroup_Size_X", "Grid_Size_X"]
    recs = [  # written out of order: the summary sorts by start time
        ["K", "void k_stage<float, 3>(x)", 5000000, 5300000, 31744, 0, 48, 256, 4096],
        ["K", "void k_stage<float, 1>(x)", 1000000, 1100000, 31744, 0, 48, 256, 4096],
        ["K", "k_finish", 5400000, 5410000, 0, 0, 8, 64, 64],
        ["K", "void k_stage<float, 2>(x)", 3000000, 3200000, 31744, 12, 48, 256, 4096],
    ]
    _write_csv(str(d / "t_kernel_trace.csv"), hdr, recs)
    out = bench.summarize_trace(str(tmp_path), "k_stage<", last=2)
    assert "| void k_stage<float, 1>(x) | 3 | 200 | 100 | 300 | 95.50 |" in out
    m = re.search(r"average duration ([0-9.]+) ms \(min ([0-9.]+), max ([0-9.]+)\)", out)
    assert m and [float(x) for x in m.groups()] == [0.25, 0.2, 0.3]
    # the two last stage dispatches and the k_finish after them: 0.2 + 0.3 + 0.01 ms
    assert "all 3 dispatches from the first of them on: 0.5100 ms, over a span of 2.4100 ms" in out
    assert "grid 4096 work-items in workgroups of 256; LDS 31744 B" in out
    assert "scratch 12 B per lane" in out  # the first of the averaged dispatches
    # fewer matching dispatches than asked for: only the kernel_stats table
    assert "average duration" not in bench.summarize_trace(str(tmp_path), "k_stage<", last=9)


def test_kernel_sha_of_the_built_library_is_stable():
    from paper_2207_05258_amd import hweno as hw
    if not os.path.exists(hw.LIB_PATH):
        pytest.skip("libhweno.so not built")
    a = bench.kernel_sha()
    assert re.fullmatch(r"[0-9a-f]{16}", a), a
    assert bench.kernel_sha() == a
    # another kernel family hashes differently, an unknown prefix finds nothing
    assert bench.kernel_sha("_ZN5hweno9k_adjointI") not in (a, "unknown")
    assert bench.kernel_sha("_ZN5hweno_no_such_kernel") == "unknown"
    # the default key covers exactly the 2D Euler stage kernels of both precisions
    assert bench.kernel_sha(bench.STAGE_2D_EULER) == a
    assert bench.kernel_sha(bench.STAGE_2D_EULER[0]) not in (a, "unknown")
    assert bench.kernel_sha("_ZN5hweno7k_stageI") not in (a, "unknown")


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu_with_a_message(argv, env):
    """The path runs on one GPU: asked for more (by flag or by a launcher's WORLD_SIZE),
    bench.py exits with status 2 and says so before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py")] + argv, cwd=root,
                       env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, (r.returncode, r.stdout, r.stderr)
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")
