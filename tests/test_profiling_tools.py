"""Host logic of the profiling helpers: counter CSVs (the rocprofv3 --pmc layout) to per-kernel
figures.  Synthetic CSVs with known values; no GPU."""
import csv

import pytest

from paper_1906_07925_amd import profsum, traffic

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for k, (name, counter, value) in enumerate(rows):
            w.writerow({"Correlation_Id": k, "Dispatch_Id": k, "Agent_Id": "Agent 1", "Queue_Id": 1, "Process_Id": 1,
                        "Thread_Id": 1, "Grid_Size": 1024, "Kernel_Id": 1, "Kernel_Name": name, "Workgroup_Size": 256,
                        "LDS_Block_Size": 0, "Scratch_Size": 0, "VGPR_Count": 64, "Accum_VGPR_Count": 0,
                        "SGPR_Count": 80, "Counter_Name": counter, "Counter_Value": value, "Start_Timestamp": 0,
                        "End_Timestamp": 1000})


def test_valu_rows(tmp_path):
    p = tmp_path / "valu.csv"
    k = "void (anonymous namespace)::pass_density_force<3, 4, false, false>(int)"
    rows = []
    for v in (1.0e9, 3.0e9):   # two launches: averages 2e9 instructions
        rows += [(k, "SQ_INSTS_VALU", v), (k, "SQ_ACTIVE_INST_VALU", v), (k, "SQ_THREAD_CYCLES_VALU", 32.0 * v)]
    write_csv(p, rows)
    (name, n, avg, util, floor_ms), = profsum.valu_rows(str(p))
    assert name == "pass_density_force<3, 4, false, false>" and n == 2
    assert avg["SQ_INSTS_VALU"] == pytest.approx(2.0e9)
    assert util == pytest.approx(0.5)                                  # 32 of 64 lanes
    assert floor_ms == pytest.approx(2.0e9 * 4 / 1024 / 2.4e6)        # 4 cycles a wave64 instruction


def test_step_table(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    mib = 512
    copy = "__amd_rocclr_copyBuffer"
    kern = "void (anonymous namespace)::pass_viscous_integrate<3, 4, false>(int)"
    # FETCH_SIZE counts half of what is read (KiB): the copy of 512 MiB reads as 256 MiB
    write_csv(fetch, [(copy, "FETCH_SIZE", mib * 1024 / 2), (kern, "FETCH_SIZE", 1000.0), (kern, "FETCH_SIZE", 3000.0)])
    write_csv(write, [(copy, "WRITE_SIZE", mib * 1024), (kern, "WRITE_SIZE", 500.0), (kern, "WRITE_SIZE", 500.0)])
    md = traffic.step_table(str(fetch), str(write), mib, 2, "t", "c", "n")
    assert "fetch scale 2.0000, write scale 1.0000" in md
    # read: 2 x (1000 + 3000) KiB over 2 steps; written: 1000 KiB over 2 steps
    row = [line for line in md.splitlines() if line.startswith("| pass_viscous_integrate")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1] == "2"
    assert float(cells[2]) == pytest.approx(2 * 4000 * 1024 / 2 / 1e6, abs=0.05)
    assert float(cells[3]) == pytest.approx(1000 * 1024 / 2 / 1e6, abs=0.05)


def test_kernel_source_digest_ignores_comments(tmp_path, monkeypatch):
    """The digest that ties committed counters to the kernels follows the code only."""
    import bench
    src = tmp_path / "k.hip"
    src.write_text("// header\nint f(int x) {  // trailing\n  return x + 1;\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    d0 = bench.kernel_source_digest()
    src.write_text("// another header\n\nint f(int x) {\n  // note\n  return x + 1;   \n}\n")
    assert bench.kernel_source_digest() == d0
    src.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_digest() != d0


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 ends at once with exit status 2 and a JSON
    message, before anything is loaded."""
    import json
    import subprocess
    import sys
    root = __import__("os").path.dirname(__import__("os").path.dirname(__file__))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
    r = subprocess.run([sys.executable, "bench.py", "--leg", "sort"], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr
