"""Host-side helpers of bench.py (no GPU): the union of kernel intervals, the
phase split of a batching/serving kernel trace, and the keys under which
counter results are stored."""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_union_ms():
    assert bench._union_ms([]) == 0
    # [0,10) and [5,20) overlap, [30,40) is apart: 20 + 10 ns
    assert bench._union_ms([(30, 40), (0, 10), (5, 20)]) == 30 / 1e6
    assert bench._union_ms([(0, 100), (10, 20), (20, 30)]) == 100 / 1e6


def test_config_key():
    assert bench._config_key(125, 8) == "delta=125,local_iters=8,split=0"
    assert bench._config_key(125, 8, None, 0, True) == "delta=125,local_iters=8,split=0,defer=1"
    assert bench._config_key(50, 4, "weight", 256) == "delta=50,local_iters=4,split=weight,grid=256"


def _trace(tmp_path, rows):
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    return path


def test_busy_summary_serving_phases(tmp_path):
    """Tuning and warm-up solves, then the sequential solves (the last `queries` pass resets before the
    first server), then one phase per rate, each starting at the server's pass reset and slot-id fill."""
    rows, t = [], 0

    def k(name, d):
        nonlocal t
        rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + d})
        t += d

    def solve():
        nonlocal t
        k("void stn::k_pass_reset(stn::VorParams)", 10)
        for _ in range(3):
            k("void stn::k_round<false>(stn::VorParams)", 100)
        t += 50  # host gap

    for _ in range(4):
        solve()  # tuning / warm-up
    for _ in range(2):
        solve()  # sequential, 2 queries: 2 * 310 ns of kernels in a 720 ns span
    for _ in range(2):  # two rates
        k("void stn::k_pass_reset(stn::VorParams)", 10)
        k("void (anonymous namespace)::k_iota(unsigned int*, unsigned int)", 10)
        for _ in range(4):
            k("void stn::k_round<false>(stn::VorParams)", 100)
        t += 1000
    line = {"value": 1.0, "unit": "queries/s", "config": {"workload": "w", "queries": 2},
            "sequential_queries_per_s": 1.0, "serving": {"rho": {"1.5": {}, "inf": {}}}}
    js = tmp_path / "line.json"
    js.write_text(json.dumps(line) + "\n")
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--busy-summary",
                          str(_trace(tmp_path, rows)), str(js)], capture_output=True, text=True, check=True).stdout
    table = [l for l in out.splitlines() if l.startswith("| ") and not l.startswith("| phase")]
    assert [l.split(" | ")[0] for l in table] == ["| sequential solves", "| server, rho = 1.5", "| server, rho = inf"]
    seq = table[0].split(" | ")
    assert seq[1] == "2" and seq[8] == "6"  # queries, k_round launches
    assert seq[5] == "92.5%"  # 620 ns of kernels in the 670 ns from the first start to the last end
    srv = table[1].split(" | ")
    assert srv[8] == "4" and srv[5] == "100.0%"  # back-to-back kernels: fully busy
