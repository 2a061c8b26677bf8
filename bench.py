"""Benchmark of the Steiner-tree hot path on one MI355X.

One step = one complete steiner_solve (Alg. 2 Steps 1-7: seed set-up, Voronoi
relaxation, pred + boundary scan, G'1 compaction, MST, pruning and
expansion, sorted edge list and D) on a graph already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

The default workload is rmat25: R-MAT scale 25, edge factor 16 (1.05 G CSR
entries after deduplication), weights U[1,1000], 10,000 seeds from the giant
component -- the largest single-GPU configuration, at the paper's largest
seed count.  Prints one JSON line.  value = GTEPS of the whole step:
undirected edges of the seeds' components divided by the mean step time
(gteps_voronoi divides by the Voronoi phase alone).  The roofline object is
for the dominant kernel (the relaxation kernel), from HIP events around each
of its launches on the graph's stream; `traffic` comes from the committed
rocprofv3 counter summary when it matches the current kernel source and the
tuned relaxation options.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS + Steiner queries/s at 1 GPU (bit-exact vs oracle); p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# inputs up to this many CSR entries get whole oracle solves in the CPU baseline; larger ones its Step 1
FULL_ORACLE_NNZ = 64 << 20
KERNEL_SRC = [os.path.join(ROOT, "paper_2205_14503_amd", "csrc", f)
              for f in ("kernels.hip", "kernels.h", "common.h", "engine.cpp", "pass.cpp")]


def algorithmic_bytes(n: int, nnz_reached: int, nnz: int):
    """Bytes a work-efficient pass must move: every (col, w) entry once (8 B),
    the row offsets once (8 B each, counted as 64-bit whatever the device
    layout), the key written at set-up and read at the end (16 B per vertex),
    and for the scan the key streamed and gathered once plus pred written
    (20 B per vertex)."""
    b_vor = 8 * nnz_reached + 8 * (n + 1) + 16 * n
    b_scan = 8 * nnz + 8 * (n + 1) + 20 * n
    return b_vor, b_scan


def copy_calibration(torch, mib: int = 1024, reps: int = 3):
    """A plain device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters to bytes."""
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": mib << 20, "bytes_written": mib << 20, "reps": reps}}),
          flush=True)


def gather_probe(torch, n: int, m: int = 1 << 26, reps: int = 5) -> float:
    """Random 8-byte gathers per second of a plain torch index_select from an n-entry int64 array (the size of
    one query's key array) at m uniformly random positions."""
    x = torch.arange(n, dtype=torch.int64, device="cuda")
    idx = torch.randint(0, n, (m,), dtype=torch.int64, device="cuda")
    out = torch.empty(m, dtype=torch.int64, device="cuda")
    torch.index_select(x, 0, idx, out=out)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.index_select(x, 0, idx, out=out)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del x, idx, out
    return m / best


def kernel_sha() -> str:
    """Hash of the sources that decide what the relaxation kernel does."""
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _pmc_per_kernel(path: str):
    """Mean counter value (KiB) per dispatch, by kernel, from a rocprofv3
    counter_collection.csv."""
    import csv
    acc = {}
    for row in csv.DictReader(open(path)):
        name = row["Kernel_Name"].split("(")[0]
        name = name.split("::")[-1].split("<")[0] if "stn::" in name else name
        acc.setdefault(name, []).append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def pmc_table(args):
    """Mean value per dispatch of every counter in rocprofv3 --pmc counter_collection.csv files, for the
    relaxation and scan kernels, with the L2 hit rate and the share of wave time spent waiting where the
    counters for them are present."""
    import csv
    acc = {}
    for path in args.pmc_table:
        for row in csv.DictReader(open(path)):
            name = _trace_name(row["Kernel_Name"])
            acc.setdefault(name, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    kernels = [k for k in ("stn::k_round", "stn::k_scan") if k in acc]
    counters = sorted({c for k in kernels for c in acc[k]})
    print("| kernel | dispatches | " + " | ".join(counters) + " | L2 hit rate | waiting share of wave cycles |")
    print("|---|---|" + "---|" * (len(counters) + 2))
    for k in kernels:
        m = {c: sum(v) / len(v) for c, v in acc[k].items()}
        hit = m.get("TCC_HIT_sum"), m.get("TCC_MISS_sum")
        rate = f"{hit[0] / (hit[0] + hit[1]):.3f}" if None not in hit and hit[0] + hit[1] else ""
        wait = m.get("SQ_WAIT_INST_ANY"), m.get("SQ_WAVE_CYCLES")
        share = f"{wait[0] / wait[1]:.3f}" if None not in wait and wait[1] else ""
        n = max(len(v) for v in acc[k].values())
        print(f"| {k} | {n} | " + " | ".join(f"{m.get(c, 0):.4g}" for c in counters) + f" | {rate} | {share} |")


def _config_key(delta, local, split=None, grid=0, defer=False) -> str:
    key = f"delta={int(delta)},local_iters={int(local)},split={split or 0}"
    return key + (f",grid={int(grid)}" if grid else "") + (",defer=1" if defer else "")


def pmc_summary(args):
    """Entry of profiles/traffic.json (workload -> relaxation options -> bytes)
    and a text table, from two counter runs of bench.py (FETCH_SIZE,
    WRITE_SIZE) and two of the copy calibration."""
    fetch, write, cfetch, cwrite = args.pmc_summary
    copy_kib = 1 << 20  # the calibration copies 1 GiB
    f_scale = copy_kib / _pmc_per_kernel(cfetch)["__amd_rocclr_copyBuffer"][0]
    w_scale = copy_kib / _pmc_per_kernel(cwrite)["__amd_rocclr_copyBuffer"][0]
    fk, wk = _pmc_per_kernel(fetch), _pmc_per_kernel(write)
    entry = {"kernel_sha": kernel_sha(), "kernel": "k_round", "fetch_scale": round(f_scale, 4),
             "write_scale": round(w_scale, 4), "per_kernel": {}}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM MB/dispatch (scaled) |",
             "|---|---|---|---|---|"]
    for name in sorted(fk, key=lambda x: -fk[x][0] * fk[x][1]):
        fv, cnt = fk[name]
        wv = wk.get(name, (0.0, 0))[0]
        mb = (fv * f_scale + wv * w_scale) * 1024 / 1e6
        entry["per_kernel"][name] = {"dispatches": cnt, "fetch_kib": round(fv, 3), "write_kib": round(wv, 3),
                                     "bytes": round(mb * 1e6)}
        if cnt and mb > 0.01:
            lines.append(f"| {name} | {cnt} | {fv:.1f} | {wv:.1f} | {mb:.3f} |")
    entry["bytes_per_launch"] = entry["per_kernel"]["k_round"]["bytes"]
    data = json.load(open(TRAFFIC_FILE)) if os.path.exists(TRAFFIC_FILE) else {}
    data.setdefault(args.workload, {})[_config_key(args.delta, args.local, args.split, args.grid,
                                                    args.defer == "on")] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(f"Copy calibration: a 1 GiB device copy reads {copy_kib / f_scale:.1f} KiB of FETCH_SIZE "
          f"(scale x{f_scale:.4f}) and writes {copy_kib / w_scale:.1f} KiB of WRITE_SIZE (scale x{w_scale:.4f}).\n")
    print("\n".join(lines))


def _trace_name(raw: str) -> str:
    """A kernel's demangled name without return type, template arguments and
    parameters ("void stn::k_round<true>(stn::VorParams)" -> "stn::k_round")."""
    name = raw.split("(")[0]
    if name.startswith("void "):
        name = name[5:]
    return name.split("<")[0]


def trace_summary(args):
    """Per-kernel durations over the timed region of one bench.py run under
    rocprofv3 --kernel-trace (its JSON line gives steps and relaxation
    launches per step; the region starts at the first of the last
    steps x launches relaxation dispatches)."""
    import csv
    trace_csv, json_file = args.trace_summary
    line = json.loads([x for x in open(json_file) if x.startswith("{")][-1])
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    nk = int(round(line["steps"] * line["roofline"]["launches_per_step"]))
    kr = [i for i, r in enumerate(rows) if _trace_name(r["Kernel_Name"]) == "stn::k_round"]
    first = kr[-nk]
    acc = {}
    for r in rows[first:]:
        name = _trace_name(r["Kernel_Name"])
        acc.setdefault(name, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in acc.values())
    print(f"Timed region: {line['steps']} steps of {line['config']['workload']}, "
          f"{line['ms_per_step']} ms per step, value {line['value']} {line['unit']}.\n")
    print("| kernel | calls | avg us | total ms per step | share of GPU time |\n|---|---|---|---|---|")
    for name, v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        print(f"| {name} | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / line['steps'] / 1e3:.4f} | "
              f"{100 * sum(v) / total:.2f}% |")
    rf = line["roofline"]
    ka = acc["stn::k_round"]
    print(f"\nk_round: rocprofv3 average {sum(ka) / len(ka):.2f} us per launch; bench.py HIP-event average "
          f"{rf['avg_launch_us']} us per launch (event pairs around chunks of launches, gaps included).")


def _union_ms(iv):
    """Length of the union of [start, end) nanosecond intervals, in ms."""
    tot, cur_s, cur_e = 0, None, None
    for a, b in sorted(iv):
        if cur_e is None or a > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot / 1e6


def busy_summary(args):
    """GPU-busy time of a batching or serving run under rocprofv3
    --kernel-trace, phase by phase.  Phases are found from marker kernels:
    every solve and every batch starts with one pass reset, and a server
    starts with a pass reset followed by its slot-id fill (k_iota).  Serving
    runs: the sequential phase is the last `queries` solves before the first
    server; then one phase per offered rate.  Batch runs: the last `steps`
    batches, then the sequential solves of the same queries."""
    import csv
    trace_csv, json_file = args.busy_summary
    line = json.loads([x for x in open(json_file) if x.startswith("{")][-1])
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    ts = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    names = [_trace_name(r["Kernel_Name"]) for r in rows]
    resets = [i for i, nm in enumerate(names) if nm == "stn::k_pass_reset"]
    phases = []  # (label, queries, first row, end row)
    if "serving" in line:
        nq = line["config"]["queries"]
        iotas = [i for i, r in enumerate(rows) if "k_iota(" in r["Kernel_Name"]]
        srv = [max(j for j in resets if j < i) for i in iotas]
        seq = [j for j in resets if j < srv[0]][-nq:]
        phases.append(("sequential solves", nq, seq[0], srv[0]))
        for p, (label, _) in enumerate(line["serving"]["rho"].items()):
            phases.append((f"server, rho = {label}", nq, srv[p], srv[p + 1] if p + 1 < len(srv) else len(rows)))
    else:
        q, steps = line["config"]["queries"], line["steps"]
        phases.append((f"batched pass ({steps} batches)", q * steps, resets[-q - steps], resets[-q]))
        phases.append(("sequential solves", q, resets[-q], len(rows)))
    print(f"Workload {line['config']['workload']}: {line['value']} {line['unit']} "
          f"({'served' if 'serving' in line else 'batched'}), "
          f"sequential {line['sequential_queries_per_s']} queries/s.\n")
    print("| phase | queries | span ms | kernel ms | GPU busy ms | busy | kernel ms per query | "
          "span ms per query | k_round launches | k_round avg us |\n|---|---|---|---|---|---|---|---|---|---|")
    for label, nq, a, b in phases:
        iv = ts[a:b]
        span = (max(e for _, e in iv) - iv[0][0]) / 1e6
        kern = sum(e - s for s, e in iv) / 1e6
        busy = _union_ms(iv)
        kr = [e - s for (s, e), nm in zip(iv, names[a:b]) if nm == "stn::k_round"]
        print(f"| {label} | {nq} | {span:.1f} | {kern:.1f} | {busy:.1f} | {100 * busy / span:.1f}% | "
              f"{kern / nq:.2f} | {span / nq:.2f} | {len(kr)} | {sum(kr) / max(len(kr), 1) / 1e3:.1f} |")


def bench_sweep(args, st, W, np, torch, stream):
    """The paper's sensitivity studies on one GPU (RMAT scale `--sweep-scale`,
    edge factor 16): bucket width from Dijkstra-like to unbounded (its
    priority-queue vs FIFO study), weight ranges [1,100]..[1,100K], seed
    counts 10..10K and the seed-selection strategies.  Relaxation attempts
    stand in for the paper's message counts.  Prints a markdown table."""
    flags = st.FLAG_TIMING | st.FLAG_COUNTERS
    scale = args.sweep_scale
    rows = []

    def measure(dg, seeds, opts, **tags):
        o = dict(opts, flags=flags | opts.get("flags", 0))
        dg.solve(seeds, o)
        ts, last = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            last = dg.solve(seeds, o)
            ts.append((time.perf_counter() - t0) * 1e3)
        x = last.stats
        row = dict(tags, ms=round(float(np.median(ts)), 3), voronoi_ms=round(x["ms_voronoi"], 3),
                   scan_ms=round(x["ms_scan"], 3), rounds=x["rounds"], messages=x["relax_attempts"],
                   atomics=x["relax_atomics"], improved=x["relax_improved"], tree_edges=len(last.a), D=last.total)
        rows.append(row)
        print(f"[sweep] {row}", file=sys.stderr, flush=True)

    def graph(whi):
        g = W.rmat(scale, 16, wlo=1, whi=whi)
        return g, W.lcc(g)

    g, cand = graph(1000)
    dg = st.Graph(g, 0, stream)
    seeds = W.sample(cand, 1000, 1, W.STREAM_SEEDS)
    for delta in (1, 16, 128, 500, 2000, 8000, 0xFFFFFFFF):
        for defer in ("off", "on"):  # large rows expanded in the next round / at the bucket's advance
            measure(dg, seeds, {"delta": delta, "flags": st.FLAG_DEFER if defer == "on" else st.FLAG_NO_DEFER},
                    study="bucket width", weights="[1,1000]", k=1000,
                    delta="unbounded" if delta == 0xFFFFFFFF else delta, defer=defer)
    for k in (10, 100, 1000, 10000):
        s = W.sample(cand, k, 1, W.STREAM_SEEDS)
        tuned = dg.tune(s)
        measure(dg, s, {}, study="seed count", weights="[1,1000]", k=k,
                delta="unbounded (tuned)" if tuned["delta"] == 0xFFFFFFFF else f"{tuned['delta']} (tuned)")
    for strat in W.SEED_STRATEGIES:
        s = W.make_seeds(g, 100, cand=cand, strategy=strat)
        measure(dg, s, {}, study="seed strategy", weights="[1,1000]", k=100, strategy=strat)
    dg.close()
    for whi in (100, 10000, 100000):
        g, cand = graph(whi)
        dg = st.Graph(g, 0, stream)
        s = W.sample(cand, 1000, 1, W.STREAM_SEEDS)
        for delta in (0xFFFFFFFF, max(1, whi // 2)):
            measure(dg, s, {"delta": delta}, study="weight range", weights=f"[1,{whi}]", k=1000,
                    delta="unbounded" if delta == 0xFFFFFFFF else delta)
        dg.close()
    cols = ["study", "weights", "k", "delta", "defer", "strategy", "ms", "voronoi_ms", "scan_ms", "rounds", "messages",
            "atomics", "improved", "tree_edges", "D"]
    print(f"RMAT scale {scale}, edge factor 16 ({g.n} vertices), one MI355X; messages = relaxation attempts.\n")
    print("| " + " | ".join(cols) + " |\n|" + "---|" * len(cols))
    for r in rows:
        print("| " + " | ".join(str(r.get(c, "")) for c in cols) + " |")


def bench_batch(args, st, W, np, torch, stream):
    """Batched multi-query pass vs one-at-a-time solves (same graph, same queries)."""
    spec = W.WORKLOADS[args.workload]
    g = W.make_graph(args.workload)
    cand = W.lcc(g)
    sets = W.make_query_set(g, spec["queries"], spec["k_lo"], spec["k_hi"], cand=cand)
    dg = st.Graph(g, 0, stream)
    if not args.no_tune:
        dg.tune(sets[len(sets) // 2])
    bopts = {"driver": args.driver} if args.driver else None
    for _ in range(args.warmup):
        dg.solve_batch(sets, bopts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch = dg.solve_batch(sets, bopts)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    single = [dg.solve(s, bopts) for s in sets]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    assert all(code == st.OK and tr.edges == sg.edges for (code, tr), sg in zip(batch, single)), \
        "batched results differ from single solves"
    q = len(sets)
    return {
        "metric": METRIC, "value": round(q / t_batch, 3), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz, "queries": q,
                   "k": [int(len(s)) for s in sets], "seed": 1},
        "sequential_queries_per_s": round(q / t_seq, 3), "batch_speedup": round(t_seq / t_batch, 3),
    }


def bench_serve(args, st, W, np, torch, stream):
    """Poisson arrivals into the continuous-batching server at rho x the
    sequential rate (rho = inf: every request submitted at once, which
    measures the server's capacity).  The sequential rate is measured on the
    same requests solved one at a time, and every served tree must equal the
    same request's solve alone."""
    import threading
    spec = W.WORKLOADS[args.workload]
    g = W.make_graph(args.workload)
    cand = W.lcc(g)
    nq = args.queries
    sets = W.make_query_set(g, nq, spec["k_lo"], spec["k_hi"], cand=cand)
    dg = st.Graph(g, 0, stream)
    if not args.no_tune:
        dg.tune(sets[0])
    sopts = {"driver": args.driver} if args.driver else None
    for s in sets[:3]:
        dg.solve(s, sopts)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = [dg.solve(s, sopts).edges for s in sets]
    mu = nq / (time.perf_counter() - t0)
    print(f"[bench] serve: {nq} requests one at a time: {mu:.2f} queries/s", file=sys.stderr, flush=True)
    budget = args.budget_gb << 30
    out = {"rho": {}}
    for rho_s in args.rhos.split(","):
        rho = float(rho_s)
        rate = rho * mu
        arrivals = W.poisson_arrivals(nq, rate, master=7) if rho != float("inf") else np.zeros(nq)
        srv = st.steiner_server_create(dg.handle, budget, args.slots, sopts)
        mem = st.steiner_server_memory(srv)
        tickets = [None] * nq
        lat = [0.0] * nq
        done = [None] * nq
        start = time.perf_counter()

        def waiter():
            for q in range(nq):
                while tickets[q] is None:
                    time.sleep(0.0002)
                tr = st.steiner_server_wait(srv, tickets[q])
                lat[q] = tr.stats["ms_total"]
                done[q] = tr
                if (q + 1) % 100 == 0:
                    print(f"[bench] serve rho={rho_s}: {q + 1} of {nq} done after {time.perf_counter() - start:.1f} s",
                          file=sys.stderr, flush=True)

        th = threading.Thread(target=waiter)
        th.start()
        for q in range(nq):
            delay = start + arrivals[q] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[q] = st.steiner_server_submit(srv, sets[q])
        th.join()
        wall = time.perf_counter() - start
        st.steiner_server_destroy(srv)
        for q in range(nq):
            assert done[q].edges == ref[q], f"served result {q} differs from the result alone"
        key = "inf" if rho == float("inf") else str(rho)
        out["rho"][key] = {"offered_qps": None if rho == float("inf") else round(rate, 2),
                           "queries_per_s": round(nq / wall, 2),
                           "p50_ms": round(float(np.percentile(lat, 50)), 3),
                           "p99_ms": round(float(np.percentile(lat, 99)), 3),
                           "slots": mem["slots"]}
        print(f"[bench] serve rho={key}: {out['rho'][key]}", file=sys.stderr, flush=True)
    best = max(v["queries_per_s"] for v in out["rho"].values())
    mid = out["rho"].get("0.9") or next(iter(out["rho"].values()))
    return {
        "metric": METRIC, "value": best, "unit": "queries/s", "n_gpus": 1, "steps": nq, "warmup": 0,
        "ms_per_step": round(1e3 / best, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz, "queries": nq, "slots": args.slots,
                   "budget_gb": args.budget_gb, "seed": 1, "k_range": [spec["k_lo"], spec["k_hi"]]},
        "sequential_queries_per_s": round(mu, 3), "served_over_sequential": round(best / mu, 3),
        "serving": out, "p50_ms": mid["p50_ms"], "p99_ms": mid["p99_ms"],
        "parity": f"all {nq} served trees equal the same requests solved alone, at every rate",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat25")
    ap.add_argument("--driver", type=int, default=0)
    ap.add_argument("--delta", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--queries", type=int, default=1000, help="serving: number of requests per rate")
    ap.add_argument("--rhos", default="0.5,0.9,1.5,inf",
                    help="serving: offered load as multiples of the sequential rate (inf: all at once)")
    ap.add_argument("--slots", type=int, default=8, help="serving: resident query slots")
    ap.add_argument("--budget-gb", type=int, default=96, help="serving: device memory budget")
    ap.add_argument("--local", type=int, default=0, help="local-queue depth (with --delta: skips the tuner)")
    ap.add_argument("--grid", type=int, default=0, help="relaxation workgroups (with --delta: skips the tuner)")
    ap.add_argument("--defer", default=None, choices=["on", "off"],
                    help="large rows expanded at the bucket's advance (with --delta: skips the tuner)")
    ap.add_argument("--split", default=None, choices=["weight"],
                    help="light/heavy edge split (with --delta: skips the tuner)")
    ap.add_argument("--seeds", default="uniform", help="seed strategy: uniform, bfs_level, eccentric, proximate")
    ap.add_argument("--sweep", action="store_true", help="run the sensitivity studies instead of the benchmark")
    ap.add_argument("--sweep-scale", type=int, default=22, help="RMAT scale of the sensitivity studies")
    ap.add_argument("--copy-calib", action="store_true", help="run only the copy kernel used to scale HBM counters")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the workload's entry of profiles/traffic.json from rocprofv3 counter runs "
                         "(with the --delta and --local those runs used)")
    ap.add_argument("--pmc-table", nargs="+", metavar="COUNTER_CSV",
                    help="per-dispatch means of rocprofv3 --pmc counters for the relaxation and scan kernels")
    ap.add_argument("--busy-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="GPU-busy time per phase of a batching or serving run under rocprofv3")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="per-kernel durations over the timed region of a bench.py run under rocprofv3")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.trace_summary:
        trace_summary(args)
        return
    if args.busy_summary:
        busy_summary(args)
        return
    if args.pmc_table:
        pmc_table(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2205_14503_amd as st
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calib:
        copy_calibration(torch)
        return
    stream = torch.cuda.current_stream()
    if args.sweep:
        bench_sweep(args, st, W, np, torch, stream)
        return
    spec = W.WORKLOADS[args.workload]
    if "queries" in spec:
        print(json.dumps(bench_batch(args, st, W, np, torch, stream)), flush=True)
        return
    if "k_lo" in spec:
        print(json.dumps(bench_serve(args, st, W, np, torch, stream)), flush=True)
        return
    t0 = time.time()
    g = W.make_graph(args.workload)
    k = spec["k"]
    seeds = W.make_seeds(g, k, strategy=args.seeds)
    labels = W.components(g)
    comp = np.isin(labels, np.unique(labels[seeds]))
    nnz_reached = int(g.degrees()[comp].sum())
    print(f"[bench] {args.workload}: n={g.n} nnz={g.nnz} k={k} reached_nnz={nnz_reached} "
          f"(generated in {time.time() - t0:.1f}s)", file=sys.stderr, flush=True)

    opts = {"flags": st.FLAG_TIMING}
    if args.driver:
        opts["driver"] = args.driver
    if args.delta:
        opts["delta"] = args.delta
    if args.local:
        opts["local_iters"] = args.local
    if args.grid:
        opts["grid"] = args.grid
    if args.split:
        opts["flags"] |= st.FLAG_SPLIT
    if args.defer:
        opts["flags"] |= st.FLAG_DEFER if args.defer == "on" else st.FLAG_NO_DEFER
    dg = st.Graph(g, 0, stream)
    tuned = None
    if not args.no_tune and not args.delta:
        t0 = time.time()
        tuned = dg.tune(seeds)  # set-up, like the upload: picks delta and the local-queue depth
        split = "weight" if tuned["flags"] & st.FLAG_SPLIT else None
        tuned = {"delta": tuned["delta"], "local_iters": tuned["local_iters"], "grid": tuned["grid"],
                 "split": split, "lazy_pred": bool(tuned["flags"] & st.FLAG_LAZY_PRED),
                 "defer": bool(tuned["flags"] & st.FLAG_DEFER), "seconds": round(time.time() - t0, 2)}
        print(f"[bench] tuned {tuned}", file=sys.stderr, flush=True)
    # Before the warm-up, outside the timed region: the relaxation's random reads (one key read per attempt,
    # counted in a solve of its own) and a plain random gather over an array of the same size, the rate that
    # bounds them.
    attempts = dg.solve(seeds, dict(opts, flags=opts["flags"] | st.FLAG_COUNTERS)).stats["relax_attempts"]
    probe_gps = gather_probe(torch, g.n)
    for _ in range(args.warmup):
        tree = dg.solve(seeds, opts)
    torch.cuda.synchronize()
    lat, relax_ms, relax_launches, scan_ms, voronoi_ms, rounds = [], [], [], [], [], []
    phase_ms = {p: [] for p in ("init", "voronoi", "scan", "compact", "mst", "expand", "total")}
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        tree = dg.solve(seeds, opts)
        lat.append((time.perf_counter() - s0) * 1e3)
        relax_ms.append(tree.stats["ms_relax_kernels"])
        relax_launches.append(tree.stats["relax_launches"])
        scan_ms.append(tree.stats["ms_scan"])
        voronoi_ms.append(tree.stats["ms_voronoi"])
        rounds.append(tree.stats["rounds"])
        for p in phase_ms:
            phase_ms[p].append(tree.stats["ms_" + p])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    gteps = (nnz_reached / 2) / (ms_per_step * 1e-3) / 1e9

    b_vor, b_scan = algorithmic_bytes(g.n, nnz_reached, g.nnz)
    mean_relax = float(np.mean(relax_ms))
    mean_launch = float(np.mean(relax_launches))
    mean_scan = float(np.mean(scan_ms))
    if mean_relax >= mean_scan:
        kname, kbytes, kms, kl = "k_round (relaxation)", b_vor, mean_relax, mean_launch
    else:
        kname, kbytes, kms, kl = "k_scan (pred + boundary)", b_scan, mean_scan, 1.0
    achieved = (kbytes / kl) / (kms / kl * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            delta = opts.get("delta", tuned and tuned["delta"])
            local = opts.get("local_iters", tuned and tuned["local_iters"])
            split = args.split or (tuned and tuned["split"])
            grid = opts.get("grid", tuned["grid"] if tuned else 0)
            defer = args.defer == "on" if args.defer else bool(tuned and tuned["defer"])
            ent = json.load(open(TRAFFIC_FILE)).get(args.workload, {}).get(
                _config_key(delta, local, split, grid, defer))
            if ent and ent.get("kernel_sha") == kernel_sha():
                traffic = ent["bytes_per_launch"]
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "algorithmic_bytes_per_step": kbytes, "launches_per_step": kl,
                "avg_launch_us": round(kms / kl * 1e3, 3)}
    roofline["random_access"] = {
        "relax_attempts_per_step": attempts,
        "relax_attempts_per_s": round(attempts / (mean_relax * 1e-3)),
        "probe_gathers_per_s": round(probe_gps),
        "probe": f"torch index_select of 2^26 random positions of a {g.n}-entry int64 array"}

    cpu, oracle_check = None, None
    if not args.no_cpu_baseline:
        import oracle
        if g.nnz <= FULL_ORACLE_NNZ:
            # whole oracle solves (all of Alg. 2) for about --cpu-seconds; the GPU tree must equal the oracle's
            times = []
            c0 = time.perf_counter()
            while not times or (time.perf_counter() - c0) < args.cpu_seconds:
                s0 = time.perf_counter()
                ref = oracle.solve(g, seeds)
                times.append(time.perf_counter() - s0)
            assert ref.code == oracle.OK and ref.edges == tree.edges and ref.total == tree.total, \
                "GPU tree differs from the oracle"
            oracle_check = "tree and D identical to the oracle's full solve"
            cpu_gteps = (nnz_reached / 2) / float(np.mean(times)) / 1e9
            cpu = {"value": round(cpu_gteps, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                   "sample": f"{len(times)} full oracle solves of the same workload (single thread), "
                             f"mean {np.mean(times):.2f} s",
                   "queries_per_s": round(1.0 / float(np.mean(times)), 4)}
        else:
            # Too large for whole oracle solves inside the benchmark (Step 2's oracle collects and sorts every
            # cross-cell edge: minutes).  The sample is the oracle's Step 1 (binary-heap multi-source Dijkstra)
            # on the same full input, once; GTEPS over that step, like gteps_voronoi.  The GPU's Voronoi keys
            # must equal the oracle's on every vertex.
            print("[bench] oracle Step 1 on the full input (single thread)", file=sys.stderr, flush=True)
            _, S = oracle.canon_seeds(g.n, seeds)
            s0 = time.perf_counter()
            dist, src = oracle.voronoi(g, S)
            t_vor = time.perf_counter() - s0
            gkey, _ = dg.voronoi(seeds)
            assert np.array_equal(gkey, oracle.packed_key(dist, src)), "GPU Voronoi keys differ from the oracle"
            oracle_check = f"Voronoi keys of all {g.n} vertices identical to the oracle's Step 1"
            cpu = {"value": round((nnz_reached / 2) / t_vor / 1e9, 6), "unit": "GTEPS", "cores": 1,
                   "kind": "oracle",
                   "sample": f"the oracle's Step 1 (Voronoi cells, binary-heap multi-source Dijkstra) on the full "
                             f"input, one run, single thread: {t_vor:.1f} s; GTEPS over that step"}
            print(f"[bench] oracle Step 1: {t_vor:.1f} s", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz, "k": k, "seed": 1, "seeds": args.seeds,
                   "weights": [spec["wlo"], spec["whi"]], "reached_nnz": nnz_reached},
        "queries_per_s": round(1e3 / ms_per_step, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "gteps_voronoi": round((nnz_reached / 2) / (float(np.mean(voronoi_ms)) * 1e-3) / 1e9, 4),
        "gteps_voronoi_scan": round((nnz_reached / 2) / ((float(np.mean(voronoi_ms)) + mean_scan) * 1e-3) / 1e9, 4),
        "phases_ms": dict({p: round(float(np.mean(v)), 4) for p, v in phase_ms.items()},
                          relax_kernels=round(mean_relax, 4), rounds=float(np.mean(rounds)),
                          relax_launches=float(np.mean(relax_launches))),
        "tree": {"edges": len(tree.a), "D": tree.total},
        "tuned": tuned,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_check": oracle_check,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
