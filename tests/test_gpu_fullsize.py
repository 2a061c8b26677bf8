"""Parity at full size: the RMAT scale-25 single query with 10,000 seeds,
solved as the benchmark solves it (tuned options).  The oracle's own solve
takes minutes there, so the GPU's intermediates are checked against
properties that determine them uniquely (the Voronoi fixed-point equations,
the exactness of G'1), and the oracle's pred, MST and expansion, run on those
verified intermediates, must reproduce the GPU's tree bit for bit."""
import sys

import numpy as np
import pytest

import props
import oracle as O
import paper_2205_14503_amd as st
import workloads as W

pytestmark = pytest.mark.gpu
U64_MAX = np.iinfo(np.uint64).max


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_stream():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)
    return torch.cuda.current_stream()


def intermediates(g, seeds, dg):
    """The GPU's Step 1 and Step 2 outputs of one query (through the C ABI)."""
    _, S = O.canon_seeds(g.n, seeds)
    key, pred = dg.voronoi(seeds)
    gi, gj, gk = dg.boundary(seeds)
    return S, key, pred, gi, gj, gk


def check_intermediates(g, S, key, pred, gi, gj, gk, tree, what):
    """The tree of one query equals the oracle's tail run on the GPU's
    intermediates, and those intermediates satisfy their defining equations.
    Host work only (the C checkers and the oracle release the GIL)."""
    k = len(S)
    assert props.voronoi_fixed_point(g, S, key) == -1, f"{what}: Voronoi keys are not the fixed point"
    reached = key != U64_MAX
    dist = np.where(reached, key >> np.uint64(32), U64_MAX).astype(np.uint64)
    src = np.where(reached, key & np.uint64(0xFFFFFFFF), np.uint64(0xFFFFFFFF)).astype(np.uint32)
    assert O.check_dist(dist) == O.OK
    assert np.array_equal(pred, O.pred(g, S, dist, src)), f"{what}: pred differs from the oracle's definition"
    pt = np.full(k * (k - 1) // 2, U64_MAX, dtype=np.uint64)
    pt[gj.astype(np.uint64) * (gj.astype(np.uint64) - 1) // 2 + gi] = gk
    assert props.boundary_exact(g, key, k, pt) == 0, f"{what}: G'1 is not the per-pair minimum"
    rc, chosen = O.mst(k, gi, gj, gk >> np.uint64(32))
    assert rc == O.OK and len(chosen) == k - 1
    sel = (gk[chosen] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    rc, a, b, w, total = O.expand(g, S, dist, src, pred, sel)
    assert rc == O.OK
    assert tree.edges == list(zip(a.tolist(), b.tolist(), w.tolist())), f"{what}: tree differs"
    assert tree.total == total, f"{what}: D differs"
    return f"{what}: tree of {len(a)} edges, D = {total}, identical"


def verify_by_properties(g, seeds, dg, tree, what):
    say(f"{what}: checking the intermediates and the oracle's tail")
    say(check_intermediates(g, *intermediates(g, seeds, dg), tree, what))


def verify_all(g, sets, dg, trees, what, workers=6):
    """verify_by_properties for every query: the GPU intermediates are fetched
    in order on this thread, the host checks run on a pool of `workers`
    threads with at most 2 x workers queries in flight (bounded memory)."""
    from concurrent.futures import ThreadPoolExecutor, wait, FIRST_COMPLETED
    pending = set()
    done_count = 0
    with ThreadPoolExecutor(max_workers=workers) as pool:
        for q, (s, tree) in enumerate(zip(sets, trees)):
            while len(pending) >= 2 * workers:
                fin, pending = wait(pending, return_when=FIRST_COMPLETED)
                for f in fin:
                    done_count += 1
                    say(f.result())
            pending.add(pool.submit(check_intermediates, g, *intermediates(g, s, dg), tree,
                                    f"{what} {q} (k={len(s)})"))
        for f in pending:
            done_count += 1
            say(f.result())
    assert done_count == len(sets)


def test_rmat25_k10000_full_size():
    stream = gpu_stream()
    say("rmat25: generating the graph")
    g = W.make_graph("rmat25")
    seeds = W.make_seeds(g, W.WORKLOADS["rmat25"]["k"])
    say(f"rmat25: n={g.n} nnz={g.nnz}; solving on the GPU")
    with st.Graph(g, 0, stream) as dg:
        dg.tune(seeds)
        tree = dg.solve(seeds)
        verify_by_properties(g, seeds, dg, tree, "rmat25")


def test_rmat22_batch64_full_size():
    """The 64-query batch of RMAT scale 22: every query equals its own solve
    and every one is verified against its defining properties and the
    oracle's tail."""
    stream = gpu_stream()
    spec = W.WORKLOADS["rmat22_batch64"]
    g = W.make_graph("rmat22_batch64")
    cand = W.lcc(g)
    sets = W.make_query_set(g, spec["queries"], spec["k_lo"], spec["k_hi"], cand=cand)
    say(f"rmat22 batch: {len(sets)} queries, k from {min(map(len, sets))} to {max(map(len, sets))}")
    with st.Graph(g, 0, stream) as dg:
        dg.tune(sets[len(sets) // 2])
        batch = dg.solve_batch(sets)
        for q, (code, tree) in enumerate(batch):
            assert code == st.OK
            assert tree.edges == dg.solve(sets[q]).edges, f"query {q}"
        verify_all(g, sets, dg, [t for _, t in batch], "rmat22 batch query")


def test_rmat24_served_full_size():
    """The served RMAT scale-24 graph: queries submitted together to the
    server equal their own solves, and every one of them is verified."""
    stream = gpu_stream()
    spec = W.WORKLOADS["rmat24_serve"]
    g = W.make_graph("rmat24_serve")
    sets = W.make_query_set(g, 16, spec["k_lo"], spec["k_hi"])
    say(f"rmat24 serve: 16 queries, k from {min(map(len, sets))} to {max(map(len, sets))}")
    with st.Graph(g, 0, stream) as dg:
        srv = st.steiner_server_create(dg.handle, 64 << 30, 8)
        try:
            tickets = [st.steiner_server_submit(srv, s) for s in sets]
            served = [st.steiner_server_wait(srv, t) for t in tickets]
        finally:
            st.steiner_server_destroy(srv)
        for q, s in enumerate(sets):
            assert served[q].edges == dg.solve(s).edges, f"query {q}"
        verify_all(g, sets, dg, served, "rmat24 served query", workers=4)
