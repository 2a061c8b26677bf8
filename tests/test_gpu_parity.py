"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

All arithmetic is integer, so every comparison is exact: Voronoi keys
(dist << 32 | seed index), canonical predecessors, the entries of G'1, the
tree's edge list, D, and the status code.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
import paper_2205_14503_amd as st
import pins
import workloads as W

pytestmark = pytest.mark.gpu

OPTION_SETS = {
    "default": None,
    "host": dict(driver=1),
    "persistent": dict(driver=2),
    "delta1": dict(delta=1),
    "unbounded": dict(delta=0xFFFFFFFF),
    "chunky": dict(small_max=1, chunk=64),
    "persist_odd": dict(driver=2, small_max=2, chunk=64, delta=3, block=1024),
    "bucketed": dict(delta=50),
    "lazy": dict(flags=st.FLAG_LAZY_PRED),
    "cluster": dict(driver=3),
    "eager": dict(flags=st.FLAG_EAGER_PRED),
    "split": dict(delta=50, flags=st.FLAG_SPLIT),
    "split_chunky": dict(delta=7, flags=st.FLAG_SPLIT, small_max=1, chunk=64, local_iters=0xFFFFFFFF),
    "graph": dict(driver=4),
    "graph_bucketed": dict(driver=4, delta=50, local_iters=2),
    "defer": dict(delta=50, flags=st.FLAG_DEFER),
    "defer_chunky": dict(delta=7, small_max=1, chunk=64, flags=st.FLAG_DEFER),
    "defer_unbounded": dict(delta=0xFFFFFFFF, flags=st.FLAG_DEFER),
    "defer_persistent": dict(driver=2, delta=50, small_max=2, flags=st.FLAG_DEFER),
    "no_defer": dict(flags=st.FLAG_NO_DEFER),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stream():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)
    st.load()
    return torch.cuda.current_stream()


def gpu_code(fn, *a, **kw):
    try:
        return st.OK, fn(*a, **kw)
    except st.SteinerError as e:
        return e.code, None


def check_case(g, seeds, stream, options, what="", flags=0):
    ref = O.solve(g, seeds)
    _, S = O.canon_seeds(g.n, seeds)
    with st.Graph(g, 0, stream, flags) as dg:
        code, tree = gpu_code(dg.solve, seeds, options)
        assert code == ref.code, f"{what}: status {code} vs oracle {ref.code}"
        if code == st.OK:
            assert tree.edges == ref.edges, f"{what}: tree differs"
            assert tree.total == ref.total
        if len(S) >= 2:
            dist, src = O.voronoi(g, S)
            ovf = O.check_dist(dist)
            code, kp = gpu_code(dg.voronoi, seeds, options)
            rc_b, pi, pj, pb, pe = O.boundary(g, dist, src, len(S)) if ovf == O.OK else (ovf, None, None, None, None)
            if ovf != O.OK or rc_b != O.OK:
                assert code == st.EOVERFLOW, f"{what}: voronoi status {code}"
            else:
                assert code == st.OK
                key, pred = kp
                assert np.array_equal(key, O.packed_key(dist, src)), f"{what}: keys differ"
                assert np.array_equal(pred, O.pred(g, S, dist, src)), f"{what}: pred differs"
                gi, gj, gk = dg.boundary(seeds, options)
                assert np.array_equal(gi, pi) and np.array_equal(gj, pj), f"{what}: G'1 pairs differ"
                assert np.array_equal(gk, (pb << np.uint64(32)) | pe.astype(np.uint64)), f"{what}: G'1 values differ"


def test_golden_cases(stream):
    """The hand-worked cases of tests/golden: every option set, in the caller's order and renumbered, gives
    the tree, D and status worked out in each file."""
    import test_golden
    for path in test_golden.CASES:
        g, seeds, code, tree, total = test_golden.load_case(path)
        for flags in (st.UPLOAD_KEEP_ORDER, st.UPLOAD_REORDER):
            with st.Graph(g, 0, stream, flags) as dg:
                for name, opt in OPTION_SETS.items():
                    got, t = gpu_code(dg.solve, seeds, opt)
                    what = f"{os.path.basename(path)} {name} flags={flags}"
                    assert got == code, f"{what}: status {got}"
                    if code == st.OK:
                        assert sorted(t.edges) == tree and t.total == total, what


def test_tiny_graphs_all_options(stream):
    cases = list(pins.tiny_cases(seed=21, count=90))
    for name, opt in OPTION_SETS.items():
        say(f"tiny graphs, options={name}")
        for t, (g, seeds) in enumerate(cases):
            check_case(g, seeds, stream, opt, f"case {t} {name}")


def test_tiny_graphs_renumbered(stream):
    """The internal degree order changes no result: ties between equal
    distances, parallel edges and self-loops are still decided on the
    caller's ids and CSR offsets."""
    cases = list(pins.tiny_cases(seed=23, count=90))
    for name in ("default", "persistent", "lazy", "eager", "cluster", "split_chunky"):
        say(f"tiny graphs renumbered, options={name}")
        for t, (g, seeds) in enumerate(cases):
            check_case(g, seeds, stream, OPTION_SETS[name], f"case {t} {name} renumbered", flags=st.UPLOAD_REORDER)


def test_error_codes_and_edge_cases(stream):
    say("error codes")
    big = 1 << 31
    cases = [
        (W.from_edges(4, [(0, 1, big), (1, 2, big), (0, 3, 1)]), [0, 3]),   # distance overflow
        (W.from_edges(3, [(0, 1, big), (1, 2, big)]), [0, 2]),              # cross-cell sum overflow
        (W.from_edges(3, [(0, 1, big - 1), (1, 2, big)]), [0, 2]),          # largest sum that fits
        (W.from_edges(2, [(0, 1, 0xFFFFFFFE)]), [0, 1]),
        (W.from_edges(5, [(0, 1, 3), (2, 3, 1), (3, 4, 2)]), [0, 4]),       # disconnected
        (W.from_edges(5, [(0, 1, 3), (2, 3, 1), (3, 4, 2)]), [2, 4, 4]),
        (W.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1)]), [2, 2, 2]),    # k = 1 after dedup
        (W.from_edges(6, []), [1, 4]),                                       # no edges at all
        (W.from_edges(4, [(0, 0, 5), (0, 1, 2), (0, 1, 1), (1, 1, 1), (1, 2, 7), (2, 3, 1), (2, 3, 1)]), [0, 3]),
    ]
    for t, (g, s) in enumerate(cases):
        for name in ("default", "persistent"):
            check_case(g, np.array(s, dtype=np.uint32), stream, OPTION_SETS[name], f"edge case {t} {name}")
        check_case(g, np.array(s, dtype=np.uint32), stream, None, f"edge case {t} renumbered", flags=st.UPLOAD_REORDER)
    g = W.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1)])
    with st.Graph(g, 0, stream) as dg:
        assert gpu_code(dg.solve, np.array([], dtype=np.uint32))[0] == st.EINVAL
        assert gpu_code(dg.solve, [0, 4])[0] == st.EINVAL
    # more distinct seeds than a query may hold (k(k-1)/2 pair indices must fit in 32 bits)
    n = 100_000
    path = W.from_edges(n, [(v, v + 1, 1) for v in range(n - 1)])
    many = np.arange(92_683, dtype=np.uint32)
    with st.Graph(path, 0, stream) as dg:
        assert gpu_code(dg.solve, many)[0] == st.EINVAL
        assert gpu_code(dg.solve_batch, [many[:3], many])[0] == st.OK  # per-query status
        codes = [c for c, _ in dg.solve_batch([many[:3], many])]
        assert codes == [st.OK, st.EINVAL]
        srv = st.steiner_server_create(dg.handle, 1 << 30, 2)
        try:
            assert gpu_code(st.steiner_server_submit, srv, many)[0] == st.EINVAL
        finally:
            st.steiner_server_destroy(srv)


def test_upload_validation(stream):
    say("upload validation")
    good = W.from_edges(3, [(0, 1, 1), (1, 2, 2)])

    def upload(rp, col, w, flags=0):
        try:
            h = st.steiner_graph_upload(3, rp, col, w, 0, stream, flags)
            st.steiner_graph_free(h)
            return st.OK
        except st.SteinerError as e:
            return e.code

    assert upload(good.row_ptr, good.col, good.w, flags=1) == st.OK
    w0 = good.w.copy(); w0[0] = 0
    assert upload(good.row_ptr, good.col, w0) == st.EINVAL
    c3 = good.col.copy(); c3[0] = 3
    assert upload(good.row_ptr, c3, good.w) == st.EINVAL
    uns = W.from_edges(3, [(1, 0, 1), (1, 2, 2)])
    cu = uns.col.copy(); cu[[1, 2]] = cu[[2, 1]]
    assert upload(uns.row_ptr, cu, uns.w) == st.EINVAL
    rp = good.row_ptr.copy(); rp[1] = 5
    assert upload(rp, good.col, good.w) == st.EINVAL
    asym = good.w.copy(); asym[0] = 9
    assert upload(good.row_ptr, good.col, asym, flags=1) == st.EINVAL
    assert upload(good.row_ptr, good.col, asym, flags=0) == st.OK
    assert upload(good.row_ptr, good.col, good.w, flags=st.UPLOAD_REORDER | st.UPLOAD_KEEP_ORDER) == st.EINVAL
    assert upload(good.row_ptr, good.col, good.w, flags=st.UPLOAD_REORDER | st.UPLOAD_SYMMETRY) == st.OK
    # renumbering needs every entry's twin: an asymmetric CSR is refused when it is forced
    assert upload(good.row_ptr, good.col, asym, flags=st.UPLOAD_REORDER) == st.EINVAL
    par = W.from_edges(3, [(0, 1, 4), (0, 1, 2), (1, 2, 2)])  # parallel entries of different weights
    assert upload(par.row_ptr, par.col, par.w, flags=st.UPLOAD_REORDER | st.UPLOAD_SYMMETRY) == st.OK


def test_device_upload_both_orders(stream):
    """Upload from device tensors, renumbered (the skewed graph's default) and
    in the caller's order: same trees, keys and preds as the oracle."""
    import torch
    g = W.rmat(13, 16, wlo=1, whi=100)
    seeds = W.sample(W.lcc(g), 120, master=4)
    ref = O.solve(g, seeds)
    _, S = O.canon_seeds(g.n, seeds)
    want_key = O.packed_key(ref.dist, ref.src)
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
    col = torch.from_numpy(g.col.view(np.int32)).cuda()
    w = torch.from_numpy(g.w.view(np.int32)).cuda()
    for flags in (0, st.UPLOAD_KEEP_ORDER, st.UPLOAD_REORDER):
        say(f"device upload flags={flags}")
        h = st.steiner_graph_upload_device(g.n, rp, col, w, 0, stream, flags)
        try:
            tree = st.steiner_solve(h, seeds)
            assert tree.edges == ref.edges and tree.total == ref.total
            key, pred = st.steiner_voronoi(h, g.n, seeds)
            assert np.array_equal(key, want_key) and np.array_equal(pred, ref.pred)
        finally:
            st.steiner_graph_free(h)


def test_er16k_config(stream):
    g = W.make_graph("er16k")
    seeds = W.make_seeds(g, 16)
    for name in ("default", "host", "persistent", "delta1", "bucketed", "split", "chunky", "lazy", "eager", "cluster"):
        say(f"er16k options={name}")
        check_case(g, seeds, stream, OPTION_SETS[name], f"er16k {name}")


def test_rmat_hubs(stream):
    g = W.rmat(16, 16, wlo=1, whi=1000)
    cand = W.lcc(g)
    for k in (2, 37, 1000):
        seeds = W.sample(cand, k, master=3)
        for name in ("default", "persistent", "chunky", "split", "eager", "cluster"):
            say(f"rmat16 k={k} options={name}")
            check_case(g, seeds, stream, OPTION_SETS[name], f"rmat16 k={k} {name}")
        for name in ("default", "eager"):  # the skewed graph is renumbered by default; also in the caller's order
            say(f"rmat16 k={k} options={name} caller order")
            check_case(g, seeds, stream, OPTION_SETS[name], f"rmat16 k={k} {name} kept", flags=st.UPLOAD_KEEP_ORDER)


def test_weight_one_ties(stream):
    g = W.rmat(13, 8, wlo=1, whi=1)
    seeds = W.sample(W.lcc(g), 300, master=5)
    for name in ("default", "persistent", "bucketed", "split_chunky", "eager", "lazy", "cluster"):
        say(f"rmat13 unit weights options={name}")
        check_case(g, seeds, stream, OPTION_SETS[name], f"unit {name}")
    gg = W.grid(61, 67, 1, 2)
    seeds = W.sample(np.arange(gg.n, dtype=np.uint32), 150, master=6)
    for name in ("default", "persistent", "lazy", "cluster"):
        say(f"grid 61x67 w in [1,2] options={name}")
        check_case(gg, seeds, stream, OPTION_SETS[name], f"grid12 {name}")
    unit_seeds = W.sample(W.lcc(g), 300, master=5)
    for name in ("default", "lazy", "eager"):
        say(f"unit weights, other vertex order, options={name}")
        check_case(g, unit_seeds, stream, OPTION_SETS[name], f"unit {name} kept", flags=st.UPLOAD_KEEP_ORDER)
        check_case(gg, seeds, stream, OPTION_SETS[name], f"grid12 {name} renumbered", flags=st.UPLOAD_REORDER)


def test_grid2048_full_size(stream):
    g = W.make_graph("grid2048")
    seeds = W.make_seeds(g, 100)
    say("grid2048 oracle")
    ref = O.solve(g, seeds)
    assert ref.code == O.OK
    want_key = O.packed_key(ref.dist, ref.src)
    with st.Graph(g, 0, stream) as dg:
        for name in ("default", "persistent", "lazy", "cluster"):
            say(f"grid2048 options={name}")
            tree = dg.solve(seeds, OPTION_SETS[name])
            assert tree.edges == ref.edges and tree.total == ref.total
            key, pred = dg.voronoi(seeds, OPTION_SETS[name])
            assert np.array_equal(key, want_key)
            assert np.array_equal(pred, ref.pred)
        # the launch configuration the benchmark times: the tuner's choice (bucket width, depth, workgroups)
        chosen = dg.tune(seeds)
        say(f"grid2048 tuned: {chosen}")
        tree = dg.solve(seeds)
        assert tree.edges == ref.edges and tree.total == ref.total
        key, pred = dg.voronoi(seeds)
        assert np.array_equal(key, want_key)
        assert np.array_equal(pred, ref.pred)


def test_tune_keeps_results(stream):
    g = W.rmat(14, 16, wlo=1, whi=1000)
    seeds = W.sample(W.lcc(g), 200, master=8)
    ref = O.solve(g, seeds)
    with st.Graph(g, 0, stream) as dg:
        say("autotune")
        chosen = dg.tune(seeds)
        assert chosen["delta"] >= 1
        tree = dg.solve(seeds)
        assert tree.edges == ref.edges and tree.total == ref.total
        other = W.sample(W.lcc(g), 77, master=9)
        assert dg.solve(other).edges == O.solve(g, other).edges
        assert gpu_code(dg.tune, [5])[0] == st.EINVAL


def test_batch_equals_single_and_oracle(stream):
    g = W.rmat(14, 16, wlo=1, whi=1000)
    cand = W.lcc(g)
    sets = [W.sample(cand, int(k), master=1, stream=200 + q) for q, k in enumerate([3, 17, 2, 64, 9, 250, 5, 1])]
    sets.append(np.array([int(cand[0])] * 3, dtype=np.uint32))  # k = 1 after dedup
    for flags, name in ((0, "default"), (0, "persistent"), (0, "cluster"), (st.UPLOAD_KEEP_ORDER, "default")):
        # the skewed graph is renumbered unless the upload keeps the caller's order;
        # a batch with driver 3 runs the frontier driver
        with st.Graph(g, 0, stream, flags) as dg:
            say(f"batch options={name} upload flags={flags}")
            res = dg.solve_batch(sets, OPTION_SETS[name])
            for q, (code, tree) in enumerate(res):
                ref = O.solve(g, sets[q])
                assert code == ref.code
                if code == st.OK:
                    assert tree.edges == ref.edges and tree.total == ref.total, f"query {q}"
                    single = dg.solve(sets[q], OPTION_SETS[name])
                    assert single.edges == tree.edges


def test_fixed_stride_rows(stream):
    """Graphs whose rows have at most four entries (grids, paths, ladders)
    run the round kernel's fixed-stride instance: no row offsets, the
    superseded test with the row load, spilled vertices claimed at the end of
    the unit.  Same trees as the oracle with and without the local queue, at
    depth 1, with the light/heavy split, and in a batch; a fifth entry in one
    row sends the same graph to the general instance."""
    shapes = [(1, 40, 1, 3), (2, 37, 1, 2), (6, 9, 1, 1), (33, 40, 1, 3), (45, 61, 1, 1000)]
    opts = {"default": None, "no_queue": dict(local_iters=0), "depth1": dict(local_iters=1),
            "split": dict(delta=5, flags=st.FLAG_SPLIT), "bucketed": dict(delta=40, local_iters=2)}
    for r, c, wlo, whi in shapes:
        g = W.grid(r, c, wlo, whi, master=r * 100 + c)
        for k in (1, 2, 7, 30):
            seeds = W.sample(np.arange(g.n, dtype=np.uint32), min(k, g.n), master=k, stream=300 + r)
            for name, opt in opts.items():
                check_case(g, seeds, stream, opt, f"grid {r}x{c} k={k} {name}")
    g = W.grid(40, 50, 1, 4, master=5)
    sets = [W.sample(np.arange(g.n, dtype=np.uint32), k, master=2, stream=400 + k) for k in (2, 9, 33, 150, 1)]
    with st.Graph(g, 0, stream) as dg:
        say("fixed-stride rows, batch")
        for q, (code, tree) in enumerate(dg.solve_batch(sets)):
            ref = O.solve(g, sets[q])
            assert code == ref.code == st.OK
            assert tree.edges == ref.edges and tree.total == ref.total, f"query {q}"
    # two interior vertices with five entries: the general instance, same results
    e = [(int(a), int(b), int(w)) for a, b, w, _ in zip(*g.edges())] + [(51, g.n - 52, 3)]
    g5 = W.from_edges(g.n, e)
    say("grid plus one long edge")
    check_case(g5, sets[2], stream, None, "grid + long edge")


def test_seed_strategies(stream):
    """The paper's seed-selection variants (BFS-level, uniform, eccentric,
    proximate) give the same trees as the oracle."""
    g = W.rmat(14, 16, wlo=1, whi=1000)
    cand = W.lcc(g)
    gg = W.grid(61, 67, 1, 1000)
    for strat in W.SEED_STRATEGIES:
        say(f"rmat14 seeds={strat}")
        check_case(g, W.make_seeds(g, 40, master=9, cand=cand, strategy=strat), stream, None, f"rmat14 {strat}")
        say(f"grid 61x67 seeds={strat}")
        check_case(gg, W.make_seeds(gg, 25, master=9, strategy=strat), stream, None, f"grid {strat}")


def test_graph_driver_replays(stream):
    """The graph-captured driver replays one instantiated graph across
    solves: with the program's own solves, batches and synchronisations in
    between, every replayed solve equals the host-stepped one and the oracle."""
    import torch
    g = W.rmat(14, 16, wlo=1, whi=1000)
    cand = W.lcc(g)
    sets = [W.sample(cand, k, master=21, stream=700 + i) for i, k in enumerate([5, 300, 40, 1000, 2])]
    refs = [O.solve(g, s) for s in sets]
    with st.Graph(g, 0, stream) as dg:
        for rep in range(3):
            for s, ref in zip(sets, refs):
                got = dg.solve(s, dict(driver=4))
                assert got.edges == ref.edges and got.total == ref.total, f"replay {rep}"
                assert dg.solve(s).edges == ref.edges
            torch.cuda.synchronize()
            batch = dg.solve_batch(sets, dict(driver=4))
            assert [t.edges for _, t in batch] == [r.edges for r in refs]
