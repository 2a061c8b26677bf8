"""Continuous-batching server: every result in the mix equals the result of
the same query alone and the oracle's, admission respects the memory budget,
and error paths report the right codes."""
import sys
import threading
import time

import numpy as np
import pytest

import oracle as O
import paper_2205_14503_amd as st
import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def graph():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)
    g = W.rmat(15, 16, wlo=1, whi=1000)
    cand = W.lcc(g)
    dg = st.Graph(g, 0, torch.cuda.current_stream())
    yield g, cand, dg
    dg.close()


SERVER_OPTIONS = {
    "default": None,
    "delta1": dict(delta=1),
    "delta50": dict(delta=50),
    "split": dict(delta=50, flags=st.FLAG_SPLIT),
    "no_local_queue": dict(local_iters=0xFFFFFFFF),
    "split_chunky": dict(delta=7, flags=st.FLAG_SPLIT, small_max=1, chunk=64, local_iters=0xFFFFFFFF),
    "graph": dict(driver=4),
    "defer": dict(delta=50, flags=st.FLAG_DEFER),
    "defer_chunky": dict(delta=7, small_max=1, chunk=64, flags=st.FLAG_DEFER),
    "no_defer": dict(flags=st.FLAG_NO_DEFER),
}


@pytest.mark.parametrize("opt", list(SERVER_OPTIONS))
def test_server_mix_equals_alone_and_oracle(graph, opt):
    """Queries seeded between rounds while other slots advance buckets, park
    vertices and relax heavy edges: every served tree equals the oracle's and
    the same query's solve alone, under each set of relaxation options."""
    g, cand, dg = graph
    ks = [3, 40, 2, 600, 17, 5, 250, 1, 90, 8, 33, 1200, 4, 64, 7, 150]
    sets = [W.sample(cand, k, master=11, stream=300 + q) for q, k in enumerate(ks)]
    say(f"server ({opt}): 16 queries, 5 slots")
    srv = st.steiner_server_create(dg.handle, 4 << 30, 5, SERVER_OPTIONS[opt])
    try:
        tickets = [st.steiner_server_submit(srv, s) for s in sets]
        trees = [st.steiner_server_wait(srv, t) for t in tickets]
    finally:
        st.steiner_server_destroy(srv)
    for q, (s, tree) in enumerate(zip(sets, trees)):
        ref = O.solve(g, s)
        assert ref.code == O.OK
        assert tree.edges == ref.edges and tree.total == ref.total, f"query {q} (k={ks[q]})"
        alone = dg.solve(s, SERVER_OPTIONS[opt])
        assert alone.edges == tree.edges


def test_server_concurrent_clients(graph):
    g, cand, dg = graph
    sets = [W.sample(cand, int(k), master=12, stream=400 + q) for q, k in enumerate(W.log_uniform_sizes(24, 3, 300, 5))]
    refs = [dg.solve(s) for s in sets]
    say("server: 4 client threads, 24 queries")
    srv = st.steiner_server_create(dg.handle, 8 << 30, 8)
    out = [None] * len(sets)
    errors = []

    def client(idx):
        try:
            for q in idx:
                t = st.steiner_server_submit(srv, sets[q])
                out[q] = st.steiner_server_wait(srv, t)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=client, args=(list(range(i, len(sets), 4)),)) for i in range(4)]
    try:
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
    finally:
        st.steiner_server_destroy(srv)
    assert not errors, errors
    for q in range(len(sets)):
        assert out[q] is not None and out[q].edges == refs[q].edges, f"query {q}"


def test_server_budget_and_errors(graph):
    g, cand, dg = graph
    probe = st.steiner_server_create(dg.handle, 1 << 30, 64)
    mem = st.steiner_server_memory(probe)
    one = st.steiner_server_query_bytes(probe, 20)
    st.steiner_server_destroy(probe)
    assert mem["fixed_bytes"] + mem["slots"] * mem["slot_bytes"] + mem["pool_bytes"] == 1 << 30
    assert mem["slot_bytes"] >= 14 * g.n
    budget = mem["fixed_bytes"] + 3 * one + (1 << 16)
    srv = st.steiner_server_create(dg.handle, budget, 64)
    try:
        m = st.steiner_server_memory(srv)
        assert m["slots"] == 3 and m["fixed_bytes"] + 3 * m["slot_bytes"] + m["pool_bytes"] == budget
        need = st.steiner_server_query_bytes(srv, 100)
        assert need >= m["slot_bytes"] + 8 * 100 * 99 // 2
        # a query whose pool region exceeds the whole pool is refused at submit
        with pytest.raises(st.SteinerError) as e:
            st.steiner_server_submit(srv, cand[:3000])
        assert e.value.code == st.ENOMEM
        with pytest.raises(st.SteinerError) as e:
            st.steiner_server_submit(srv, [g.n + 5])
        assert e.value.code == st.EINVAL
        # k = 1 completes at once
        t = st.steiner_server_submit(srv, [int(cand[0])] * 4)
        tree = st.steiner_server_wait(srv, t, 10_000_000)
        assert tree.total == 0 and len(tree.a) == 0
        # at most 3 queries fit the budget at a time; all still finish correctly
        sets = [W.sample(cand, 20, master=13, stream=500 + q) for q in range(9)]
        tickets = [st.steiner_server_submit(srv, s) for s in sets]
        for s, t in zip(sets, tickets):
            assert st.steiner_server_wait(srv, t).edges == dg.solve(s).edges
        with pytest.raises(st.SteinerError) as e:
            st.steiner_server_wait(srv, 987654321)
        assert e.value.code == st.EINVAL
    finally:
        st.steiner_server_destroy(srv)
    with pytest.raises(st.SteinerError):
        st.steiner_server_create(dg.handle, 10, 4)


def test_server_disconnected_query(graph):
    g, cand, dg = graph
    comp = W.components(g)
    other = np.nonzero(comp != comp[cand[0]])[0]
    srv = st.steiner_server_create(dg.handle, 2 << 30, 4)
    try:
        t = st.steiner_server_submit(srv, [int(cand[0]), int(other[0])])
        with pytest.raises(st.SteinerError) as e:
            st.steiner_server_wait(srv, t)
        assert e.value.code == st.EDISCONNECTED
        t = st.steiner_server_submit(srv, cand[:10])
        assert st.steiner_server_wait(srv, t).edges == O.solve(g, cand[:10]).edges
    finally:
        st.steiner_server_destroy(srv)


def test_server_fixed_stride_rows(graph):
    """A grid (every row at most four entries) is served by the round kernel's
    fixed-stride instance: same trees in the mix, alone and by the oracle."""
    import torch
    g = W.grid(60, 70, 1, 5, master=3)
    allv = np.arange(g.n, dtype=np.uint32)
    ks = [2, 31, 5, 120, 9, 1, 64, 17]
    sets = [W.sample(allv, k, master=13, stream=500 + q) for q, k in enumerate(ks)]
    with st.Graph(g, 0, torch.cuda.current_stream()) as gg:
        say("server: grid 60x70, 8 queries, 3 slots")
        srv = st.steiner_server_create(gg.handle, 1 << 30, 3)
        try:
            tickets = [st.steiner_server_submit(srv, s) for s in sets]
            trees = [st.steiner_server_wait(srv, t) for t in tickets]
        finally:
            st.steiner_server_destroy(srv)
        for q, (s, tree) in enumerate(zip(sets, trees)):
            ref = O.solve(g, s)
            assert ref.code == O.OK
            assert tree.edges == ref.edges and tree.total == ref.total, f"query {q} (k={ks[q]})"
            assert gg.solve(s).edges == tree.edges


def test_server_round_wrap(graph, monkeypatch):
    """A server's pass lives for ever, so its round numbers wrap (at 3 * 2^28, a multiple of the list parity and
    of the three rotating counters): a pass started just below the wrap serves every query through it with the
    results of the same queries solved alone."""
    g, cand, dg = graph
    monkeypatch.setenv("STEINER_SERVER_ROUND_BASE", str((3 << 28) - 7))
    ks = [2, 40, 600, 9, 150, 1200, 3, 64]
    sets = [W.sample(cand, k, master=15, stream=700 + q) for q, k in enumerate(ks)]
    for opt in (None, dict(delta=50)):
        say(f"server round wrap ({opt}): 8 queries, 3 slots")
        srv = st.steiner_server_create(dg.handle, 2 << 30, 3, opt)
        try:
            tickets = [st.steiner_server_submit(srv, s) for s in sets]
            trees = [st.steiner_server_wait(srv, t) for t in tickets]
        finally:
            st.steiner_server_destroy(srv)
        for q, (s, tree) in enumerate(zip(sets, trees)):
            assert tree.edges == dg.solve(s, opt).edges, f"query {q} (k={ks[q]})"


def test_server_timeout_and_cancel(graph):
    """A wait that runs out of time returns ETIMEDOUT and leaves the request
    pending; waiters blocked when the server is destroyed get ECANCELED."""
    g, cand, dg = graph
    sets = [W.sample(cand, 1200, master=14, stream=600 + q) for q in range(40)]
    srv = st.steiner_server_create(dg.handle, 4 << 30, 1)
    codes = {}
    try:
        tickets = [st.steiner_server_submit(srv, s) for s in sets]
        with pytest.raises(st.SteinerError) as e:
            st.steiner_server_wait(srv, tickets[-1], 0)
        assert e.value.code == st.ETIMEDOUT
        first = st.steiner_server_wait(srv, tickets[0])  # still pending after the time-out elsewhere
        assert first.edges == dg.solve(sets[0]).edges

        def waiter(q):
            try:
                st.steiner_server_wait(srv, tickets[q])
                codes[q] = st.OK
            except st.SteinerError as ex:
                codes[q] = ex.code

        threads = [threading.Thread(target=waiter, args=(q,)) for q in range(35, 40)]
        for th in threads:
            th.start()
        time.sleep(0.05)
    finally:
        st.steiner_server_destroy(srv)
    for th in threads:
        th.join(timeout=60)
    assert sorted(codes) == list(range(35, 40))
    assert all(c == st.ECANCELED for c in codes.values()), codes
