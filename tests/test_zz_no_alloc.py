"""steiner_solve_noalloc (the entry point for callers that cannot allocate)
against steiner_solve through the C ABI: identical trees and D, on two calls
in a row with the second on a smaller input, and its limits."""
import sys

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
def stream():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)
    st.load()
    return torch.cuda.current_stream()


def code_of(fn, *a, **kw):
    try:
        fn(*a, **kw)
        return st.OK
    except st.SteinerError as e:
        return e.code


@pytest.mark.parametrize("options", [None, dict(flags=st.FLAG_EAGER_PRED), dict(delta=50, local_iters=2)])
def test_noalloc_equals_solve_twice_second_smaller(stream, options):
    big = W.rmat(16, 16, wlo=1, whi=1000)               # renumbered at upload (skewed degrees)
    small = W.er(2048, 16384, 1, 100, master=1)
    cases = [(big, W.sample(W.lcc(big), 300, master=1)), (small, W.sample(W.lcc(small), 16, master=1))]
    for rep, (g, seeds) in enumerate(cases):
        say(f"noalloc call {rep}: n={g.n} k={len(seeds)} options={options}")
        with st.Graph(g, 0, stream) as dg:
            ref = st.steiner_solve(dg.handle, seeds, options)
            got = st.steiner_solve_noalloc(dg.handle, seeds, g.n, options)
        assert got.edges == ref.edges, f"call {rep}: tree differs from steiner_solve"
        assert got.total == ref.total
        orc = O.solve(g, seeds)
        assert orc.code == O.OK and got.edges == orc.edges and got.total == orc.total


def test_noalloc_limits_and_codes(stream):
    g = W.er(2048, 16384, 1, 100, master=1)
    cand = W.lcc(g)
    with st.Graph(g, 0, stream) as dg:
        seeds = W.sample(cand, 40, master=2)
        ref = st.steiner_solve(dg.handle, seeds)
        m = len(ref.a)
        # too small an output: ENOMEM, then the same call with room succeeds
        assert code_of(st.steiner_solve_noalloc, dg.handle, seeds, m - 1) == st.ENOMEM
        assert st.steiner_solve_noalloc(dg.handle, seeds, m).edges == ref.edges
        # k = 1 after deduplication: empty tree; seed out of range: EINVAL; too many seeds: ENOMEM
        one = st.steiner_solve_noalloc(dg.handle, [int(cand[0])] * 3, 0)
        assert one.total == 0 and len(one.a) == 0
        assert code_of(st.steiner_solve_noalloc, dg.handle, [0, g.n], 10) == st.EINVAL
        assert code_of(st.steiner_solve_noalloc, dg.handle, np.zeros(9000, dtype=np.uint32), 10) == st.ENOMEM
    # disconnected seeds
    d = W.from_edges(5, [(0, 1, 3), (2, 3, 1), (3, 4, 2)])
    with st.Graph(d, 0, stream) as dg:
        assert code_of(st.steiner_solve_noalloc, dg.handle, [0, 4], 10) == st.EDISCONNECTED
        assert st.steiner_solve_noalloc(dg.handle, [2, 4], 10).edges == st.steiner_solve(dg.handle, [2, 4]).edges
    # a graph whose solve needs more than the scratch
    huge = W.grid(2400, 2400, 1, 1000, master=1)
    with st.Graph(huge, 0, stream) as dg:
        assert code_of(st.steiner_solve_noalloc, dg.handle, [0, 5, 99], 100) == st.ENOMEM
