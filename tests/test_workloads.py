"""Input generators: determinism and CSR well-formedness (no GPU)."""
import numpy as np
import pytest

import workloads as W


def _check_csr(g, wlo, whi, simple=True):
    rp = g.row_ptr.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(g.col) == len(g.w)
    r = g.rows().astype(np.int64)
    c = g.col.astype(np.int64)
    assert np.all(c < g.n)
    # rows sorted strictly (no duplicates) and no self-loops
    same_row = r[1:] == r[:-1]
    assert np.all(c[1:][same_row] > c[:-1][same_row])
    assert not np.any(r == c)
    assert g.w.min() >= wlo and g.w.max() <= whi
    # symmetry with equal weights
    fwd = np.lexsort((c, r))
    bwd = np.lexsort((r, c))
    assert np.array_equal(r[fwd], c[bwd]) and np.array_equal(c[fwd], r[bwd])
    assert np.array_equal(g.w[fwd], g.w[bwd])


def test_er_shape_and_determinism():
    g = W.make_graph("er16k")
    assert g.n == 16384 and g.nnz == 2 * 131072
    _check_csr(g, 1, 100)
    h = W.make_graph("er16k")
    assert np.array_equal(g.col, h.col) and np.array_equal(g.w, h.w)
    other = W.er(16384, 131072, 1, 100, master=2)
    assert not np.array_equal(g.col, other.col)


def test_grid_shape():
    g = W.grid(37, 53, 1, 1000)
    assert g.n == 37 * 53 and g.nnz == 2 * (37 * 52 + 36 * 53)
    _check_csr(g, 1, 1000)
    d = g.degrees()
    assert d.max() == 4 and d.min() == 2


def test_rmat_small():
    g = W.rmat(12, 16, wlo=1, whi=1000)
    _check_csr(g, 1, 1000)
    assert g.nnz <= 2 * 16 * 4096
    d = g.degrees()
    assert d.max() > 20 * np.median(d[d > 0])  # heavy-tailed
    g2 = W.rmat(12, 16, wlo=1, whi=1000)
    assert np.array_equal(g.row_ptr, g2.row_ptr) and np.array_equal(g.col, g2.col)


def test_lcc_and_sampling():
    g = W.from_edges(7, [(0, 1, 1), (1, 2, 1), (3, 4, 1), (5, 6, 1), (4, 5, 1)])
    assert W.lcc(g).tolist() == [3, 4, 5, 6]
    lab = W.components(g)
    assert lab.tolist() == [0, 0, 0, 3, 3, 3, 3]
    cand = np.arange(100, dtype=np.uint32)
    s = W.sample(cand, 30, master=1)
    assert len(set(s.tolist())) == 30
    assert np.array_equal(s, W.sample(cand, 30, master=1))
    with pytest.raises(ValueError):
        W.sample(cand, 101)


def test_query_sizes_log_uniform():
    ks = W.log_uniform_sizes(2000, 3, 4096)
    assert ks.min() >= 3 and ks.max() <= 4096
    # log-uniform: about half the mass below the geometric midpoint
    mid = np.sqrt(3 * 4097)
    assert 0.4 < np.mean(ks < mid) < 0.6
    t = W.poisson_arrivals(1000, rate=50.0)
    assert np.all(np.diff(t) > 0) and 15 < t[-1] < 25


def _py_bfs(g, src):
    from collections import deque
    lv = [None] * g.n
    lv[src] = 0
    q = deque([src])
    while q:
        v = q.popleft()
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            u = int(g.col[e])
            if lv[u] is None:
                lv[u] = lv[v] + 1
                q.append(u)
    return [0xFFFFFFFF if x is None else x for x in lv]


def test_bfs_levels_match_python():
    for g in (W.er(300, 500, 1, 9, 3), W.grid(13, 17, 1, 5, 4), W.rmat(9, 8, wlo=1, whi=9, master=5)):
        for src in (0, g.n // 2, g.n - 1):
            assert W.bfs_levels(g, src).tolist() == _py_bfs(g, src)


def test_kbfs_seed_strategies_by_definition():
    g = W.rmat(9, 8, wlo=1, whi=9, master=6)
    cand = W.lcc(g)
    for mode in ("eccentric", "proximate"):
        s = W.seeds_kbfs(g, 12, mode, master=2, cand=cand)
        assert len(set(s.tolist())) == 12 and set(s.tolist()) <= set(cand.tolist())
        acc = {int(v): 0 for v in cand}
        for i in range(1, 12):  # each further seed extremises the level sum over the seeds before it
            lv = _py_bfs(g, int(s[i - 1]))
            for v in acc:
                acc[v] += lv[v]
            rest = [v for v in acc if v not in set(int(x) for x in s[:i])]
            key = (lambda v: (-acc[v], v)) if mode == "eccentric" else (lambda v: (acc[v], v))
            assert int(s[i]) == min(rest, key=key), (mode, i)
    gg = W.grid(20, 20, 1, 3, 7)
    prox = W.seeds_kbfs(gg, 2, "proximate", master=3)
    assert _py_bfs(gg, int(prox[0]))[int(prox[1])] == 1  # the nearest other vertex is a neighbour
    ecc = W.seeds_kbfs(gg, 2, "eccentric", master=3)
    lv = _py_bfs(gg, int(ecc[0]))
    assert lv[int(ecc[1])] == max(lv)


def test_bfs_level_seeds_follow_level_sizes():
    g = W.grid(40, 50, 1, 9, 8)
    cand = np.arange(g.n, dtype=np.uint32)
    s = W.seeds_bfs_level(g, 60, master=4, cand=cand)
    assert len(s) == 60 and len(set(s.tolist())) == 60
    root = int(W.sample(cand, 1, 4, W.STREAM_SEEDS)[0])
    lv = W.bfs_levels(g, root)
    sizes = np.bincount(lv)
    got = np.bincount(lv[s], minlength=len(sizes))
    assert np.all(np.abs(got - sizes * 60 / g.n) < 1.0 + 1e-9)  # largest-remainder quotas
    assert np.array_equal(W.make_seeds(g, 60, master=4, cand=cand, strategy="bfs_level"), s)
