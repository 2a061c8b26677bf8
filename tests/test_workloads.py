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
