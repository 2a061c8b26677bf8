"""Pins of the CPU oracle (runs without a GPU)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
import pins


@pytest.fixture(scope="module")
def lib():
    return O.load()


@pytest.fixture(scope="module")
def cases():
    return list(pins.tiny_cases(seed=11, count=240))


def test_voronoi_equals_floyd_warshall(lib, cases):
    pins.check_voronoi(lib, cases)


def test_pred_canonical_and_paths(lib, cases):
    pins.check_pred(lib, cases)


def test_boundary_bruteforce_and_mehlhorn(lib, cases):
    pins.check_boundary(lib, cases)


def test_solve_invariants_and_ratio(lib, cases):
    pins.check_solve(lib, cases)


def test_mst_matches_textbook_kruskal(lib):
    pins.check_mst_direct(lib)


def test_special_cases(lib):
    pins.check_special_cases(lib, seed=3, count=60)


def test_ratio_against_dreyfus_wagner_larger_k(lib):
    """Bound k*D <= 2(k-1)*D_min with k up to 8 on denser graphs."""
    from brute import dreyfus_wagner, check_tree
    rng = np.random.default_rng(5)
    worst = 1.0
    for t in range(25):
        n = int(rng.integers(8, 15))
        g = W.random_small(rng, n, 0.35, 1, 20, connected=True)
        k = int(rng.integers(3, min(8, n) + 1))
        S = rng.choice(n, size=k, replace=False)
        sol = O.solve(g, S, lib)
        assert sol.code == O.OK
        check_tree(g, S, sol.edges, sol.total)
        dmin = dreyfus_wagner(g, S)
        assert k * sol.total <= 2 * (k - 1) * dmin
        worst = max(worst, sol.total / dmin)
    assert worst < 2.0


def test_seed_order_and_duplicates_do_not_matter(lib):
    rng = np.random.default_rng(9)
    for _ in range(20):
        g = W.random_small(rng, 15, 0.3, 1, 2, connected=True)
        S = rng.choice(15, size=6, replace=False)
        base = O.solve(g, S, lib)
        shuffled = np.concatenate([rng.permutation(S), S[:3]])
        again = O.solve(g, shuffled, lib)
        assert base.code == again.code == O.OK
        assert base.edges == again.edges and base.total == again.total


def test_error_codes(lib):
    g = W.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1)])
    assert O.solve(g, np.array([], dtype=np.uint32), lib).code == O.EINVAL
    assert O.solve(g, [0, 4], lib).code == O.EINVAL
    one = O.solve(g, [2, 2, 2], lib)
    assert one.code == O.OK and one.total == 0 and len(one.a) == 0
    # two components
    g2 = W.from_edges(5, [(0, 1, 3), (2, 3, 1), (3, 4, 2)])
    assert O.solve(g2, [0, 4], lib).code == O.EDISCONNECTED
    assert O.solve(g2, [2, 4], lib).code == O.OK
    # zero weight, column out of range, unsorted row
    bad = W.from_edges(3, [(0, 1, 1), (1, 2, 1)])
    bad.w = bad.w.copy()
    bad.w[0] = 0
    assert O.check_graph(bad, lib) == O.EINVAL
    bad = W.from_edges(3, [(0, 1, 1), (1, 2, 1)])
    bad.col = bad.col.copy()
    bad.col[0] = 3
    assert O.check_graph(bad, lib) == O.EINVAL
    bad = W.from_edges(3, [(0, 1, 1), (0, 2, 1)])
    bad.col = bad.col.copy()
    bad.col[[0, 1]] = bad.col[[1, 0]]
    assert O.check_graph(bad, lib) == O.EINVAL
    bad = W.from_edges(3, [(0, 1, 1)])
    bad.row_ptr = bad.row_ptr.copy()
    bad.row_ptr[-1] += 1
    assert O.check_graph(bad, lib) == O.EINVAL


def test_overflow_rules(lib):
    big = 1 << 31
    # distance overflow: vertex 2 is at 2^32 from seed 0
    g = W.from_edges(4, [(0, 1, big), (1, 2, big), (0, 3, 1)])
    assert O.solve(g, [0, 3], lib).code == O.EOVERFLOW
    # largest representable distance 2^32-2 is fine
    g = W.from_edges(2, [(0, 1, 0xFFFFFFFE)])
    dist, src = O.voronoi(g, np.array([0], dtype=np.uint32), lib)
    assert int(dist[1]) == 0xFFFFFFFE and O.check_dist(dist, lib) == O.OK
    g = W.from_edges(2, [(0, 1, 0xFFFFFFFF)])
    dist, _ = O.voronoi(g, np.array([0], dtype=np.uint32), lib)
    assert O.check_dist(dist, lib) == O.EOVERFLOW
    # cross-cell sum overflow with all distances representable:
    # 0 -(2^31)- 1 -(2^31)- 2, seeds {0, 2}; vertex 1 ties and joins cell 0,
    # the cross edge (1,2) sums to 2^31 + 2^31 + 0 = 2^32.
    g = W.from_edges(3, [(0, 1, big), (1, 2, big)])
    assert O.solve(g, [0, 2], lib).code == O.EOVERFLOW
    g = W.from_edges(3, [(0, 1, big - 1), (1, 2, big)])
    sol = O.solve(g, [0, 2], lib)
    assert sol.code == O.OK and sol.total == 2 * big - 1


def test_tie_rules_by_hand(lib):
    """Square 0-1-2-3-0 with unit weights and seeds {0, 2}: vertices 1 and 3
    are equidistant; the smaller seed index (seed 0) takes both.  The cross
    edges (1,2) and (2,3) tie on d1+d+d1 = 2; the smaller edge id, the half
    edge 1->2, is kept, so the tree is 0-1-2."""
    g = W.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1), (0, 3, 1)])
    sol = O.solve(g, [2, 0], lib)
    assert sol.code == O.OK
    assert sol.src.tolist() == [0, 0, 1, 0]
    assert sol.edges == [(0, 1, 1), (1, 2, 1)] and sol.total == 2
