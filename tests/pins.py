"""Checks that pin the CPU oracle to facts it does not compute itself.

Each check takes a loaded oracle library (the real one, or a deliberately
broken copy in the mutation test) and raises AssertionError on a mismatch.
References: Floyd-Warshall distances, brute-force minima over edges by
definition, Mehlhorn's theorem (every MST of G'1 is an MST of G1, Section II),
the KMB/Mehlhorn 2(1-1/l) bound against exact Dreyfus-Wagner trees
(Section I, Section III), and closed-form special cases: k = 2 gives a
shortest path, k = n gives the MST of G, a tree graph gives its minimal
subtree spanning S.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import workloads as W
from brute import (BIG, check_tree, dreyfus_wagner, floyd_warshall, kruskal_weight, prim_dense_weight,
                   prune_tree_to_seeds, voronoi_fw)


def tiny_cases(seed: int, count: int, nmax: int = 18):
    """Seeded tiny graphs with seed sets, mixing tie-heavy weights,
    multigraphs, self-loops and disconnected pieces."""
    rng = np.random.default_rng(seed)
    for t in range(count):
        n = int(rng.integers(2, nmax + 1))
        style = t % 6
        if style == 0:
            g = W.random_small(rng, n, 0.3, 1, 10, connected=True)
        elif style == 1:
            g = W.random_small(rng, n, 0.35, 1, 1, connected=True)  # all weights 1: maximal ties
        elif style == 2:
            g = W.random_small(rng, n, 0.3, 1, 2, multi=0.3, loops=0.2, connected=True)
        elif style == 3:
            g = W.random_small(rng, n, 0.15, 1, 5)  # may be disconnected
        elif style == 4:
            g = W.random_tree(rng, n, 1, 3)
        else:
            g = W.random_small(rng, n, 0.5, 1, 3, multi=0.2, connected=True)
        k = int(rng.integers(1, n + 1))
        seeds = rng.choice(n, size=k, replace=False).astype(np.uint32)
        yield g, seeds


def check_voronoi(lib, cases) -> None:
    """dist/src equal Floyd-Warshall's min over seeds with the smaller-index tie rule."""
    for g, seeds in cases:
        rc, S = O.canon_seeds(g.n, seeds, lib)
        assert rc == O.OK
        dist, src = O.voronoi(g, S, lib)
        fd, fs, reached = voronoi_fw(g, S)
        assert np.array_equal(dist != O.DIST_INF, reached)
        assert np.array_equal(dist[reached].astype(np.int64), fd[reached])
        assert np.array_equal(src[reached].astype(np.int64), fs[reached])
        assert np.all(src[~reached] == O.IDX_NONE)


def check_pred(lib, cases) -> None:
    """pred is the first in-cell shortest-path neighbour in row order (checked
    against Floyd-Warshall distances), and following pred from any reached
    vertex reaches its own seed with total weight dist(v)."""
    for g, seeds in cases:
        _, S = O.canon_seeds(g.n, seeds, lib)
        dist, src = O.voronoi(g, S, lib)
        pr = O.pred(g, S, dist, src, lib)
        fd, fs, reached = voronoi_fw(g, S)
        seedset = {int(s): i for i, s in enumerate(S)}
        rp = g.row_ptr.astype(np.int64)
        for v in range(g.n):
            if not reached[v]:
                assert pr[v] == O.IDX_NONE
                continue
            if v in seedset:
                assert pr[v] == v
                continue
            want = None
            for e in range(rp[v], rp[v + 1]):
                u = int(g.col[e])
                if reached[u] and fs[u] == fs[v] and fd[u] + int(g.w[e]) == fd[v]:
                    want = u
                    break
            assert want is not None and int(pr[v]) == want
            x, acc, steps = v, 0, 0
            while x not in seedset:
                p = int(pr[x])
                assert fs[p] == fs[v]
                acc += int(fd[x] - fd[p])
                x = p
                steps += 1
                assert steps <= g.n
            assert int(S[fs[v]]) == x and acc == fd[v]


def brute_boundary(g, S, fd, fs, reached):
    best = {}
    rp = g.row_ptr.astype(np.int64)
    for a in range(g.n):
        for e in range(rp[a], rp[a + 1]):
            b = int(g.col[e])
            if a < b and reached[a] and reached[b] and fs[a] != fs[b]:
                i, j = sorted((int(fs[a]), int(fs[b])))
                cand = (int(fd[a]) + int(g.w[e]) + int(fd[b]), e)
                if (i, j) not in best or cand < best[(i, j)]:
                    best[(i, j)] = cand
    return best


def check_boundary(lib, cases) -> None:
    """G'1 equals the per-pair minimum of (d1 + d + d1, edge id) over all
    cross-cell edges, computed by brute force from Floyd-Warshall distances;
    and Mehlhorn's theorem: MST weight of G'1 == MST weight of G1 (the
    complete distance graph on the seeds, KMB step 1)."""
    for g, seeds in cases:
        _, S = O.canon_seeds(g.n, seeds, lib)
        k = len(S)
        dist, src = O.voronoi(g, S, lib)
        rc, pi, pj, pb, pe = O.boundary(g, dist, src, k, lib)
        assert rc == O.OK
        D = floyd_warshall(g)
        fd, fs, reached = voronoi_fw(g, S, D)
        best = brute_boundary(g, S, fd, fs, reached)
        got = {(int(i), int(j)): (int(b), int(e)) for i, j, b, e in zip(pi, pj, pb, pe)}
        assert got == best
        # Mehlhorn's theorem on the seeds' own component structure.
        G1 = D[np.ix_(S.astype(np.int64), S.astype(np.int64))]
        w1, c1 = kruskal_weight(k, [(i, j, int(G1[i, j])) for i in range(k) for j in range(i + 1, k)
                                    if G1[i, j] < BIG])
        w2, c2 = kruskal_weight(k, [(i, j, b) for (i, j), (b, _) in best.items()])
        assert (w1, c1) == (w2, c2)
        if c1 == k - 1:
            assert prim_dense_weight(G1) == w2


def check_solve(lib, cases, dw_kmax: int = 6, dw_nmax: int = 14) -> None:
    """End-to-end: tree invariants, D <= MST(G1) <= 2(1-1/k) D_min (exact
    Dreyfus-Wagner on small instances), EDISCONNECTED exactly when the seeds
    span several components."""
    for g, seeds in cases:
        sol = O.solve(g, seeds, lib)
        _, S = O.canon_seeds(g.n, seeds, lib)
        k = len(S)
        D = floyd_warshall(g)
        G1 = D[np.ix_(S.astype(np.int64), S.astype(np.int64))]
        connected = bool(np.all(G1 < BIG))
        if k == 1:
            assert sol.code == O.OK and sol.total == 0 and len(sol.a) == 0
            continue
        if not connected:
            assert sol.code == O.EDISCONNECTED
            continue
        assert sol.code == O.OK
        check_tree(g, S, sol.edges, sol.total)
        mst1 = prim_dense_weight(G1)
        assert sol.total <= mst1
        if k <= dw_kmax and g.n <= dw_nmax:
            dmin = dreyfus_wagner(g, S)
            assert dmin <= sol.total
            assert k * sol.total <= 2 * (k - 1) * dmin


def check_mst_direct(lib, seed: int = 4, count: int = 200) -> None:
    """oracle_mst on shuffled, tie-heavy G'1 lists picks exactly the pairs a
    textbook Kruskal picks under the strict order (weight, i, j)."""
    rng = np.random.default_rng(seed)
    for _ in range(count):
        k = int(rng.integers(2, 12))
        pairs = [(i, j) for i in range(k) for j in range(i + 1, k) if rng.random() < 0.6]
        pairs += [(i, i + 1) for i in range(k - 1) if rng.random() < 0.5 and (i, i + 1) not in pairs]
        rng.shuffle(pairs)
        ws = rng.integers(1, 4, size=len(pairs))
        pi = np.array([p[0] for p in pairs], dtype=np.uint32)
        pj = np.array([p[1] for p in pairs], dtype=np.uint32)
        pb = ws.astype(np.uint64)
        rc, ch = O.mst(k, pi, pj, pb, lib)
        par = list(range(k))

        def f(x):
            while par[x] != x:
                par[x] = par[par[x]]
                x = par[x]
            return x

        want = []
        for (i, j), w in sorted(zip(pairs, ws.tolist()), key=lambda t: (t[1], t[0][0], t[0][1])):
            a, b = f(i), f(j)
            if a != b:
                par[a] = b
                want.append((i, j))
        got = sorted((int(pi[c]), int(pj[c])) for c in ch)
        assert got == sorted(want)
        assert rc == (O.OK if len(want) == k - 1 else O.EDISCONNECTED)


def check_special_cases(lib, seed: int = 7, count: int = 30) -> None:
    """k = 2: a shortest path of weight FW(s0, s1).  k = n: the MST of G under
    the order (w, a, b).  G a tree: the minimal subtree spanning S."""
    rng = np.random.default_rng(seed)
    for t in range(count):
        n = int(rng.integers(3, 16))
        g = W.random_small(rng, n, 0.4, 1, 3 if t % 2 else 1, connected=True, multi=0.2 if t % 3 == 0 else 0.0)
        D = floyd_warshall(g)
        # k = 2
        s = rng.choice(n, size=2, replace=False)
        sol = O.solve(g, s, lib)
        assert sol.code == O.OK and sol.total == int(D[s[0], s[1]])
        deg = {}
        for a, b, _ in sol.edges:
            deg[a] = deg.get(a, 0) + 1
            deg[b] = deg.get(b, 0) + 1
        assert all(d <= 2 for d in deg.values())
        # k = n: textbook Kruskal on (w, a, b) over the lightest parallel edge
        sol = O.solve(g, np.arange(n), lib)
        A = {}
        for a, b, w in zip(g.rows().tolist(), g.col.tolist(), g.w.tolist()):
            if a < b and ((a, b) not in A or w < A[(a, b)]):
                A[(a, b)] = w
        par = list(range(n))

        def f(x):
            while par[x] != x:
                par[x] = par[par[x]]
                x = par[x]
            return x

        mst = []
        for (a, b), w in sorted(A.items(), key=lambda kv: (kv[1], kv[0][0], kv[0][1])):
            ra, rb = f(a), f(b)
            if ra != rb:
                par[ra] = rb
                mst.append((a, b, w))
        assert sol.code == O.OK and sol.edges == sorted(mst)
        # tree graph
        tg = W.random_tree(rng, n, 1, 4)
        k = int(rng.integers(2, n + 1))
        S = rng.choice(n, size=k, replace=False)
        sol = O.solve(tg, S, lib)
        tedges = [(int(a), int(b), int(w)) for a, b, w, _ in zip(*tg.edges())]
        assert sol.code == O.OK and sol.total == prune_tree_to_seeds(n, tedges, S)


def run_all(lib, seed: int = 1, count: int = 60) -> None:
    cases = list(tiny_cases(seed, count))
    check_voronoi(lib, cases)
    check_pred(lib, cases)
    check_boundary(lib, cases)
    check_solve(lib, cases)
    check_mst_direct(lib)
    check_special_cases(lib)
