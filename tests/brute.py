"""Brute-force references used to pin the oracle on tiny graphs.

Written independently of both the oracle and the GPU library, from textbook
definitions: Floyd-Warshall all-pairs distances, Dreyfus-Wagner exact Steiner
minimal trees, dense Prim MST, Kruskal MST, iterative leaf pruning, and tree
invariant checks.
"""
from __future__ import annotations

import itertools

import numpy as np

BIG = np.int64(1) << 60  # 'no path'; sums of two stay below 2^63


def adjacency_min(g) -> np.ndarray:
    """n x n matrix of the lightest edge between u and v (BIG if none); self-loops ignored."""
    n = g.n
    A = np.full((n, n), BIG, dtype=np.int64)
    rows = g.rows().astype(np.int64)
    col = g.col.astype(np.int64)
    w = g.w.astype(np.int64)
    for u, v, wt in zip(rows, col, w):
        if u != v and wt < A[u, v]:
            A[u, v] = wt
    return A


def floyd_warshall(g) -> np.ndarray:
    D = adjacency_min(g)
    np.fill_diagonal(D, 0)
    for m in range(g.n):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    return np.minimum(D, BIG)


def voronoi_fw(g, S, D=None):
    """dist[v] = min over seeds of FW distance; src = smallest seed index attaining it."""
    if D is None:
        D = floyd_warshall(g)
    S = np.asarray(S, dtype=np.int64)
    sub = D[S, :]  # k x n
    dist = sub.min(axis=0)
    src = sub.argmin(axis=0)  # first (smallest index) minimiser
    reached = dist < BIG
    return dist, src, reached


def kruskal_weight(k: int, edges) -> tuple[int, int]:
    """Weight and edge count of a minimum spanning forest of (i, j, w) triples."""
    par = list(range(k))

    def f(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    tot = cnt = 0
    for i, j, w in sorted(edges, key=lambda t: (t[2], t[0], t[1])):
        a, b = f(i), f(j)
        if a != b:
            par[a] = b
            tot += w
            cnt += 1
    return tot, cnt


def prim_dense_weight(M: np.ndarray) -> int:
    """MST weight of a complete graph given as a dense symmetric matrix (Prim)."""
    k = M.shape[0]
    if k <= 1:
        return 0
    in_tree = np.zeros(k, dtype=bool)
    in_tree[0] = True
    best = M[0].copy()
    tot = 0
    for _ in range(k - 1):
        cand = np.where(in_tree, BIG, best)
        j = int(np.argmin(cand))
        tot += int(cand[j])
        in_tree[j] = True
        best = np.minimum(best, M[j])
    return tot


def dreyfus_wagner(g, S) -> int:
    """Exact Steiner minimal tree weight D_min (Dreyfus & Wagner 1971)."""
    D = floyd_warshall(g)
    S = list(S)
    k = len(S)
    if k <= 1:
        return 0
    n = g.n
    full = (1 << k) - 1
    dp = np.full((1 << k, n), BIG, dtype=np.int64)
    for i, s in enumerate(S):
        dp[1 << i] = D[s]
    for mask in range(1, full + 1):
        if mask & (mask - 1) == 0:
            continue
        best = np.full(n, BIG, dtype=np.int64)
        sub = (mask - 1) & mask
        while sub:
            if sub < (mask ^ sub):  # each split once
                best = np.minimum(best, dp[sub] + dp[mask ^ sub])
            sub = (sub - 1) & mask
        # dp[mask][v] = min_u best[u] + D[u][v]
        dp[mask] = np.minimum((np.minimum(best, BIG)[:, None] + D).min(axis=0), BIG)
    return int(dp[full].min())


def prune_tree_to_seeds(n: int, edges, S) -> int:
    """Weight of the minimal subtree of a tree spanning S (repeatedly drop non-seed leaves)."""
    S = set(int(s) for s in S)
    adj = {v: {} for v in range(n)}
    for a, b, w in edges:
        adj[a][b] = w
        adj[b][a] = w
    changed = True
    while changed:
        changed = False
        for v in list(adj):
            if v not in S and len(adj[v]) <= 1:
                for u in adj[v]:
                    del adj[u][v]
                del adj[v]
                changed = True
    return sum(w for a in adj for b, w in adj[a].items() if a < b)


def check_tree(g, S, edges, total: int) -> None:
    """Tree invariants: every edge exists in G with that weight; acyclic; connected;
    spans all seeds; every leaf is a seed; |E| = |V| - 1; D = sum of weights."""
    S = sorted(set(int(s) for s in S))
    assert total == sum(w for _, _, w in edges)
    if len(S) <= 1:
        assert edges == []
        return
    have = {}
    for u, v, w in zip(g.rows().tolist(), g.col.tolist(), g.w.tolist()):
        have.setdefault((u, v), set()).add(w)
    verts = set()
    seen = set()
    for a, b, w in edges:
        assert a < b, "edges are reported with a < b"
        assert (a, b) not in seen, "duplicate edge"
        seen.add((a, b))
        assert w in have.get((a, b), set()), f"edge ({a},{b},{w}) not in G"
        verts.update((a, b))
    assert set(S) <= verts
    assert len(edges) == len(verts) - 1
    # connectivity via union-find
    par = {v: v for v in verts}

    def f(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    for a, b, _ in edges:
        ra, rb = f(a), f(b)
        assert ra != rb, "cycle"
        par[ra] = rb
    assert len({f(v) for v in verts}) == 1
    deg = {v: 0 for v in verts}
    for a, b, _ in edges:
        deg[a] += 1
        deg[b] += 1
    for v, d in deg.items():
        if d == 1:
            assert v in S, f"leaf {v} is not a seed"


def all_subsets(seq, kmin=1, kmax=None):
    kmax = len(seq) if kmax is None else kmax
    for r in range(kmin, kmax + 1):
        yield from itertools.combinations(seq, r)
