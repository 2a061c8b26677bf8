"""Seeded synthetic inputs shared by the GPU library's tests, the benchmark and
the CPU oracle's tests.

Nothing in this package computes any part of the Steiner-tree method: it makes
graphs (CSR with uint32 weights), draws seed sets, query sizes and arrival
times, and nothing else.  The heavy generators live in ``gen.c`` (OpenMP,
counter-based SplitMix64 draws, so the bytes do not depend on thread count);
tiny graphs for brute-force tests are built here in numpy.

Graph recipes follow the paper's workload shapes (symmetric edges with positive
integer weights drawn from a range, Section V "Graph Datasets"; seeds drawn
from the largest connected component, Section V "Seed Vertex Selection" and
Table V's uniform strategy).  The five named workloads are listed in
``WORKLOADS``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwlgen.so")
_lib = None

# Independent random streams under one master seed.
STREAM_GRAPH, STREAM_WEIGHT, STREAM_PERM, STREAM_SEEDS, STREAM_QSIZE, STREAM_ARRIVAL = 1, 2, 3, 4, 5, 6


def build(verbose: bool = False) -> str:
    """Compile gen.c into libwlgen.so next to this file (always recompiles)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
           "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "gen.c")]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    global _lib
    _lib = None
    return _LIB_PATH


class _WlGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nnz", ctypes.c_uint64),
                ("row_ptr", ctypes.POINTER(ctypes.c_uint64)),
                ("col", ctypes.POINTER(ctypes.c_uint32)),
                ("w", ctypes.POINTER(ctypes.c_uint32))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() or workloads.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    u32, u64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    gp = ctypes.POINTER(_WlGraph)
    lib.wl_draw.restype = u64
    lib.wl_draw.argtypes = [u64, u64]
    lib.wl_stream_key.restype = u64
    lib.wl_stream_key.argtypes = [u64, u64]
    lib.wl_gen_er.restype = gp
    lib.wl_gen_er.argtypes = [u32, u64, u32, u32, u64]
    lib.wl_gen_grid.restype = gp
    lib.wl_gen_grid.argtypes = [u32, u32, u32, u32, u64]
    lib.wl_gen_rmat.restype = gp
    lib.wl_gen_rmat.argtypes = [u32, u32, dbl, dbl, dbl, u32, u32, ctypes.c_int, u64]
    lib.wl_graph_free.restype = None
    lib.wl_graph_free.argtypes = [gp]
    lib.wl_components.restype = None
    lib.wl_components.argtypes = [u32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.wl_lcc.restype = u32
    lib.wl_lcc.argtypes = [u32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.wl_sample.restype = ctypes.c_int
    lib.wl_sample.argtypes = [ctypes.c_void_p, u32, u32, u64, ctypes.c_void_p]
    lib.wl_num_threads.restype = ctypes.c_int
    lib.wl_bfs_levels.restype = None
    lib.wl_bfs_levels.argtypes = [u32, ctypes.c_void_p, ctypes.c_void_p, u32, ctypes.c_void_p]
    lib.wl_kbfs_seeds.restype = ctypes.c_int
    lib.wl_kbfs_seeds.argtypes = [u32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, u32, u32, u32,
                                  ctypes.c_int, ctypes.c_void_p]
    _lib = lib
    return lib


@dataclass
class Graph:
    """Undirected graph as a symmetric CSR (rows sorted by column)."""
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[nnz]
    w: np.ndarray        # uint32[nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def rows(self) -> np.ndarray:
        """Row index of every CSR entry."""
        return np.repeat(np.arange(self.n, dtype=np.uint32), self.degrees())

    def edges(self):
        """Undirected edge list as (a, b, w, e) with a < b, e = CSR offset in row a."""
        r = self.rows()
        keep = r < self.col
        e = np.nonzero(keep)[0]
        return r[keep], self.col[keep], self.w[keep], e


class _Owner:
    def __init__(self, lib, ptr):
        self._lib, self._ptr = lib, ptr

    def __del__(self):
        try:
            self._lib.wl_graph_free(self._ptr)
        except Exception:
            pass


def _wrap(ptr, name: str) -> Graph:
    lib = _load()
    if not ptr:
        raise ValueError(f"generator rejected the parameters for {name}")
    g = ptr.contents
    owner = _Owner(lib, ptr)

    def view(p, count, ctype, dtype):
        if count == 0:
            return np.zeros(0, dtype=dtype)
        arr_t = ctype * count
        buf = arr_t.from_address(ctypes.addressof(p.contents))
        buf._owner = owner
        return np.frombuffer(buf, dtype=dtype)

    row_ptr = view(g.row_ptr, g.n + 1, ctypes.c_uint64, np.uint64)
    col = view(g.col, g.nnz, ctypes.c_uint32, np.uint32)
    w = view(g.w, g.nnz, ctypes.c_uint32, np.uint32)
    return Graph(int(g.n), row_ptr, col, w, name=name)


def stream_key(master: int, stream_id: int) -> int:
    return int(_load().wl_stream_key(master, stream_id))


def draw(key: int, i: int) -> int:
    return int(_load().wl_draw(key, i))


def er(n: int, m: int, wlo: int = 1, whi: int = 100, master: int = 1) -> Graph:
    return _wrap(_load().wl_gen_er(n, m, wlo, whi, master), f"er_n{n}_m{m}_w{wlo}-{whi}_s{master}")


def grid(rows: int, cols: int, wlo: int = 1, whi: int = 1000, master: int = 1) -> Graph:
    return _wrap(_load().wl_gen_grid(rows, cols, wlo, whi, master), f"grid_{rows}x{cols}_w{wlo}-{whi}_s{master}")


def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wlo: int = 1, whi: int = 1000, master: int = 1, permute: bool = True) -> Graph:
    return _wrap(_load().wl_gen_rmat(scale, edgefactor, a, b, c, wlo, whi, int(permute), master),
                 f"rmat{scale}_ef{edgefactor}_w{wlo}-{whi}_s{master}")


def components(g: Graph) -> np.ndarray:
    """Component label (smallest vertex id in the component) of every vertex."""
    lab = np.empty(g.n, dtype=np.uint32)
    _load().wl_components(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, lab.ctypes.data)
    return lab


def lcc(g: Graph) -> np.ndarray:
    """Ascending vertex ids of the largest connected component."""
    out = np.empty(g.n, dtype=np.uint32)
    cnt = _load().wl_lcc(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, out.ctypes.data)
    return out[:cnt].copy()


def sample(cand: np.ndarray, k: int, master: int = 1, stream: int = STREAM_SEEDS) -> np.ndarray:
    """k distinct entries of `cand`, uniform without replacement, in draw order."""
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    out = np.empty(k, dtype=np.uint32)
    if _load().wl_sample(cand.ctypes.data, len(cand), k, stream_key(master, stream), out.ctypes.data) != 0:
        raise ValueError("k exceeds the candidate count")
    return out


def uniforms(count: int, master: int, stream: int, offset: int = 0) -> np.ndarray:
    """count uniforms in [0,1) from the top 53 bits of successive draws."""
    key = stream_key(master, stream)
    lib = _load()
    return np.array([(lib.wl_draw(key, offset + i) >> 11) * (1.0 / (1 << 53)) for i in range(count)])


def log_uniform_sizes(count: int, lo: int, hi: int, master: int = 1, stream: int = STREAM_QSIZE) -> np.ndarray:
    """Seed-set sizes k = floor(exp(U(ln lo, ln(hi+1)))), capped at hi."""
    u = uniforms(count, master, stream)
    k = np.floor(np.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).astype(np.int64)
    return np.minimum(np.maximum(k, lo), hi)


def poisson_arrivals(count: int, rate: float, master: int = 1, stream: int = STREAM_ARRIVAL) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    u = uniforms(count, master, stream)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


# ----------------------------------------------------------------------------
# Tiny graphs for brute-force tests (pure numpy, seeded).
# ----------------------------------------------------------------------------

def from_edges(n: int, edges, name: str = "edges") -> Graph:
    """Symmetric CSR from undirected (u, v, w) triples.  Parallel edges and
    self-loops are kept as given; entries of a row are ordered by (col, w)."""
    us, vs, ws = [], [], []
    for (u, v, w) in edges:
        us.append(u); vs.append(v); ws.append(w)
        if u != v:
            us.append(v); vs.append(u); ws.append(w)
        else:
            us.append(u); vs.append(u); ws.append(w)
    if us:
        src = np.array(us, dtype=np.int64)
        dst = np.array(vs, dtype=np.int64)
        wt = np.array(ws, dtype=np.int64)
        order = np.lexsort((wt, dst, src))
        src, dst, wt = src[order], dst[order], wt[order]
    else:
        src = dst = wt = np.zeros(0, dtype=np.int64)
    counts = np.bincount(src, minlength=n) if len(src) else np.zeros(n, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    row_ptr[1:] = np.cumsum(counts)
    return Graph(n, row_ptr, dst.astype(np.uint32), wt.astype(np.uint32), name=name)


def random_small(rng: np.random.Generator, n: int, p: float, wlo: int = 1, whi: int = 10,
                 multi: float = 0.0, loops: float = 0.0, connected: bool = False) -> Graph:
    """Small G(n,p) graph; with probability `multi` an edge gets a parallel
    copy (own weight), `loops` adds self-loops; `connected` adds a random
    spanning path first."""
    edges = []
    if connected and n > 1:
        perm = rng.permutation(n)
        for i in range(n - 1):
            edges.append((int(perm[i]), int(perm[i + 1]), int(rng.integers(wlo, whi + 1))))
    present = {(min(a, b), max(a, b)) for a, b, _ in edges}
    for u in range(n):
        for v in range(u + 1, n):
            if (u, v) not in present and rng.random() < p:
                edges.append((u, v, int(rng.integers(wlo, whi + 1))))
    extra = []
    for (u, v, _) in edges:
        if rng.random() < multi:
            extra.append((u, v, int(rng.integers(wlo, whi + 1))))
    edges += extra
    for u in range(n):
        if rng.random() < loops:
            edges.append((u, u, int(rng.integers(wlo, whi + 1))))
    return from_edges(n, edges, name=f"small_n{n}")


def random_tree(rng: np.random.Generator, n: int, wlo: int = 1, whi: int = 10) -> Graph:
    edges = [(int(rng.integers(0, v)), v, int(rng.integers(wlo, whi + 1))) for v in range(1, n)]
    perm = rng.permutation(n)
    edges = [(int(perm[a]), int(perm[b]), w) for a, b, w in edges]
    return from_edges(n, edges, name=f"tree_n{n}")


# ----------------------------------------------------------------------------
# The named workloads.
# ----------------------------------------------------------------------------

WORKLOADS = {
    "er16k": dict(kind="er", n=16384, m=131072, wlo=1, whi=100, k=16, seeds_from="lcc"),
    "grid2048": dict(kind="grid", rows=2048, cols=2048, wlo=1, whi=1000, k=100, seeds_from="all"),
    "rmat25": dict(kind="rmat", scale=25, edgefactor=16, wlo=1, whi=1000, k=10000, seeds_from="lcc"),
    "rmat22_batch64": dict(kind="rmat", scale=22, edgefactor=16, wlo=1, whi=1000, queries=64,
                           k_lo=3, k_hi=4096, seeds_from="lcc"),
    "rmat24_serve": dict(kind="rmat", scale=24, edgefactor=16, wlo=1, whi=1000, k_lo=3, k_hi=10000,
                         seeds_from="lcc"),
    # batching where one query leaves the GPU mostly idle (high diameter: latency bound)
    "grid2048_batch32": dict(kind="grid", rows=2048, cols=2048, wlo=1, whi=1000, queries=32, k_lo=10, k_hi=1000,
                             seeds_from="all"),
    # serving where one query leaves the GPU mostly idle
    "grid2048_serve": dict(kind="grid", rows=2048, cols=2048, wlo=1, whi=1000, k_lo=10, k_hi=1000,
                           seeds_from="all"),
}


def make_graph(name: str, master: int = 1, **override) -> Graph:
    spec = dict(WORKLOADS[name], **override)
    if spec["kind"] == "er":
        g = er(spec["n"], spec["m"], spec["wlo"], spec["whi"], master)
    elif spec["kind"] == "grid":
        g = grid(spec["rows"], spec["cols"], spec["wlo"], spec["whi"], master)
    else:
        g = rmat(spec["scale"], spec["edgefactor"], 0.57, 0.19, 0.19, spec["wlo"], spec["whi"], master)
    g.name = name
    g.meta = spec
    return g


def seed_candidates(g: Graph) -> np.ndarray:
    if g.meta.get("seeds_from") == "all":
        return np.arange(g.n, dtype=np.uint32)
    return lcc(g)


def bfs_levels(g: Graph, src: int) -> np.ndarray:
    """Hop counts from src; 0xFFFFFFFF where unreached."""
    out = np.empty(g.n, dtype=np.uint32)
    _load().wl_bfs_levels(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, int(src), out.ctypes.data)
    return out


SEED_STRATEGIES = ("uniform", "bfs_level", "eccentric", "proximate")


def seeds_bfs_level(g: Graph, k: int, master: int = 1, stream: int = STREAM_SEEDS, cand=None) -> np.ndarray:
    """The paper's default seed selection (Section V): BFS levels of the
    candidates from a random root, then a uniform sample from every level
    with quotas proportional to the level sizes (largest remainder), level l
    drawing from stream `stream * 1000 + 1 + l`."""
    if cand is None:
        cand = seed_candidates(g)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    if k > len(cand):
        raise ValueError("k exceeds the candidate count")
    root = int(sample(cand, 1, master, stream)[0])
    lv = bfs_levels(g, root)[cand]
    levels, counts = np.unique(lv, return_counts=True)
    exact = counts * (k / len(cand))
    quota = np.floor(exact).astype(np.int64)
    order = np.lexsort((levels, -(exact - quota)))
    quota[order[:k - int(quota.sum())]] += 1
    out = []
    for l, q in zip(levels, quota):
        if q:
            out.append(sample(cand[lv == l], int(q), master, stream * 1000 + 1 + int(l)))
    return np.concatenate(out).astype(np.uint32)


def seeds_kbfs(g: Graph, k: int, mode: str, master: int = 1, stream: int = STREAM_SEEDS, cand=None) -> np.ndarray:
    """"eccentric" (seeds far apart) or "proximate" (seeds close together):
    the paper's k-BFS seed selection (Section V); the first seed is a uniform
    draw from the candidates, which must lie in one component.  One BFS per
    seed, so meant for modest k."""
    if cand is None:
        cand = seed_candidates(g)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    first = int(sample(cand, 1, master, stream)[0])
    out = np.empty(k, dtype=np.uint32)
    m = {"eccentric": 0, "proximate": 1}[mode]
    if _load().wl_kbfs_seeds(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, cand.ctypes.data, len(cand), first, k, m,
                             out.ctypes.data) != 0:
        raise ValueError("k exceeds the candidate count")
    return out


def make_seeds(g: Graph, k: int, master: int = 1, stream: int = STREAM_SEEDS, cand=None,
               strategy: str = "uniform") -> np.ndarray:
    """k seeds of graph g by one of SEED_STRATEGIES (uniform from the seed
    candidates unless asked otherwise)."""
    if cand is None:
        cand = seed_candidates(g)
    if strategy == "uniform":
        return sample(cand, k, master, stream)
    if strategy == "bfs_level":
        return seeds_bfs_level(g, k, master, stream, cand)
    if strategy in ("eccentric", "proximate"):
        return seeds_kbfs(g, k, strategy, master, stream, cand)
    raise ValueError(f"unknown seed strategy {strategy!r}")


def make_query_set(g: Graph, count: int, k_lo: int, k_hi: int, master: int = 1, cand=None):
    """`count` seed sets with log-uniform sizes; query q uses seed stream 100+q."""
    if cand is None:
        cand = seed_candidates(g)
    ks = log_uniform_sizes(count, k_lo, k_hi, master)
    return [sample(cand, int(min(k, len(cand))), master, 100 + q) for q, k in enumerate(ks)]
