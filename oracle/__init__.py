"""CPU oracle for the Voronoi-cell 2-approximation Steiner tree (arXiv:2205.14503,
Alg. 2 with Mehlhorn's distance graph, Section II).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the GPU library (``paper_2205_14503_amd``) and neither imports the other.

The arithmetic lives in ``oracle.c`` (plain sequential C, one function per
step of Alg. 2); this module only marshals numpy arrays through ctypes.

Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
Floyd-Warshall distances, exact Dreyfus-Wagner Steiner trees, Mehlhorn's
theorem, closed-form special cases and tree invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EDISCONNECTED, EOVERFLOW = 0, -1, -2, -3, -4
CODE_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDISCONNECTED: "EDISCONNECTED",
              EOVERFLOW: "EOVERFLOW"}
DIST_INF = np.uint64(0xFFFFFFFFFFFFFFFF)
IDX_NONE = np.uint32(0xFFFFFFFF)


def build(src: str | None = None, out: str | None = None, verbose: bool = False) -> str:
    """Compile oracle.c (or another source, for mutation tests) to a shared library."""
    src = src or os.path.join(_HERE, "oracle.c")
    out = out or _LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", out + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    global _lib
    if out == _LIB_PATH:
        _lib = None
    return out


def _bind(lib):
    vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    sigs = {
        "oracle_check_graph": [u32, u64, vp, vp, vp],
        "oracle_canon_seeds": [u32, vp, u32, vp, vp],
        "oracle_voronoi": [u32, vp, vp, vp, u32, vp, vp, vp],
        "oracle_pred": [u32, vp, vp, vp, u32, vp, vp, vp, vp],
        "oracle_check_dist": [u32, vp],
        "oracle_boundary": [u32, vp, vp, vp, vp, vp, u64, vp, vp, vp, vp, vp],
        "oracle_mst": [u32, u64, vp, vp, vp, vp, vp],
        "oracle_expand": [u32, vp, vp, vp, u32, vp, vp, vp, vp, u32, vp, u64, vp, vp, vp, vp, vp],
        "oracle_solve": [u32, vp, vp, vp, vp, u32, vp, vp, vp, vp, vp, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None if name == "oracle_pred" else ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load the compiled oracle (the default build, or an explicit path)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run oracle.build()")
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data


def _csr(g):
    return (np.ascontiguousarray(g.row_ptr, dtype=np.uint64), np.ascontiguousarray(g.col, dtype=np.uint32),
            np.ascontiguousarray(g.w, dtype=np.uint32))


def check_graph(g, lib=None) -> int:
    lib = lib or load()
    rp, col, w = _csr(g)
    return lib.oracle_check_graph(g.n, int(rp[-1]), _p(rp), _p(col), _p(w))


def canon_seeds(n: int, seeds, lib=None):
    lib = lib or load()
    s = np.ascontiguousarray(seeds, dtype=np.uint32)
    out = np.empty(max(len(s), 1), dtype=np.uint32)
    kk = np.zeros(1, dtype=np.uint32)
    rc = lib.oracle_canon_seeds(n, _p(s), len(s), _p(out), _p(kk))
    return rc, out[: int(kk[0])].copy()


def voronoi(g, S, lib=None):
    lib = lib or load()
    rp, col, w = _csr(g)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    dist = np.empty(g.n, dtype=np.uint64)
    src = np.empty(g.n, dtype=np.uint32)
    rc = lib.oracle_voronoi(g.n, _p(rp), _p(col), _p(w), len(S), _p(S), _p(dist), _p(src))
    if rc:
        raise MemoryError("oracle_voronoi")
    return dist, src


def pred(g, S, dist, src, lib=None):
    lib = lib or load()
    rp, col, w = _csr(g)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    out = np.empty(g.n, dtype=np.uint32)
    lib.oracle_pred(g.n, _p(rp), _p(col), _p(w), len(S), _p(S), _p(dist), _p(src), _p(out))
    return out


def check_dist(dist, lib=None) -> int:
    lib = lib or load()
    dist = np.ascontiguousarray(dist, dtype=np.uint64)
    return lib.oracle_check_dist(len(dist), _p(dist))


def boundary(g, dist, src, k: int, lib=None):
    """(rc, i, j, bsum, e) sorted by (i, j)."""
    lib = lib or load()
    rp, col, w = _csr(g)
    cap = max(1, min(k * (k - 1) // 2, g.nnz // 2 + 1))
    pi = np.empty(cap, dtype=np.uint32)
    pj = np.empty(cap, dtype=np.uint32)
    pb = np.empty(cap, dtype=np.uint64)
    pe = np.empty(cap, dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_boundary(g.n, _p(rp), _p(col), _p(w), _p(dist), _p(src), cap, _p(pi), _p(pj), _p(pb),
                             _p(pe), _p(cnt))
    m = int(cnt[0]) if rc == OK else 0
    return rc, pi[:m].copy(), pj[:m].copy(), pb[:m].copy(), pe[:m].copy()


def mst(k: int, pi, pj, pb, lib=None):
    """(rc, chosen positions in the G'1 list, in Kruskal acceptance order)."""
    lib = lib or load()
    pi = np.ascontiguousarray(pi, dtype=np.uint32)
    pj = np.ascontiguousarray(pj, dtype=np.uint32)
    pb = np.ascontiguousarray(pb, dtype=np.uint64)
    ch = np.empty(max(k, 1), dtype=np.uint32)
    nch = np.zeros(1, dtype=np.uint32)
    rc = lib.oracle_mst(k, len(pi), _p(pi), _p(pj), _p(pb), _p(ch), _p(nch))
    return rc, ch[: int(nch[0])].copy()


def expand(g, S, dist, src, pred_, sel_e, lib=None):
    """(rc, a, b, w, D) for the selected cross-cell edge ids."""
    lib = lib or load()
    rp, col, w = _csr(g)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    sel = np.ascontiguousarray(sel_e, dtype=np.uint32)
    cap = g.n
    oa = np.empty(cap, dtype=np.uint32)
    ob = np.empty(cap, dtype=np.uint32)
    ow = np.empty(cap, dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_expand(g.n, _p(rp), _p(col), _p(w), len(S), _p(S), _p(dist), _p(src), _p(pred_), len(sel),
                           _p(sel), cap, _p(oa), _p(ob), _p(ow), _p(cnt), _p(tot))
    m = int(cnt[0])
    return rc, oa[:m].copy(), ob[:m].copy(), ow[:m].copy(), int(tot[0])


@dataclass
class Solution:
    code: int
    a: np.ndarray
    b: np.ndarray
    w: np.ndarray
    total: int
    dist: np.ndarray
    src: np.ndarray
    pred: np.ndarray

    @property
    def edges(self):
        return list(zip(self.a.tolist(), self.b.tolist(), self.w.tolist()))


def solve(g, seeds, lib=None) -> Solution:
    """Alg. 2 end to end.  For k == 1 (after deduplication) the per-vertex
    arrays are left unfilled (no Voronoi pass runs)."""
    lib = lib or load()
    rp, col, w = _csr(g)
    s = np.ascontiguousarray(seeds, dtype=np.uint32)
    dist = np.full(g.n, DIST_INF, dtype=np.uint64)
    src = np.full(g.n, IDX_NONE, dtype=np.uint32)
    pr = np.full(g.n, IDX_NONE, dtype=np.uint32)
    cap = g.n
    oa = np.empty(cap, dtype=np.uint32)
    ob = np.empty(cap, dtype=np.uint32)
    ow = np.empty(cap, dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.uint64)
    rc = lib.oracle_solve(g.n, _p(rp), _p(col), _p(w), _p(s), len(s), _p(dist), _p(src), _p(pr), _p(oa), _p(ob),
                          _p(ow), _p(cnt), _p(tot))
    m = int(cnt[0]) if rc == OK else 0
    return Solution(rc, oa[:m].copy(), ob[:m].copy(), ow[:m].copy(), int(tot[0]) if rc == OK else 0, dist, src, pr)


def packed_key(dist, src):
    """(dist << 32) | src with all-ones for unreached: the 64-bit vertex key form."""
    dist = np.asarray(dist, dtype=np.uint64)
    src = np.asarray(src, dtype=np.uint64)
    key = (dist << np.uint64(32)) | src
    key[dist == DIST_INF] = DIST_INF
    return key
