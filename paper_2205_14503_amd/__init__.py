"""MI355X (gfx950) Voronoi-cell 2-approximation Steiner trees (arXiv:2205.14503).

Thin ctypes binding over ``libsteiner.so`` (declared in ``include/steiner.h``):
the functions named ``steiner_*`` below mirror the C entry points one to one
and only marshal arguments; every step of the method runs in the library's HIP
kernels and host engine.  PyTorch is used for device memory and streams only
(``torch`` is imported first so the library binds to the HIP runtime torch
loaded).  There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

try:  # the HIP runtime must be the one torch uses
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsteiner.so")

OK, EINVAL, ENOMEM, EDISCONNECTED, EOVERFLOW, EDEVICE, ETIMEDOUT, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
CODE_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDISCONNECTED: "EDISCONNECTED",
              EOVERFLOW: "EOVERFLOW", EDEVICE: "EDEVICE", ETIMEDOUT: "ETIMEDOUT", ECANCELED: "ECANCELED"}
FLAG_TIMING = 1
FLAG_COUNTERS = 2
FLAG_SPLIT = 4
FLAG_LAZY_PRED = 8
FLAG_EAGER_PRED = 16
FLAG_DEFER = 32
FLAG_NO_DEFER = 64
MAX_SEEDS = 92682
UPLOAD_SYMMETRY = 1
UPLOAD_REORDER = 2
UPLOAD_KEEP_ORDER = 4
DRIVER_DEFAULT, DRIVER_HOST, DRIVER_PERSISTENT = 0, 1, 2

EXPORTS = [
    "steiner_graph_upload", "steiner_graph_upload_device", "steiner_graph_free", "steiner_graph_tune", "steiner_solve",
    "steiner_solve_noalloc", "steiner_solve_batch", "steiner_result_edges", "steiner_result_total", "steiner_result_stats",
    "steiner_result_free", "steiner_voronoi", "steiner_boundary", "steiner_server_create",
    "steiner_server_submit", "steiner_server_wait", "steiner_server_query_bytes", "steiner_server_memory",
    "steiner_server_destroy",
    "steiner_strerror", "steiner_last_error",
]


class SteinerError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class steiner_options(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in
                ("delta", "driver", "block", "grid", "small_max", "chunk", "flags", "local_iters")]


class steiner_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in
                ("rounds", "advances", "pairs", "tree_edges", "relax_launches", "reserved")] + [
        (name, ctypes.c_double) for name in
        ("ms_init", "ms_voronoi", "ms_scan", "ms_compact", "ms_mst", "ms_expand", "ms_total", "ms_relax_kernels")] + [
        (name, ctypes.c_uint64) for name in
        ("relax_attempts", "relax_atomics", "relax_improved", "pushes_local", "pushes_next", "parked", "items",
         "scan_entries", "scan_gathers", "scan_candidates", "scan_atomics", "relax_attempts_large")]


_lib = None


def load(path: str | None = None):
    """Load libsteiner.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, u32, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
    sigs = {
        "steiner_graph_upload": (i32, [u32, u64, vp, vp, vp, i32, vp, u32, vp]),
        "steiner_graph_upload_device": (i32, [u32, u64, vp, vp, vp, i32, vp, u32, vp]),
        "steiner_graph_free": (i32, [vp]),
        "steiner_graph_tune": (i32, [vp, vp, u32, vp]),
        "steiner_solve": (i32, [vp, vp, u32, vp, vp]),
        "steiner_solve_noalloc": (i32, [vp, vp, u32, vp, u64, vp, vp, vp, vp, vp]),
        "steiner_solve_batch": (i32, [vp, u32, vp, vp, vp, vp, vp]),
        "steiner_result_edges": (i32, [vp, vp, vp, vp, vp]),
        "steiner_result_total": (u64, [vp]),
        "steiner_result_stats": (i32, [vp, vp]),
        "steiner_result_free": (None, [vp]),
        "steiner_voronoi": (i32, [vp, vp, u32, vp, vp, vp]),
        "steiner_boundary": (i32, [vp, vp, u32, vp, vp, vp, vp, vp, u64]),
        "steiner_server_create": (i32, [vp, u64, u32, vp, vp]),
        "steiner_server_submit": (i32, [vp, vp, u32, vp]),
        "steiner_server_wait": (i32, [vp, u64, i64, vp]),
        "steiner_server_query_bytes": (u64, [vp, u32]),
        "steiner_server_memory": (i32, [vp, vp, vp, vp, vp]),
        "steiner_server_destroy": (i32, [vp]),
        "steiner_strerror": (ctypes.c_char_p, [i32]),
        "steiner_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise SteinerError(rc, load().steiner_last_error().decode(errors="replace"))


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _opts(options) -> ctypes.c_void_p | None:
    if options is None:
        return None
    if isinstance(options, dict):
        o = steiner_options(**options)
    else:
        o = options
    return ctypes.cast(ctypes.pointer(o), ctypes.c_void_p), o


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


# ------------------------------------------------------ C entry points

def steiner_graph_upload(n, row_ptr, col, w, device: int = 0, stream=None, flags: int = 0) -> int:
    """Upload host arrays; returns the graph handle (int)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    c = _u32(col)
    ww = _u32(w)
    out = ctypes.c_void_p()
    _check(load().steiner_graph_upload(n, int(rp[-1]), rp.ctypes.data, c.ctypes.data, ww.ctypes.data, device,
                                       _stream_ptr(stream), flags, ctypes.byref(out)))
    return out.value


def steiner_graph_upload_device(n, row_ptr_t, col_t, w_t, device: int = 0, stream=None, flags: int = 0) -> int:
    """Upload from torch device tensors (int64 row_ptr, int32 col and w, contiguous)."""
    out = ctypes.c_void_p()
    nnz = int(col_t.numel())
    _check(load().steiner_graph_upload_device(n, nnz, row_ptr_t.data_ptr(), col_t.data_ptr(), w_t.data_ptr(),
                                              device, _stream_ptr(stream), flags, ctypes.byref(out)))
    return out.value


def steiner_graph_free(g: int) -> None:
    _check(load().steiner_graph_free(g))


def steiner_graph_tune(g: int, seeds) -> dict:
    """Pick the graph's default relaxation settings on a sample seed set."""
    s = _u32(seeds)
    o = steiner_options()
    _check(load().steiner_graph_tune(g, s.ctypes.data if len(s) else None, len(s), ctypes.byref(o)))
    return {name: getattr(o, name) for name, _ in steiner_options._fields_}


@dataclass
class Tree:
    a: np.ndarray
    b: np.ndarray
    w: np.ndarray
    total: int
    stats: dict

    @property
    def edges(self):
        return list(zip(self.a.tolist(), self.b.tolist(), self.w.tolist()))


def steiner_result_edges(r: int):
    """(a, b, w) copies of a result's edge arrays."""
    m = ctypes.c_uint64()
    pa, pb, pw = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    _check(load().steiner_result_edges(r, ctypes.byref(m), ctypes.byref(pa), ctypes.byref(pb), ctypes.byref(pw)))
    cnt = m.value

    def arr(p):
        if cnt == 0:
            return np.zeros(0, dtype=np.uint32)
        return np.ctypeslib.as_array((ctypes.c_uint32 * cnt).from_address(p.value)).copy()

    return arr(pa), arr(pb), arr(pw)


def steiner_result_total(r: int) -> int:
    return int(load().steiner_result_total(r))


def steiner_result_stats(r: int) -> dict:
    st = steiner_stats()
    _check(load().steiner_result_stats(r, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in steiner_stats._fields_}


def steiner_result_free(r: int) -> None:
    load().steiner_result_free(r)


def _take_result(r: int) -> Tree:
    a, b, w = steiner_result_edges(r)
    tree = Tree(a, b, w, steiner_result_total(r), steiner_result_stats(r))
    steiner_result_free(r)
    return tree


def steiner_solve(g: int, seeds, options=None) -> Tree:
    s = _u32(seeds)
    out = ctypes.c_void_p()
    o = _opts(options)
    _check(load().steiner_solve(g, s.ctypes.data if len(s) else None, len(s), o[0] if o else None,
                                ctypes.byref(out)))
    return _take_result(out.value)


NOALLOC_SCRATCH_BYTES = 256 << 20


def steiner_solve_noalloc(g: int, seeds, cap: int, options=None) -> Tree:
    """steiner_solve without allocation inside the library: the tree lands in
    host arrays of capacity `cap` allocated here by the caller's side."""
    s = _u32(seeds)
    a = np.empty(max(cap, 1), dtype=np.uint32)
    b = np.empty(max(cap, 1), dtype=np.uint32)
    w = np.empty(max(cap, 1), dtype=np.uint32)
    m = ctypes.c_uint64()
    tot = ctypes.c_uint64()
    o = _opts(options)
    _check(load().steiner_solve_noalloc(g, s.ctypes.data if len(s) else None, len(s), o[0] if o else None, cap,
                                        ctypes.byref(m), a.ctypes.data, b.ctypes.data, w.ctypes.data,
                                        ctypes.byref(tot)))
    k = m.value
    return Tree(a[:k].copy(), b[:k].copy(), w[:k].copy(), tot.value, {})


def steiner_solve_batch(g: int, seed_sets, options=None):
    """Returns a list of (status, Tree or None)."""
    sets = [_u32(s) for s in seed_sets]
    q = len(sets)
    ptrs = (ctypes.c_void_p * q)(*[s.ctypes.data if len(s) else None for s in sets])
    ks = (ctypes.c_uint32 * q)(*[len(s) for s in sets])
    outs = (ctypes.c_void_p * q)()
    st = (ctypes.c_int * q)()
    o = _opts(options)
    _check(load().steiner_solve_batch(g, q, ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(ks, ctypes.c_void_p),
                                      o[0] if o else None, ctypes.cast(outs, ctypes.c_void_p),
                                      ctypes.cast(st, ctypes.c_void_p)))
    res = []
    for i in range(q):
        res.append((st[i], _take_result(outs[i]) if st[i] == OK else None))
    return res


def steiner_voronoi(g: int, n: int, seeds, options=None):
    """(key u64[n], pred u32[n])."""
    s = _u32(seeds)
    key = np.empty(n, dtype=np.uint64)
    pred = np.empty(n, dtype=np.uint32)
    o = _opts(options)
    _check(load().steiner_voronoi(g, s.ctypes.data if len(s) else None, len(s), o[0] if o else None,
                                  key.ctypes.data, pred.ctypes.data))
    return key, pred


def steiner_boundary(g: int, seeds, cap: int, options=None):
    """(i, j, packed) of G'1 sorted by (i, j)."""
    s = _u32(seeds)
    cap = max(int(cap), 1)
    pi = np.empty(cap, dtype=np.uint32)
    pj = np.empty(cap, dtype=np.uint32)
    pk = np.empty(cap, dtype=np.uint64)
    m = ctypes.c_uint64()
    o = _opts(options)
    _check(load().steiner_boundary(g, s.ctypes.data if len(s) else None, len(s), o[0] if o else None,
                                   ctypes.byref(m), pi.ctypes.data, pj.ctypes.data, pk.ctypes.data, cap))
    k = m.value
    return pi[:k].copy(), pj[:k].copy(), pk[:k].copy()


def steiner_server_create(g: int, mem_budget_bytes: int, max_slots: int, options=None) -> int:
    out = ctypes.c_void_p()
    o = _opts(options)
    _check(load().steiner_server_create(g, mem_budget_bytes, max_slots, o[0] if o else None, ctypes.byref(out)))
    return out.value


def steiner_server_submit(s: int, seeds) -> int:
    a = _u32(seeds)
    t = ctypes.c_uint64()
    _check(load().steiner_server_submit(s, a.ctypes.data if len(a) else None, len(a), ctypes.byref(t)))
    return t.value


def steiner_server_wait(s: int, ticket: int, timeout_us: int = -1) -> Tree:
    out = ctypes.c_void_p()
    _check(load().steiner_server_wait(s, ticket, timeout_us, ctypes.byref(out)))
    return _take_result(out.value)


def steiner_server_query_bytes(s: int, k: int) -> int:
    return int(load().steiner_server_query_bytes(s, k))


def steiner_server_memory(s: int) -> dict:
    """How the server's budget is split: fixed + slots * slot_bytes + pool = budget."""
    f, sb, p = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    n = ctypes.c_uint32()
    _check(load().steiner_server_memory(s, ctypes.byref(f), ctypes.byref(sb), ctypes.byref(n), ctypes.byref(p)))
    return {"fixed_bytes": f.value, "slot_bytes": sb.value, "slots": n.value, "pool_bytes": p.value}


def steiner_server_destroy(s: int) -> None:
    _check(load().steiner_server_destroy(s))


def steiner_strerror(code: int) -> str:
    return load().steiner_strerror(code).decode()


def steiner_last_error() -> str:
    return load().steiner_last_error().decode(errors="replace")


# ------------------------------------------------------------ convenience

class Graph:
    """A graph resident on one GPU.  Accepts any object with n / row_ptr / col / w
    (numpy) attributes, e.g. ``workloads.Graph``."""

    def __init__(self, g, device: int = 0, stream=None, flags: int = 0):
        self.n = int(g.n)
        self.nnz = int(g.row_ptr[-1])
        self.handle = steiner_graph_upload(self.n, g.row_ptr, g.col, g.w, device, stream, flags)

    def solve(self, seeds, options=None) -> Tree:
        return steiner_solve(self.handle, seeds, options)

    def tune(self, seeds) -> dict:
        return steiner_graph_tune(self.handle, seeds)

    def solve_batch(self, seed_sets, options=None):
        return steiner_solve_batch(self.handle, seed_sets, options)

    def voronoi(self, seeds, options=None):
        return steiner_voronoi(self.handle, self.n, seeds, options)

    def boundary(self, seeds, options=None):
        k = len(np.unique(np.asarray(seeds)))
        cap = min(k * (k - 1) // 2, self.nnz // 2 + 1)
        return steiner_boundary(self.handle, seeds, cap, options)

    def close(self):
        if self.handle:
            steiner_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
