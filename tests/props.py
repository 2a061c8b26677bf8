"""Binding of the test-side property verifier (tests/props.c): the Voronoi
fixed-point equations and the exactness of G'1, for sizes the oracle's full
solve cannot reach in a test."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "props.c")
LIB = os.path.join(HERE, "libprops.so")
_lib = None


def stale() -> bool:
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)


def build() -> str:
    subprocess.run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC],
                   check=True)
    os.replace(LIB + ".tmp", LIB)
    global _lib
    _lib = None
    return LIB


def _load():
    global _lib
    if _lib is None:
        if stale():
            build()
        lib = ctypes.CDLL(LIB)
        vp, u32 = ctypes.c_void_p, ctypes.c_uint32
        lib.chk_voronoi_fixed_point.restype = ctypes.c_int64
        lib.chk_voronoi_fixed_point.argtypes = [u32, vp, vp, vp, u32, vp, vp]
        lib.chk_boundary.restype = ctypes.c_int
        lib.chk_boundary.argtypes = [u32, vp, vp, vp, vp, u32, vp]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data


def voronoi_fixed_point(g, S, key) -> int:
    """-1 if key is the relaxation's fixed point, else the first failing vertex."""
    S = np.ascontiguousarray(S, dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    return int(_load().chk_voronoi_fixed_point(g.n, _p(g.row_ptr), _p(g.col), _p(g.w), len(S), _p(S), _p(key)))


def boundary_exact(g, key, k, pt) -> int:
    """0 if the dense pair table pt is exactly Step 2's per-pair minimum."""
    key = np.ascontiguousarray(key, dtype=np.uint64)
    pt = np.ascontiguousarray(pt, dtype=np.uint64)
    return int(_load().chk_boundary(g.n, _p(g.row_ptr), _p(g.col), _p(g.w), _p(key), k, _p(pt)))
