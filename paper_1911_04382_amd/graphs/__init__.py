"""Seeded synthetic graph generators (inputs only; no arithmetic of the method).

Every generator returns a :class:`Graph` holding a canonical edge list: ``src < dst``,
sorted by ``(src, dst)``, no duplicates, edge id = position, int32 node ids and
float64 weights. The draw order is fixed (topology first, then one weight per
edge in canonical order), so ``(family, sizes, seed)`` names exactly one graph.

The families stand in for the paper's benchmark matrices, which are not
available here (Sec. V): 2-D/3-D meshes (thermal / FEM problems, Tables III, V),
a grid with long-range edges (on-chip power grids, Tables I, II), random
geometric graphs, and preferential-attachment networks (the social / data
networks of Table VII).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgrassgen.so")
_SRC = os.path.join(_HERE, "gen.c")

W_UNIFORM, W_LOGUNIFORM10, W_LOGNORMAL, W_CONST = 0, 1, 2, 3


class _GenGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("src", ctypes.POINTER(ctypes.c_int32)),
        ("dst", ctypes.POINTER(ctypes.c_int32)),
        ("w", ctypes.POINTER(ctypes.c_double)),
    ]


def build(force: bool = True) -> str:
    """Compile the generator library in place with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        import subprocess

        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_GenGraph)
        i64, dbl, u64, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int
        lib.gen_grid2d.argtypes = [i64, i64, i32, dbl, dbl, u64, P]
        lib.gen_mesh3d.argtypes = [i64, i64, i64, i32, dbl, dbl, u64, P]
        lib.gen_grid2d_longrange.argtypes = [i64, dbl, i64, i32, dbl, dbl, u64, P]
        lib.gen_rgg.argtypes = [i64, dbl, i32, dbl, dbl, u64, P]
        lib.gen_ba.argtypes = [i64, i64, i32, dbl, dbl, u64, P]
        lib.gen_cycle.argtypes = [i64, i32, dbl, dbl, u64, P]
        lib.gen_complete.argtypes = [i64, i32, dbl, dbl, u64, P]
        lib.gen_random_connected.argtypes = [i64, i64, i32, dbl, dbl, u64, P]
        lib.gen_free.argtypes = [P]
        for f in ("gen_grid2d", "gen_mesh3d", "gen_grid2d_longrange", "gen_rgg", "gen_ba",
                  "gen_cycle", "gen_complete", "gen_random_connected"):
            getattr(lib, f).restype = ctypes.c_int
        lib.gen_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Canonical weighted undirected graph (host arrays)."""

    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    w: np.ndarray  # float64 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _call(fn, *args, name=""):
    lib = _load()
    g = _GenGraph()
    rc = getattr(lib, fn)(*args, ctypes.byref(g))
    if rc != 0:
        raise ValueError(f"{fn}{args}: generator rejected its arguments")
    try:
        m = int(g.m)
        src = np.ctypeslib.as_array(g.src, shape=(max(m, 1),))[:m].copy()
        dst = np.ctypeslib.as_array(g.dst, shape=(max(m, 1),))[:m].copy()
        w = np.ctypeslib.as_array(g.w, shape=(max(m, 1),))[:m].copy()
        return Graph(int(g.n), src, dst, w, name)
    finally:
        lib.gen_free(ctypes.byref(g))


def _wargs(weights):
    kind, a, b = weights
    return int(kind), float(a), float(b)


def grid2d(nx, ny, weights=(W_UNIFORM, 1.0, 10.0), seed=0):
    """nx x ny 4-neighbour grid; node id y*nx + x."""
    return _call("gen_grid2d", nx, ny, *_wargs(weights), seed, name=f"grid2d_{nx}x{ny}")


def mesh3d(nx, ny, nz, weights=(W_UNIFORM, 1.0, 10.0), seed=0):
    """nx x ny x nz 7-point mesh; node id (z*ny + y)*nx + x."""
    return _call("gen_mesh3d", nx, ny, nz, *_wargs(weights), seed, name=f"mesh3d_{nx}x{ny}x{nz}")


def grid2d_longrange(side, frac=0.01, maxhops=200, weights=(W_LOGNORMAL, 0.0, 2.0), seed=0):
    """side x side grid plus floor(frac * grid edges) long-range edges within maxhops hops."""
    return _call("gen_grid2d_longrange", side, frac, maxhops, *_wargs(weights), seed,
                 name=f"powergrid_{side}x{side}")


def rgg(n0, avgdeg=8.0, weights=(W_UNIFORM, 1.0, 10.0), seed=0):
    """Random geometric graph (unit square), largest component kept."""
    return _call("gen_rgg", n0, avgdeg, *_wargs(weights), seed, name=f"rgg_{n0}")


def ba(n, m0=5, weights=(W_UNIFORM, 0.1, 1.0), seed=0):
    """Barabasi-Albert preferential attachment, m0 edges per new node."""
    return _call("gen_ba", n, m0, *_wargs(weights), seed, name=f"ba_{n}")


def cycle(n, weights=(W_CONST, 1.0, 0.0), seed=0):
    return _call("gen_cycle", n, *_wargs(weights), seed, name=f"cycle_{n}")


def complete(n, weights=(W_UNIFORM, 1.0, 10.0), seed=0):
    return _call("gen_complete", n, *_wargs(weights), seed, name=f"complete_{n}")


def random_connected(n, extra, weights=(W_UNIFORM, 1.0, 10.0), seed=0):
    return _call("gen_random_connected", n, extra, *_wargs(weights), seed, name=f"randconn_{n}")


def hair_comb_mask(g: Graph, nx: int, ny: int) -> np.ndarray:
    """Edge mask of the 'hair-comb' spanning tree of an nx x ny grid (Sec. V-C):
    the spine is the bottom row (y = 0) and every column is a tooth."""
    u = g.src.astype(np.int64)
    v = g.dst.astype(np.int64)
    vertical = (v - u) == nx
    bottom = ((v - u) == 1) & (u // nx == 0)
    return (vertical | bottom).astype(np.uint8)


# ----------------------------------------------------------------- workloads
def config_c1(seed=0):
    """64x64 grid, weights U[1,10), seed 0: the small FP64 case."""
    return grid2d(64, 64, (W_UNIFORM, 1.0, 10.0), seed)


def config_c2(side=100, seed=0):
    """side^3 7-point mesh, weights 10^U(-3,3) (ill-conditioned FEM-like)."""
    return mesh3d(side, side, side, (W_LOGUNIFORM10, -3.0, 3.0), seed)


def config_c3(side=2000, seed=0):
    """Power-grid-like: side^2 grid + 1% long-range edges within 200 hops, lognormal(0, 2)."""
    return grid2d_longrange(side, 0.01, 200, (W_LOGNORMAL, 0.0, 2.0), seed)


def config_c4_sizes(count=256, lo=1e3, hi=2e5, seed=0):
    """Node counts log-uniform in [lo, hi] and family cycle {2-D mesh, 3-D mesh, RGG}."""
    rng = np.random.Generator(np.random.Philox(key=seed + 0x5EED))
    out = []
    for i in range(count):
        n = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        out.append((("mesh2d", "mesh3d", "rgg")[i % 3], n))
    return out


def config_c4_graph(kind, n, seed):
    w = (W_UNIFORM, 1.0, 10.0)
    if kind == "mesh2d":
        s = max(2, int(round(math.sqrt(n))))
        return grid2d(s, s, w, seed)
    if kind == "mesh3d":
        s = max(2, int(round(n ** (1.0 / 3.0))))
        return mesh3d(s, s, s, w, seed)
    return rgg(n, 8.0, w, seed)


def config_c5_sizes(count, lo=1e4, hi=2e6, seed=1):
    """Request sizes from the bounded continuous power law p(n) ~ n^-2 on [lo, hi]."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    u = rng.uniform(size=count)
    # inverse CDF of p(n) ~ n^-2 on [lo, hi]
    inv = 1.0 / lo - u * (1.0 / lo - 1.0 / hi)
    return np.floor(1.0 / inv).astype(np.int64)


def config_c5_graph(n, seed):
    return ba(int(n), 5, (W_UNIFORM, 0.1, 1.0), seed)
