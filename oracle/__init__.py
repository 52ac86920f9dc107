"""GRASS oracle: ctypes binding of the plain FP64 CPU implementation in
``grass_oracle.c``.

TEST INFRASTRUCTURE ONLY: the product package never imports this module. It is
used by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of
``bench.py``. It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libgrass_oracle.so")
_SRC = os.path.join(_HERE, "grass_oracle.c")

OK, NOT_CONVERGED, ERR_INVALID, ERR_DISCONNECTED = 0, 1, -1, -2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (single-threaded, strict IEEE: no -ffast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class Opts(ctypes.Structure):
    _fields_ = [
        ("sigma2", ctypes.c_double),
        ("k", ctypes.c_int32),
        ("t", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("max_iters", ctypes.c_int32),
        ("budget_frac", ctypes.c_double),
        ("sim_hops", ctypes.c_int32),
        ("lambda_steps", ctypes.c_int32),
        ("pcg_rtol", ctypes.c_double),
        ("pcg_max_iters", ctypes.c_int32),
    ]


class PassStats(ctypes.Structure):
    _fields_ = [
        ("pass_", ctypes.c_int64),
        ("lambda_max", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("heat_max", ctypes.c_double),
        ("m_off", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("accepted", ctypes.c_int64),
        ("added_total", ctypes.c_int64),
        ("pcg_iters", ctypes.c_int64),
        ("pcg_resid", ctypes.c_double),
    ]

    def as_dict(self):
        return {f[0].rstrip("_"): getattr(self, f[0]) for f in self._fields_}


class Summary(ctypes.Structure):
    _fields_ = [
        ("lambda_max", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("heat_max", ctypes.c_double),
        ("pcg_resid", ctypes.c_double),
        ("passes", ctypes.c_int32),
        ("tree_edges", ctypes.c_int64),
        ("added_edges", ctypes.c_int64),
        ("scored_edges", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i64, i32, dbl, u64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        L.orc_validate.argtypes = [i64, i64, vp, vp, vp]
        L.orc_validate.restype = i32
        L.orc_max_spanning_tree.argtypes = [i64, i64, vp, vp, vp, vp]
        L.orc_max_spanning_tree.restype = i64
        L.orc_laplacian_apply.argtypes = [i64, i64, vp, vp, vp, vp, i32, vp, vp]
        L.orc_laplacian_apply.restype = None
        L.orc_weighted_degree.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        L.orc_weighted_degree.restype = None
        L.orc_root_tree.argtypes = [i64, i64, vp, vp, vp, vp, i64, vp, vp, vp]
        L.orc_root_tree.restype = i32
        L.orc_tree_solve.argtypes = [i64, vp, vp, vp, i32, vp, vp]
        L.orc_tree_solve.restype = None
        L.orc_pcg.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, dbl, i32, vp]
        L.orc_pcg.restype = i32
        L.orc_sdd_solve.argtypes = [i64, i64, vp, vp, vp, vp, i32, vp, vp, vp, i32, vp, vp, dbl, i32, dbl, vp]
        L.orc_sdd_solve.restype = i32
        L.orc_low_stretch_tree.argtypes = [i64, i64, vp, vp, vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, vp]
        L.orc_low_stretch_tree.restype = i64
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_philox4x64_10.restype = None
        L.orc_gauss_vectors.argtypes = [i64, i32, u64, i64, vp]
        L.orc_gauss_vectors.restype = None
        L.orc_embed.argtypes = [i64, i64, vp, vp, vp, vp, i32, i32, i32, u64, i64, dbl, i32, vp,
                                ctypes.POINTER(PassStats)]
        L.orc_embed.restype = i32
        L.orc_theta.argtypes = [dbl, dbl, dbl, i32]
        L.orc_theta.restype = dbl
        L.orc_filter_select.argtypes = [i64, i64, vp, vp, vp, vp, dbl, dbl, i32, i64, vp]
        L.orc_filter_select.restype = i64
        L.orc_sparsify.argtypes = [i64, i64, vp, vp, vp, ctypes.POINTER(Opts), vp, vp, vp,
                                   ctypes.POINTER(Summary), ctypes.POINTER(PassStats), i32]
        L.orc_sparsify.restype = i32
        L.orc_tree_stretch.argtypes = [i64, i64, vp, vp, vp, vp, vp]
        L.orc_tree_stretch.restype = dbl
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def _edges(g):
    src = np.ascontiguousarray(g.src, dtype=np.int32)
    dst = np.ascontiguousarray(g.dst, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.float64)
    return src, dst, w


def make_opts(sigma2=100.0, k=8, t=2, seed=0, max_iters=50, budget_frac=0.01, sim_hops=1,
              lambda_steps=0, pcg_rtol=1e-12, pcg_max_iters=100000) -> Opts:
    return Opts(sigma2, k, t, seed, max_iters, budget_frac, sim_hops, lambda_steps, pcg_rtol, pcg_max_iters)


def validate(g) -> int:
    s, d, w = _edges(g)
    return lib().orc_validate(g.n, g.m, _p(s), _p(d), _p(w))


def max_spanning_tree(g) -> np.ndarray:
    s, d, w = _edges(g)
    mask = np.zeros(g.m, np.uint8)
    lib().orc_max_spanning_tree(g.n, g.m, _p(s), _p(d), _p(w), _p(mask))
    return mask


def laplacian_apply(g, x, use=None):
    s, d, w = _edges(g)
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty_like(x)
    u = None if use is None else np.ascontiguousarray(use, dtype=np.uint8)
    lib().orc_laplacian_apply(g.n, g.m, _p(s), _p(d), _p(w), _p(u), k, _p(x), _p(y))
    return y


def weighted_degree(g, use=None):
    s, d, w = _edges(g)
    deg = np.empty(g.n, np.float64)
    u = None if use is None else np.ascontiguousarray(use, dtype=np.uint8)
    lib().orc_weighted_degree(g.n, g.m, _p(s), _p(d), _p(w), _p(u), _p(deg))
    return deg


def root_tree(g, tree_mask, root=0):
    s, d, w = _edges(g)
    tm = np.ascontiguousarray(tree_mask, dtype=np.uint8)
    parent = np.empty(g.n, np.int64)
    pw = np.empty(g.n, np.float64)
    order = np.empty(g.n, np.int64)
    rc = lib().orc_root_tree(g.n, g.m, _p(s), _p(d), _p(w), _p(tm), root, _p(parent), _p(pw), _p(order))
    if rc != 0:
        raise ValueError("tree edges do not span the graph")
    return parent, pw, order


def tree_solve(tree, b):
    parent, pw, order = tree
    b = np.ascontiguousarray(b, dtype=np.float64)
    k = 1 if b.ndim == 1 else b.shape[1]
    x = np.empty_like(b)
    lib().orc_tree_solve(parent.shape[0], _p(parent), _p(pw), _p(order), k, _p(b), _p(x))
    return x


def pcg(g, inP, tree, b, rtol=1e-12, maxit=100000):
    s, d, w = _edges(g)
    parent, pw, order = tree
    b = np.ascontiguousarray(b, dtype=np.float64)
    k = 1 if b.ndim == 1 else b.shape[1]
    x = np.empty_like(b)
    res = ctypes.c_double(0.0)
    P = np.ascontiguousarray(inP, dtype=np.uint8)
    it = lib().orc_pcg(g.n, g.m, _p(s), _p(d), _p(w), _p(P), _p(parent), _p(pw), _p(order), k, _p(b), _p(x),
                       rtol, maxit, ctypes.byref(res))
    return x, it, res.value


def sdd_solve(g, p_mask, b, rtol=1e-3, maxit=1000, rtol_inner=1e-12):
    """Sec. V-E: PCG on the grounded L_G preconditioned by the sparsifier P.
    p_mask uses the sparsify convention (1 = spanning-tree edge, 2 = added edge);
    P is the tree alone when no edge is marked 2. Returns (x, outer iterations
    (largest over the columns), largest final ||r|| / ||b||)."""
    s, d, w = _edges(g)
    mask = np.asarray(p_mask)
    tree = root_tree(g, (mask == 1).astype(np.uint8))
    parent, pw, order = tree
    inP = np.ascontiguousarray(mask != 0, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.float64)
    k = 1 if b.ndim == 1 else b.shape[1]
    x = np.empty_like(b)
    res = ctypes.c_double(0.0)
    it = lib().orc_sdd_solve(g.n, g.m, _p(s), _p(d), _p(w), _p(inP), int(not (mask == 2).any()), _p(parent),
                             _p(pw), _p(order), k, _p(b), _p(x), rtol, maxit, rtol_inner, ctypes.byref(res))
    return x, it, res.value


def partition(g, p_mask, steps=5, seed=0, rtol=1e-3, maxit=1000):
    """Sec. V-F: a few inverse power iterations for the Fiedler vector of L_G, each
    step solving L_G x = u with the sparsifier-preconditioned PCG of sdd_solve,
    then removing the mean and normalizing; the sign cut gives the two parts.
    u0 is the Philox Gaussian vector of eq. (28) (pass 0, mean removed). Returns
    (u, side) with side[v] = 1 where u[v] >= 0."""
    u = gauss_vectors(g.n, 1, seed, 0)[:, 0].copy()
    u /= np.linalg.norm(u)
    for _ in range(steps):
        x, _, _ = sdd_solve(g, p_mask, u, rtol=rtol, maxit=maxit)
        x = x - x.mean()
        u = x / np.linalg.norm(x)
    return u, (u >= 0).astype(np.uint8)


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    kk = np.asarray(key, dtype=np.uint64)
    out = np.empty(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(kk), _p(out))
    return out


def gauss_vectors(n, k, seed, pass_=0):
    h = np.empty((n, k), np.float64)
    lib().orc_gauss_vectors(n, k, seed, pass_, _p(h))
    return h


@dataclass
class EmbedResult:
    heat: np.ndarray
    stats: dict


def embed(g, inP, k=8, t=2, seed=0, pass_=0, lambda_steps=0, pcg_rtol=1e-12, pcg_max_iters=100000):
    s, d, w = _edges(g)
    P = np.ascontiguousarray(inP, dtype=np.uint8)
    heat = np.empty(g.m, np.float64)
    st = PassStats()
    rc = lib().orc_embed(g.n, g.m, _p(s), _p(d), _p(w), _p(P), k, t, lambda_steps, seed, pass_, pcg_rtol,
                         pcg_max_iters, _p(heat), ctypes.byref(st))
    if rc != 0:
        raise ValueError("tree edges do not span the graph")
    return EmbedResult(heat, st.as_dict())


def theta(sigma2, lambda_min, lambda_max, t):
    return lib().orc_theta(sigma2, lambda_min, lambda_max, t)


def filter_select(g, heat, inP, theta_, heat_max, sim_hops=1, budget=0):
    s, d, _ = _edges(g)
    h = np.ascontiguousarray(heat, dtype=np.float64)
    P = np.array(inP, dtype=np.uint8, copy=True)
    nc = ctypes.c_int64(0)
    acc = lib().orc_filter_select(g.n, g.m, _p(s), _p(d), _p(h), _p(P), theta_, heat_max, sim_hops, budget,
                                  ctypes.byref(nc))
    return P, int(acc), int(nc.value)


@dataclass
class SparsifyResult:
    status: int
    mask: np.ndarray
    scores: np.ndarray
    summary: dict
    trace: list = field(default_factory=list)


def sparsify(g, opts: Opts | None = None, init_mask=None, trace_cap=256, **kw) -> SparsifyResult:
    if opts is None:
        opts = make_opts(**kw)
    s, d, w = _edges(g)
    mask = np.zeros(g.m, np.uint8)
    scores = np.zeros(g.m, np.float64)
    summ = Summary()
    tr = (PassStats * trace_cap)()
    im = None if init_mask is None else np.ascontiguousarray(init_mask, dtype=np.uint8)
    rc = lib().orc_sparsify(g.n, g.m, _p(s), _p(d), _p(w), ctypes.byref(opts), _p(im), _p(mask), _p(scores),
                            ctypes.byref(summ), tr, trace_cap)
    if rc < 0:
        return SparsifyResult(rc, mask, scores, {}, [])
    sd = {f[0]: getattr(summ, f[0]) for f in Summary._fields_}
    trace = [tr[i].as_dict() for i in range(min(summ.passes, trace_cap))]
    return SparsifyResult(rc, mask, scores, sd, trace)


def low_stretch_tree(g, seed=0, class_bits=2, max_rounds=0):
    """Low-stretch spanning tree (AKPW over weight classes with exponential
    start-time clustering, Sec. III-A; see orc_low_stretch_tree). Returns the
    tree mask (m, uint8) and the final cluster of every node."""
    s, d, w = _edges(g)
    mask = np.zeros(g.m, np.uint8)
    cluster = np.empty(g.n, np.int64)
    rc = lib().orc_low_stretch_tree(g.n, g.m, _p(s), _p(d), _p(w), seed, class_bits, max_rounds, _p(mask),
                                    _p(cluster))
    if rc < 0:
        raise ValueError("class_bits must be >= 1")
    return mask, cluster


def tree_stretch(g, tree_mask):
    s, d, w = _edges(g)
    tm = np.ascontiguousarray(tree_mask, dtype=np.uint8)
    st = np.empty(g.m, np.float64)
    total = lib().orc_tree_stretch(g.n, g.m, _p(s), _p(d), _p(w), _p(tm), _p(st))
    return st, total
