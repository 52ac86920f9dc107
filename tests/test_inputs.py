"""The seeded synthetic inputs (paper_1911_04382_amd/graphs) against the recipe they
stand in for: sizes, canonical edge lists, weight distributions, structure (stencil
offsets, the long-range edges' share and hop bound, heavy-tailed degrees, the
log-uniform and power-law size draws), connectivity and determinism."""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.stats as ss

from paper_1911_04382_amd import graphs as G


def _canonical(g):
    s, d = g.src.astype(np.int64), g.dst.astype(np.int64)
    assert g.src.dtype == np.int32 and g.dst.dtype == np.int32 and g.w.dtype == np.float64
    assert (s >= 0).all() and (s < d).all() and (d < g.n).all()
    assert (np.diff(s * g.n + d) > 0).all()  # sorted by (src, dst), no repeated edge


def _connected(g):
    a = sp.coo_matrix((np.ones(g.m), (g.src, g.dst)), shape=(g.n, g.n))
    return csg.connected_components(a, directed=False)[0] == 1


def test_c1_grid():
    g = G.config_c1()
    assert (g.n, g.m) == (4096, 8064)
    _canonical(g)
    assert _connected(g)
    assert g.w.min() >= 1.0 and g.w.max() < 10.0
    assert ss.kstest(g.w, "uniform", args=(1.0, 9.0)).pvalue > 1e-3


def test_c2_mesh_at_full_size():
    g = G.config_c2(100)
    assert (g.n, g.m) == (1_000_000, 2_970_000)
    _canonical(g)
    # 7-point stencil: every edge joins nodes one step apart along one axis
    assert set(np.unique(g.dst - g.src).tolist()) == {1, 100, 10_000}
    lw = np.log10(g.w)
    assert lw.min() >= -3.0 and lw.max() <= 3.0
    assert ss.kstest(lw[::97], "uniform", args=(-3.0, 6.0)).pvalue > 1e-3


def test_c2_family_is_connected():
    assert _connected(G.config_c2(20))


def test_c3_power_grid_at_full_size():
    side = 2000
    g = G.config_c3(side)
    s, d = g.src.astype(np.int64), g.dst.astype(np.int64)
    grid = ((d - s == 1) & (s // side == d // side)) | (d - s == side)
    assert g.n == side * side and grid.sum() == 2 * side * (side - 1)
    assert (~grid).sum() == round(0.01 * grid.sum())  # long-range edges: 1% of the grid's
    ls, ld = s[~grid], d[~grid]
    hops = np.abs(ls % side - ld % side) + np.abs(ls // side - ld // side)
    assert hops.min() >= 2 and hops.max() <= 200
    _canonical(g)
    lw = np.log(g.w)
    assert abs(lw.mean()) < 0.01 and abs(lw.std() - 2.0) < 0.01
    assert ss.kstest(lw[::101], "norm", args=(0.0, 2.0)).pvalue > 1e-3


def test_c4_sizes_and_families():
    sizes = G.config_c4_sizes()
    assert len(sizes) == 256
    assert [k for k, _ in sizes[:6]] == ["mesh2d", "mesh3d", "rgg"] * 2
    n = np.array([v for _, v in sizes], dtype=np.float64)
    assert n.min() >= 1e3 and n.max() <= 2e5
    assert ss.kstest(np.log(n), "uniform", args=(math.log(1e3), math.log(2e5) - math.log(1e3))).pvalue > 1e-3
    for kind in ("mesh2d", "mesh3d", "rgg"):
        g = G.config_c4_graph(kind, 5000, 7)
        _canonical(g)
        assert _connected(g)
        assert g.w.min() >= 1.0 and g.w.max() < 10.0
    r = G.config_c4_graph("rgg", 20000, 5)
    assert 0.95 * 20000 <= r.n <= 20000  # the largest component of the geometric graph
    assert abs(2 * r.m / r.n - 8.0) < 0.5  # mean degree 8


def test_c5_sizes_and_preferential_attachment():
    lo, hi = 1e4, 2e6
    n = G.config_c5_sizes(2000)
    assert n.min() >= lo and n.max() <= hi
    # bounded power law p(n) ~ n^-2: F(n) = (1/lo - 1/n) / (1/lo - 1/hi)
    cdf = lambda x: (1.0 / lo - 1.0 / np.asarray(x, dtype=np.float64)) / (1.0 / lo - 1.0 / hi)  # noqa: E731
    assert ss.kstest(n + 0.5, cdf).pvalue > 1e-3
    g = G.config_c5_graph(20000, 3)
    _canonical(g)
    assert _connected(g)
    assert g.m == 15 + 5 * (g.n - 6)  # a seed clique of 6, then 5 edges per new node
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert deg.min() >= 5 and deg.max() > 20 * deg.mean()  # heavy-tailed degrees
    assert g.w.min() >= 0.1 and g.w.max() < 1.0


def test_generators_are_deterministic_in_the_seed():
    for mk in (lambda s: G.config_c2(12, s), lambda s: G.config_c3(60, s), lambda s: G.config_c5_graph(3000, s),
               lambda s: G.rgg(3000, seed=s)):
        a, b, c = mk(1), mk(1), mk(2)
        assert a.n == b.n and np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
        assert np.array_equal(a.w, b.w)
        assert not (a.m == c.m and np.array_equal(a.src, c.src) and np.array_equal(a.w, c.w))
