"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
never against the oracle itself: dense generalized eigendecompositions and
pseudo-inverses (numpy/scipy), scipy's graph Laplacian and spanning tree,
numpy's independent Philox implementation, closed forms, brute force on tiny
graphs, and the paper's hair-comb figure (tests/golden/hair_comb.txt).
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle as O
from paper_1911_04382_amd import graphs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers
def adjacency(g, use=None):
    sel = np.ones(g.m, bool) if use is None else np.asarray(use) != 0
    s, d, w = g.src[sel], g.dst[sel], g.w[sel]
    return sp.coo_matrix((np.r_[w, w], (np.r_[s, d], np.r_[d, s])), shape=(g.n, g.n)).tocsr()


def dense_laplacian(g, use=None):
    return np.asarray(csg.laplacian(adjacency(g, use)).todense())


def grounded(M, root=0):
    keep = np.arange(M.shape[0]) != root
    return M[np.ix_(keep, keep)]


def pencil_eigs(g, inP, root=0):
    """Nonzero generalized eigenvalues of L_G u = lambda L_P u (eq. 4), from the
    grounded (root row/column removed) pair, which is SPD for connected P."""
    LG = grounded(dense_laplacian(g), root)
    LP = grounded(dense_laplacian(g, inP), root)
    return sla.eigh(LG, LP, eigvals_only=True)


def small_graphs():
    out = [
        G.grid2d(5, 4, seed=3),
        G.random_connected(18, 25, seed=7),
        G.complete(7, seed=1),
        G.cycle(9, weights=(G.W_UNIFORM, 0.5, 2.0), seed=2),
        G.mesh3d(3, 3, 3, weights=(G.W_LOGUNIFORM10, -3, 3), seed=4),
        G.random_connected(30, 60, weights=(G.W_LOGNORMAL, 0.0, 2.0), seed=11),
    ]
    return out


SMALL = small_graphs()


# ------------------------------------------------------------- validation
def test_validate_rejects_bad_inputs():
    g = G.grid2d(4, 4)
    assert O.validate(g) == O.OK
    bad = G.Graph(g.n, g.src.copy(), g.dst.copy(), g.w.copy())
    bad.w[3] = 0.0
    assert O.validate(bad) == O.ERR_INVALID
    bad.w[3] = float("nan")
    assert O.validate(bad) == O.ERR_INVALID
    swp = G.Graph(g.n, g.dst.copy(), g.src.copy(), g.w.copy())  # src > dst
    assert O.validate(swp) == O.ERR_INVALID
    uns = G.Graph(g.n, g.src[::-1].copy(), g.dst[::-1].copy(), g.w.copy())  # unsorted
    assert O.validate(uns) == O.ERR_INVALID
    dup = G.Graph(g.n, np.r_[g.src[:1], g.src], np.r_[g.dst[:1], g.dst], np.r_[g.w[:1], g.w])
    assert O.validate(dup) == O.ERR_INVALID
    # two components: drop every edge touching node 0
    keep = (g.src != 0) & (g.dst != 0)
    disc = G.Graph(g.n, g.src[keep], g.dst[keep], g.w[keep])
    assert O.validate(disc) == O.ERR_DISCONNECTED
    one = G.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert O.validate(one) == O.ERR_INVALID


# ------------------------------------------------------ P1: Laplacian (eqs. 1-2)
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_laplacian_matches_scipy_and_quadratic_form(g):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((g.n, 3))
    y = O.laplacian_apply(g, x)
    L = dense_laplacian(g)  # scipy's own Laplacian of the adjacency matrix
    np.testing.assert_allclose(y, L @ x, rtol=1e-12, atol=1e-12 * np.abs(L).max() * np.abs(x).max())
    # zero row sums: L 1 = 0
    ones = np.ones((g.n, 1))
    assert np.abs(O.laplacian_apply(g, ones)).max() < 1e-12 * g.w.max() * 8
    # symmetry: x'Ly = y'Lx
    z = rng.standard_normal((g.n, 1))
    lhs = float((x[:, :1].T @ O.laplacian_apply(g, z))[0, 0])
    rhs = float((z.T @ O.laplacian_apply(g, x[:, :1]))[0, 0])
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)
    # eq. (2): x'Lx equals the Joule heat sum over edges
    heat = (g.w * (x[g.src, 0] - x[g.dst, 0]) ** 2).sum()
    assert abs(float(x[:, 0] @ y[:, 0]) - heat) <= 1e-11 * heat
    # weighted degrees are the diagonal of eq. (1)
    np.testing.assert_allclose(O.weighted_degree(g), np.diag(L), rtol=1e-14)


# ---------------------------------------------------------- P2: spanning tree
def _is_spanning_tree(n, edges):
    par = list(range(n))

    def f(x):
        while par[x] != x:
            x = par[x]
        return x

    for u, v in edges:
        a, b = f(u), f(v)
        if a == b:
            return False
        par[a] = b
    return True


def test_tree_brute_force_distinct_weights():
    # enumerate every spanning tree of small graphs; the maximum-weight one is unique
    for seed in range(6):
        g = G.random_connected(6, 6, weights=(G.W_UNIFORM, 1.0, 10.0), seed=seed)
        best, best_w = None, -1.0
        for comb in itertools.combinations(range(g.m), g.n - 1):
            if _is_spanning_tree(g.n, [(g.src[e], g.dst[e]) for e in comb]):
                tw = g.w[list(comb)].sum()
                if tw > best_w:
                    best, best_w = set(comb), tw
        mask = O.max_spanning_tree(g)
        assert set(np.flatnonzero(mask)) == best


@pytest.mark.parametrize("seed", range(4))
def test_tree_matches_scipy_mst(seed):
    g = G.random_connected(300, 900, weights=(G.W_UNIFORM, 1.0, 10.0), seed=seed)
    # scipy minimum spanning tree of (C - w) is the maximum spanning tree of w
    C = g.w.max() + 1.0
    A = sp.coo_matrix((C - g.w, (g.src, g.dst)), shape=(g.n, g.n)).tocsr()
    T = csg.minimum_spanning_tree(A).tocoo()
    ref = set(zip(np.minimum(T.row, T.col).tolist(), np.maximum(T.row, T.col).tolist()))
    mask = O.max_spanning_tree(g)
    got = set(zip(g.src[mask == 1].tolist(), g.dst[mask == 1].tolist()))
    assert got == ref


@pytest.mark.parametrize("wkind", ["ints", "equal"])
def test_tree_cycle_property_with_ties(wkind):
    # tie-heavy weights: every off-tree edge must be the last, in the total order
    # (w desc, id asc), on its fundamental cycle; that characterises the unique tree
    rng = np.random.default_rng(5)
    g = G.random_connected(120, 300, seed=9)
    w = rng.integers(1, 4, g.m).astype(float) if wkind == "ints" else np.ones(g.m)
    g = G.Graph(g.n, g.src, g.dst, w)
    mask = O.max_spanning_tree(g)
    assert mask.sum() == g.n - 1
    parent, pw, order = O.root_tree(g, mask)
    # parent edge id per node
    pe = np.full(g.n, -1)
    for e in np.flatnonzero(mask):
        a, b = g.src[e], g.dst[e]
        pe[b if parent[b] == a else a] = e
    depth = np.zeros(g.n, int)
    for v in order[1:]:
        depth[v] = depth[parent[v]] + 1

    def rank_key(e):
        return (-g.w[e], e)

    for e in np.flatnonzero(mask == 0):
        a, b = int(g.src[e]), int(g.dst[e])
        path = []
        while a != b:
            if depth[a] >= depth[b]:
                path.append(pe[a]); a = parent[a]
            else:
                path.append(pe[b]); b = parent[b]
        assert all(rank_key(f) < rank_key(e) for f in path)


# ----------------------------------------------------------- P3: tree solve
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_tree_solve_is_grounded_pseudo_inverse(g):
    mask = O.max_spanning_tree(g)
    tree = O.root_tree(g, mask)
    rng = np.random.default_rng(1)
    b = rng.standard_normal((g.n, 4))
    b -= b.mean(0)  # b orthogonal to the all-ones vector
    x = O.tree_solve(tree, b)
    assert np.all(x[0] == 0.0)  # grounded at the root
    LT = dense_laplacian(g, mask)
    xp = np.linalg.pinv(LT) @ b
    np.testing.assert_allclose(x - x.mean(0), xp, rtol=1e-9, atol=1e-9 * np.abs(xp).max())
    # for a general b, L_T x = b - (sum b) e_root
    b2 = rng.standard_normal((g.n, 2))
    x2 = O.tree_solve(tree, b2)
    r = LT @ x2 - b2
    r[0] += b2.sum(0)
    assert np.abs(r).max() < 1e-9 * np.abs(b2).max() * g.n


def test_tree_solve_root_invariance():
    g = G.random_connected(40, 50, seed=3)
    mask = O.max_spanning_tree(g)
    b = np.random.default_rng(2).standard_normal((g.n, 3))
    b -= b.mean(0)
    x0 = O.tree_solve(O.root_tree(g, mask, 0), b)
    x7 = O.tree_solve(O.root_tree(g, mask, 7), b)
    d = x0 - x7
    np.testing.assert_allclose(d - d[0], 0.0, atol=1e-10 * np.abs(x0).max())


# ---------------------------------------------------------------- P4: PCG
def test_pcg_dense_and_iteration_bound():
    g = G.random_connected(40, 50, seed=12)
    tmask = O.max_spanning_tree(g)
    tree = O.root_tree(g, tmask)
    b = np.random.default_rng(3).standard_normal((g.n, 2))
    b -= b.mean(0)
    off = np.flatnonzero(tmask == 0)
    for s_count in (0, 1, 3, 5):
        inP = tmask.copy()
        inP[off[:s_count]] = 2
        x, it, res = O.pcg(g, inP, tree, b, rtol=1e-13)
        LP = dense_laplacian(g, inP)
        xp = np.linalg.pinv(LP) @ b
        np.testing.assert_allclose(x - x.mean(0), xp, rtol=1e-9, atol=1e-9 * np.abs(xp).max())
        assert res <= 1e-13
        # L_T^+ L_P has at most |S| eigenvalues different from 1 (rank-|S| update):
        # CG terminates in at most |S| + 1 steps in exact arithmetic
        assert it <= s_count + 2, (s_count, it)
        if s_count == 0:
            assert it == 1


def test_sdd_solve_dense_and_iteration_bound():
    """Sec. V-E solver: PCG on L_G with the sparsifier as preconditioner. Pinned to
    the dense pseudo-inverse, and to the rank argument: with P = G minus s edges,
    L_P^+ L_G - I has rank <= s, so CG stops within s + 1 steps (exact arithmetic)."""
    g = G.random_connected(40, 50, seed=12)
    tmask = O.max_spanning_tree(g)
    b = np.random.default_rng(5).standard_normal((g.n, 2))
    b -= b.mean(0)
    xd = np.linalg.pinv(dense_laplacian(g)) @ b
    x, it, res = O.sdd_solve(g, tmask, b, rtol=1e-13)
    np.testing.assert_allclose(x - x.mean(0), xd, rtol=1e-9, atol=1e-9 * np.abs(xd).max())
    assert res <= 1e-13 and it <= g.n
    off = np.flatnonzero(tmask == 0)
    for s_count in (0, 1, 3, 5):
        mask = tmask.copy()
        mask[off] = 2
        mask[off[:s_count]] = 0
        x, it, res = O.sdd_solve(g, mask, b, rtol=1e-12)
        np.testing.assert_allclose(x - x.mean(0), xd, rtol=1e-9, atol=1e-9 * np.abs(xd).max())
        assert it <= s_count + 2, (s_count, it)
        if s_count == 0:
            assert it == 1


def test_partition_converges_to_dense_fiedler_vector():
    """Sec. V-F partitioner: enough inverse power steps give the eigenvector of the
    smallest nonzero eigenvalue of L_G (dense eigh), whatever the preconditioner."""
    g = G.grid2d(9, 7, seed=4)
    w, V = np.linalg.eigh(dense_laplacian(g))
    f = V[:, 1]
    assert w[2] - w[1] > 1e-3 * w[1]  # a simple Fiedler value
    tmask = O.max_spanning_tree(g)
    u, side = O.partition(g, tmask, steps=300, seed=2, rtol=1e-12)
    assert abs(float(u @ f)) >= 1 - 1e-9
    np.testing.assert_array_equal(side, (u >= 0).astype(np.uint8))


def test_partition_splits_two_clusters_at_the_bridge():
    """Two 12-cliques joined by one weak edge: the sign cut is the two cliques."""
    n1 = 12
    edges = [(a, b) for a in range(n1) for b in range(a + 1, n1)]
    edges += [(n1 + a, n1 + b) for a in range(n1) for b in range(a + 1, n1)]
    edges.append((n1 - 1, n1))
    edges.sort()
    src = np.array([e[0] for e in edges], np.int32)
    dst = np.array([e[1] for e in edges], np.int32)
    w = np.where((src == n1 - 1) & (dst == n1), 1e-3, 1.0)
    g = G.Graph(name="two_cliques", n=2 * n1, src=src, dst=dst, w=w)
    u, side = O.partition(g, O.max_spanning_tree(g), steps=6, seed=1, rtol=1e-12)
    assert len(set(side[:n1])) == 1 and len(set(side[n1:])) == 1 and side[0] != side[-1]


# ------------------------------------------- P5/P6: power iteration and heat
@pytest.mark.parametrize("g", SMALL[:5], ids=lambda g: g.name)
@pytest.mark.parametrize("t", [1, 2, 3])
def test_embedding_matches_dense_power_iteration(g, t):
    k = 4
    tmask = O.max_spanning_tree(g)
    inP = tmask.copy()
    off = np.flatnonzero(tmask == 0)
    inP[off[: max(0, len(off) // 3)]] = 2  # a subgraph with extra edges too
    for P in (tmask, inP):
        res = O.embed(g, P, k=k, t=t, seed=5, pass_=1)
        h = O.gauss_vectors(g.n, k, 5, 1)
        LG = dense_laplacian(g)
        LPp = np.linalg.pinv(dense_laplacian(g, P))
        for _ in range(t):  # eq. (29): h_t = (L_P^+ L_G)^t h_0
            h = LPp @ (LG @ h)
        d = h[g.src] - h[g.dst]
        heat = g.w * (d * d).sum(1)  # eqs. (31), (55)
        np.testing.assert_allclose(res.heat, heat, rtol=1e-8, atol=1e-10 * heat.max())
        # eq. (33)-(35): the off-P heat of vector j equals h_j'(L_G - L_P)h_j
        dL = LG - dense_laplacian(g, P)
        offP = P == 0
        for j in range(k):
            qf = h[:, j] @ dL @ h[:, j]
            sj = (g.w[offP] * d[offP, j] ** 2).sum()
            assert abs(qf - sj) <= 1e-8 * max(1.0, abs(qf))


# --------------------------------------------- P7/P8: eigenvalue estimates
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_lambda_estimates_bracket_dense_spectrum(g):
    tmask = O.max_spanning_tree(g)
    inP = tmask.copy()
    off = np.flatnonzero(tmask == 0)
    inP[off[::4]] = 2
    for P in (tmask, inP):
        lam = pencil_eigs(g, P)
        res = O.embed(g, P, k=8, t=2, seed=1).stats
        # Courant-Fischer (eq. 24, Sec. IV-C.1): a Rayleigh quotient never exceeds lambda_max
        assert res["lambda_max"] <= lam.max() * (1 + 1e-9)
        # eq. (61): min degree ratio is an upper bound of lambda_min; and lambda_min >= 1
        # for a subgraph with the original weights (Sec. II-C)
        assert lam.min() >= 1 - 1e-9
        assert lam.min() <= res["lambda_min"] * (1 + 1e-9)
        # continued power iterations converge to lambda_max (Sec. IV-C.1)
        long = O.embed(g, P, k=8, t=2, seed=1, lambda_steps=400).stats
        assert abs(long["lambda_max"] - lam.max()) <= 2e-3 * lam.max()
        # the Rayleigh quotient of eq. (2)/(4) equals 1 + off-P heat / P heat
        assert long["kappa"] == pytest.approx(long["lambda_max"] / long["lambda_min"])


# ------------------------------------------------------------ P9: trace (eq. 8)
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_trace_equals_total_stretch(g):
    tmask = O.max_spanning_tree(g)
    st, total = O.tree_stretch(g, tmask)
    lam = pencil_eigs(g, tmask)
    # eq. (8): Tr(L_P^+ L_G) = st_P(G); tree edges have stretch 1 (eq. 7)
    assert abs(lam.sum() - total) <= 1e-8 * total
    assert np.allclose(st[tmask == 1], 1.0)
    assert lam.max() <= total * (1 + 1e-12)


# ------------------------------------------------ P10: cycle closed form
@pytest.mark.parametrize("n", [5, 9, 16])
def test_cycle_closed_form(n):
    g = G.cycle(n)  # unit weights
    tmask = O.max_spanning_tree(g)
    # ties everywhere: the tree drops the last edge in (w desc, id asc) order
    assert tmask.sum() == n - 1 and tmask[-1] == 0
    lam = np.sort(pencil_eigs(g, tmask))
    # spectrum of a unit cycle against its path: 1 (n-2 times) and n = 1 + stretch
    np.testing.assert_allclose(lam[:-1], 1.0, atol=1e-9)
    assert lam[-1] == pytest.approx(float(n), rel=1e-9)
    long = O.embed(g, tmask, k=4, t=2, lambda_steps=60).stats
    assert long["lambda_max"] == pytest.approx(float(n), rel=1e-9)
    # adding the single off-tree edge brings every eigenvalue to 1 (Sec. III-F)
    r = O.sparsify(g, sigma2=1.5, k=4, t=2, max_iters=5)
    assert r.status == O.OK
    assert r.summary["added_edges"] == 1 and r.summary["kappa"] == 1.0
    assert r.scores[-1] == 1.0  # the only off-tree edge has normalized heat 1


# ---------------------------------------------- P11: interlacing / monotonicity
def test_adding_edges_never_raises_eigenvalues():
    g = G.grid2d(6, 5, seed=8)
    tmask = O.max_spanning_tree(g)
    off = np.flatnonzero(tmask == 0)
    prev = np.sort(pencil_eigs(g, tmask))
    P = tmask.copy()
    for e in off[::3]:
        P[e] = 2
        cur = np.sort(pencil_eigs(g, P))
        assert np.all(cur <= prev + 1e-9)  # eqs. (43)-(53): rank-one updates interlace
        prev = cur
    P[:] = np.where(tmask == 1, 1, 2)
    np.testing.assert_allclose(pencil_eigs(g, P), 1.0, atol=1e-9)


# --------------------------------------------- Philox and start vectors (eq. 28)
def test_philox_matches_numpy_bit_generator():
    rng = np.random.default_rng(4)
    for _ in range(20):
        ctr = rng.integers(1, 2**63, 4, dtype=np.uint64)
        key = rng.integers(0, 2**63, 2, dtype=np.uint64)
        # numpy increments its (256-bit) counter before producing a block
        before = [int(ctr[0]) - 1] + [int(c) for c in ctr[1:]]
        bg = np.random.Philox(counter=before, key=key)
        ref = bg.random_raw(4).astype(np.uint64)
        got = O.philox4x64_10(ctr, key)
        assert np.array_equal(ref, got)


def test_gauss_vectors_distribution_and_mean():
    from scipy import stats

    h = O.gauss_vectors(20000, 4, 123, 0)
    assert np.abs(h.sum(0)).max() < 1e-9  # 1'h_0 = 0 (eq. 28)
    for j in range(4):
        assert stats.kstest(h[:, j], "norm").pvalue > 1e-4
    # counter-based: distinct passes and seeds give independent streams; same inputs repeat
    assert np.array_equal(h, O.gauss_vectors(20000, 4, 123, 0))
    assert abs(np.corrcoef(h[:, 0], O.gauss_vectors(20000, 4, 123, 1)[:, 0])[0, 1]) < 0.05


# ------------------------------------------------------- threshold (eq. 58)
def test_theta_closed_form():
    for s2, lmin, lmax, t in [(100.0, 1.0, 9571.5, 2), (50.0, 1.3, 700.0, 3), (100.0, 1.0, 90.0, 1)]:
        assert O.theta(s2, lmin, lmax, t) == pytest.approx(math.pow(s2 * lmin / lmax, 2 * t + 1), rel=1e-14)


def test_filter_select_properties():
    g = G.grid2d(12, 12, seed=2)
    tmask = O.max_spanning_tree(g)
    res = O.embed(g, tmask, k=8, t=2)
    st = res.stats
    th = O.theta(4.0, st["lambda_min"], st["lambda_max"], 2)
    assert st["kappa"] > 4.0  # so theta < 1 and the hottest edge is a candidate
    # no similarity check, no budget: every candidate is taken (literal eq. 58)
    P, acc, nc = O.filter_select(g, res.heat, tmask, th, st["heat_max"], sim_hops=-1, budget=0)
    cand = (tmask == 0) & (res.heat >= th * st["heat_max"])
    assert acc == nc == cand.sum() and np.array_equal(P == 2, cand)
    # with a budget and the similarity check: accepted edges are the top of the ranking
    # order restricted to dissimilar edges, at most `budget` of them
    P2, acc2, nc2 = O.filter_select(g, res.heat, tmask, th, st["heat_max"], sim_hops=0, budget=5)
    assert acc2 <= 5 and set(np.flatnonzero(P2 == 2)) <= set(np.flatnonzero(cand))
    top = np.flatnonzero(cand)[np.argsort(-res.heat[cand], kind="stable")]
    assert P2[top[0]] == 2  # the hottest edge always enters


# ------------------------------------------------ full loop (Sec. IV-D)
def test_sparsify_loop_invariants():
    g = G.grid2d(16, 16, seed=1)
    r = O.sparsify(g, sigma2=20.0, k=8, t=2, max_iters=30)
    assert r.status in (O.OK, O.NOT_CONVERGED)
    assert (r.mask == 1).sum() == g.n - 1
    assert np.array_equal(r.mask == 1, O.max_spanning_tree(g) == 1)
    budget = max(1, int(0.01 * g.n))
    assert (r.mask == 2).sum() <= budget * (r.summary["passes"] - 1)
    if r.status == O.OK:
        assert r.summary["kappa"] <= 20.0
    lam = pencil_eigs(g, r.mask)
    # the final estimates bracket the true pencil (Sec. IV-C)
    assert r.summary["lambda_max"] <= lam.max() * (1 + 1e-9)
    assert lam.min() <= r.summary["lambda_min"] * (1 + 1e-9)
    # determinism (same seed => identical output bits)
    r2 = O.sparsify(g, sigma2=20.0, k=8, t=2, max_iters=30)
    assert np.array_equal(r.mask, r2.mask) and np.array_equal(r.scores, r2.scores)
    # densification reduces the true lambda_max (eqs. 43-53)
    lam_tree = pencil_eigs(g, O.max_spanning_tree(g))
    assert lam.max() < lam_tree.max()


def test_sparsify_c1_one_pass():
    g = G.config_c1()
    r = O.sparsify(g, sigma2=100.0, k=8, t=2, seed=0, max_iters=1)
    assert r.summary["passes"] == 2 and r.summary["added_edges"] == 40
    assert r.trace[0]["m_off"] == 3969 and r.trace[0]["candidates"] > 0
    assert np.isclose(r.scores.max(), 1.0)


# ------------------------------------ P12: the paper's hair-comb example (Sec. V-C)
def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def test_hair_comb_lambda_max_matches_paper():
    gold = _read_golden("hair_comb.txt")
    side = int(gold["side"])
    g = G.grid2d(side, side, (G.W_CONST, 1.0, 0.0))
    comb = G.hair_comb_mask(g, side, side)
    assert comb.sum() == g.n - 1
    st = O.embed(g, comb, k=4, t=1, lambda_steps=20).stats
    assert st["lambda_max"] == pytest.approx(gold["sigma2_before"], rel=gold["rel_tol"])
    # lambda_min of a spanning tree of G is >= 1; the degree ratio bound is exact here
    assert st["lambda_min"] >= 1.0


@pytest.mark.slow
def test_hair_comb_against_sparse_eigensolver():
    from scipy.sparse.linalg import eigsh

    g = G.grid2d(200, 200, (G.W_CONST, 1.0, 0.0))
    comb = G.hair_comb_mask(g, 200, 200)
    keep = np.arange(1, g.n)
    LG = csg.laplacian(adjacency(g)).tocsr()[keep][:, keep]
    LP = csg.laplacian(adjacency(g, comb)).tocsr()[keep][:, keep]
    lam = eigsh(LG.tocsc(), k=1, M=LP.tocsc(), which="LA", return_eigenvectors=False, tol=1e-10)[0]
    st = O.embed(g, comb, k=4, t=1, lambda_steps=400).stats
    assert st["lambda_max"] <= lam * (1 + 1e-9)
    assert st["lambda_max"] == pytest.approx(lam, rel=2e-3)


# ------------------------------------------- low-stretch spanning tree (Sec. III-A)
def _tree_spans(g, mask):
    if int(np.asarray(mask).sum()) != g.n - 1:
        return False
    ncomp, _ = csg.connected_components(adjacency(g, mask), directed=False)
    return ncomp == 1


LSST_GRAPHS = [
    G.grid2d(12, 9, weights=(G.W_CONST, 1.0, 1.0)),
    G.mesh3d(5, 4, 3, weights=(G.W_LOGUNIFORM10, -3, 3), seed=4),
    G.random_connected(60, 150, weights=(G.W_LOGNORMAL, 0.0, 2.0), seed=11),
    G.ba(80, 3, seed=5),
    G.complete(9, seed=1),
]


@pytest.mark.parametrize("g", LSST_GRAPHS, ids=lambda g: g.name)
@pytest.mark.parametrize("class_bits", [1, 2, 5])
def test_lsst_is_a_spanning_tree(g, class_bits):
    mask, cl = O.low_stretch_tree(g, seed=3, class_bits=class_bits)
    assert _tree_spans(g, mask)
    assert np.all(cl == cl[0])  # one cluster at the end


def test_lsst_of_a_tree_is_the_tree():
    g = G.random_connected(50, 0, seed=9)  # no extra edges: a random tree
    assert g.m == g.n - 1
    mask, _ = O.low_stretch_tree(g, seed=1)
    assert np.all(mask == 1)


def _shift(seed, u, j):
    """The shift of cluster u in round j, read from the generator's output bits."""
    o = [int(x) for x in O.philox4x64_10([u, j, 0x4C535354, 0], [seed, 0])]
    bits = [(o[i // 64] >> (i % 64)) & 1 for i in range(256)]
    for gi in range(85):
        if bits[3 * gi] | bits[3 * gi + 1] | bits[3 * gi + 2] == 0:
            return gi
    return 85


def test_lsst_shift_is_geometric():
    # P(d >= k) = (7/8)^k; mean 7
    d = np.array([_shift(11, u, 0) for u in range(4000)])
    assert abs(d.mean() - 7.0) < 0.4
    for k in (1, 4, 10):
        assert abs((d >= k).mean() - (7 / 8) ** k) < 0.03


def _hops_from(g, u):
    return csg.shortest_path(adjacency(g) > 0, unweighted=True, directed=False, indices=u)


@pytest.mark.parametrize("g", [G.random_connected(40, 60, seed=2), G.ba(60, 2, seed=3), G.grid2d(7, 6, seed=1)],
                         ids=lambda g: g.name)
def test_lsst_round_is_min_shifted_distance(g):
    """One round from single nodes with every edge in class 0 equals the direct
    definition: center(v) = argmin_u hops(u, v) + (85 - d_u), ties to the smaller
    u; v joins through the heaviest FP32 edge to a neighbour one hop nearer to
    its center inside its cluster (smaller id on ties)."""
    mask, cl = O.low_stretch_tree(g, seed=7, class_bits=64, max_rounds=1)
    start = np.array([85 - _shift(7, u, 0) for u in range(g.n)], dtype=float)
    D = np.stack([_hops_from(g, u) for u in range(g.n)])  # D[u, v]
    key = D + start[:, None]
    best = key.min(axis=0)
    center = np.array([np.flatnonzero(key[:, v] == best[v]).min() for v in range(g.n)])
    assert np.array_equal(cl, center)
    w32 = g.w.astype(np.float32)
    want = np.zeros(g.m, np.uint8)
    for v in range(g.n):
        c = center[v]
        if c == v:
            continue
        cands = []
        for e in range(g.m):
            a, b = int(g.src[e]), int(g.dst[e])
            if v not in (a, b):
                continue
            x = b if a == v else a
            if center[x] == c and D[c, x] == D[c, v] - 1:
                cands.append((-float(w32[e]), e))
        want[min(cands)[1]] = 1
    assert np.array_equal(mask, want)


def test_lsst_lowers_stretch_on_a_uniform_grid():
    # with equal weights the maximum-weight tree (ties by edge id) is a comb, whose
    # total stretch grows like n^1.5; the low-stretch tree stays within m log^2 n
    g = G.grid2d(48, 48, weights=(G.W_CONST, 1.0, 1.0))
    mask, _ = O.low_stretch_tree(g, seed=1)
    _, s_ls = O.tree_stretch(g, mask)
    _, s_mst = O.tree_stretch(g, O.max_spanning_tree(g))
    assert s_ls < 0.5 * s_mst
    assert s_ls < g.m * math.log2(g.n) ** 2


def test_lsst_classes_follow_binary_exponents():
    # weights 1, 2, 4, ..., 2^9 on a path: class_bits = 3 puts edges of exponents
    # 9..7 in class 0, 6..4 in class 1, 3..1 in class 2, 0 in class 3. Each class
    # is a set of path edges, so every round keeps joining along the path and the
    # tree is the path itself whatever the classes; with a chord of weight 2^20
    # the chord (class 0 alone) must be in the tree.
    n = 11
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    w = 2.0 ** np.arange(n - 1)
    path = G.Graph(n, src, dst, w, "path")
    mask, _ = O.low_stretch_tree(path, seed=2, class_bits=3)
    assert np.all(mask == 1)
    s2 = np.r_[src, np.int32(0)]
    d2 = np.r_[dst, np.int32(5)]
    order = np.lexsort((d2, s2))
    chord = G.Graph(n, s2[order], d2[order], np.r_[w, 2.0 ** 20][order], "path_chord")
    mask, _ = O.low_stretch_tree(chord, seed=2, class_bits=3)
    assert _tree_spans(chord, mask)
    assert mask[np.flatnonzero((chord.src == 0) & (chord.dst == 5))[0]] == 1


# ------------------------- the estimators and the greedy, each pinned to its definition
def _dense_power_vectors(g, inP, k, t, seed, pass_):
    """h_t = (L_P^+ L_G)^t h_0 with dense pseudo-inverses (eq. 29); h_0 from eq. (28)."""
    h = O.gauss_vectors(g.n, k, seed, pass_)
    LG = dense_laplacian(g)
    LPp = np.linalg.pinv(dense_laplacian(g, inP))
    for _ in range(t):
        h = LPp @ (LG @ h)
        h /= np.abs(h).max(axis=0)  # the quotient below is scale-invariant per vector
    return h


def _subgraphs(g):
    tmask = O.max_spanning_tree(g)
    P = tmask.copy()
    off = np.flatnonzero(tmask == 0)
    P[off[::3]] = 2
    return tmask, P


@pytest.mark.parametrize("g", SMALL[:5], ids=lambda g: g.name)
@pytest.mark.parametrize("lambda_steps", [0, 4])
def test_lambda_max_is_the_largest_rayleigh_quotient_over_vectors(g, lambda_steps):
    """Sec. IV-C.1: the estimate is the largest of the k Rayleigh quotients
    h_j'L_G h_j / h_j'L_P h_j (eqs. 2, 4) of the power vectors, computed here from
    dense matrices; with lambda_steps > t the same vectors continue."""
    k, t = 6, 2
    for inP in _subgraphs(g):
        st = O.embed(g, inP, k=k, t=t, seed=3, pass_=2, lambda_steps=lambda_steps).stats
        h = _dense_power_vectors(g, inP, k, max(t, lambda_steps), 3, 2)
        LG, LP = dense_laplacian(g), dense_laplacian(g, inP)
        rq = np.einsum("ij,ij->j", h, LG @ h) / np.einsum("ij,ij->j", h, LP @ h)
        assert st["lambda_max"] == pytest.approx(rq.max(), rel=1e-9)
        if not np.all(inP != 0):
            # the k quotients differ, so an aggregate other than the maximum would fail
            assert rq.max() > rq.mean() * (1 + 1e-6)


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_lambda_min_is_the_smallest_degree_ratio(g):
    """eq. (61): lambda_min is estimated by min over nodes of L_G(v,v) / L_P(v,v),
    the diagonals taken from scipy's graph Laplacians."""
    for inP in _subgraphs(g):
        st = O.embed(g, inP, k=2, t=1, seed=0).stats
        ratio = np.diag(dense_laplacian(g)) / np.diag(dense_laplacian(g, inP))
        assert st["lambda_min"] == pytest.approx(ratio.min(), rel=1e-12)
        if not np.all(inP != 0):
            assert ratio.max() > ratio.min() * (1 + 1e-9)  # only the minimum passes


@pytest.mark.parametrize("n", [5, 9, 16])
def test_lambda_min_of_a_cycle_against_its_path(n):
    """Closed form: a unit n-cycle has degree 2 everywhere; its path has degree 1
    at the two ends and 2 inside, so the degree ratios are 1 (inside) and 2 (ends)
    and the eq. (61) estimate is 1, the true lambda_min of this pencil."""
    g = G.cycle(n)
    tmask = O.max_spanning_tree(g)
    st = O.embed(g, tmask, k=2, t=1).stats
    assert st["lambda_min"] == 1.0
    assert np.sort(pencil_eigs(g, tmask))[0] == pytest.approx(1.0, abs=1e-9)


def _hand_graph():
    """Six nodes; the path 0-1-2-3-4-5 is the tree and five chords are off-tree:
    (0,2) (0,5) (1,3) (2,4) (3,5). Canonical order (src < dst, sorted)."""
    e = [(0, 1), (0, 2), (0, 5), (1, 2), (1, 3), (2, 3), (2, 4), (3, 4), (3, 5), (4, 5)]
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    g = G.Graph(6, src, dst, np.ones(len(e)), "hand6")
    tree = np.array([1 if (b - a) == 1 else 0 for a, b in e], np.uint8)
    heat = np.zeros(len(e))
    for (a, b), h in {(0, 2): 10.0, (3, 5): 9.0, (1, 3): 8.0, (2, 4): 7.0, (0, 5): 6.0}.items():
        heat[e.index((a, b))] = h
    return g, e, tree, heat


@pytest.mark.parametrize(
    "sim_hops,budget,theta,expect",
    [
        # worked by hand from the reading of Sec. IV-D step 6: taking (0,2) marks 0, 2
        # and their G-neighbours {1, 2, 5} and {0, 1, 3, 4}: every node, so no other
        # chord is dissimilar
        (1, 0, 0.5, [(0, 2)]),
        # endpoint marks only: (3,5) and (1,3) and (2,4) each bring an unmarked
        # endpoint; (0,5) then has both ends marked
        (0, 0, 0.5, [(0, 2), (3, 5), (1, 3), (2, 4)]),
        (0, 2, 0.5, [(0, 2), (3, 5)]),
        # no similarity check: every candidate with heat >= 0.65 * 10 (eq. 58)
        (-1, 0, 0.65, [(0, 2), (3, 5), (1, 3), (2, 4)]),
    ],
)
def test_greedy_hand_worked_example(sim_hops, budget, theta, expect):
    g, e, tree, heat = _hand_graph()
    P, acc, nc = O.filter_select(g, heat, tree, theta, heat.max(), sim_hops=sim_hops, budget=budget)
    got = sorted(e[i] for i in np.flatnonzero(P == 2))
    assert got == sorted(expect) and acc == len(expect)


@pytest.mark.parametrize("sim_hops", [0, 1])
@pytest.mark.parametrize("budget", [0, 15])
def test_greedy_defining_property(sim_hops, budget):
    """Sec. IV-D step 6 under the reading of the similarity check: walking the
    candidates in rank order (heat desc, id asc), an edge is taken exactly when at
    least one endpoint is unmarked by the edges taken before it; a taken edge marks
    its endpoints and, with sim_hops = 1, their neighbours in G; nothing is taken
    once `budget` edges are in."""
    g = G.random_connected(30, 200, seed=5)
    tmask = O.max_spanning_tree(g)
    rng = np.random.default_rng(9)
    heat = np.round(rng.uniform(0, 10, g.m), 1)  # coarse values: ties by id occur
    thr = 0.3
    P, acc, nc = O.filter_select(g, heat, tmask, thr, heat.max(), sim_hops=sim_hops, budget=budget)
    cand = np.flatnonzero((tmask == 0) & (heat >= thr * heat.max()))
    order = cand[np.lexsort((cand, -heat[cand]))]
    taken = set(np.flatnonzero(P == 2).tolist())
    assert taken <= set(cand.tolist()) and nc == len(cand) and acc == len(taken)
    A = adjacency(g).tolil().rows
    marked = np.zeros(g.n, bool)
    count, skipped_similar = 0, 0
    for e in order:
        p, q = int(g.src[e]), int(g.dst[e])
        if budget and count == budget:
            assert e not in taken
            continue
        if e in taken:
            assert not (marked[p] and marked[q])
            count += 1
            marked[[p, q]] = True
            if sim_hops >= 1:
                marked[A[p]] = True
                marked[A[q]] = True
        else:
            assert marked[p] and marked[q]
            skipped_similar += 1
    assert skipped_similar > 0  # the case exercises the similarity check
