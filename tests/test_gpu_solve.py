"""The sparsifier as a preconditioner (Sec. V-E) and the partitioner built on it
(Sec. V-F).

grass_solve (flexible PCG on the
grounded L_G, preconditioner L_P^+) against the oracle's PCG with an exact inner
solve, on the same seeded graphs, subgraphs and right-hand sides.

Bars: FP64 with tight tolerances: solution within 1e-8 (relative, max norm) of the
oracle's; outer iteration counts within max(2, 5%) of the oracle's (over a hundred
CG steps, inner products summed in a different order move the stopping step by a
few). FP32 at the paper's 1e-3: the FP64 residual of the returned x, recomputed on
the host, within 1.05 x 1e-3 per column; at most 1.5x + 2 the oracle's (FP64)
iteration count (FP32 recurrences on weights spread over six decades lose
orthogonality and take some extra steps); fewer iterations with the sparsifier
than with the tree."""
import numpy as np
import pytest

import oracle as O
from paper_1911_04382_amd import graphs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1911_04382_amd as grass  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = grass.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def sparsifier_mask(g, k=8):
    """Tree plus one pass of the oracle's filtering (values 1 and 2)."""
    tmask = O.max_spanning_tree(g)
    r0 = O.embed(g, tmask, k=k, t=2, seed=0)
    th = O.theta(100.0, r0.stats["lambda_min"], r0.stats["lambda_max"], 2)
    P, acc, _ = O.filter_select(g, r0.heat, tmask, th, r0.stats["heat_max"], sim_hops=1, budget=max(1, g.n // 50))
    assert acc > 0
    return tmask, P


def rhs(n, k, seed, dtype):
    b = np.random.default_rng(seed).standard_normal((n, k))
    b -= b.mean(0)
    return b.astype(dtype).astype(np.float64)  # the values the GPU sees


def close_count(a, b):
    return abs(a - b) <= max(2, 0.05 * b)


def host_resid(g, x, b):
    """max_j ||b_j - L_G x_j|| / ||b_j|| in FP64, grounded at node 0."""
    r = b - O.laplacian_apply(g, x)
    r[0] = 0.0
    bb = b.copy()
    bb[0] = 0.0
    return (np.linalg.norm(r, axis=0) / np.linalg.norm(bb, axis=0)).max()


@pytest.mark.parametrize("with_edges", [False, True])
def test_solve_fp64_matches_oracle(ctx, with_edges):
    g = G.grid2d(40, 40, seed=3)
    tmask, P = sparsifier_mask(g)
    mask = P if with_edges else tmask
    k = 8
    b = rhs(g.n, k, 1, np.float64)
    say("solve fp64:", g.name, "added edges", int((mask == 2).sum()))
    xo, ito, reso = O.sdd_solve(g, mask, b, rtol=1e-10)
    dg = grass.to_device(g, DEV)
    opts = grass.make_opts(k=k, precision=64, pcg_rtol=1e-13)
    pm = torch.as_tensor(mask).to(DEV)
    rc, x, info = grass.grass_solve(ctx, dg, torch.as_tensor(b, device=DEV), opts, p_mask=pm, rtol=1e-10)
    x = x.cpu().numpy()
    err = np.abs(x - xo).max() / np.abs(xo).max()
    say(f"  oracle {ito} iterations, GPU {info['iters']} (inner {info['inner_iters']}), resid {info['resid']:.2e},"
        f" max error {err:.2e}")
    assert rc == 0
    assert info["added_edges"] == int((mask == 2).sum())
    assert close_count(info["iters"], ito)
    assert err <= 1e-8
    assert host_resid(g, x, b) <= 1.05e-10


def test_solve_tree_default_mask(ctx):
    """p_mask None means the maximum-weight spanning tree."""
    g = G.grid2d(30, 33, seed=5)
    tmask = O.max_spanning_tree(g)
    b = rhs(g.n, 4, 2, np.float64)
    xo, ito, _ = O.sdd_solve(g, tmask, b, rtol=1e-10)
    dg = grass.to_device(g, DEV)
    rc, x, info = grass.grass_solve(ctx, dg, torch.as_tensor(b, device=DEV), grass.make_opts(k=4, precision=64),
                                    rtol=1e-10)
    assert rc == 0 and info["added_edges"] == 0 and info["inner_iters"] == 0
    assert close_count(info["iters"], ito)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-8 * np.abs(xo).max()


# (name, graph, k, compare iteration counts with the oracle: its exact inner solves
# take minutes on the power-law case, whose check is the residual bound)
CASES = [
    ("mesh", lambda: G.mesh3d(16, 15, 14, weights=(G.W_LOGUNIFORM10, -3, 3), seed=4), 16, True),
    ("ba_hubs", lambda: G.ba(12000, seed=5), 16, False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solve_fp32_to_paper_tolerance(ctx, case):
    name, mk, k, with_oracle = case
    g = mk()
    tmask, P = sparsifier_mask(g)
    b = rhs(g.n, k, 3, np.float32)
    dg = grass.to_device(g, DEV)
    opts = grass.make_opts(k=k, precision=32)
    bt = torch.as_tensor(b.astype(np.float32), device=DEV)
    its = {}
    for label, mask in (("tree", tmask), ("sparsifier", P)):
        ito = O.sdd_solve(g, mask, b, rtol=1e-3)[1] if with_oracle else None
        rc, x, info = grass.grass_solve(ctx, dg, bt, opts, p_mask=torch.as_tensor(mask).to(DEV), rtol=1e-3)
        res = host_resid(g, x.cpu().numpy().astype(np.float64), b)
        say(f"  {name} {label}: oracle {ito} iterations, GPU {info['iters']} (inner {info['inner_iters']}),"
            f" FP64 residual of x {res:.3e}")
        assert rc == 0
        assert res <= 1.05e-3
        if with_oracle:
            assert info["iters"] <= 1.5 * ito + 2
        its[label] = info["iters"]
    assert its["sparsifier"] < its["tree"]


def test_solve_rejects_bad_arguments(ctx):
    g = G.grid2d(8, 8, seed=1)
    dg = grass.to_device(g, DEV)
    b = torch.zeros((g.n, 2), dtype=torch.float32, device=DEV)
    with pytest.raises(grass.GrassError):
        grass.grass_solve(ctx, dg, b, grass.make_opts(k=2), rtol=0.0)
    bad = torch.full((g.m,), 3, dtype=torch.uint8, device=DEV)
    with pytest.raises(grass.GrassError):
        grass.grass_solve(ctx, dg, b, grass.make_opts(k=2), p_mask=bad)


# ------------------------------------------------------------ Sec. V-F partitioner
def test_partition_fp64_matches_oracle(ctx):
    g = G.grid2d(30, 33, seed=5)
    tmask, P = sparsifier_mask(g)
    uo, so = O.partition(g, P, steps=5, seed=3, rtol=1e-10)
    dg = grass.to_device(g, DEV)
    opts = grass.make_opts(precision=64, seed=3, pcg_rtol=1e-13)
    rc, u, side, info = grass.grass_partition(ctx, dg, opts, p_mask=torch.as_tensor(P).to(DEV), steps=5, rtol=1e-10)
    u, side = u.cpu().numpy(), side.cpu().numpy()
    err = np.abs(u - uo).max()
    say(f"partition fp64: {info}, max |u - u_oracle| {err:.2e}")
    assert rc == 0 and info["steps"] == 5 and info["inner_iters"] > 0
    assert err <= 1e-7
    assert abs(np.linalg.norm(u) - 1.0) <= 1e-12 and abs(u.sum()) <= 1e-9
    sure = np.abs(uo) > 1e-6
    np.testing.assert_array_equal(side[sure], so[sure])


def test_partition_fp32_sparsifier_vs_exact_solves(ctx):
    """The paper's comparison: sign cut with the sparsifier-preconditioned solver at
    1e-3 against the one from exact solves (the oracle, tight tolerance): it reports
    0.07% to 4% of nodes on different sides; the bar is 5%. In FP32 the solution's
    smooth component (about 1e3 x b on this mesh) puts the attainable residual near
    1e-3, so a step may end just above it (status 1, outputs valid): the residual
    bar is 2e-3."""
    g = G.grid2d(100, 100, seed=8)
    tmask, P = sparsifier_mask(g)
    uo, so = O.partition(g, tmask, steps=5, seed=4, rtol=1e-10)
    dg = grass.to_device(g, DEV)
    # the preconditioner solves need little accuracy inside flexible CG
    rc, u, side, info = grass.grass_partition(ctx, dg, grass.make_opts(precision=32, seed=4, pcg_rtol=1e-2),
                                              p_mask=torch.as_tensor(P).to(DEV), steps=5, rtol=1e-3)
    u = u.cpu().numpy().astype(np.float64)
    side = side.cpu().numpy()
    diff = float((side != so).mean())
    cos = abs(float(u @ uo))
    say(f"partition fp32: {info}, sides differ on {100 * diff:.2f}% of nodes, |cos| {cos:.5f}")
    assert rc in (0, 1) and info["resid"] <= 2e-3
    assert diff <= 0.05 and cos >= 0.99
