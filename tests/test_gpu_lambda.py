"""lambda_max from continued generalized power iterations (Sec. IV-C.1; the
paper's Table IV compares such estimates with exact extreme eigenvalues): the
gfx950 estimate through the C ABI against the oracle's (FP64, same seeds) and
against the exact largest eigenvalue of the grounded pencil (L_G, L_P)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

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


def _lap(g, use):
    sel = np.asarray(use) != 0
    s, d, w = g.src[sel], g.dst[sel], g.w[sel]
    A = sp.coo_matrix((np.r_[w, w], (np.r_[s, d], np.r_[d, s])), shape=(g.n, g.n)).tocsr()
    return np.asarray(csg.laplacian(A).todense())[1:, 1:]  # grounded at node 0


def exact_lambda_max(g, P):
    return float(sla.eigh(_lap(g, np.ones(g.m)), _lap(g, P), eigvals_only=True).max())


def cases():
    g1 = G.mesh3d(6, 5, 4, weights=(G.W_LOGUNIFORM10, -3, 3), seed=4)
    t1 = O.max_spanning_tree(g1)
    g2 = G.grid2d(14, 12, seed=3)
    t2 = O.max_spanning_tree(g2)
    p2 = t2.copy()
    off = np.flatnonzero(t2 == 0)
    p2[off[::5]] = 2
    return [("mesh_tree", g1, t1), ("grid_sparsifier", g2, p2)]


@pytest.mark.parametrize("steps", [8, 300])
@pytest.mark.parametrize("idx", [0, 1])
def test_lambda_steps_parity_and_accuracy(ctx, idx, steps):
    name, g, P = cases()[idx]
    print("lambda_steps:", name, "steps", steps, flush=True)
    dg = grass.to_device(g, DEV)
    pm = torch.as_tensor(P).to(DEV)
    opts = grass.make_opts(k=8, t=2, precision=64, seed=1, lambda_steps=steps, pcg_rtol=1e-12)
    heat, st = grass.grass_embed(ctx, dg, pm, opts, pass_=0)
    ref = O.embed(g, P, k=8, t=2, seed=1, lambda_steps=steps).stats
    assert st["lambda_max"] == pytest.approx(ref["lambda_max"], rel=1e-8)
    exact = exact_lambda_max(g, P)
    assert st["lambda_max"] <= exact * (1 + 1e-9)  # a Rayleigh quotient (Courant-Fischer)
    if steps >= 300:
        assert abs(st["lambda_max"] - exact) <= 2e-3 * exact
    # the scores use t steps only: identical to the run without extra steps
    heat0, _ = grass.grass_embed(ctx, dg, pm, grass.make_opts(k=8, t=2, precision=64, seed=1, pcg_rtol=1e-12),
                                 pass_=0)
    assert torch.equal(heat, heat0)


def test_fp32_sparsify_with_eight_step_lambda(ctx):
    """FP32 sparsify of a 40^3 mesh of the benchmark's family (weights 10^U(-3,3),
    k = 32, t = 2) with lambda_max from 8 continued power steps: every L_P solve
    reaches pcg_rtol although the continued vectors grow nearly parallel, the loop
    stops at kappa_est <= sigma^2, and the 8-step estimate of the final pass is
    close to the sparsifier's lambda_max continued to 100 steps on one vector in
    FP64 (a Rayleigh quotient: at most that value, and the paper reports errors of
    a few percent with fewer than ten steps)."""
    g = G.config_c2(40)
    print("lambda_steps = 8 sparsify:", g.n, g.m, flush=True)
    dg = grass.to_device(g, DEV)
    sigma2 = 100.0
    r = grass.grass_sparsify(ctx, dg, grass.make_opts(k=32, t=2, sigma2=sigma2, precision=32, seed=1,
                                                       lambda_steps=8))
    print(f"  {r.summary['passes']} passes, kappa_est {r.summary['kappa']:.2f}", flush=True)
    assert r.status == grass.OK
    assert all(t["pcg_resid64"] <= 1e-6 for t in r.trace[1:])
    assert all(t["flags"] == 0 for t in r.trace)
    assert r.summary["kappa"] <= sigma2
    _, st = grass.grass_embed(ctx, dg, r.mask, grass.make_opts(k=1, t=2, lambda_steps=100, precision=64, seed=1),
                              pass_=1000)
    est, ref = r.summary["lambda_max"], st["lambda_max"]
    print(f"  lambda_max: 8-step estimate {est:.3f}, 100 steps {ref:.3f}", flush=True)
    assert est <= ref * (1 + 1e-3)
    assert est >= 0.9 * ref
