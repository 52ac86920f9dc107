"""Failure detection through the C ABI: an L_P solve that misses its FP64
target (eq. 29), values that overflow the working precision, invalid weights and
the pass cap of the densification loop (Sec. IV-D). Each condition is forced
from the host (iteration caps, weights near the FP32 limit); every kernel still
exits normally."""
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


@pytest.mark.parametrize("precision", [32, 64])
def test_failed_lp_solve_is_reported(ctx, precision):
    """One block-PCG iteration per solve cannot reach pcg_rtol: the first pass
    that needs an L_P solve returns GRASS_ERR_SOLVE, is flagged in the trace, and
    selects nothing from its heats; the mask keeps the tree pass's additions."""
    g = G.grid2d(40, 40, seed=2)
    say("failed solve:", g.name, "precision", precision)
    dg = grass.to_device(g, DEV)
    opts = grass.make_opts(k=8, t=2, precision=precision, sigma2=10.0, pcg_max_iters=1, pcg_max_outer=1)
    with pytest.raises(grass.GrassError) as e:
        grass.grass_sparsify(ctx, dg, opts)
    assert e.value.status == grass.ERR_SOLVE
    part = e.value.result
    tr = part.trace
    assert part.summary["passes"] == 2 and len(tr) == 2
    assert tr[0]["flags"] == 0 and tr[0]["accepted"] > 0
    assert tr[1]["flags"] & grass.PASS_SOLVE_FAILED and tr[1]["pcg_resid64"] > 1e-6
    assert tr[1]["accepted"] == 0 and tr[1]["candidates"] == 0
    mask = part.mask.cpu().numpy()
    assert (mask == 1).sum() == g.n - 1 and (mask == 2).sum() == tr[0]["accepted"]
    # the same subgraph through grass_embed
    with pytest.raises(grass.GrassError) as e2:
        grass.grass_embed(ctx, dg, part.mask, opts, pass_=1)
    assert e2.value.status == grass.ERR_SOLVE
    assert e2.value.result["flags"] & grass.PASS_SOLVE_FAILED
    # with the default iteration limits the same subgraph solves to pcg_rtol
    ok = grass.make_opts(k=8, t=2, precision=precision, sigma2=10.0)
    heat, st = grass.grass_embed(ctx, dg, part.mask, ok, pass_=1)
    assert st["flags"] == 0 and st["pcg_resid64"] <= ok.pcg_rtol


def test_fp32_overflow_is_reported(ctx):
    """Weights near the FP32 limit are valid input, but the FP32 products
    overflow: the call returns GRASS_ERR_NONFINITE instead of scores. FP64 runs
    the same graph."""
    g = G.grid2d(16, 16, seed=1)
    big = G.Graph(g.n, g.src, g.dst, g.w * 3.0e37)  # w in [3e37, 3e38): each below FLT_MAX
    say("overflow:", big.name, float(big.w.max()))
    dg = grass.to_device(big, DEV)
    with pytest.raises(grass.GrassError) as e:
        grass.grass_sparsify(ctx, dg, grass.make_opts(k=8, t=2, precision=32, max_iters=3))
    assert e.value.status == grass.ERR_NONFINITE
    res = grass.grass_sparsify(ctx, dg, grass.make_opts(k=8, t=2, precision=64, max_iters=3))
    assert res.status in (grass.OK, grass.NOT_CONVERGED)
    assert np.isfinite(res.scores.cpu().numpy()).all()


@pytest.mark.parametrize("bad", [np.nan, np.inf, 0.0, -2.0])
def test_invalid_weight_is_rejected(ctx, bad):
    g = G.grid2d(8, 8, seed=3)
    w = g.w.copy()
    w[17] = bad
    say("invalid weight:", bad)
    dg = grass.to_device(G.Graph(g.n, g.src, g.dst, w), DEV)
    with pytest.raises(grass.GrassError) as e:
        grass.grass_sparsify(ctx, dg, grass.make_opts(k=4))
    assert e.value.status == grass.ERR_INVALID
    assert O.validate(G.Graph(g.n, g.src, g.dst, w)) == O.ERR_INVALID


def test_pass_cap_returns_not_converged(ctx):
    """max_iters passes without reaching kappa <= sigma2: GRASS_NOT_CONVERGED with
    valid outputs, matching the oracle (FP64)."""
    g = G.grid2d(30, 30, seed=4)
    say("pass cap:", g.name)
    dg = grass.to_device(g, DEV)
    opts = grass.make_opts(k=8, t=2, precision=64, sigma2=2.0, max_iters=2, pcg_rtol=1e-12)
    res = grass.grass_sparsify(ctx, dg, opts)
    ref = O.sparsify(g, sigma2=2.0, k=8, t=2, max_iters=2)
    assert res.status == grass.NOT_CONVERGED and ref.status == O.NOT_CONVERGED
    assert res.summary["passes"] == 3 and res.summary["kappa"] > 2.0
    assert np.array_equal(res.mask.cpu().numpy(), ref.mask)
