"""Degenerate inputs of the method through the C ABI, against the oracle: a graph
that is its own spanning tree (no off-tree edge to score: the pass estimates
kappa = 1 and the loop stops at once, Sec. III-F) and the smallest graph, two
nodes and one edge."""
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


def _path(n):
    s = np.arange(n - 1, dtype=np.int32)
    return G.Graph(n, s, s + 1, np.linspace(1.0, 9.0, n - 1))


def _random_tree(n, seed):
    # every node v > 0 hangs off a uniformly chosen earlier node; edges stored (lo, hi)
    # in sorted order as the graph format requires
    rng = np.random.default_rng(seed)
    par = np.array([rng.integers(0, v) for v in range(1, n)], dtype=np.int32)
    child = np.arange(1, n, dtype=np.int32)
    order = np.lexsort((child, par))
    return G.Graph(n, par[order], child[order], rng.uniform(1.0, 10.0, n - 1)[order])


CASES = [("path_1000", lambda: _path(1000)), ("random_tree_5000", lambda: _random_tree(5000, 3)),
         ("two_nodes", lambda: G.Graph(2, np.array([0], np.int32), np.array([1], np.int32), np.array([3.0])))]


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_without_off_tree_edges(ctx, case, prec):
    name, mk = case
    g = mk()
    print("no off-tree edges:", name, g.n, g.m, prec, flush=True)
    ref = O.sparsify(g, sigma2=100.0, k=8, t=2, seed=0)
    r = grass.grass_sparsify(ctx, grass.to_device(g, DEV), grass.make_opts(k=8, t=2, precision=prec, seed=0))
    assert r.status == grass.OK
    assert r.summary["passes"] == ref.summary["passes"] == 1
    assert r.summary["added_edges"] == ref.summary["added_edges"] == 0
    assert r.summary["scored_edges"] == ref.summary["scored_edges"] == 0
    assert r.summary["tree_edges"] == g.m
    assert r.summary["kappa"] == pytest.approx(1.0, abs=1e-6)
    assert r.summary["lambda_min"] == pytest.approx(ref.summary["lambda_min"], abs=1e-12)
    assert (r.mask.cpu().numpy() == 1).all()
    assert (r.scores.cpu().numpy() == 0).all()
