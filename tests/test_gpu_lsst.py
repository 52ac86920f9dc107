"""Low-stretch spanning tree (Sec. III-A): the gfx950 construction through the C
ABI against the oracle on the same seeded graphs. Integer work, so the bar is
bit-exact: the same tree mask."""
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


def cases():
    return [
        (G.grid2d(64, 48, weights=(G.W_CONST, 1.0, 1.0)), 1, 2),
        (G.mesh3d(20, 18, 16, weights=(G.W_LOGUNIFORM10, -3, 3), seed=2), 5, 2),
        (G.mesh3d(20, 18, 16, weights=(G.W_LOGUNIFORM10, -3, 3), seed=2), 5, 1),
        (G.random_connected(3000, 6000, weights=(G.W_UNIFORM, 1.0, 4.0), seed=3), 2, 5),
        (G.Graph(*(lambda g: (g.n, g.src, g.dst, np.floor(g.w)))(G.random_connected(2000, 5000, seed=4))), 9, 2),
        (G.cycle(257), 0, 2),
        (G.ba(4000, seed=2), 4, 2),
        (G.rgg(3000, seed=1), 6, 3),
        (G.config_c1(), 0, 2),
    ]


@pytest.mark.parametrize("idx", range(9))
def test_low_stretch_tree_bit_exact(ctx, idx):
    g, seed, bits = cases()[idx]
    say("lsst parity:", g.name, g.n, g.m, "seed", seed, "class_bits", bits)
    dg = grass.to_device(g, DEV)
    mask = grass.grass_low_stretch_tree(ctx, dg, seed=seed, class_bits=bits).cpu().numpy()
    ref, _ = O.low_stretch_tree(g, seed=seed, class_bits=bits)
    assert int(mask.sum()) == g.n - 1
    assert np.array_equal(mask, ref)


def test_low_stretch_tree_large_mesh(ctx):
    # a 60^3 mesh with the weight spread of the benchmark graph, in the caller's workspace
    g = G.mesh3d(60, 60, 60, weights=(G.W_LOGUNIFORM10, -3, 3), seed=7)
    say("lsst parity (large):", g.name, g.n, g.m)
    dg = grass.to_device(g, DEV)
    ws = grass.low_stretch_tree_workspace(dg, DEV)
    mask = grass.grass_low_stretch_tree(ctx, dg, seed=1, class_bits=2, ws=ws).cpu().numpy()
    ref, _ = O.low_stretch_tree(g, seed=1, class_bits=2)
    assert np.array_equal(mask, ref)


def test_low_stretch_tree_errors(ctx):
    # two components, and class_bits out of range
    a = G.grid2d(6, 5, seed=1)
    off = a.n
    g = G.Graph(2 * a.n, np.r_[a.src, a.src + off].astype(np.int32), np.r_[a.dst, a.dst + off].astype(np.int32),
                np.r_[a.w, a.w], "two_grids")
    dg = grass.to_device(g, DEV)
    with pytest.raises(grass.GrassError) as ei:
        grass.grass_low_stretch_tree(ctx, dg, seed=0)
    assert ei.value.status == grass.ERR_DISCONNECTED
    dg = grass.to_device(a, DEV)
    with pytest.raises(grass.GrassError) as ei:
        grass.grass_low_stretch_tree(ctx, dg, class_bits=0)
    assert ei.value.status == grass.ERR_INVALID


def test_sparsify_on_the_low_stretch_tree(ctx):
    # one FP64 pass of the sparsifier built on it (opts.init_mask): it keeps the
    # tree and adds the edges the oracle adds on the same tree
    g = G.grid2d(40, 30, weights=(G.W_CONST, 1.0, 1.0))
    dg = grass.to_device(g, DEV)
    tree = grass.grass_low_stretch_tree(ctx, dg, seed=3)
    opts = grass.make_opts(k=8, t=2, sigma2=50.0, precision=64, seed=0, max_iters=1, init_mask=tree)
    res = grass.grass_sparsify(ctx, dg, opts)
    mask = res.mask.cpu().numpy()
    t = tree.cpu().numpy()
    assert np.array_equal(mask == 1, t == 1)
    ref = O.sparsify(g, sigma2=50.0, k=8, t=2, seed=0, max_iters=1, init_mask=t)
    assert np.array_equal(mask, ref.mask)
    assert res.summary["lambda_max"] == pytest.approx(ref.summary["lambda_max"], rel=1e-8)
