"""Host-side checks of the C-ABI library (no GPU needed): the shared library
loads, exports every function include/grass.h declares, and its host-only
entry points behave."""
import ctypes
import os

import pytest

import paper_1911_04382_amd as grass


def test_library_exports_every_declared_symbol():
    lib = grass.load_library()
    declared = grass.exported_symbols_declared_in_header()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/grass.h but not exported"


def test_header_declares_the_boundary_calls():
    declared = set(grass.exported_symbols_declared_in_header())
    for name in ("grass_create", "grass_destroy", "grass_last_error", "grass_opts_default", "grass_workspace_bytes",
                 "grass_sparsify", "grass_spanning_tree", "grass_embed", "grass_select", "grass_start_vectors",
                 "grass_sparsify_batch", "grass_batch_workspace_bytes", "grass_server_create", "grass_server_submit",
                 "grass_solve", "grass_solve_workspace_bytes", "grass_partition",
                 "grass_partition_workspace_bytes", "grass_low_stretch_tree",
                 "grass_low_stretch_tree_workspace_bytes"):
        assert name in declared


def test_opts_defaults():
    o = grass.load_library().grass_opts_default()
    assert o.sigma2 == 100.0 and o.k == 16 and o.t == 2 and o.max_iters == 50
    assert o.budget_frac == 0.01 and o.sim_hops == 1 and o.precision == 32
    assert o.pcg_rtol == 1e-6 and o.init_mask is None


def test_opts_defaults_match_the_header():
    """Every bracketed default in the grass_opts declaration of include/grass.h is
    the value grass_opts_default() returns."""
    import re

    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "grass.h")).read()
    body = hdr[hdr.index("/* Options (grass_opts_default()"):hdr.index("} grass_opts;")]
    fields = re.findall(r"\b(?:double|int32_t|uint64_t)\s+(\w+);\s*/\*(.*?)\*/", body, re.S)
    assert len(fields) >= 12
    o = grass.load_library().grass_opts_default()
    for name, doc in fields:
        m = re.search(r"\[([^\]=]+?)(?:\s*=.*)?\]", doc)
        assert m, f"{name}: no default in brackets"
        want = float(m.group(1))
        assert float(getattr(o, name)) == want, f"{name}: header says {want}, library returns {getattr(o, name)}"


def test_workspace_bytes_monotone_and_rejects_bad_sizes():
    lib = grass.load_library()
    o = lib.grass_opts_default()
    small = lib.grass_workspace_bytes(1000, 3000, ctypes.byref(o))
    big = lib.grass_workspace_bytes(100000, 300000, ctypes.byref(o))
    assert 0 < small < big
    o.k = 32
    assert lib.grass_workspace_bytes(1000, 3000, ctypes.byref(o)) > small
    o.precision = 64
    assert lib.grass_workspace_bytes(1000, 3000, ctypes.byref(o)) > small
    assert lib.grass_workspace_bytes(1, 0, ctypes.byref(o)) == 0
    o.k = 65
    assert lib.grass_workspace_bytes(1000, 3000, ctypes.byref(o)) == 0


def test_low_stretch_tree_workspace_bytes():
    lib = grass.load_library()
    small = lib.grass_low_stretch_tree_workspace_bytes(1000, 3000)
    assert 1000 * 28 + 3000 * 4 <= small < lib.grass_low_stretch_tree_workspace_bytes(100000, 300000)
    assert lib.grass_low_stretch_tree_workspace_bytes(-1, 3) == 0


def test_null_context_is_rejected():
    lib = grass.load_library()
    assert lib.grass_sparsify(None, None, None, None, 0, None, None) == grass.ERR_INVALID
    assert lib.grass_last_error(None) == b"no context"


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib

    mod = importlib.import_module("paper_1911_04382_amd")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(ImportError):
            mod.load_library(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved


def test_solve_workspace_covers_the_sparsify_workspace():
    lib = grass.load_library()
    o = grass.make_opts(k=16)
    for n, m in ((1000, 3000), (100000, 400000)):
        a = lib.grass_workspace_bytes(n, m, ctypes.byref(o))
        b = lib.grass_solve_workspace_bytes(n, m, ctypes.byref(o))
        assert b > a > 0
    assert lib.grass_solve_workspace_bytes(1, 0, ctypes.byref(o)) == 0
