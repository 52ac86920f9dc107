"""AddressSanitizer + UndefinedBehaviorSanitizer over the CPU code (no GPU): the
oracle and the generators built by gcc, and the host runtime of the library
(every .hip file's host code, built by hipcc with the instrumentation on the host
side only), each exercised in a child process with its sanitizer runtime
preloaded. Any report fails the test (UBSan is fatal, leaks are not checked: the
HIP runtime keeps allocations until exit)."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-O1", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

ORACLE_RUN = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle as O
from paper_1911_04382_amd import graphs as G
O._LIB = LIB_ORACLE
G._LIB_PATH = LIB_GEN
gs = [G.grid2d(12, 10, seed=1), G.mesh3d(5, 4, 4, weights=(G.W_LOGUNIFORM10, -3, 3), seed=2),
      G.ba(300, 5, seed=3), G.rgg(300, seed=4), G.grid2d_longrange(20, seed=5), G.cycle(9),
      G.complete(6, seed=6), G.random_connected(40, 60, weights=(G.W_LOGNORMAL, 0.0, 2.0), seed=7)]
for g in gs:
    assert O.validate(g) == 0
    r = O.sparsify(g, sigma2=10.0, k=4, t=2, max_iters=4)
    tm = O.max_spanning_tree(g)
    e = O.embed(g, r.mask, k=3, t=2, lambda_steps=4)
    P, acc, nc = O.filter_select(g, e.heat, tm, 0.1, e.stats["heat_max"], sim_hops=1, budget=3)
    O.low_stretch_tree(g, seed=1)
    b = O.gauss_vectors(g.n, 2, 0, 0)
    O.sdd_solve(g, r.mask, b, rtol=1e-6)
bad = G.Graph(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, -1.0]))
assert O.validate(bad) != 0
print("oracle-ok")
"""

HOST_RUN = r"""
import ctypes, sys
sys.path.insert(0, ROOT)
import paper_1911_04382_amd as grass
from paper_1911_04382_amd import graphs as G
L = grass.load_library(LIB_HOST)
o = L.grass_opts_default()
for n, m in ((1000, 3000), (100000, 400000), (1, 0)):
    for k in (1, 5, 16, 32, 64, 65):
        for prec in (32, 64):
            o.k, o.precision = k, prec
            L.grass_workspace_bytes(n, m, ctypes.byref(o))
            L.grass_solve_workspace_bytes(n, m, ctypes.byref(o))
            L.grass_partition_workspace_bytes(n, m, ctypes.byref(o))
L.grass_low_stretch_tree_workspace_bytes(1000, 3000)
assert L.grass_sparsify(None, None, None, None, 0, None, None) == grass.ERR_INVALID
assert L.grass_last_error(None) == b"no context"
h = ctypes.c_void_p()
assert L.grass_create(0, ctypes.byref(h)) in (grass.OK, grass.ERR_DEVICE)
print("host-ok")
"""


def _run(code, env, preload, **paths):
    src = code
    for k, v in dict(ROOT=ROOT, **paths).items():
        src = src.replace(k, repr(v))
    e = dict(env, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, "-c", src], env=e, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    gcc = ["gcc", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off"] + SAN
    lo, lg = str(tmp_path / "liboracle_san.so"), str(tmp_path / "libgen_san.so")
    subprocess.check_call(gcc + ["-o", lo, os.path.join(ROOT, "oracle", "grass_oracle.c"), "-lm"])
    subprocess.check_call(gcc + ["-o", lg, os.path.join(ROOT, "paper_1911_04382_amd", "graphs", "gen.c"), "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    out = _run(ORACLE_RUN, ENV, asan, LIB_ORACLE=lo, LIB_GEN=lg)
    assert "oracle-ok" in out


@pytest.mark.slow
def test_host_runtime_under_asan_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("clang's sanitizer runtime or hipcc is not installed")
    from paper_1911_04382_amd import build as B

    lib = B.build(sanitize=True, out=str(tmp_path / "libgrass_san.so"))
    out = _run(HOST_RUN, ENV, rt[-1], LIB_HOST=lib)
    assert "host-ok" in out
