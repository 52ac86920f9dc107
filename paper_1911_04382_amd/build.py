"""Build the gfx950 library libgrass.so in place with hipcc.

Usage: python -m paper_1911_04382_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgrass.so")
SOURCES = ["prim.hip", "graph.hip", "embed.hip", "bpcg.hip", "select.hip", "api.hip", "serve.hip", "sdd.hip", "lsst.hip"]
ARCH = os.environ.get("GRASS_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 instructions.
HIPFLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Host-code sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) for a CPU
# check of the host runtime; the device code is built as usual. The runtime is
# clang's, preloaded by the process that loads the library.
SANITIZE_HOST = shlex.split("-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=undefined "
                            "-Xarch_host -fno-omit-frame-pointer")


def build(verbose: bool = False, jobs: int = 5, sanitize: bool = False, out: str = LIB) -> str:
    """Compile every HIP source and link libgrass.so (always recompiles); with
    sanitize, the host code is instrumented and the library is written to `out`."""
    tmpdir = tempfile.mkdtemp(prefix="grass_build_")
    objs, procs = [], []
    extra = SANITIZE_HOST if sanitize else []
    for src in SOURCES:
        obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
        cmd = [hipcc()] + HIPFLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}"] + extra + ["-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(lines))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
