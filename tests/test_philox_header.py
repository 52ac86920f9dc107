"""The device Philox4x64-10 (csrc/philox.h, whose output the low-stretch tree's
shifts are read from) compiled for the host with g++ and checked bit for bit
against numpy's Philox bit generator, the published reference implementation
(Salmon et al., SC'11). The device-only qualifiers and the high half of the
64 x 64 product are supplied by the test program."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_04382_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <cstdlib>
#define __device__
#define __forceinline__ inline
static inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
    return (unsigned long long)(((unsigned __int128)a * b) >> 64);
}
#include "philox.h"
int main(int argc, char **argv) {
    // argv: c0 c1 c2 c3 k0 k1, decimal
    unsigned long long c[4], k[2];
    for (int i = 0; i < 4; i++) c[i] = std::strtoull(argv[1 + i], nullptr, 10);
    for (int i = 0; i < 2; i++) k[i] = std::strtoull(argv[5 + i], nullptr, 10);
    grass::philox4x64_10(c, k[0], k[1]);
    std::printf("%llu %llu %llu %llu\n", c[0], c[1], c[2], c[3]);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_device_philox_matches_numpy(tmp_path):
    src, exe = tmp_path / "philox.cpp", tmp_path / "philox"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-I", CSRC, str(src), "-o", str(exe)])
    rng = np.random.default_rng(11)
    for i in range(12):
        ctr = [int(x) for x in rng.integers(1, 2**63, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        if i == 0:
            ctr, key = [1, 0, 0, 0], [0, 0]
        # numpy increments its 256-bit counter before producing a block
        ref = np.random.Philox(counter=[ctr[0] - 1] + ctr[1:], key=key).random_raw(4).astype(np.uint64)
        out = subprocess.check_output([str(exe)] + [str(x) for x in ctr + key], text=True).split()
        assert [int(x) for x in out] == [int(x) for x in ref]
