"""Host logic of the launch schedule's autotuner (csrc/launch_sched.h, plain C++): built with
g++ (with the address and undefined-behaviour sanitizers) into a small program that feeds
it timings and prints its choices."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_04382_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "launch_sched.h"
using namespace grass;
int main() {
    Tuner t;
    const int a = Tuner::key(1000, 16), b = Tuner::key(1 << 20, 32);
    // size classes: rounded log2 of the node count and the padded width
    std::printf("keys %d %d %d\n", a == Tuner::key(1100, 16), a != Tuner::key(1000, 32), a != b);
    // exploration: every candidate is tried kSchedSamples times, fewest samples first
    const double cost[kSchedCands] = {5.0, 4.0, 2.0, 3.0, 6.0};  // seconds per iteration
    int seen[kSchedCands] = {};
    for (int r = 0; r < kSchedCands * kSchedSamples; r++) {
        const int i = t.pick(a);
        seen[i]++;
        t.record(a, i, cost[i]);
    }
    std::printf("seen");
    for (int i = 0; i < kSchedCands; i++) std::printf(" %d", seen[i]);
    std::printf("\n");
    // then the fastest is kept, and later timings do not change it
    const int c = t.pick(a);
    t.record(a, c, 100.0);
    std::printf("choice %d %d chunks %d\n", c, t.pick(a), kSchedCand[c]);
    // another class explores on its own
    std::printf("other %d\n", t.pick(b));
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tuner_explores_every_candidate_then_keeps_the_fastest(tmp_path):
    src = tmp_path / "tuner.cpp"
    exe = tmp_path / "tuner"
    src.write_text(PROGRAM)
    # address and undefined-behaviour sanitizers on the host-only tuner code
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", CSRC, str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    assert out[0] == "keys 1 1 1"
    samples = out[1].split()[1:]
    assert samples == ["3"] * 5  # each candidate timed three times
    choice = out[2].split()
    assert choice[1] == "2" and choice[2] == "2"  # the 2.0 s candidate, kept after a slow phase
    assert choice[4] == "2"  # candidate 2 replays two chunks per host read
    assert out[3] == "other 0"
