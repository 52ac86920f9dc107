"""The pins hold the oracle to facts outside itself strongly enough to catch plausible
mistakes: each case plants one mistake in a copy of the oracle's C source (CPU only),
builds that copy and runs the pin that covers the step, which must then fail.

- lambda_max (Sec. IV-C.1) as the mean of the vectors' Rayleigh quotients instead
  of their maximum;
- lambda_min (eq. 61) as the largest degree ratio instead of the smallest;
- the similarity check (Sec. IV-D step 6) without the marks on q's neighbours."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("lambda_max_mean_over_vectors",
     "        if (j == 0 || r > lmax) lmax = r;\n    }",
     "        lmax += r / k;\n    }",
     "lambda_max_is_the_largest_rayleigh_quotient"),
    ("lambda_min_largest_degree_ratio",
     "if (v == 0 || r < lmin) lmin = r;",
     "if (v == 0 || r > lmin) lmin = r;",
     "lambda_min_is_the_smallest_degree_ratio or lambda_min_of_a_cycle"),
    ("greedy_without_neighbour_marks_of_q",
     "                for (int64_t a = rp[q]; a < rp[q + 1]; a++) mark[adj[a]] = 1;\n",
     "",
     "greedy"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_a_planted_oracle_mistake(tmp_path, name, old, new, pins):
    dst = tmp_path / "repo"
    shutil.copytree(ROOT, dst, ignore=shutil.ignore_patterns(".git", "_work", "gpurun_out", "__pycache__",
                                                             ".pytest_cache", ".hypothesis", "_build"))
    src = dst / "oracle" / "grass_oracle.c"
    text = src.read_text()
    assert text.count(old) == 1, f"{name}: the site to change is not in the oracle once"
    src.write_text(text.replace(old, new))
    subprocess.check_call([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=dst)
    # the same pins pass on the unchanged oracle (test_oracle_pins.py itself); here they must fail
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-p", "no:cacheprovider",
                        "-k", pins], cwd=dst, capture_output=True, text=True, timeout=600)
    tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else r.stderr[-500:]
    assert r.returncode == 1 and " failed" in tail, f"{name}: pins did not fail ({tail})"
