"""The library's host orchestration on the CPU: the real host code of every
source (graph capture and the graph cache, stream forks and joins, the
solver's chunk loop, the batched relaxed-FISTA step, single-context calls),
built without device code and with AddressSanitizer on the host, run against a
host-only stand-in of the HIP runtime (tests/host_harness/hip_stub.cpp) that
checks the stream, event and graph rules and scripts the solver's open-system
counts.  Kernels do not run, so no number is compared; what must hold is that
the host side touches no memory out of bounds or after free and breaks none of
the modelled rules, also when more solver graphs are captured than the cache
holds (evictions) and with the 32-problem batched recipe's seven grid groups."""

import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HARNESS = os.path.join(HERE, "host_harness")


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists("/opt/rocm/llvm/bin/clang++"):
        pytest.skip("ROCm clang++ not available")
    sys.path.insert(0, HARNESS)
    import build_harness
    return build_harness.build()


def _run(driver, tmp_path, problems, steps):
    f = tmp_path / "problems.txt"
    f.write_text("".join(f"{n} {T}\n" for n, T in problems))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([driver, str(f), str(steps)], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:] + r.stdout[-2000:]
    assert "ERROR: AddressSanitizer" not in r.stderr
    words = r.stdout.split()
    return {words[i]: int(words[i + 1]) for i in range(0, len(words) - 1, 2)}


def test_uneven_batch_with_graph_cache_evictions(driver, tmp_path):
    """Seven grid groups, scripted counts that vary the set of open groups from
    chunk to chunk: far more solver graphs are captured than the cache's 32
    slots, so entries are evicted and destroyed while the batch keeps stepping."""
    problems = [(8, 3), (12, 5), (16, 4), (24, 6), (32, 3), (40, 5), (48, 4), (8, 2), (16, 7), (24, 3)]
    rep = _run(driver, tmp_path, problems, 20)
    assert rep["groups"] == 7 and rep["violations"] == 0
    assert rep["graphs_instantiated"] > 2 * 32 + 10          # evictions happened
    assert rep["count_reads"] > 100 and rep["graph_launches"] > 100


def test_full_batched_recipe_host_side(driver, tmp_path):
    """The 32-problem recipe (grids 64^2-512^2, 8-64 transmitters, M = 4T): its
    real buffer layout, arena and geometry set-up, three steps of each start
    mode and a batched forward solve."""
    sys.path.insert(0, os.path.dirname(HERE))
    from synth.workloads import batched_uneven
    problems = [(w.n, w.T) for w in batched_uneven()]
    rep = _run(driver, tmp_path, problems, 3)
    assert rep["groups"] == 7 and rep["problems"] == 32 and rep["violations"] == 0
