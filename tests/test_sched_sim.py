"""The serving scheduler on the CPU, against a simulated executor.

serve.cpp, planner.cpp and arena.cpp are built unchanged with the host
compiler and linked with ``tests/sched_sim/fake_exec.cpp``, which stands in
for the device: tables are sizes only, every size is a fixed function of the
pattern or of the joined tables, and memory follows the library's rules
(exact-size arena blocks, join scratch held while a join runs, a batch's
results in one shared block).  Each scenario runs its queries alone through
the plain planner first, then all together through submit / serve_step /
poll_next, over a grid of arena sizes, admission budgets, arrival and poll
schedules.  What must hold in every scenario:

* the round loop ends well within its limit, and no round reports an error;
* every arena byte comes back;
* with a caller that polls, a query completes exactly when it completes
  alone, with the same row count, and fails with the status it has alone
  (memory failures are all reported as TOO_LARGE by the server); a query
  whose plain run failed only for memory may complete when served (its
  memory then happened to be laid out differently);
* with a caller that never polls while queries run, the loop still ends:
  a step that waits for unpolled results fails with TOO_LARGE after a
  bounded number of rounds.

A second build of the same host sources under AddressSanitizer (leak
detection on) and UndefinedBehaviorSanitizer runs a subset of the scenarios;
any report fails the test.
"""
import itertools
import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1702_03484_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("serve.cpp", "planner.cpp", "arena.cpp")] + [
    os.path.join(HERE, "sched_sim", "fake_exec.cpp")]
MEMORY = (-3, -4)  # CAPACITY, TOO_LARGE


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("sched_sim") / "sim")
    subprocess.run([cxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
                    *SOURCES, "-o", exe], check=True, capture_output=True, text=True)
    return exe


@pytest.fixture(scope="module")
def sim_sanitized(tmp_path_factory):
    """The same host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer (any report aborts the run)."""
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("sched_sim_san") / "sim")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
    r = subprocess.run([cxx, "-std=c++17", "-O1", *flags, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + CSRC, *SOURCES, "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    return exe


def run(exe, seed, nq, arena_mb, budget_permille, arrive_every, poll_every, max_active):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe, str(seed), str(nq), str(arena_mb), str(budget_permille), str(arrive_every),
                          str(poll_every), str(max_active)], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stderr[-4000:]
    return json.loads(out.stdout)


def check(d, polls):
    assert d["terminated"] and d["rounds"] < 20000, d["rounds"]
    assert d["step_errors"] == 0
    assert d["free_end"] == d["free0"], "arena bytes leaked"
    assert d["free_alone"] == d["free0"]
    for i, (a, s) in enumerate(zip(d["alone"], d["served"])):
        if polls:
            if a[0] == 0:
                assert s == a, f"query {i}: alone {a}, served {s}"
            elif a[0] in MEMORY:
                assert s[0] == -4 or s[0] == 0, f"query {i}: alone {a}, served {s}"
            else:
                assert s[0] == a[0], f"query {i}: alone {a}, served {s}"
        else:
            assert s == a or s[0] == -4 or (a[0] in MEMORY and s[0] == 0), f"query {i}: alone {a}, served {s}"


@pytest.mark.parametrize("seed", range(1, 9))
def test_served_outcomes_equal_alone(sim, seed):
    """Outcomes as alone over arena sizes, budgets, arrival schedules and
    in-flight limits, with a caller that polls every round or every third."""
    for arena, budget, arrive, poll, maxa in itertools.product([256, 1024, 4096, 16384], [300, 1000, 3000], [0, 1, 3],
                                                               [1, 3], [0, 4]):
        check(run(sim, seed, 40, arena, budget, arrive, poll, maxa), polls=True)


@pytest.mark.parametrize("seed", [101, 104, 106, 125])
def test_many_queries_under_memory_pressure(sim, seed):
    """200 queries at once or spread out, small and large arenas."""
    for arena, budget, arrive, poll, maxa in itertools.product([512, 2048, 8192], [600, 3000], [0, 1], [1, 3], [0, 8]):
        check(run(sim, seed, 200, arena, budget, arrive, poll, maxa), polls=True)


@pytest.mark.parametrize("seed", range(1, 5))
def test_loop_ends_without_polls(sim, seed):
    """A caller that polls only once nothing is in flight: finished results
    keep their memory, and every query still ends (completed, or failed
    with TOO_LARGE where it needed that memory)."""
    for arena, budget, arrive, maxa in itertools.product([256, 1024, 4096], [300, 3000], [0, 1], [0, 4]):
        check(run(sim, seed, 40, arena, budget, arrive, 0, maxa), polls=False)


@pytest.mark.parametrize("seed", [3, 104])
def test_scheduler_under_sanitizers(sim_sanitized, seed):
    """The scheduler, planner and arena under AddressSanitizer (with leak
    detection) and UndefinedBehaviorSanitizer: polling and non-polling
    callers, tight and roomy arenas, every scenario clean and its outcomes
    as in the plain build's checks."""
    for arena, budget, arrive, poll, maxa in itertools.product([256, 4096], [300, 3000], [0, 1], [0, 1], [0, 4]):
        check(run(sim_sanitized, seed, 60, arena, budget, arrive, poll, maxa), polls=poll > 0)
