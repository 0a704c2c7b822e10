"""The column library's host code and the plan executor under AddressSanitizer and
UndefinedBehaviorSanitizer, driven through the C ABI the way the benchmark drives them.

csrc/ms_api.hip and csrc/ms_plan.hip are compiled with the host compiler against the host
model of the HIP runtime (tests/plan_host) and stand-ins for the kernel launchers that write
what each kernel writes over the extents its contract gives.  Allocator callbacks free in
stream order, as a caching allocator does.  The replay encodes the star workload's inputs,
runs the probe plan with statistics and footprint steps, and for every output-format policy
runs a plan eagerly, autotunes another through the tune cache, replays and inspects its
graph, re-tunes a third to one branch, runs and replays a fourth with batched persistent
launches (the recorder, task tables, tickets); then plans over inputs morphed into every
format.
Any out-of-bounds access, use after free, leak or undefined behaviour fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "plan_host")
CSRC = os.path.join(ROOT, "paper_2004_09350_amd", "csrc")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("api_host")
    exe = str(d / "api_replay")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(HERE, "include"), "-I", HERE,
           "-x", "c++", os.path.join(CSRC, "ms_api.hip"), os.path.join(CSRC, "ms_plan.hip"),
           os.path.join(CSRC, "ms_batch.hip"), "-x", "none",
           os.path.join(HERE, "hip_model.cpp"), os.path.join(HERE, "kernels_model.cpp"),
           os.path.join(HERE, "api_replay.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe, d


def test_api_replay_is_clean_under_sanitizers(replay):
    exe, d = replay
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    cache = str(d / "tune_cache.txt")
    r = subprocess.run([exe, cache], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "api replay ok" in r.stdout, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    # the autotuner wrote one line per plan signature and read the mixed policy's back
    lines = open(cache).read().split("\n")
    assert len([x for x in lines if x.strip()]) >= 8
