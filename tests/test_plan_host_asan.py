"""The plan executor's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

csrc/ms_plan.hip is compiled with the host compiler against a host-only model of the
HIP runtime (tests/plan_host: asynchronous queues, stream capture with its documented
join rules, executable graphs that run through their own objects) and stand-ins for the
column operators that read and write their buffers when their work runs.  The replay
drives the sequences of the benchmarks and tests: the star plan launched as a graph on
parallel branches, run eagerly and autotuned right after the eager run, re-formatted,
relaunched and destroyed without a sync; a 512-step batch plan run eagerly on one and
eight branches then autotuned; a capture that fails half way.  Any use after free,
double free, leak of a freed arena into a replay, unjoined capture or undefined behaviour
fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "plan_host")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("plan_host")
    exe = str(d / "replay")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(HERE, "include"), "-I", HERE,
           "-x", "c++", os.path.join(ROOT, "paper_2004_09350_amd", "csrc", "ms_plan.hip"), "-x", "none",
           os.path.join(HERE, "hip_model.cpp"), os.path.join(HERE, "ops_model.cpp"), os.path.join(HERE, "replay.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe, d


def test_plan_executor_replay_is_clean_under_sanitizers(replay):
    exe, d = replay
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(d / "tune_cache.txt")], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "replay ok" in r.stdout, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
