"""Host code under test on the CPU, plain and under the sanitizers: the
serving core (paper_2207_00257_amd/csrc/nrm_sched.h) with a fake executor
(tests/cpu/sched_test.cpp), and the C oracle (oracle/*.c) driven over its
edge cases (tests/cpu/oracle_san.c). Builds with g++/gcc only: no GPU code
is involved."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_00257_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SCHED_TEST = os.path.join(ROOT, "tests", "cpu", "sched_test.cpp")
ORACLE_DRIVER = os.path.join(ROOT, "tests", "cpu", "oracle_san.c")
ORACLE_SRCS = [os.path.join(ROOT, "oracle", f) for f in sorted(os.listdir(os.path.join(ROOT, "oracle")))
               if f.endswith(".c")]

SANITIZERS = {
    "plain": [],
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=300)
    return r.returncode, r.stdout + r.stderr


def _build_and_run(compiler, srcs, flags, out, extra):
    rc, log = _run([compiler, "-O1", "-g", "-I" + INCLUDE, "-I" + CSRC] + flags + srcs + ["-o", out] + extra)
    assert rc == 0, log
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    rc, log = _run([out], env=env)
    assert rc == 0, log
    return log


@pytest.mark.parametrize("san", list(SANITIZERS))
def test_scheduler_core_with_fake_executor(san, tmp_path):
    log = _build_and_run("g++", [SCHED_TEST], ["-std=c++17", "-pthread"] + SANITIZERS[san],
                         str(tmp_path / ("sched_" + san)), [])
    assert "all passed" in log


@pytest.mark.parametrize("san", ["plain", "asan_ubsan"])
def test_oracle_under_sanitizers(san, tmp_path):
    log = _build_and_run("gcc", [ORACLE_DRIVER] + ORACLE_SRCS, ["-std=c11"] + SANITIZERS[san],
                         str(tmp_path / ("oracle_" + san)), ["-lm"])
    assert "all passed" in log
