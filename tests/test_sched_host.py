"""The serving loop's scheduler (csrc/sched.hpp, shared with the GPU server)
driven by a fake device on the CPU, in sanitizer builds of the host code:

* AddressSanitizer + UndefinedBehaviorSanitizer (leaks, use after free,
  double release of a request, signed overflow in the counters);
* ThreadSanitizer (the lock over requests, queue and counters, shared by the
  client calls and the worker thread).

The cases (tests/sched_fake.cpp): admission under both limits in submission
order, head-of-line blocking, rejection at submission, cancel of queued and
running requests, release only in a terminal state, LM_NOT_CONVERGED, a
failed start, a failed round, destruction with requests queued and running,
four client threads submitting, cancelling and releasing at random, and the
release of kept device memory only after the worker has stayed idle.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_fake.cpp")
INC = [os.path.join(ROOT, "paper_2511_12450_amd", "csrc"), os.path.join(ROOT, "include")]

CASES = ["admission_fifo", "head_of_line", "reject", "cancel_queued", "cancel_running", "release", "not_converged",
         "start_failure", "round_failure", "destroy_in_flight", "concurrent_clients", "idle_release"]

SANITIZERS = {"asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
              "tsan": ["-fsanitize=thread"]}


def _build(tmp_path_factory, kind):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp(kind) / "sched_fake")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", "-Wall", "-Werror"]
    cmd += SANITIZERS[kind] + [f"-I{d}" for d in INC] + [SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


@pytest.fixture(scope="module")
def asan_bin(tmp_path_factory):
    return _build(tmp_path_factory, "asan_ubsan")


@pytest.fixture(scope="module")
def tsan_bin(tmp_path_factory):
    return _build(tmp_path_factory, "tsan")


def _run(exe, case, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe, case], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0 and f"ok {case}" in r.stdout, f"{case}: rc={r.returncode}\n{r.stdout}\n{r.stderr[-4000:]}"


@pytest.mark.parametrize("case", CASES)
def test_scheduler_asan_ubsan(asan_bin, case):
    _run(asan_bin, case, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                          "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


@pytest.mark.parametrize("case", CASES)
def test_scheduler_tsan(tsan_bin, case):
    _run(tsan_bin, case, {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
