"""Host-side native tests under the compilers' sanitizers (CPU only).

* The server's scheduler (paper_0904_4152_amd/csrc/scheduler.h, the same
  header the HIP server uses) against a fake executor with a simulated clock
  (tests/native/sched_fake.cpp): admission in arrival order, the memory
  budget, least-recently-used eviction, no overtaking of a waiting request,
  two iterations in flight, status mapping of failures and NaN results --
  built plain, with ThreadSanitizer and with AddressSanitizer +
  UndefinedBehaviorSanitizer.
* The oracle (oracle/mg_oracle.c) driven through every function on small
  inputs (tests/native/oracle_sanitize.c) under AddressSanitizer +
  UndefinedBehaviorSanitizer.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_0904_4152_amd", "csrc")]
# ThreadSanitizer from the ROCm LLVM toolchain: the system GCC 11 runtime does
# not intercept pthread_cond_clockwait (condition_variable::wait_until on the
# steady clock) and then reports false lock-order errors.
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_ERRORS = ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "runtime error:",
              "ERROR: LeakSanitizer")


def _build_and_run(tmp, name, cmd, timeout=180):
    exe = os.path.join(tmp, name)
    subprocess.check_call(cmd + ["-o", exe])
    env = dict(os.environ)
    env.setdefault("ASAN_OPTIONS", "detect_leaks=1:abort_on_error=1")
    env.setdefault("TSAN_OPTIONS", "halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ALL PASS" in r.stdout, out[-4000:]
    for marker in SAN_ERRORS:
        assert marker not in out, out[-4000:]
    return r.stdout


SCHED = os.path.join(NATIVE, "sched_fake.cpp")
COMMON = ["-std=c++17", "-g", "-pthread"] + INC + [SCHED]


def test_scheduler_plain(tmp_path):
    out = _build_and_run(str(tmp_path), "sched", ["g++", "-O2"] + COMMON)
    for s in ("concurrent", "budget", "lru_eviction", "no_overtaking", "latency", "statuses",
              "executor_failure"):
        assert "PASS " + s in out


def test_scheduler_thread_sanitizer(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang++ not found")
    _build_and_run(str(tmp_path), "sched_tsan", [CLANG, "-O1", "-fsanitize=thread"] + COMMON)


def test_scheduler_address_ub_sanitizers(tmp_path):
    _build_and_run(str(tmp_path), "sched_asan",
                   ["g++", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer"] + COMMON)


def test_oracle_address_ub_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    _build_and_run(str(tmp_path), "oracle_san",
                   ["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-I", os.path.join(ROOT, "oracle"), os.path.join(NATIVE, "oracle_sanitize.c"),
                    os.path.join(ROOT, "oracle", "mg_oracle.c"), "-lm"])
