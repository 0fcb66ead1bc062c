"""Sanitizer builds of the host code (CPU only, no GPU call):

* the planner (network construction, greedy and TreeSA optimizers with trials
  on several threads, slicing, open vertices, explicit trees, executor
  program) under AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
  ThreadSanitizer, driven by tests/sanitize/planner_driver.cpp;
* the CPU oracle (brute force, elimination in every algebra, polynomial
  elimination, plan follower with slices) under AddressSanitizer +
  UndefinedBehaviorSanitizer, driven by tests/sanitize/oracle_driver.c.

Each sanitizer aborts the driver on a finding, so a zero exit status is the
pass.  The GPU-side code (kernels, executors, server) is not covered here:
GPU sanitizers are not available for it.
"""
import concurrent.futures as cf
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_00227_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
CXX = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
       "-I" + os.path.join(ROOT, "include")]

pytestmark = pytest.mark.slow


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def _planner(tmp, flags):
    objs = []
    with cf.ThreadPoolExecutor(3) as ex:
        futs = []
        for f in ("net", "optimize", "plan"):
            o = os.path.join(tmp, f + ".o")
            objs.append(o)
            futs.append(ex.submit(_run, CXX + flags + ["-c", os.path.join(CSRC, f + ".cpp"), "-o", o]))
        for f in futs:
            f.result()
    exe = os.path.join(tmp, "planner_driver")
    _run(CXX + flags + [os.path.join(SAN, "planner_driver.cpp")] + objs + ["-o", exe, "-lpthread"])
    return exe


def test_planner_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = _planner(str(tmp_path), ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    r = _run([exe, "16"], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "0 failed checks" in r.stdout


def test_planner_threads_under_thread_sanitizer(tmp_path):
    exe = _planner(str(tmp_path), ["-fsanitize=thread"])
    r = _run([exe, "8"], env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert "0 failed checks" in r.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "0 failed checks" in r.stdout
