"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (gcc) and the library's scheduling code (scheduler.cpp and
stages.cpp; hipcc, sanitizers on the host side only) are built with the
sanitizers and driven by the programs in tests/sanitize/, which also check
their results. Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
REPORTS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")


def run_clean(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert not any(s in r.stderr for s in REPORTS), r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fopenmp", "-D_GNU_SOURCE", "-std=c11", os.path.join(ROOT, "oracle", "qsim_oracle.c"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    assert "ok" in run_clean(exe)


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")), reason="no hipcc")
def test_scheduler_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    exe = str(tmp_path / "sched_driver")
    csrc = os.path.join(ROOT, "paper_1704_01127_amd", "csrc")
    # sanitizers on the host pass only (-Xarch_host before each flag)
    cmd = [hipcc, "-x", "hip", "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-command-line-argument",
           "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
           os.path.join(ROOT, "tests", "sanitize", "sched_driver.cpp"), os.path.join(csrc, "scheduler.cpp"),
           os.path.join(csrc, "stages.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    assert "ok" in run_clean(exe)
