"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the oracle's C entry points (built with gcc) and the library's host-side
pattern checks and sweep schedules (analysis.cpp, built with hipcc with the
sanitizers on the host side only), each driven by a small program in
tests/sanitize/ on seeded inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(HERE, "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "mpk_oracle.c"), "-lm"])
    _run(exe)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_host_schedules_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-std=c++20", "-O1",
                           "-g"] + host + ["-I", os.path.join(ROOT, "include"),
                                           os.path.join(HERE, "plan_check.cpp"),
                                           os.path.join(ROOT, "paper_2504_14498_amd", "csrc",
                                                        "analysis.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    _run(exe)
