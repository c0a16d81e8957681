"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a driver
(oracle/sanitize_main.c) that includes the oracle source calls every entry
point on a small scene (SH degrees 0 and 2; FP32, BF16 and FP64 targets; one
and two OpenMP threads).  The sanitized build must run clean, leaks included;
a build with a planted out-of-bounds read must be reported, which shows that
the instrumentation is active."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "oracle", "sanitize_main.c")
FLAGS = ["-std=gnu11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-fopenmp"]


def _build(tmp_path, extra=()):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oc_san")
    r = subprocess.run([gcc, *FLAGS, *extra, "-I", os.path.join(ROOT, "oracle"), DRIVER, "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_clean_under_sanitizers(tmp_path):
    r = _run(_build(tmp_path))
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report
    assert "ERROR: LeakSanitizer" not in report, report
    assert "ran clean" in r.stdout


def test_sanitizer_reports_a_planted_read(tmp_path):
    r = _run(_build(tmp_path, ["-DOC_SANITIZE_SELFTEST"]))
    assert r.returncode != 0
    # whichever sanitizer sees it first: ASan's heap check or UBSan's object-size check
    assert "heap-buffer-overflow" in r.stderr or "insufficient space for an object" in r.stderr, r.stderr
