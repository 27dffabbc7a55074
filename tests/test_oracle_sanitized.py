"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): every C entry point on small 2D and 3D grids at orders 4 and 16, with
sparse points on the grid's last cell and in the layer, records of 1, 2 and
9 samples and several checkpoint segments (tests/sanitize/oracle_driver.c).
A control program with a one-element heap overflow, built the same way,
must be stopped by the sanitizers, so a clean run means something."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-static-libasan", "-fopenmp", "-std=c11"]

CONTROL = r"""
#include <stdlib.h>
int main(void) { volatile int* a = malloc(4 * sizeof(int)); a[4] = 1; int r = a[0]; free((void*)a); return r; }
"""


def _build(src, out, tmp_path):
    r = subprocess.run(["gcc"] + FLAGS + ["-o", str(out), str(src), "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("AddressSanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_sanitizer_catches_a_heap_overflow(tmp_path):
    src = tmp_path / "control.c"
    src.write_text(CONTROL)
    exe = tmp_path / "control"
    _build(src, exe, tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode != 0 and ("AddressSanitizer" in r.stderr or "runtime error" in r.stderr)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    _build(os.path.join(HERE, "sanitize", "oracle_driver.c"), exe, tmp_path)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle sanitized run ok" in r.stdout
