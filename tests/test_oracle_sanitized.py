"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's source is compiled with -fsanitize=address,undefined into a
temporary library and the whole pin suite (tests/test_oracle_pins.py) runs
against it in a subprocess, with the sanitizer runtimes preloaded into the
Python interpreter: any out-of-bounds access, use after free or undefined
operation in the oracle aborts the run.  A planted one-past-the-end write
checks that the sanitized build really is the one being exercised."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bjp_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


ASAN, UBSAN = _runtime("libasan.so"), _runtime("libubsan.so")
pytestmark = pytest.mark.skipif(not (ASAN and UBSAN), reason="gcc sanitizer runtimes not installed")


def _build(src_text, out):
    c = out.with_suffix(".c")
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-Wno-unknown-pragmas", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", str(out), str(c), "-lm"])
    return out


def _run_pins(lib, k=None):
    env = dict(os.environ, BJP_ORACLE_LIB=str(lib), LD_PRELOAD=f"{ASAN}:{UBSAN}",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    # -s: a sanitizer report goes to the real stderr (fd capture would hide it)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", PINS]
    if k:
        cmd += ["-k", k]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def test_pins_pass_under_sanitizers(tmp_path):
    res = _run_pins(_build(open(SRC).read(), tmp_path / "liboracle_san.so"))
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out


def test_sanitized_build_catches_planted_overflow(tmp_path):
    """r[n] written one past the end of the PCG's residual: the sanitized run
    must abort with an AddressSanitizer report."""
    src = open(SRC).read()
    old = "        for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];\n"
    assert src.count(old) == 1
    lib = _build(src.replace(old, old.replace("i < n", "i <= n")), tmp_path / "liboracle_bad.so")
    res = _run_pins(lib, k="pcg_single_block")
    assert res.returncode != 0
    assert "heap-buffer-overflow" in res.stdout + res.stderr
