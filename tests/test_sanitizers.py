"""Address and undefined-behaviour sanitizer builds of the host C code (CPU only).

The oracle (oracle/oracle.c) and the seeded input generators (gen/gen.c) are compiled with
gcc's -fsanitize=address,undefined into a scratch directory; the oracle pins, the generator
tests and the strong-baseline tests then run in a child Python process that loads those
instrumented copies (SPLIT_ORACLE_LIB, SPLIT_GEN_LIB) with the sanitizer runtimes preloaded.
Any report (out-of-bounds access, use after free, signed overflow, misaligned or oversized
shift, ...) aborts the child and fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _build(src, out, extra):
    subprocess.check_call(["gcc", "-std=gnu11", "-fPIC", "-shared", "-pthread", *SAN, "-o",
                           out, src, *extra])


@pytest.mark.slow
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    olib = str(tmp_path / "liboracle_san.so")
    glib = str(tmp_path / "libsplitgen_san.so")
    _build(os.path.join(ROOT, "oracle", "oracle.c"), olib, [])
    _build(os.path.join(ROOT, "gen", "gen.c"), glib, ["-lm"])
    env = dict(os.environ)
    # the sanitizer runtimes go first; anything already preloaded stays after them
    preload = ":".join(p for p in (asan, ubsan, os.environ.get("LD_PRELOAD", "")) if p)
    env.update({
        "SPLIT_ORACLE_LIB": olib,
        "SPLIT_GEN_LIB": glib,
        "LD_PRELOAD": preload,
        # the Python interpreter itself is not instrumented: its allocations are not leaks
        # of ours
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "OMP_NUM_THREADS": "4",
    })
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_oracle.py", "test_gen.py", "test_cpu_baseline.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                          "-p", "no:cacheprovider", *tests],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout[-4000:] + res.stderr[-4000:]
    assert res.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    # the setup does catch a planted heap overflow in a library loaded the same way
    bad_c = tmp_path / "planted.c"
    bad_c.write_text("#include <stdlib.h>\n"
                     "int planted(int i) { int *a = malloc(4 * sizeof(int));\n"
                     "  for (int k = 0; k < 4; ++k) a[k] = k;\n"
                     "  int v = a[i]; free(a); return v; }\n")
    bad_so = str(tmp_path / "libplanted.so")
    _build(str(bad_c), bad_so, [])
    planted = subprocess.run(
        [sys.executable, "-c",
         f"import ctypes; l = ctypes.CDLL({bad_so!r}); print(l.planted(4))"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert planted.returncode != 0, planted.stdout
    assert "heap-buffer-overflow" in planted.stderr or "runtime error" in planted.stderr
    # the child really loaded the instrumented copies
    probe = subprocess.run(
        [sys.executable, "-c",
         "import oracle, gen; oracle._load(); gen._load(); "
         "print(oracle._LIB); print(gen._LIB)"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert olib in probe.stdout and glib in probe.stdout
