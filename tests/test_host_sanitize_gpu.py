"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the GPU.

build() compiles tests/host_sanitize_driver.cpp together with every library source into one
program whose host code (the C-ABI layer, the search and surrogate host code) is instrumented;
the device code is the library's. The program drives every C-ABI entry point on small seeded
inputs -- every kernel form and block length, enqueued and blocking calls, the batch, the
autotuner, a captured graph, the allocation-free entry point, the surrogate (prediction,
gradient, training, checkpoint, shortlist, screening), the search, and the error paths -- and
requires all evaluation paths to agree bit for bit. A sanitizer report (heap or stack overflow,
use after free, a leak of the host layer, signed overflow, a misaligned or oversized shift)
aborts it and fails the test. Leaks inside the HIP runtime's own libraries are not ours and are
suppressed.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "_build", "host_sanitize_driver")


def test_c_abi_host_code_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(BIN):
        pytest.fail(f"{BIN} is missing: run __graft_entry__.build() first")
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler-register\n"
                    "leak:libdrm\nleak:libnuma\n")
    env = dict(os.environ)
    env.update({
        "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1:halt_on_error=1",
        "LSAN_OPTIONS": f"suppressions={supp}:print_suppressions=0",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    print("[host-sanitize] running the instrumented C-ABI driver", flush=True)
    res = subprocess.run([BIN, str(tmp_path)], env=env, capture_output=True, text=True,
                         timeout=240)
    out = res.stdout[-6000:] + res.stderr[-6000:]
    print(out, flush=True)
    assert res.returncode == 0, out
    assert "all checks passed" in res.stdout
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out
    assert "runtime error" not in out
