"""Build libsplitgpu.so (HIP kernels + C-ABI host layer) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsplitgpu.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("split_kernels.hip", "split_host.cpp", "nn_kernels.hip", "nn_host.cpp",
            "search_host.cpp")]
ARCH = os.environ.get("SPLITGPU_ARCH", "gfx950")


def hipcc_command(out: str) -> list[str]:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed-FP32 instructions anywhere in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-command-line-argument",
        "-o", out, *SOURCES,
    ]


# A test program that drives every C-ABI entry point with the host code (the C-ABI layer, the
# search and surrogate host code, the test program itself) under AddressSanitizer and
# UndefinedBehaviorSanitizer; the device code is compiled as in the library.
ROOT = os.path.dirname(HERE)
SAN_DRIVER = os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")
SAN_BIN = os.path.join(ROOT, "_build", "host_sanitize_driver")
HOST_SAN_FLAGS = ("-Xarch_host -g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                  "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer")


def host_sanitize_command(out: str) -> list[str]:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        *HOST_SAN_FLAGS.split(),
        "-Wall", "-Wno-unused-command-line-argument",
        "-o", out, SAN_DRIVER, *SOURCES,
    ]


def build_host_sanitize_driver(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(SAN_BIN), exist_ok=True)
    tmp = SAN_BIN + ".tmp"
    cmd = host_sanitize_command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{res.stderr}")
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, SAN_BIN)
    return SAN_BIN


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{' '.join(cmd)}\n{res.stderr}")
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_host_sanitize_driver(verbose=True))
