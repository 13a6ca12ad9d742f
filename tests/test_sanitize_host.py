"""Address and undefined-behaviour sanitizer runs of the host code (CPU only).

* The oracle (gcc, -fsanitize=address,undefined) under tests/sanitize/oracle_driver.c:
  every routine on degenerate and random small grids.
* The library's host code -- argument validation, workspace sizing, batch
  descriptions, the tuner's and status query's checks -- built with hipcc
  with the sanitizers on the host side only (-Xarch_host; the gfx950 device
  code is compiled normally and never launched), under
  tests/sanitize/abi_driver.cpp.

Builds are cached under tests/sanitize/_build keyed by a hash of their
sources and flags, so the library build (about a minute) runs only after a
change.
"""

import glob
import hashlib
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
BUILD = os.path.join(SAN, "_build")
CSRC = os.path.join(ROOT, "paper_2106_15869_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ORACLE_FLAGS = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
                "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
LIB_FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
             "-Xarch_host", "-fsanitize=address,undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _cached_build(name, sources, cmd_fn):
    h = hashlib.sha256()
    for p in sources:
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(cmd_fn("OUT")).encode())
    exe = os.path.join(BUILD, f"{name}-{h.hexdigest()[:16]}")
    if not os.path.exists(exe):
        os.makedirs(BUILD, exist_ok=True)
        for old in glob.glob(os.path.join(BUILD, f"{name}-*")):
            os.remove(old)
        tmp = exe + ".tmp%d" % os.getpid()
        r = subprocess.run(cmd_fn(tmp), capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        os.replace(tmp, exe)
    return exe


def _run(exe, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers():
    src = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "eik_oracle.c")]
    exe = _cached_build("oracle_driver", src,
                        lambda out: ["gcc"] + ORACLE_FLAGS + ["-o", out] + src + ["-lm"])
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                     "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "clean" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_address_and_ub_sanitizers():
    hips = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    deps = hips + sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [os.path.join(ROOT, "include", "eik.h"),
                                                                    os.path.join(SAN, "abi_driver.cpp")]
    exe = _cached_build("abi_driver", deps,
                        lambda out: [HIPCC] + LIB_FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", out,
                                                           os.path.join(SAN, "abi_driver.cpp")] + hips)
    # the HIP runtime's own allocations at exit are not this library's: leak
    # checking off, everything else on
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "clean" in out
