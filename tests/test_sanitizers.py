"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

Two small drivers exercise the oracle's C entry points and the host-only
paths of the library's C ABI; each is built with both sanitizers (host code
only: device code is built as usual) and must run to completion with no
report.  The sanitizers abort on the first finding."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2109_07527_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_driver")
        subprocess.check_call(["gcc", "-std=c11", "-O1", "-g"] + SAN +
                              ["-o", exe, os.path.join(HERE, "oracle_driver.c"),
                               os.path.join(ROOT, "oracle", "crmc_oracle.c"), "-lm"])
        assert "oracle driver ok" in _run(exe)


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p if os.path.exists(p) else None


@pytest.mark.skipif(_hipcc() is None, reason="no hipcc")
def test_library_host_paths_under_sanitizers():
    hipcc = _hipcc()
    base = ["-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    # host-only sanitizer flags: each one right after -Xarch_host
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        host_san += ["-Xarch_host", f]
    # the kernel translation units (device code and thin launchers) are built
    # as the product builds them; the host paths under test at -O1 -g
    kernel_flags = ["-O3"] + base[1:]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src, san in (("crmc_kernels.hip", False), ("crmc_learn.hip", False), ("crmc_md.hip", False),
                         ("crmc_api.cpp", True)):
            o = os.path.join(d, src + ".o")
            flags = (base + host_san) if san else kernel_flags
            subprocess.check_call([hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", o],
                                  stderr=subprocess.DEVNULL)
            objs.append(o)
        drv = os.path.join(d, "host_driver.o")
        subprocess.check_call([hipcc] + base + host_san + ["-c", os.path.join(HERE, "host_driver.cpp"), "-o", drv],
                              stderr=subprocess.DEVNULL)
        exe = os.path.join(d, "host_driver")
        subprocess.check_call([hipcc, "--offload-arch=gfx950"] + host_san[:4] + ["-o", exe, drv] + objs,
                              stderr=subprocess.DEVNULL)
        assert "host driver ok" in _run(exe)
