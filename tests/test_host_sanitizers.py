"""The host half of the C-ABI (validation, planning, sizing) built with
AddressSanitizer and UBSan and driven on the CPU by tests/asan_host_paths.c.

The instrumented object holds the library's host code (capi.cpp); it is
linked ahead of libpdhg.so, so its pdhg_* definitions are the ones the driver
calls, while the kernel launchers come from the library.  Device code cannot
be sanitized on this hardware; its bounds are checked on the host before
every launch and by the GPU tests."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2508_16806_amd")
SAN = {"address": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined"],
       "thread": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=thread"]}
INC = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def built():
    from paper_2508_16806_amd import build as hb

    if hb.stale():
        hb.build()
    return hb.LIB


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_paths_under_sanitizers(built, tmp_path, kind):
    """AddressSanitizer + UBSan, then ThreadSanitizer (batches are validated
    and binned on several host threads)."""
    capi = os.path.join(PKG, "csrc", "capi.cpp")
    drv = os.path.join(ROOT, "tests", "asan_host_paths.c")
    flags = SAN[kind]
    _run(["g++", "-std=c++17"] + flags + INC + ["-c", capi, "-o", str(tmp_path / "capi.o")])
    _run(["gcc", "-std=c11"] + flags + INC + ["-c", drv, "-o", str(tmp_path / "drv.o")])
    exe = str(tmp_path / "host_paths")
    _run(["g++"] + flags + [str(tmp_path / "drv.o"), str(tmp_path / "capi.o"), built,
                            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=87"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "host paths ok" in r.stdout, out[-4000:]
