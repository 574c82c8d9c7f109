"""The library's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer: a sanitizer build of every source (host side
only; the device code is compiled as usual) and a plain-C driver of the
host-only entry points (tests/san_host_checks.c).  Runs on the CPU."""
import glob
import importlib.util
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "_rdm_build", os.path.join(ROOT, "paper_2204_08147_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists("/opt/rocm/bin/hipcc")),
                    reason="needs the ROCm compilers")
def test_host_code_under_sanitizers(tmp_path):
    lib = _build_module().build(sanitize=True)
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    assert rt, "no sanitizer runtime"
    rtdir = os.path.dirname(rt[-1])
    exe = str(tmp_path / "san_host_checks")
    cmd = [CLANG, "-g", "-shared-libsan", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "san_host_checks.c"),
           "-L" + os.path.dirname(lib), "-lrdm_san", "-Wl,-rpath," + os.path.dirname(lib),
           "-Wl,-rpath," + rtdir, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "host checks passed" in r.stdout, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr, r.stderr
