"""Build the gfx950 shared library ``librdm.so`` in-tree with hipcc.

Every HIP/C++ source under ``csrc/`` is compiled for gfx950 and linked into
one C-ABI shared library next to this file.  Packed FP32 instructions are
disabled for all device code (``-packed-fp32-ops``); hipcc's host pass warns
that it does not know the feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librdm.so")
BUILD_DIR = os.path.join(ROOT, "_build", "librdm")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CXXFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f"-I{os.path.join(ROOT, 'include')}"]


# host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# compiled as usual): a separate library for the CPU tests of the host code
SAN_DIR = os.path.join(ROOT, "_build", "librdm_san")
SAN_LIB = os.path.join(SAN_DIR, "librdm_san.so")
SANFLAGS = ["-g", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_DIR if sanitize else BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC, *CXXFLAGS, *(SANFLAGS if sanitize else []), *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link ``librdm.so`` (sanitize: the host-side
    sanitizer build ``_build/librdm_san/librdm_san.so``); returns its path."""
    out_dir, lib = (SAN_DIR, SAN_LIB) if sanitize else (BUILD_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, sanitize), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrocprofiler-sdk-roctx",
           "-lpthread"]
    if sanitize:
        # host runtimes only: the device code carries no sanitizer
        cmd[1:1] = ["-shared-libsan", "-fsanitize=address,undefined", "-fno-gpu-sanitize"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
