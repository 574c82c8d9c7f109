"""The C ABI from plain C: the example client compiles and links against
include/rdm.h and librdm.so with gcc; without a GPU it fails cleanly with the
library's error message; on the GPU its results match the oracle."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2204_08147_amd")


def _build(tmp_path):
    exe = str(tmp_path / "solve_chain")
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", f"-I{ROOT}/include", os.path.join(PKG, "examples", "solve_chain.c"),
           f"-L{PKG}", "-lrdm", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def _instance():
    from workloads import Instance
    cps = [(i, i + 1, 1.0, 1.0, 1.0) for i in range(3)]
    return Instance(1, 3, cps, np.zeros(4), np.full(4, 0.2), np.array([0.5, 2.0]), 4, 16, 7)


def test_c_client_builds_and_fails_cleanly_without_a_gpu(tmp_path):
    if not os.path.exists(os.path.join(PKG, "librdm.so")):
        pytest.skip("librdm.so not built")
    exe = _build(tmp_path)
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present; the GPU test runs the client")
    except ImportError:
        pass
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 1
    assert "rdm_solve failed" in r.stderr


@pytest.mark.gpu
def test_c_client_matches_oracle(tmp_path):
    from oracle import lanczos as olz
    exe = _build(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = {}
    for line in r.stdout.splitlines():
        name, b, *rest = line.split()
        vals[(name, int(b))] = np.array([float(x) for x in rest])
    want = olz.solve(_instance())["results"]
    tol = 1e-12  # FP64 path, as the other FP64 solve parity tests
    for b in range(2):
        assert np.abs(vals[("rho", b)].reshape(2, 2) - want[b]["rho"]).max() < tol
        assert np.abs(vals[("h_star", b)].reshape(2, 2) - want[b]["h_star"]).max() < tol * 10
        assert abs(vals[("log_z", b)][0] - want[b]["log_z"]) < tol
        assert abs(vals[("entropy", b)][0] - want[b]["entropy"]) < tol
