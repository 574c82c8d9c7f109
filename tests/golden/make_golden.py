"""Writes the stored reference results ``o3_<case>.json`` of this folder: the
oracle's FP64 run of the path (O3: per-column Lanczos, function
approximation of exp(-beta H/2), Gram, bath quadrature, finalisation) on
instances too large to recompute inside a test.

It calls only ``oracle`` and ``workloads``.  The columns run in a process
pool on the merged operator form (both pinned to the plain serial run by the
CPU tests).  Usage, from the repository root:

    python tests/golden/make_golden.py [case ...]     (default: every case)

The 2 + 18 case is the long-range workload of the benchmark itself (64 start
columns, k = 60, four temperatures); it takes about 20 minutes on 8 cores.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import lanczos as olz  # noqa: E402
from workloads import cfg_long_range, long_range_xx_zz, tfim_request  # noqa: E402

# name -> instance; the GPU tests rebuild the same instances from this table
CASES = {
    # the benchmark's workload: 2 + 18 spins, h = 0.5, n_v = 16, k = 60, 4 betas
    "lr_2+18_h0.5": lambda: cfg_long_range(0),
    # 22 bits: transverse-field chain request (1 + 21 spins)
    "tfim_1+21": lambda: tfim_request(3, n_range=(22, 22), n_v=2, k=30),
    # 21 bits: long-range XX+ZZ (1 + 20 spins)
    "lr_1+20": lambda: long_range_xx_zz(1, 20, 1.0, 81, betas=(0.5, 2.0), n_v=2, k=30),
}


def path(name: str) -> str:
    return os.path.join(HERE, f"o3_{name}.json")


def load(name: str) -> dict:
    with open(path(name)) as f:
        d = json.load(f)
    for r in d["results"]:
        for key in ("rho", "h_star"):
            r[key] = np.asarray(r[key])
    return d


def write(name: str, nproc: int) -> None:
    inst = CASES[name]()
    t0 = time.time()
    with mp.get_context("spawn").Pool(nproc) as pool:
        out = olz.solve(inst, merged=True, mapper=lambda f, tasks: pool.imap(f, tasks))
    keys = ("rho", "h_star", "log_z", "log_z_t", "log_z_b", "entropy")
    doc = {
        "what": "oracle O3 (FP64) results, written by tests/golden/make_golden.py",
        "case": name, "instance": inst.name, "n_s": inst.n_s, "n_b": inst.n_b,
        "n_v": inst.n_v, "k": inst.k, "seed": inst.seed, "betas": list(map(float, inst.betas)),
        "e0": out["e0"], "e0b": out["e0b"],
        "seconds": round(time.time() - t0, 1), "processes": nproc,
        "results": [{key: (np.asarray(r[key]).tolist() if key in ("rho", "h_star") else float(r[key]))
                     for key in keys} for r in out["results"]],
    }
    with open(path(name), "w") as f:
        json.dump(doc, f, indent=1)
    print(f"{name}: {doc['seconds']} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        write(n, max(1, min(8, os.cpu_count() or 1)))
