"""Parameter scans and observables on top of the solver (the paper's
numerical experiments on long-range chains): entropy over a grid of
temperatures and fields, the internal-energy deviation tr(H* rho*) -
tr(H_s rho_s), and the system-bath coupling sweep.  Every solve and the
deviation run through the C ABI (batched: one Lanczos run per Hamiltonian
serves all its temperatures); this module only arranges the results.
"""
from __future__ import annotations

from typing import Callable, Iterable, List, Sequence

import numpy as np

from . import Hamiltonian, solve_batch


def run(instances: Iterable, **opts) -> List[dict]:
    """One batched solve over the instances (each with its own temperatures,
    bath vectors, k and seed).  Returns per-instance result dicts with the
    instance's H_s and the internal-energy deviation tr(H* rho*) -
    tr(H_s rho_s) per temperature (Section "Deviation in internal energy",
    computed by the library) attached."""
    insts = list(instances)
    hs = [Hamiltonian.from_instance(i) for i in insts]
    try:
        items = [dict(h=h, betas=i.betas, n_v=i.n_v, k=i.k, seed=i.seed) for h, i in zip(hs, insts)]
        out = solve_batch(items, **opts)
        for o, h, i in zip(out, hs, insts):
            o["h_s"] = h.system_matrix()
            if o["status"] == 0:
                o["deviation"] = h.energy_deviation(i.betas, o["rho"], o["h_star"])
    finally:
        for h in hs:
            h.close()
    return out


def entropy_grid(make: Callable[[float], object], fields: Sequence[float], **opts) -> np.ndarray:
    """von Neumann entropy S(field, beta): make(field) returns an instance
    whose betas are the temperature grid (the paper's entropy phase plot).
    Shape (len(fields), len(betas))."""
    res = run((make(f) for f in fields), **opts)
    for r in res:
        if r["status"] != 0:
            raise RuntimeError(f"solve failed with status {r['status']}")
    return np.array([r["entropy"] for r in res])


def deviation_scan(make: Callable[[float], object], values: Sequence[float], **opts) -> np.ndarray:
    """Internal-energy deviation for each parameter value (e.g. the power-law
    exponent alpha or the coupling scale eps); make(value) returns the
    instance.  Shape (len(values), len(betas))."""
    insts = [make(v) for v in values]
    res = run(insts, **opts)
    rows = []
    for r, i in zip(res, insts):
        if r["status"] != 0:
            raise RuntimeError(f"solve failed with status {r['status']}")
        rows.append(r["deviation"])
    return np.array(rows)
