"""Parameter scans and observables on top of the solver (the paper's
numerical experiments on long-range chains): entropy over a grid of
temperatures and fields, the internal-energy deviation tr(H* rho*) -
tr(H_s rho_s), and the system-bath coupling sweep.  Every solve runs through
the C ABI (batched: one Lanczos run per Hamiltonian serves all its
temperatures); only d_s x d_s post-processing happens here.
"""
from __future__ import annotations

from typing import Callable, Iterable, List, Sequence

import numpy as np

from . import Hamiltonian, solve_batch


def bare_system_rho(hs: np.ndarray, beta: float) -> np.ndarray:
    """rho_s(beta) = exp(-beta H_s) / tr exp(-beta H_s) of the bare system."""
    w, v = np.linalg.eigh(hs)
    p = np.exp(-beta * (w - w.min()))
    p /= p.sum()
    return (v * p) @ v.T


def energy_deviation(result: dict, hs: np.ndarray, betas: Sequence[float]) -> np.ndarray:
    """tr(H*(beta) rho*(beta)) - tr(H_s rho_s(beta)) per temperature (Section
    "Deviation in internal energy"): zero when the system-bath coupling
    vanishes, where H* = H_s."""
    out = []
    for b, beta in enumerate(betas):
        out.append(float(np.trace(result["h_star"][b] @ result["rho"][b])
                         - np.trace(hs @ bare_system_rho(hs, beta))))
    return np.array(out)


def run(instances: Iterable, **opts) -> List[dict]:
    """One batched solve over the instances (each with its own temperatures,
    bath vectors, k and seed).  Returns per-instance result dicts with the
    instance's H_s attached."""
    insts = list(instances)
    hs = [Hamiltonian.from_instance(i) for i in insts]
    try:
        items = [dict(h=h, betas=i.betas, n_v=i.n_v, k=i.k, seed=i.seed) for h, i in zip(hs, insts)]
        out = solve_batch(items, **opts)
        for o, h in zip(out, hs):
            o["h_s"] = h.system_matrix()
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
        rows.append(energy_deviation(r, r["h_s"], i.betas))
    return np.array(rows)
