"""O8: the low-temperature limit (Section "High and low temperature limits"
and the appendix deriving them).

Test infrastructure only (see ``oracle/__init__``).

As beta -> infinity the total state tends to the uniform mixture of the r
ground states of H_t, so rho*(inf) = (1/r) sum_i tr_b |psi_i><psi_i|, and
H*(inf) = (E_t - E_b) I with E_t, E_b the ground energies of H_t and H_b.

``exact`` evaluates this by dense diagonalisation.  ``lanczos_ritz`` follows
the algorithm the library uses, step by step: a plain Lanczos run on each of
n_v seeded full-space Rademacher vectors, the lowest Ritz pair of each T, the
columns whose lowest Ritz value reached the smallest one, their Ritz vectors'
Gram matrix, an orthonormal basis of its dominant eigenvectors (the ground
space), and the partial trace of the projector onto it.
"""
from __future__ import annotations

import numpy as np

from .exact import partial_trace_bath
from .lanczos import lanczos
from .rng import bath_vector
from .spin import bath_terms, dense_hamiltonian, sparse_bath_hamiltonian, sparse_hamiltonian


def _entropy(rho: np.ndarray) -> float:
    p = np.clip(np.linalg.eigvalsh(rho), 0.0, None)
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


def exact(inst, rel_tol: float = 1e-9) -> dict:
    """Dense ground space of H_t (eigenvalues within rel_tol * spread of the
    lowest), its partial trace, and the ground energies."""
    h = dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    w, v = np.linalg.eigh(h)
    tol = rel_tol * max(1.0, float(np.abs(w).max()))
    g = v[:, w <= w[0] + tol]
    r = g.shape[1]
    rho = partial_trace_bath(g @ g.T, inst.d_s, inst.d_b) / r
    bc, bhx, bhz = bath_terms(inst.n_s, inst.couplings, inst.hx, inst.hz)
    e_b = float(np.linalg.eigvalsh(dense_hamiltonian(inst.n_b, bc, bhx, bhz))[0])
    return {"rho": rho, "e_total": float(w[0]), "e_bath": e_b, "degeneracy": r,
            "entropy": _entropy(rho), "h_star": (w[0] - e_b) * np.eye(inst.d_s)}


def lanczos_ritz(inst, n_v: int, k: int, seed: int, e_rel: float = 1e-9, m_rel: float = 1e-6) -> dict:
    """The library's algorithm in FP64 on the same seeded start vectors."""
    op = sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    opb = sparse_bath_hamiltonian(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    runs = []
    for c in range(n_v):
        x0 = bath_vector(seed, c, inst.n)
        a, b, q, _ = lanczos(op.apply, x0, min(k, inst.dim), keep_q=True)
        t = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        th, s = np.linalg.eigh(t)
        runs.append((th[0], q @ s[:, 0], np.abs(th).max()))
    e_t = min(r[0] for r in runs)
    scale = max(1.0, max(r[2] for r in runs))
    psi = np.stack([r[1] for r in runs if r[0] <= e_t + e_rel * scale], axis=1)
    m = psi.T @ psi
    lam, u = np.linalg.eigh(0.5 * (m + m.T))
    keep = lam > m_rel * lam[-1]
    phi = psi @ (u[:, keep] / np.sqrt(lam[keep]))
    r = phi.shape[1]
    rho = partial_trace_bath(phi @ phi.T, inst.d_s, inst.d_b)
    rho = 0.5 * (rho + rho.T) / np.trace(rho)
    e_b = min(float(np.linalg.eigvalsh(np.diag(a) + np.diag(b, 1) + np.diag(b, -1))[0])
              for a, b, _, _ in (lanczos(opb.apply, bath_vector(seed, c, inst.n_b), min(k, inst.d_b),
                                         keep_q=False) for c in range(n_v)))
    return {"rho": rho, "e_total": float(e_t), "e_bath": e_b, "degeneracy": r, "entropy": _entropy(rho),
            "h_star": (e_t - e_b) * np.eye(inst.d_s)}
