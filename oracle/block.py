"""O4: the paper's block Lanczos (Algorithm 1) with block Gauss quadrature.

Test infrastructure only (see ``oracle/__init__``).

Algorithm 1 started from V_j = I_s (x) |v_j> (dim x d_s, V^T V = I):
    Q_1 = V; for j = 1..k:  Z = H Q_j - Q_{j-1} B_{j-1}^T;  A_j = Q_j^T Z;
                           Z = Z - Q_j A_j;  (Q_{j+1}, B_j) = QR(Z)
builds the block tridiagonal T (A_j on the diagonal, B_j below, B_j^T above).
The quadratic form (I_s (x) <v|) f(H) (I_s (x) |v>) is approximated by
E_1^T f(T) E_1 (eqn:fT; exact for polynomials of degree <= 2k-1), and the
partial-trace estimator averages it over j (eqn:trB_est).  The exponential is
shifted by E0 = the smallest eigenvalue over all T_j (overflow remedy of the
section on the mean force Hamiltonian).
"""
from __future__ import annotations

import numpy as np

from .exact import finalize
from .lanczos import lanczos, quad_weight, min_ritz, TAU_FP64
from .rng import bath_vectors
from .spin import sparse_bath_hamiltonian, sparse_hamiltonian


def block_lanczos(apply, v: np.ndarray, k: int):
    """Algorithm 1.  Returns the block tridiagonal T (k*b x k*b)."""
    dim, b = v.shape
    q = v.copy()
    q_prev = np.zeros_like(q)
    b_prev = np.zeros((b, b))
    t = np.zeros((k * b, k * b))
    for j in range(k):
        z = apply(q) - q_prev @ b_prev.T
        a = q.T @ z
        z = z - q @ a
        q_next, b_j = np.linalg.qr(z)
        t[j * b:(j + 1) * b, j * b:(j + 1) * b] = 0.5 * (a + a.T)
        if j + 1 < k:
            t[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = b_j
            t[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = b_j.T
        q_prev, q, b_prev = q, q_next, b_j
    return t


def block_quadrature(t: np.ndarray, b: int, beta: float, e0: float) -> np.ndarray:
    th, s = np.linalg.eigh(t)
    s1 = s[:b, :]
    return (s1 * np.exp(-beta * (th - e0))) @ s1.T


def solve(inst, betas=None) -> dict:
    betas = np.asarray(inst.betas if betas is None else betas, float)
    op = sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    opb = sparse_bath_hamiltonian(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    d_s, d_b, n_v = inst.d_s, inst.d_b, inst.n_v
    v = bath_vectors(inst.seed, n_v, inst.n_b)
    ts = []
    for j in range(n_v):
        vj = np.zeros((inst.dim, d_s))
        for m in range(d_s):
            vj[m * d_b:(m + 1) * d_b, m] = v[:, j]
        ts.append(block_lanczos(op.apply, vj, inst.k))
    e0 = min(float(np.linalg.eigvalsh(t)[0]) for t in ts)
    bath = [lanczos(opb.apply, v[:, j], inst.k, TAU_FP64, keep_q=False) for j in range(n_v)]
    e0b = min(min_ritz(a, b) for a, b, _, _ in bath)
    results = []
    for bt in betas:
        m = sum(block_quadrature(t, d_s, bt, e0) for t in ts) / n_v
        m_b = sum(nx * nx * quad_weight(a, b, bt, e0b) for a, b, _, nx in bath) / n_v
        results.append(finalize(m, m_b, e0, e0b, bt, d_b) | {"m": m, "m_b": m_b})
    return {"results": results, "e0": e0, "e0b": e0b}
