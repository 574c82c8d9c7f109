"""O1 (dense exact answer) and O2 (exact typicality with the same bath vectors).

Test infrastructure only (see ``oracle/__init__``).

O1 follows the paper's definitions directly: rho*(beta) = tr_b exp(-beta H_t) /
Z_t, Z* = Z_t / Z_b and H*(beta) = -(1/beta) ln[tr_b exp(-beta H_t) / Z_b]
(Introduction, eqn:HMF); the von Neumann entropy is -tr rho* ln rho*
(Section "von Neumann entropy").  The matrix exponential comes from a dense
symmetric eigendecomposition, shifted by the ground energy to avoid overflow.

O2 replaces the partial trace by the n_v-sample average of eqn:trace_est with
the *same* seeded Rademacher vectors as the Krylov path, but evaluates each
quadratic form exactly (dense).  It isolates the stochastic error from the
Krylov error.
"""
from __future__ import annotations

import numpy as np

from .rng import bath_vectors
from .spin import bath_terms, dense_hamiltonian


def partial_trace_bath(a: np.ndarray, d_s: int, d_b: int) -> np.ndarray:
    """tr_b of an operator on C^{d_s} (x) C^{d_b} (system index major)."""
    return np.trace(a.reshape(d_s, d_b, d_s, d_b), axis1=1, axis2=3)


def _logsumexp(x: np.ndarray) -> float:
    m = x.max()
    return float(m + np.log(np.exp(x - m).sum()))


def finalize(m: np.ndarray, m_b: float, e0: float, e0b: float, beta: float, d_b: int) -> dict:
    """Turn the averaged d_s x d_s matrix M ~ V^T exp(-beta (H_t - e0)) V and the
    bath scalar m_b ~ v^T exp(-beta (H_b - e0b)) v into the outputs.

    With E[v v^T] = I/d_b:  E[M] = exp(beta e0) tr_b exp(-beta H_t) / d_b and
    E[m_b] = exp(beta e0b) Z_b / d_b, hence
      rho*   = M / tr M                          (ratio of sums, eqn:rho_est)
      ln Z_t = ln tr M - beta e0 + ln d_b
      ln Z_b = ln m_b - beta e0b + ln d_b
      ln Z*  = ln Z_t - ln Z_b
      H*     = U diag(-(1/beta) ln(mu_i / m_b) + e0 - e0b) U^T   (eqn:H_est),
    taken through the eigenvalues mu_i of M as the paper suggests (no matrix
    logarithm).  mu_i is clamped at mu_max * 2^-52 before the logarithm; the
    entropy uses 0 ln 0 = 0."""
    m = 0.5 * (m + m.T)
    mu, u = np.linalg.eigh(m)
    tr = float(np.trace(m))
    rho = m / tr
    log_z_t = np.log(tr) - beta * e0 + np.log(d_b)
    log_z_b = np.log(m_b) - beta * e0b + np.log(d_b)
    mu_c = np.maximum(mu, mu.max() * 2.0 ** -52)
    h_eig = -np.log(mu_c / m_b) / beta + e0 - e0b
    h_star = (u * h_eig) @ u.T
    p = np.clip(mu / mu.sum(), 0.0, None)
    nz = p > 0
    ent = float(-(p[nz] * np.log(p[nz])).sum())
    return {"rho": rho, "h_star": h_star, "log_z": float(log_z_t - log_z_b),
            "log_z_t": float(log_z_t), "log_z_b": float(log_z_b), "entropy": ent,
            "mu": mu}


def exact_rdm(inst, beta: float) -> dict:
    """O1: exact rho*, H*, ln Z*, S of an instance at one beta (dense, N <= 13)."""
    n, d_s, d_b = inst.n, inst.d_s, inst.d_b
    h = dense_hamiltonian(n, inst.couplings, inst.hx, inst.hz)
    e, u = np.linalg.eigh(h)
    e0 = e[0]
    a = (u * np.exp(-beta * (e - e0))) @ u.T            # exp(-beta (H - e0))
    r = partial_trace_bath(a, d_s, d_b)                 # exp(beta e0) tr_b exp(-beta H)
    r = 0.5 * (r + r.T)
    bc, bhx, bhz = bath_terms(inst.n_s, inst.couplings, inst.hx, inst.hz)
    eb = np.linalg.eigvalsh(dense_hamiltonian(inst.n_b, bc, bhx, bhz))
    log_z_t = float(np.log(np.trace(r)) - beta * e0)
    log_z_b = _logsumexp(-beta * eb)
    mu, w = np.linalg.eigh(r)
    h_eig = -(np.log(mu) - beta * e0 - log_z_b) / beta
    p = mu / mu.sum()
    p = p[p > 0]
    return {"rho": r / np.trace(r), "h_star": (w * h_eig) @ w.T,
            "log_z": log_z_t - log_z_b, "log_z_t": log_z_t, "log_z_b": log_z_b,
            "entropy": float(-(p * np.log(p)).sum()), "e_t": float(e0),
            "e_b": float(eb[0]), "mu": mu}


def start_columns(inst) -> np.ndarray:
    """(dim, d_s*n_v) start block: column c = j*d_s + m is |m> (x) |v_j>."""
    d_s, d_b, n_v = inst.d_s, inst.d_b, inst.n_v
    v = bath_vectors(inst.seed, n_v, inst.n_b)
    x = np.zeros((inst.dim, d_s * n_v))
    for j in range(n_v):
        for m in range(d_s):
            x[m * d_b:(m + 1) * d_b, j * d_s + m] = v[:, j]
    return x


def exact_typicality(inst, betas=None) -> list:
    """O2: the n_v-sample average with the same bath vectors, each quadratic
    form evaluated exactly with the dense exponential."""
    betas = inst.betas if betas is None else betas
    n, d_s, d_b, n_v = inst.n, inst.d_s, inst.d_b, inst.n_v
    h = dense_hamiltonian(n, inst.couplings, inst.hx, inst.hz)
    e, u = np.linalg.eigh(h)
    bc, bhx, bhz = bath_terms(inst.n_s, inst.couplings, inst.hx, inst.hz)
    eb, ub = np.linalg.eigh(dense_hamiltonian(inst.n_b, bc, bhx, bhz))
    x = start_columns(inst)
    v = bath_vectors(inst.seed, n_v, inst.n_b)
    ux = u.T @ x
    ubv = ub.T @ v
    out = []
    for beta in betas:
        g = ux * np.exp(-beta * (e - e[0]))[:, None]
        full = ux.T @ g                                   # C x C
        m = np.zeros((d_s, d_s))
        for j in range(n_v):
            sl = slice(j * d_s, (j + 1) * d_s)
            m += full[sl, sl]
        m /= n_v
        m_b = float((ubv ** 2 * np.exp(-beta * (eb - eb[0]))[:, None]).sum() / n_v)
        out.append(finalize(m, m_b, e[0], eb[0], beta, d_b) | {"m": m, "m_b": m_b})
    return out
