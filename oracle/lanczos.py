"""O3: the hot path's algorithm, step by step, in FP64 on the CPU.

Test infrastructure only (see ``oracle/__init__``).

For each start column x_c = |m> (x) |v_j> (c = j*d_s + m) this runs the
scalar case of Algorithm 1 (block size one, Section "Algorithm"): the
three-term Lanczos recurrence from q_1 = x / |x|, in which each new direction
is H q_j with its components along q_j and q_(j-1) removed and normalised,
a_j and b_j being the removed component along q_j and the norm of the rest.
There is no reorthogonalisation (Section "Finite precision arithmetic").
The run stops early (k_c = j) when b_j <= tau * max(|a_1..a_j|, b_1..b_{j-1}).
T = tridiag(b, a, b) of order k_c.  A Lanczos function approximation of
exp(-beta (H - E0)/2) x is  psi = |x| Q exp(-beta (T - E0)/2) e_1, where E0 is
the smallest Ritz value over all columns of the solve (the overflow shift of
Section "An algorithm for the mean force Hamiltonian").  Then

    M(beta) = (1/n_v) sum_j Psi_j^T Psi_j,   Psi_j = [psi_{j*d_s+m}]_m,

which equals V_j^T exp(-beta (H-E0)) V_j up to the Krylov error: the per-column
form of the block quadrature (eqn:fT, eqn:trB_est), exact when f = g^2 with
deg g <= k-1.  The bath scalar m_b(beta) is the Gauss quadrature
e_1^T exp(-beta (T_b - E0b)) e_1 of a Lanczos run on H_b from the same v_j
(eqn:H_est), averaged over j.  ``exact.finalize`` produces rho*, H*, ln Z*, S.
"""
from __future__ import annotations

import numpy as np

from .exact import finalize
from .rng import bath_vectors
from .spin import (merged_bath_hamiltonian, merged_hamiltonian, sparse_bath_hamiltonian,
                   sparse_hamiltonian)

TAU_FP64 = 1e-12


def lanczos(apply, x: np.ndarray, k: int, tau: float = TAU_FP64, keep_q: bool = True):
    """Plain Lanczos on one vector.  Returns (alpha[k_c], beta[k_c-1], Q or
    None, |x|)."""
    nx = float(np.sqrt(np.dot(x, x)))
    q = x / nx
    q_prev = np.zeros_like(q)
    b_prev = 0.0
    alphas, betas, qs = [], [], [q] if keep_q else None
    scale = 0.0
    for j in range(1, k + 1):
        w = apply(q) - b_prev * q_prev
        a = float(np.dot(q, w))
        w = w - a * q
        alphas.append(a)
        scale = max(scale, abs(a))
        if j == k:
            break
        b = float(np.sqrt(np.dot(w, w)))
        if b <= tau * scale:
            break
        scale = max(scale, b)
        betas.append(b)
        q_prev, q, b_prev = q, w / b, b
        if keep_q:
            qs.append(q)
    qmat = np.stack(qs, axis=1) if keep_q else None
    return np.array(alphas), np.array(betas), qmat, nx


def tridiag(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    return np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)


def fa_weights(alpha, beta, beta_t: float, e0: float) -> np.ndarray:
    """y = exp(-beta_t (T - e0)/2) e_1 through the eigendecomposition of T."""
    th, s = np.linalg.eigh(tridiag(alpha, beta))
    return s @ (np.exp(-0.5 * beta_t * (th - e0)) * s[0, :])


def quad_weight(alpha, beta, beta_t: float, e0: float) -> float:
    """Gauss quadrature e_1^T exp(-beta_t (T - e0)) e_1."""
    th, s = np.linalg.eigh(tridiag(alpha, beta))
    return float((s[0, :] ** 2 * np.exp(-beta_t * (th - e0))).sum())


def min_ritz(alpha, beta) -> float:
    return float(np.linalg.eigvalsh(tridiag(alpha, beta))[0])


_OPS = {}


def _operator(inst, which: int, merged: bool):
    """H_t (which = 0) or H_b (which = 1) of an instance, matrix-free
    (``merged`` = True: the merged form, fast enough for full-size reference
    runs).  A few operators are kept per process for repeated column runs."""
    key = (inst.n_s, inst.n_b, tuple(map(tuple, inst.couplings)), tuple(inst.hx), tuple(inst.hz),
           which, merged)
    if key not in _OPS:
        if len(_OPS) >= 4:
            _OPS.pop(next(iter(_OPS)))
        if which == 0:
            make = merged_hamiltonian if merged else sparse_hamiltonian
            _OPS[key] = make(inst.n, inst.couplings, inst.hx, inst.hz)
        else:
            make = merged_bath_hamiltonian if merged else sparse_bath_hamiltonian
            _OPS[key] = make(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    return _OPS[key]


def column_task(task):
    """One Lanczos run of a solve.  task = (inst, which, c, tau, merged,
    weights): start column c of H_t (which = 0, column c = j*d_s + m is
    |m> (x) |v_j>) or bath vector c on H_b (which = 1).  Without weights it
    returns (alpha, beta, |x|); with weights = (betas, E0) it returns, for an
    H_t column, psi = |x| Q exp(-b (T - E0)/2) e_1 for every b (dim x n_beta).
    The basis Q is rebuilt by running the same recurrence again, which
    repeats it exactly, so a run never holds more than one column's basis."""
    inst, which, c, tau, merged, weights = task
    op = _operator(inst, which, merged)
    if which == 0:
        v = bath_vectors(inst.seed, c // inst.d_s + 1, inst.n_b)[:, c // inst.d_s]
        x = np.zeros(inst.dim)
        m = c % inst.d_s
        x[m * inst.d_b:(m + 1) * inst.d_b] = v
    else:
        x = bath_vectors(inst.seed, c + 1, inst.n_b)[:, c]
    a, b, q, nx = lanczos(op.apply, x, inst.k, tau, keep_q=weights is not None)
    if weights is None:
        return a, b, nx
    betas, e0 = weights
    return np.stack([q @ (nx * fa_weights(a, b, bt, e0)) for bt in betas], axis=1)


def solve(inst, betas=None, tau: float = TAU_FP64, merged: bool = False, mapper=map) -> dict:
    """Run the whole path for one instance.  Returns per-beta outputs plus the
    intermediate Lanczos coefficients (for coefficient-level comparisons).
    ``mapper`` runs the independent column runs (the builtin map, or a process
    pool's); ``merged`` selects the merged operator form."""
    betas = np.asarray(inst.betas if betas is None else betas, float)
    d_s, d_b, n_v = inst.d_s, inst.d_b, inst.n_v
    n_cols = inst.n_cols
    # every column's recurrence coefficients; the common shifts
    runs = list(mapper(column_task, [(inst, 0, c, tau, merged, None) for c in range(n_cols)] +
                       [(inst, 1, j, tau, merged, None) for j in range(n_v)]))
    cols, bath = runs[:n_cols], runs[n_cols:]
    e0 = min(min_ritz(a, b) for a, b, _ in cols)
    e0b = min(min_ritz(a, b) for a, b, _ in bath)
    # the recombined columns for every temperature, then the Gram per bath
    # vector and the n_v average
    psis = list(mapper(column_task, [(inst, 0, c, tau, merged, (betas, e0)) for c in range(n_cols)]))
    results = []
    for t, bt in enumerate(betas):
        m = np.zeros((d_s, d_s))
        for j in range(n_v):
            psi = np.stack([psis[j * d_s + mm][:, t] for mm in range(d_s)], axis=1)
            m += psi.T @ psi
        m /= n_v
        m_b = sum(nx * nx * quad_weight(a, b, bt, e0b) for a, b, nx in bath) / n_v
        results.append(finalize(m, m_b, e0, e0b, bt, d_b) | {"m": m, "m_b": m_b})
    return {"results": results, "e0": e0, "e0b": e0b,
            "alpha": [c[0] for c in cols], "beta": [c[1] for c in cols],
            "bath_alpha": [b[0] for b in bath], "bath_beta": [b[1] for b in bath]}
