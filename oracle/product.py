"""O10: the product-state (rank-one) estimator of the appendix "A consistent
partial trace estimator".

Test infrastructure only (see ``oracle/__init__``).

A sample is a unit product vector x_j = |v_s^(j)> (x) |v_b^(j)> (system index
major).  The bath factor v_b^(j) is the bath vector j of the partial-trace
estimator (same seed); the system factor is the same published sign rule
applied to the n_s system bits with the seed XOR ``SYS_SEED_XOR``.  With
E[x x^T] = I/D (D = 2^N), D <x|A|x> is an unbiased estimate of tr A, and for
fixed v_s (fixed v_b) its mean over the other factor is the quadratic form
of the partial trace tr_b A (tr_s A), so trace and partial-trace estimates
agree.  For A = exp(-beta H_t) this estimates Z_t from n_v single columns;
the bath partition function comes from the bath vectors as in the
partial-trace estimator (eqn:H_est), and ln Z* = ln Z_t - ln Z_b.

``exact_samples`` evaluates each <x_j|exp(-beta H_t)|x_j> densely;
``lanczos_estimate`` follows the library's steps: plain Lanczos from each
x_j, the Gauss quadrature e_1^T exp(-beta (T_j - E0)) e_1 with E0 the
smallest Ritz value over the columns, the same for the bath.
"""
from __future__ import annotations

import numpy as np

from .lanczos import TAU_FP64, lanczos, min_ritz, quad_weight
from .rng import bath_vector
from .spin import dense_hamiltonian, sparse_bath_hamiltonian, sparse_hamiltonian

SYS_SEED_XOR = 0x9E3779B97F4A7C15


def system_vector(seed: int, j: int, n_s: int) -> np.ndarray:
    """Unit Rademacher system vector of sample j."""
    return bath_vector(seed ^ SYS_SEED_XOR, j, n_s)


def product_vector(seed: int, j: int, n_s: int, n_b: int) -> np.ndarray:
    """x_j = v_s^(j) (x) v_b^(j) over the 2^(n_s + n_b) basis states."""
    return np.kron(system_vector(seed, j, n_s), bath_vector(seed, j, n_b))


def _logmeanexp_rows(lw: np.ndarray) -> np.ndarray:
    m = lw.max(axis=1, keepdims=True)
    return (m + np.log(np.exp(lw - m).mean(axis=1, keepdims=True)))[:, 0]


def exact_samples(inst, betas, n_v: int, seed: int) -> dict:
    """Dense per-sample ln(D <x_j|exp(-beta H_t)|x_j>), their average as ln Z_t."""
    h = dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    e, u = np.linalg.eigh(h)
    xs = np.stack([product_vector(seed, j, inst.n_s, inst.n_b) for j in range(n_v)], axis=1)
    c2 = (u.T @ xs) ** 2
    lw = np.array([[np.log((c2[:, j] * np.exp(-b * (e - e[0]))).sum()) - b * e[0] + inst.n * np.log(2.0)
                    for j in range(n_v)] for b in betas])
    return {"log_z_t_samples": lw, "log_z_t": _logmeanexp_rows(lw)}


def lanczos_estimate(inst, betas, n_v: int, k: int, seed: int, tau: float = TAU_FP64) -> dict:
    """ln Z_t, ln Z_b, ln Z* and the per-sample ln Z_t estimates by Lanczos
    quadrature on the product vectors (and the bath vectors for Z_b)."""
    betas = np.asarray(betas, float)
    op = sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    opb = sparse_bath_hamiltonian(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    tot = [lanczos(op.apply, product_vector(seed, j, inst.n_s, inst.n_b), min(k, inst.dim), tau, keep_q=False)
           for j in range(n_v)]
    bath = [lanczos(opb.apply, bath_vector(seed, j, inst.n_b), min(k, inst.d_b), tau, keep_q=False)
            for j in range(n_v)]
    e0 = min(min_ritz(a, b) for a, b, _, _ in tot)
    e0b = min(min_ritz(a, b) for a, b, _, _ in bath)
    # x^T f(H) x = |x|^2 e_1^T f(T) e_1 (Gauss quadrature from a start vector of norm |x|)
    lw = np.array([[np.log(nx * nx * quad_weight(a, b, bt, e0)) - bt * e0 + inst.n * np.log(2.0)
                    for a, b, _, nx in tot] for bt in betas])
    lb = np.array([[np.log(nx * nx * quad_weight(a, b, bt, e0b)) - bt * e0b + inst.n_b * np.log(2.0)
                    for a, b, _, nx in bath] for bt in betas])
    log_z_t, log_z_b = _logmeanexp_rows(lw), _logmeanexp_rows(lb)
    return {"log_z_t": log_z_t, "log_z_b": log_z_b, "log_z": log_z_t - log_z_b, "log_z_t_samples": lw,
            "e0": e0, "e0b": e0b}
