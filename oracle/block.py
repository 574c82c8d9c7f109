"""O4: the paper's block estimator -- block Gauss quadrature on the block
Krylov space of each bath vector's start block (Algorithm 1, eqn:fT,
eqn:trB_est).

Test infrastructure only (see ``oracle/__init__``).

The quantity Algorithm 1 computes is a property of the block Krylov space
K_k = span{V, HV, ..., H^(k-1) V} of the start block V = I_s (x) |v_j>
(dim x d_s, V^T V = I): with Q any orthonormal basis of K_k whose first d_s
columns are V, the projected operator T = Q^T H Q gives the quadrature
E_1^T f(T) E_1 (E_1 the first d_s unit vectors), exact for polynomials of
degree at most 2k - 1 (Section "Block Gauss quadrature").  The value does not
depend on which such basis is taken: another one is Q U with U orthogonal and
U E_1 = E_1, and f(U^T T U) = U^T f(T) U.  Algorithm 1 builds one particular
basis by a three-term block recurrence, for which T comes out block
tridiagonal; this oracle instead builds the space directly -- every new block
is H times the previous one, orthogonalised against all earlier basis vectors
(twice) and orthonormalised -- and projects H onto it.  It therefore shares
no step with a recurrence implementation, and differs from one only by
rounding (and by the recurrence's loss of orthogonality, which the Gauss
quadrature tolerates).

The partial-trace estimator averages E_1^T exp(-beta (T_j - E0)) E_1 over the
bath vectors; E0 is the smallest eigenvalue over all T_j (the overflow shift
of the section on the mean force Hamiltonian).
"""
from __future__ import annotations

import numpy as np

from .exact import finalize
from .lanczos import lanczos, quad_weight, min_ritz, TAU_FP64
from .rng import bath_vectors
from .spin import sparse_bath_hamiltonian, sparse_hamiltonian


def krylov_basis(apply, v: np.ndarray, k: int, tau: float = TAU_FP64):
    """Orthonormal basis Q (dim x n, n <= k*b) of span{V, HV, ..., H^(k-1) V}
    with V (dim x b, orthonormal columns) as its first block, and H Q.  Each
    new block is H times the previous one with its components along the basis
    removed (twice) and orthonormalised by an SVD.  The space stops growing at
    the first new block whose smallest singular value after that is at most
    tau times the largest entry of H projected on the basis so far: the space
    is then (numerically) invariant."""
    blocks, images = [v], []
    scale = 0.0
    while True:
        w = apply(blocks[-1])
        images.append(w)
        if len(blocks) == k:
            break
        q = np.hstack(blocks)
        scale = max(scale, float(np.abs(q.T @ w).max()))
        for _ in range(2):
            w = w - q @ (q.T @ w)
        u, s, _ = np.linalg.svd(w, full_matrices=False)
        if s.min() <= tau * scale:
            break
        blocks.append(u)
    return np.hstack(blocks), np.hstack(images)


def krylov_projection(apply, v: np.ndarray, k: int) -> np.ndarray:
    """T = Q^T H Q on the basis of ``krylov_basis`` (symmetrised)."""
    q, hq = krylov_basis(apply, v, k)
    t = q.T @ hq
    return 0.5 * (t + t.T)


def block_quadrature(t: np.ndarray, b: int, beta: float, e0: float) -> np.ndarray:
    """E_1^T exp(-beta (T - e0)) E_1 through the eigendecomposition of T."""
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
        ts.append(krylov_projection(op.apply, vj, inst.k))
    e0 = min(float(np.linalg.eigvalsh(t)[0]) for t in ts)
    bath = [lanczos(opb.apply, v[:, j], inst.k, TAU_FP64, keep_q=False) for j in range(n_v)]
    e0b = min(min_ritz(a, b) for a, b, _, _ in bath)
    results = []
    for bt in betas:
        m = sum(block_quadrature(t, d_s, bt, e0) for t in ts) / n_v
        m_b = sum(nx * nx * quad_weight(a, b, bt, e0b) for a, b, _, nx in bath) / n_v
        results.append(finalize(m, m_b, e0, e0b, bt, d_b) | {"m": m, "m_b": m_b})
    return {"results": results, "e0": e0, "e0b": e0b}
