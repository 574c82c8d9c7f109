"""O9: the estimator's high-temperature offset (Section "A note on high
temperatures"; the appendix deriving the high-temperature limit).

Test infrastructure only (see ``oracle/__init__``).

Split H_t = H_s (x) I_b + I_s (x) H_b + H_sb, where H_sb holds the couplings
with one site in the system and one in the bath.  As beta -> 0 the exact
H*(beta) tends to H_s + tr_b(H_sb)/d_b = H_s, but the n_v-sample estimate
built from unit bath vectors v_j tends to H_s + C with

    C = (1/n_v) sum_j (I_s (x) <v_j|) H_sb (I_s (x) |v_j>).

``offset`` evaluates that definition as written: H_sb applied matrix-free
(the spin module's scatter form, restricted to the cross couplings) to the
columns |m> (x) |v_j>, then the d_s x d_s quadratic forms, averaged over j.
``bath_sx`` gives the averaged single-site expectations <v_j| sx_c |v_j>.
"""
from __future__ import annotations

import numpy as np

from .rng import bath_vectors
from .spin import sparse_hamiltonian


def cross_couplings(n_s: int, couplings) -> list:
    """The couplings of H_sb: exactly one site in the system."""
    return [c for c in couplings if (c[0] < n_s) != (c[1] < n_s)]


def offset_from_vectors(n_s: int, n_b: int, couplings, v: np.ndarray) -> np.ndarray:
    """C for given unit bath vectors (columns of v, shape (d_b, n_v))."""
    n, d_s, d_b = n_s + n_b, 1 << n_s, 1 << n_b
    hsb = sparse_hamiltonian(n, cross_couplings(n_s, couplings), np.zeros(n), np.zeros(n))
    c = np.zeros((d_s, d_s))
    for j in range(v.shape[1]):
        x = np.zeros((d_s * d_b, d_s))                  # columns |m> (x) |v_j>
        for m in range(d_s):
            x[m * d_b:(m + 1) * d_b, m] = v[:, j]
        c += x.T @ hsb.apply(x)
    return c / v.shape[1]


def offset(inst, n_v: int | None = None, seed: int | None = None) -> np.ndarray:
    """C for the bath vectors of a solve of ``inst`` (its seed and n_v unless given)."""
    n_v = inst.n_v if n_v is None else n_v
    seed = inst.seed if seed is None else seed
    return offset_from_vectors(inst.n_s, inst.n_b, inst.couplings, bath_vectors(seed, n_v, inst.n_b))


def bath_sx(inst, n_v: int | None = None, seed: int | None = None) -> np.ndarray:
    """(1/n_v) sum_j <v_j| sx_c |v_j> for bath sites c = n_s .. N-1."""
    n_v = inst.n_v if n_v is None else n_v
    seed = inst.seed if seed is None else seed
    v = bath_vectors(seed, n_v, inst.n_b)
    out = np.zeros(inst.n_b)
    for t in range(inst.n_b):
        field = np.zeros(inst.n_b)
        field[t] = 1.0
        sx = sparse_hamiltonian(inst.n_b, [], field, np.zeros(inst.n_b))
        out[t] = float(np.einsum("bj,bj->", v, sx.apply(v))) / n_v
    return out
