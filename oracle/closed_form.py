"""O5: closed forms that pin the dense oracle and the Hamiltonian convention.

Test infrastructure only (see ``oracle/__init__``).

1. The open XX chain H = -(J/2) sum_i (sx_i sx_{i+1} + sy_i sy_{i+1})
   + (h/2) sum_i sz_i with the system the first two sites (paper appendix
   "Solution to the spin chain", after Campisi, Zueco & Talkner).  Two formulas
   there are garbled in the source text and are read as follows:
     * the occupation factor is N_k = 1 / (1 + exp(beta lambda_k));
     * the magnetisation is <sz_j> = (4/(N+1)) sum_k sin^2(j k pi/(N+1)) N_k - 1
       (the printed form lacks the "- 1" and has the opposite sign), and delta
       uses <sz_1> - <sz_2>.
2. Two spins, one system and one bath, H = J (sx sx + sy sy) + Jz sz sz
   + h1 sz_1 + h2 sz_2, derived here: |00> and |11> are eigenstates with
   energies Jz + h1 + h2 and Jz - h1 - h2; on {|01>, |10>} the block is
   -Jz I + [[d, 2J], [2J, -d]], d = h1 - h2, with eigenvalues -Jz +- r,
   r = sqrt(d^2 + 4 J^2).  Tracing out the bath spin gives a diagonal rho*.
"""
from __future__ import annotations

import numpy as np


def xx_chain_rdm(n: int, J: float, h: float, beta: float, n_b: int | None = None) -> dict:
    """Eigenvalues p_1..p_4 of rho*, ln Z_N, ln Z*, eigenvalues of H* and the
    entropy for the N-site open XX chain with a two-site system."""
    def lam(nn):
        k = np.arange(1, nn + 1)
        return h - 2.0 * J * np.cos(k * np.pi / (nn + 1)), k

    lk, k = lam(n)
    occ = 1.0 / (1.0 + np.exp(beta * lk))
    s = lambda j: np.sin(j * k * np.pi / (n + 1))
    xx = -4.0 / (n + 1) * np.sum(s(1) * s(2) * occ)
    z1 = 4.0 / (n + 1) * np.sum(s(1) ** 2 * occ) - 1.0
    z2 = 4.0 / (n + 1) * np.sum(s(2) ** 2 * occ) - 1.0
    zz = z1 * z2 - xx ** 2
    delta = np.sqrt(4.0 * xx ** 2 + (z1 - z2) ** 2)
    p = np.array([(1 + z1 + z2 + zz) / 4, (1 - delta - zz) / 4,
                  (1 + delta - zz) / 4, (1 - z1 - z2 + zz) / 4])

    def log_z(nn):
        l, _ = lam(nn)
        return beta * nn * h / 2.0 + np.sum(np.log1p(np.exp(-beta * l)))

    nb = n - 2 if n_b is None else n_b
    lzs = log_z(n) - log_z(nb)
    h_eig = -(lzs + np.log(p)) / beta
    return {"p": p, "log_z_n": log_z(n), "log_z": lzs, "h_eig": h_eig,
            "entropy": float(-(p * np.log(p)).sum())}


def two_spin_rdm(J: float, Jz: float, h1: float, h2: float, beta: float) -> dict:
    """rho* (2x2), ln Z_t and ln Z_b for the two-spin model above."""
    d = h1 - h2
    r = np.sqrt(d * d + 4.0 * J * J)
    e_up = np.exp(-beta * (Jz + h1 + h2))
    e_dn = np.exp(-beta * (Jz - h1 - h2))
    c, sh = np.cosh(beta * r), np.sinh(beta * r)
    r00 = e_up + np.exp(beta * Jz) * (c - d / r * sh)
    r11 = np.exp(beta * Jz) * (c + d / r * sh) + e_dn
    z_t = e_up + e_dn + 2.0 * np.exp(beta * Jz) * c
    z_b = 2.0 * np.cosh(beta * h2)
    rho = np.diag([r00, r11]) / z_t
    return {"rho": rho, "log_z_t": float(np.log(z_t)), "log_z_b": float(np.log(z_b)),
            "log_z": float(np.log(z_t) - np.log(z_b))}
