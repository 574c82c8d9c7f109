"""Truncation bounds of the Krylov quadratures (Section "Error analysis",
subsection "Block Gauss quadrature").

Test infrastructure only (see ``oracle/__init__``).

For V with orthonormal columns and the block Lanczos T built from V, the
quadratic form V^T p(H) V equals E_1^T p(T) E_1 for every polynomial p of
degree at most 2k-1.  The paper subtracts such a p from f on both sides and
bounds each side by the largest deviation of f from p on the spectral interval
[lambda_min, lambda_max] (the Ritz values lie inside it), giving

    || V^T f(H) V - E_1^T f(T) E_1 ||_2 <= 2 min_{deg p <= 2k-1} max |f - p|.

The per-column path reproduces g(H) x (unit x) through |x| Q g(T) e_1, which
is exact for deg g <= k-1; the same argument gives
|| Q g(T) e_1 - g(H) x || <= 2 E_{k-1}(g).  With g = exp(-beta (x - E0)/2),
psi = g(H) X + Delta for the d_s start columns X of one bath vector
(X^T X = I), ||Delta||_2 <= sqrt(d_s) 2 E_{k-1}(g) and ||g(H) X||_2 <=
max g =: G, so the Gram Psi^T Psi differs from X^T g(H)^2 X by at most
||Delta|| (2 G + ||Delta||).  Both bounds survive the n_v average (triangle
inequality).

E_n(f) is bounded above by the error of one particular degree-n polynomial,
the interpolant of f in the n+1 Chebyshev points of [lambda_min, lambda_max];
its error is evaluated on a fine grid.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as cheb


def chebyshev_interpolation_error(beta: float, lo: float, hi: float, shift: float, n: int,
                                  grid: int = 40001) -> float:
    """max over [lo, hi] of |f - p_n| for f(x) = exp(-beta (x - shift)) and p_n
    its interpolant in the n+1 Chebyshev points of the first kind."""
    t = np.cos(np.pi * (np.arange(n + 1) + 0.5) / (n + 1))
    mid, half = 0.5 * (hi + lo), 0.5 * (hi - lo)
    c = cheb.chebfit(t, np.exp(-beta * (mid + half * t - shift)), n)
    tg = np.linspace(-1.0, 1.0, grid)
    return float(np.abs(cheb.chebval(tg, c) - np.exp(-beta * (mid + half * tg - shift))).max())


def block_quadrature_bound(beta: float, lo: float, hi: float, e0: float, k: int) -> float:
    """Bound on || avg_j (V_j^T exp(-beta (H - e0)) V_j - E_1^T exp(-beta (T_j - e0)) E_1) ||_2
    after k block Lanczos steps."""
    return 2.0 * chebyshev_interpolation_error(beta, lo, hi, e0, 2 * k - 1)


def per_column_gram_bound(beta: float, lo: float, hi: float, e0: float, k: int, d_s: int) -> float:
    """Bound on || avg_j (Psi_j^T Psi_j - X_j^T exp(-beta (H - e0)) X_j) ||_2 for the
    per-column function approximation of exp(-beta (H - e0)/2) after k steps."""
    delta = np.sqrt(d_s) * 2.0 * chebyshev_interpolation_error(0.5 * beta, lo, hi, e0, k - 1)
    g_max = np.exp(0.5 * beta * (e0 - lo))
    return float(delta * (2.0 * g_max + delta))
