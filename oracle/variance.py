"""O6: exact variance of one Rademacher sample of the partial-trace estimator.

Test infrastructure only (see ``oracle/__init__``).

Write A = sum_{m,n} |m><n| (x) A_mn (Section "Trace estimators").  Entry (m,n)
of one sample is v^T A_mn v = v^T S v with S = (A_mn + A_mn^T)/2.  For
v_a = eps_a / sqrt(d_b), eps_a = +-1 independent and fair,
    E[v^T S v] = tr S / d_b,   Var[v^T S v] = (2 / d_b^2) sum_{a != b} S_ab^2,
since E[eps_a eps_b eps_c eps_d] is 1 exactly when the indices pair up.
"""
from __future__ import annotations

import numpy as np


def entry_variance(a: np.ndarray, d_s: int, d_b: int) -> np.ndarray:
    """Per-entry variance (d_s x d_s) of one sample (I_s (x) <v|) A (I_s (x) |v>)."""
    blocks = a.reshape(d_s, d_b, d_s, d_b)
    var = np.zeros((d_s, d_s))
    for m in range(d_s):
        for n in range(d_s):
            s = blocks[m, :, n, :]
            s = 0.5 * (s + s.T)
            off = s - np.diag(np.diag(s))
            var[m, n] = 2.0 * (off ** 2).sum() / d_b ** 2
    return var
