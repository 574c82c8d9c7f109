"""Spin-1/2 Hamiltonians of the paper's form (eqn:Ht), dense and matrix-free.

Test infrastructure only (see ``oracle/__init__``).

Reading of eqn:Ht used throughout (Section "Spin systems"): Pauli matrices;
each unordered pair (i<j) once with coefficients (J^x, J^y, J^z) on
sx_i sx_j, sy_i sy_j, sz_i sz_j; one-site fields hx_i sx_i + hz_i sz_i (the
paper's (h/2) sz_i is hz_i = h/2).  sigma_i acts on the i-th Kronecker factor
counting from the left (0-based here), so site i is bit (N-1-i) of a basis
index and the system (first n_s sites) occupies the top n_s bits.  sz|0> = +|0>.
"""
from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = {"x": SX, "y": SY, "z": SZ}


def site_operator(p: np.ndarray, i: int, n: int) -> np.ndarray:
    """I x ... x p x ... x I with p on the i-th factor from the left."""
    out = np.ones((1, 1), dtype=np.complex128)
    for s in range(n):
        out = np.kron(out, p if s == i else I2)
    return out


def dense_terms(n: int, couplings: Iterable, hx: Sequence[float], hz: Sequence[float],
                keep=lambda i, j: True) -> np.ndarray:
    """Dense complex Hamiltonian built from Kronecker products; ``keep`` selects
    which pairs (and fields, passed as (i, i)) are included."""
    d = 1 << n
    h = np.zeros((d, d), dtype=np.complex128)
    ops = {a: [site_operator(PAULI[a], s, n) for s in range(n)] for a in "xyz"}
    for (i, j, jx, jy, jz) in couplings:
        if not keep(i, j):
            continue
        for a, c in (("x", jx), ("y", jy), ("z", jz)):
            if c != 0.0:
                h += c * (ops[a][i] @ ops[a][j])
    for s in range(n):
        if not keep(s, s):
            continue
        if hx[s] != 0.0:
            h += hx[s] * ops["x"][s]
        if hz[s] != 0.0:
            h += hz[s] * ops["z"][s]
    return h


def dense_hamiltonian(n: int, couplings, hx, hz) -> np.ndarray:
    """Real symmetric dense H_t (the imaginary part of a real combination of
    XX, YY, ZZ and x/z fields vanishes identically)."""
    h = dense_terms(n, couplings, hx, hz)
    assert np.abs(h.imag).max(initial=0.0) == 0.0
    return h.real.copy()


def split_dense(n_s: int, n_b: int, couplings, hx, hz):
    """(H_s on C^{d_s}, H_b on C^{d_b}, H_sb on the full space), following the
    decomposition H_t = H_s (x) I_b + I_s (x) H_b + H_sb."""
    n = n_s + n_b
    in_s = lambda s: s < n_s
    hs = dense_terms(n_s, [c for c in couplings if in_s(c[0]) and in_s(c[1])],
                     hx[:n_s], hz[:n_s]).real
    bc = [(i - n_s, j - n_s, a, b, c) for (i, j, a, b, c) in couplings
          if not in_s(i) and not in_s(j)]
    hb = dense_terms(n_b, bc, hx[n_s:], hz[n_s:]).real
    hsb = dense_terms(n, couplings, hx, hz,
                      keep=lambda i, j: i != j and (in_s(i) != in_s(j))).real
    return hs, hb, hsb


def bath_terms(n_s: int, couplings, hx, hz):
    """Couplings and fields of H_b, re-indexed to bath-local sites."""
    bc = [(i - n_s, j - n_s, a, b, c) for (i, j, a, b, c) in couplings
          if i >= n_s and j >= n_s]
    return bc, np.asarray(hx[n_s:], float), np.asarray(hz[n_s:], float)


# ---------------------------------------------------------------------------
# Matrix-free form.  Each Pauli string maps a basis state |p> to a phase times a
# single basis state |p'>.  The operator is stored as a list of
# (out_index_array, phase_array) per term and applied by scatter-add:
#     Y[out(p)] += coef * phase(p) * X[p]
# This is the column action of H, built independently of the dense form.
# ---------------------------------------------------------------------------

def _pauli_action(kind: str, bits: np.ndarray):
    """Action of one Pauli on a site with current bit values: returns
    (flip?, phase array).  sx|b> = |1-b>; sy|0> = i|1>, sy|1> = -i|0>;
    sz|b> = (1-2b)|b>."""
    if kind == "x":
        return True, np.ones(bits.shape, np.complex128)
    if kind == "y":
        return True, np.where(bits == 0, 1j, -1j)
    return False, (1 - 2 * bits).astype(np.complex128)


class SparseSpinOperator:
    """Matrix-free H as a sum of Pauli strings.

    Each term is kept symbolically as (flip mask, phase function) and its
    action on an array of basis indices is evaluated on demand, so the full
    operator never needs dim-sized tables per term."""

    def __init__(self, n: int, couplings, hx, hz):
        self.n = n
        # symbolic terms: list of (kind_i, site_i, kind_j, site_j, coef);
        # single-site terms use site_j = -1
        self.terms = []
        for (i, j, jx, jy, jz) in couplings:
            for kind, c in (("x", jx), ("y", jy), ("z", jz)):
                if c != 0.0:
                    self.terms.append((kind, i, kind, j, float(c)))
        for s in range(n):
            if hx[s] != 0.0:
                self.terms.append(("x", s, "", -1, float(hx[s])))
            if hz[s] != 0.0:
                self.terms.append(("z", s, "", -1, float(hz[s])))
        self._cache = None

    @property
    def dim(self) -> int:
        return 1 << self.n

    def _action(self, term, p: np.ndarray):
        """Image basis index and real phase of one term acting on states p."""
        ka, i, kb, j, c = term
        n = self.n
        out = p.copy()
        ph = np.full(p.shape, c, dtype=np.complex128)
        for kind, s in ((ka, i), (kb, j)):
            if s < 0:
                continue
            b = (p >> (n - 1 - s)) & 1
            flip, phase = _pauli_action(kind, b)
            ph = ph * phase
            if flip:
                out = out ^ (1 << (n - 1 - s))
        assert np.abs(ph.imag).max(initial=0.0) == 0.0
        return out, ph.real

    def apply(self, x: np.ndarray) -> np.ndarray:
        """Y = H X for X of shape (dim,) or (dim, C), by scatter of the column
        action: Y[out(p)] += phase(p) X[p]."""
        x = np.asarray(x, dtype=np.float64)
        p = np.arange(self.dim, dtype=np.int64)
        y = np.zeros_like(x)
        shape = (-1,) + (1,) * (x.ndim - 1)
        if self._cache is None and self.dim <= (1 << 16):
            # small spaces: keep each term's (image, phase) table between calls
            self._cache = [self._action(t, p) for t in self.terms]
        for i, t in enumerate(self.terms):
            out, ph = self._cache[i] if self._cache is not None else self._action(t, p)
            # every term is an involution on basis states, so ``out`` is a
            # permutation and an indexed add has no repeated targets
            y[out] += ph.reshape(shape) * x
        return y

    def rows(self, idx: np.ndarray, x: np.ndarray) -> np.ndarray:
        """(H X)[idx] for a set of rows, without forming H X: a term maps p to
        out(p) with phase(p), and being an involution its row idx is hit by
        p = out(idx)."""
        idx = np.asarray(idx, dtype=np.int64)
        shape = (-1,) + (1,) * (x.ndim - 1)
        val = np.zeros((len(idx),) + x.shape[1:])
        for t in self.terms:
            p, _ = self._action(t, idx)
            _, ph = self._action(t, p)
            val += ph.reshape(shape) * x[p]
        return val


class MergedSpinOperator:
    """The same matrix-free H with its Pauli strings merged by the basis state
    they reach.  A string whose flips are the bit set f maps |p> to a phase
    times |p ^ f>, so

        (H X)[q] = d(q) X[q] + sum_{f != 0} c_f(q) X[q ^ f],

    with d the summed phases of the strings that flip nothing and c_f(q) the
    summed phase, read at the source state q ^ f, of every string that flips
    f.  Both are evaluated once from the matrix-free form's own term actions
    (kept as a scalar when constant over q).  X[q ^ f] for all q is X with the
    index axes of the bits in f reversed (a view of X as a 2 x ... x 2
    tensor), which is what makes this form fast enough for full-size
    reference runs; it is pinned to the matrix-free and dense forms."""

    def __init__(self, n: int, couplings, hx, hz):
        base = SparseSpinOperator(n, couplings, hx, hz)
        self.n = n
        p = np.arange(1 << n, dtype=np.int64)
        self.diag = np.zeros(1 << n)
        coef = {}
        for t in base.terms:
            f = 0
            for s in (t[1], t[3]):
                if s >= 0 and t[0 if s == t[1] else 2] in "xy":
                    f |= 1 << (n - 1 - s)
            if f == 0:
                out, ph = base._action(t, p)
                self.diag += ph
                continue
            out, ph = base._action(t, p ^ f)          # phase read at the source q ^ f
            assert np.array_equal(out, p)
            coef[f] = coef.get(f, 0.0) + ph
        self.hops = []
        for f, c in coef.items():
            c = np.asarray(c)
            if np.all(c == c.flat[0]):
                c = float(c.flat[0])
            if np.any(c != 0.0):
                self.hops.append((f, c))

    @property
    def dim(self) -> int:
        return 1 << self.n

    def _partner(self, x: np.ndarray, f: int) -> np.ndarray:
        n = self.n
        axes = [n - 1 - b for b in range(n) if (f >> b) & 1]
        t = x.reshape((2,) * n + x.shape[1:])
        return np.flip(t, axis=axes).reshape(x.shape)

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        shape = (-1,) + (1,) * (x.ndim - 1)
        y = self.diag.reshape(shape) * x
        for f, c in self.hops:
            xf = self._partner(x, f)
            if isinstance(c, float):
                y += c * xf
            else:
                y += c.reshape(shape) * xf
        return y


def merged_hamiltonian(n: int, couplings, hx, hz) -> MergedSpinOperator:
    return MergedSpinOperator(n, couplings, hx, hz)


def merged_bath_hamiltonian(n_s: int, n_b: int, couplings, hx, hz) -> MergedSpinOperator:
    bc, bhx, bhz = bath_terms(n_s, couplings, hx, hz)
    return MergedSpinOperator(n_b, bc, bhx, bhz)


def sparse_hamiltonian(n: int, couplings, hx, hz) -> SparseSpinOperator:
    return SparseSpinOperator(n, couplings, hx, hz)


def sparse_bath_hamiltonian(n_s: int, n_b: int, couplings, hx, hz) -> SparseSpinOperator:
    bc, bhx, bhz = bath_terms(n_s, couplings, hx, hz)
    return SparseSpinOperator(n_b, bc, bhx, bhz)
