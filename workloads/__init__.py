"""Seeded synthetic spin-Hamiltonian workloads.

This module only *draws inputs*: coupling lists, fields, inverse temperatures,
sample counts and seeds.  It holds none of the method's arithmetic, so both the
CPU oracle and the HIP path may import it without sharing any computation.

Conventions (the paper's Hamiltonian, eqn:Ht in the "Spin systems" section):

* sites are 0-based; site 0 is the leftmost Kronecker factor and the system is
  the first ``n_s`` sites;
* a coupling ``(i, j, jx, jy, jz)`` with ``i < j`` contributes
  ``jx*sx_i sx_j + jy*sy_i sy_j + jz*sz_i sz_j`` in Pauli matrices, each
  unordered pair once (the paper's ordered double sum is read as a sum over
  unordered pairs carrying the full coefficient);
* ``hx[i]`` / ``hz[i]`` are the coefficients of ``sx_i`` / ``sz_i``; a "field of
  strength h" in the paper's sense is the coefficient ``h/2``.

Random couplings use NumPy's PCG64 ``default_rng(seed)``; the bath vectors are
*not* drawn here (both sides generate them from the counter-based rule
described with the solver's seed argument).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Coupling = Tuple[int, int, float, float, float]


@dataclass
class Instance:
    """One solve: Hamiltonian terms plus the estimator's parameters."""

    n_s: int
    n_b: int
    couplings: List[Coupling]
    hx: np.ndarray
    hz: np.ndarray
    betas: np.ndarray
    n_v: int
    k: int
    seed: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n_s + self.n_b

    @property
    def dim(self) -> int:
        return 1 << self.n

    @property
    def d_s(self) -> int:
        return 1 << self.n_s

    @property
    def d_b(self) -> int:
        return 1 << self.n_b

    @property
    def n_cols(self) -> int:
        return self.d_s * self.n_v


def _zeros(n: int) -> np.ndarray:
    return np.zeros(n, dtype=np.float64)


def nn_xxz_chain(n_s: int, n_b: int, seed: int, *, sb_strength: float | None = 1.0,
                 h: float = 0.5, betas: Sequence[float] = (1.0,), n_v: int = 4,
                 k: int = 30, name: str = "") -> Instance:
    """Nearest-neighbour XXZ chain, J_xy and J_z ~ U(-1,1) per bond, uniform
    z-field of strength ``h`` (coefficient h/2).  The bond joining the last
    system site to the first bath site is set to ``sb_strength`` for both
    J_xy and J_z (None keeps the random draw)."""
    n = n_s + n_b
    rng = np.random.default_rng(seed)
    cps: List[Coupling] = []
    for i in range(n - 1):
        jxy = float(rng.uniform(-1.0, 1.0))
        jz = float(rng.uniform(-1.0, 1.0))
        if sb_strength is not None and i == n_s - 1:
            jxy = jz = float(sb_strength)
        cps.append((i, i + 1, jxy, jxy, jz))
    hz = np.full(n, h / 2.0)
    return Instance(n_s, n_b, cps, _zeros(n), hz, np.asarray(betas, float), n_v, k,
                    seed, name or f"xxz_chain_{n_s}+{n_b}")


def cfg_small_chain() -> Instance:
    """1 system spin + 9 bath spins (dim 1024), nearest-neighbour XXZ chain with
    J_xy, J_z ~ U(-1,1), z-field h = 0.5, system-bath bond of strength 1,
    beta = 1, 4 Rademacher bath vectors, 30 Lanczos steps, FP64."""
    return nn_xxz_chain(1, 9, 1001, sb_strength=1.0, h=0.5, betas=(1.0,), n_v=4,
                        k=30, name="xxz_chain_1+9")


def long_range_xx_zz(n_s: int, n_b: int, h: float, seed: int, *, alpha: float = 1.5,
                     betas: Sequence[float] = (0.5, 1.0, 2.0, 4.0), n_v: int = 16,
                     k: int = 60, name: str = "") -> Instance:
    """All pairs J^x = J^z = |i-j|^-alpha, J^y = 0, transverse x-field of
    strength h (coefficient h/2)."""
    n = n_s + n_b
    cps = []
    for i in range(n):
        for j in range(i + 1, n):
            c = float(abs(i - j)) ** (-alpha)
            cps.append((i, j, c, 0.0, c))
    hx = np.full(n, h / 2.0)
    return Instance(n_s, n_b, cps, hx, _zeros(n), np.asarray(betas, float), n_v, k,
                    seed, name or f"lr_xxzz_{n_s}+{n_b}_h{h}", {"h": h})


LR_FIELDS = (0.5, 1.0, 1.5)


def cfg_long_range(h_index: int = 0, *, n_b: int = 18) -> Instance:
    """2 system + 18 bath spins (dim 2^20), long-range XX+ZZ, J=1, alpha=1.5,
    x-field h in {0.5, 1.0, 1.5}, beta in {0.5,1,2,4}, n_v=16, k=60."""
    h = LR_FIELDS[h_index]
    return long_range_xx_zz(2, n_b, h, 2001 + h_index, name=f"lr_xxzz_2+{n_b}_h{h}")


def random_sparse_xxz(seed: int, *, n_range=(12, 22), n_s_choices=(1, 2, 3),
                      n_v: int = 8, k: int = 50) -> Instance:
    """Random XXZ couplings U(-1,1) on a uniformly random simple graph with 2N
    edges (average degree 4), no field, beta log-uniform in [0.1, 10]."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    n_s = int(rng.choice(n_s_choices))
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    m = min(2 * n, len(pairs))
    pick = rng.choice(len(pairs), size=m, replace=False)
    cps = []
    for p in sorted(int(x) for x in pick):
        i, j = pairs[p]
        jxy = float(rng.uniform(-1.0, 1.0))
        jz = float(rng.uniform(-1.0, 1.0))
        cps.append((i, j, jxy, jxy, jz))
    beta = float(10.0 ** rng.uniform(-1.0, 1.0))
    return Instance(n_s, n - n_s, cps, _zeros(n), _zeros(n), np.asarray([beta]), n_v, k,
                    seed, f"sparse_xxz_{n_s}+{n - n_s}")


def cfg_batch(n_instances: int = 64, **kw) -> List[Instance]:
    """64 independent random-sparse-XXZ instances, seeds 3000..3063."""
    return [random_sparse_xxz(3000 + i, **kw) for i in range(n_instances)]


def long_range_xxz(n_s: int, n_b: int, seed: int, *, alpha: float = 1.2, delta: float = 0.8,
                   hx_field: float = 1.0, betas=(2.0,), n_v: int = 4, k: int = 80) -> Instance:
    """All pairs J^x = J^y = |i-j|^-alpha, J^z = delta*|i-j|^-alpha, x-field of
    strength hx_field (coefficient hx_field/2)."""
    n = n_s + n_b
    cps = []
    for i in range(n):
        for j in range(i + 1, n):
            c = float(abs(i - j)) ** (-alpha)
            cps.append((i, j, c, c, delta * c))
    hx = np.full(n, hx_field / 2.0)
    return Instance(n_s, n_b, cps, hx, _zeros(n), np.asarray(betas, float), n_v, k, seed,
                    f"lr_xxz_{n_s}+{n_b}")


def cfg_large(n_b: int = 23) -> Instance:
    """3 system + 23 bath spins (dim 2^26), long-range XXZ alpha=1.2, Delta=0.8,
    x-field 1.0, beta=2, n_v=4 (32 columns), k=80."""
    return long_range_xxz(3, n_b, 4001)


def tfim_request(r: int, *, n_range=(14, 24), n_v: int = 8, k: int = 60) -> Instance:
    """Serving request r: ZZ chain J=1 with x-field h ~ U(0,2) (coefficient
    h/2), N ~ U{14..24}, d_s in {2,4}, beta log-uniform in [0.1, 10]."""
    rng = np.random.default_rng(5000 + r)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    n_s = int(rng.choice((1, 2)))
    h = float(rng.uniform(0.0, 2.0))
    beta = float(10.0 ** rng.uniform(-1.0, 1.0))
    cps = [(i, i + 1, 0.0, 0.0, 1.0) for i in range(n - 1)]
    hx = np.full(n, h / 2.0)
    return Instance(n_s, n - n_s, cps, hx, _zeros(n), np.asarray([beta]), n_v, k, 5000 + r,
                    f"tfim_{n_s}+{n - n_s}", {"h": h})


def xy_power_law(n_s: int, n_b: int, alpha: float, h: float, seed: int, *, J: float = 1.0,
                 eps: float = 1.0, betas: Sequence[float] = (1.0,), n_v: int = 100,
                 k: int = 60) -> Instance:
    """The family of the paper's long-range experiments: isotropic XY chain
    with J^x = J^y = J |i-j|^-alpha (alpha = inf: nearest neighbours only),
    J^z = 0, z-field h (coefficient h/2 on every site); the system-bath pairs
    are scaled by eps (H_s + H_b + eps H_sb)."""
    n = n_s + n_b
    cps = []
    for i in range(n):
        for j in range(i + 1, n):
            d = j - i
            c = J * (1.0 if d == 1 else 0.0) if np.isinf(alpha) else J * float(d) ** (-alpha)
            if c == 0.0:
                continue
            if (i < n_s) != (j < n_s):
                c *= eps
            cps.append((i, j, c, c, 0.0))
    hz = np.full(n, h / 2.0)
    return Instance(n_s, n_b, cps, _zeros(n), hz, np.asarray(betas, float), n_v, k, seed,
                    f"xy_a{alpha}_h{h}_e{eps}_{n_s}+{n_b}", {"alpha": alpha, "h": h, "eps": eps})


def poisson_arrivals(n: int, rate: float, seed: int = 5999) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def xx_chain(n: int, n_s: int, J: float, h: float, *, betas=(1.0,), n_v: int = 4, k: int = 30,
             seed: int = 0) -> Instance:
    """Open XX chain H = -(J/2) sum (sx sx + sy sy) + (h/2) sum sz: the solvable
    chain of the paper's experiments."""
    cps = [(i, i + 1, -J / 2.0, -J / 2.0, 0.0) for i in range(n - 1)]
    return Instance(n_s, n - n_s, cps, _zeros(n), np.full(n, h / 2.0),
                    np.asarray(betas, float), n_v, k, seed, f"xx_chain_{n_s}+{n - n_s}")


def random_dense_terms(n_s: int, n_b: int, seed: int, *, density: float = 0.6,
                       betas=(1.0,), n_v: int = 3, k: int = 20) -> Instance:
    """Every term type with random coefficients (XX, YY, ZZ with independent
    strengths, x- and z-fields) on a random subset of pairs: used to exercise
    all code paths at small sizes."""
    n = n_s + n_b
    rng = np.random.default_rng(seed)
    cps = []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.uniform() < density:
                cps.append((i, j, float(rng.normal()), float(rng.normal()), float(rng.normal())))
    hx = rng.normal(size=n) * 0.5
    hz = rng.normal(size=n) * 0.5
    return Instance(n_s, n_b, cps, hx, hz, np.asarray(betas, float), n_v, k, seed,
                    f"random_terms_{n_s}+{n_b}")
