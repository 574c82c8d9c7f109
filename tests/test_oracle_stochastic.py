"""Statistical pins of the partial-trace typicality estimator (eqn:vivj,
eqn:trace_est) and of the exact-variance formula O6."""
import itertools

import numpy as np

from oracle import exact, spin, variance
from oracle.rng import bath_vectors
from workloads import cfg_small_chain, random_dense_terms


def _shifted_exp(inst, beta):
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    e, u = np.linalg.eigh(H)
    return (u * np.exp(-beta * (e - e[0]))) @ u.T


def _estimate(a, d_s, d_b, v):
    """(1/n_v) sum_j (I (x) <v_j|) A (I (x) |v_j>)."""
    blocks = a.reshape(d_s, d_b, d_s, d_b)
    av = np.einsum("ajbk,kv->ajbv", blocks, v, optimize=True)
    return np.einsum("ajbv,jv->ab", av, v, optimize=True) / v.shape[1]


def test_variance_formula_by_enumeration():
    # all 2^8 sign patterns of a d_b = 8 Rademacher vector
    inst = random_dense_terms(1, 3, 41)
    a = _shifted_exp(inst, 0.7)
    d_s, d_b = 2, 8
    samples = []
    for signs in itertools.product((-1.0, 1.0), repeat=d_b):
        v = np.array(signs)[:, None] / np.sqrt(d_b)
        samples.append(_estimate(a, d_s, d_b, v))
    samples = np.array(samples)
    mean = samples.mean(axis=0)
    assert np.abs(mean - exact.partial_trace_bath(a, d_s, d_b) / d_b).max() < 1e-15
    assert np.abs(samples.var(axis=0) - variance.entry_variance(a, d_s, d_b)).max() < 1e-15


def test_estimator_error_matches_exact_variance():
    inst = cfg_small_chain()
    a = _shifted_exp(inst, 1.0)
    d_s, d_b, n_v = inst.d_s, inst.d_b, inst.n_v
    target = exact.partial_trace_bath(a, d_s, d_b) / d_b
    var = variance.entry_variance(a, d_s, d_b)
    errs = np.array([_estimate(a, d_s, d_b, bath_vectors(seed, n_v, inst.n_b)) - target
                     for seed in range(200)])
    ratio = (errs ** 2).mean(axis=0) / (var / n_v)
    assert np.all((ratio > 0.75) & (ratio < 1.3)), ratio
    # unbiased: the mean error over 200 seeds is within 5 standard errors
    assert np.all(np.abs(errs.mean(axis=0)) < 5 * np.sqrt(var / n_v / 200))
    # every single run lies within 5 sigma
    assert np.all(np.abs(errs) <= 5 * np.sqrt(var / n_v))


def test_error_shrinks_as_inverse_sqrt_nv():
    inst = cfg_small_chain()
    a = _shifted_exp(inst, 1.0)
    d_s, d_b = inst.d_s, inst.d_b
    target = exact.partial_trace_bath(a, d_s, d_b) / d_b
    nvs = [4, 16, 64, 256]
    rms = []
    for n_v in nvs:
        e = [np.linalg.norm(_estimate(a, d_s, d_b, bath_vectors(100 + s, n_v, inst.n_b)) - target)
             for s in range(60)]
        rms.append(np.sqrt(np.mean(np.square(e))))
    slope = np.polyfit(np.log(nvs), np.log(rms), 1)[0]
    assert abs(slope + 0.5) < 0.06, slope


def test_union_bound_holds():
    # Section "Trace estimators": per-entry Chebyshev bounds at eps/d_s and
    # delta/d_s^2 give P[|| estimate - tr_b(A)/d_b || > eps] < delta
    inst = cfg_small_chain()
    a = _shifted_exp(inst, 1.0)
    d_s, d_b, n_v = inst.d_s, inst.d_b, inst.n_v
    target = exact.partial_trace_bath(a, d_s, d_b) / d_b
    var = variance.entry_variance(a, d_s, d_b)
    delta = 1e-2
    # Chebyshev per entry: P[|err| > t] <= var/(n_v t^2) = delta/d_s^2
    t = np.sqrt(var.max() / n_v / (delta / d_s ** 2))
    eps = t * d_s
    viol = 0
    for seed in range(200):
        err = _estimate(a, d_s, d_b, bath_vectors(seed, n_v, inst.n_b)) - target
        viol += np.linalg.norm(err, 2) > eps
    assert viol / 200 < delta + 0.02
