"""Pins of O10, the product-state estimator (appendix "A consistent partial
trace estimator"): unbiasedness over every product sign vector, the
conditional means equal to the partial traces' quadratic forms (which fixes
the Kronecker order), the link to the partial-trace estimator's samples, and
Lanczos quadrature = dense quadratic form at convergence."""
import itertools

import numpy as np
import pytest

from oracle import lanczos as olz, product
from oracle.exact import partial_trace_bath
from oracle.rng import bath_vector
from oracle.spin import dense_hamiltonian
from workloads import random_dense_terms


def _expm(inst, beta):
    e, u = np.linalg.eigh(dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz))
    return (u * np.exp(-beta * e)) @ u.T


def _signs(d):
    return [np.array(s, float) / np.sqrt(d) for s in itertools.product((1.0, -1.0), repeat=d)]


def test_unbiased_and_consistent_over_all_product_vectors():
    inst = random_dense_terms(1, 2, 7, density=1.0)
    d_s, d_b = inst.d_s, inst.d_b
    a = _expm(inst, 0.7)
    vs_all, vb_all = _signs(d_s), _signs(d_b)
    q = np.array([[np.kron(vs, vb) @ a @ np.kron(vs, vb) for vb in vb_all] for vs in vs_all])
    # E[x x^T] = I / D: D * mean = tr A
    assert abs(d_s * d_b * q.mean() - np.trace(a)) < 1e-12 * np.trace(a)
    # mean over the bath factor = <v_s| tr_b A |v_s> / d_b
    trb = partial_trace_bath(a, d_s, d_b)
    for i, vs in enumerate(vs_all):
        assert abs(q[i].mean() - vs @ trb @ vs / d_b) < 1e-13
    # mean over the system factor = <v_b| tr_s A |v_b> / d_s
    trs = np.trace(a.reshape(d_s, d_b, d_s, d_b), axis1=0, axis2=2)
    for i, vb in enumerate(vb_all):
        assert abs(q[:, i].mean() - vb @ trs @ vb / d_s) < 1e-13
    # the Kronecker order matters: the swapped order misses tr_b for this H
    trb_wrong = np.trace(a.reshape(d_b, d_s, d_b, d_s), axis1=0, axis2=2)
    assert max(abs(q[i].mean() - vs @ trb_wrong @ vs / d_b) for i, vs in enumerate(vs_all)) > 1e-3


def test_sample_is_the_partial_trace_sample_seen_through_v_s():
    # <v_s (x) v_j| A |v_s (x) v_j> = v_s^T M_j v_s with M_j = (I (x) <v_j|) A (I (x) |v_j>)
    inst = random_dense_terms(2, 5, 23)
    a = _expm(inst, 1.3)
    for j in range(3):
        vb = bath_vector(inst.seed, j, inst.n_b)
        vmat = np.kron(np.eye(inst.d_s), vb[:, None])
        mj = vmat.T @ a @ vmat
        vs = product.system_vector(inst.seed, j, inst.n_s)
        x = product.product_vector(inst.seed, j, inst.n_s, inst.n_b)
        assert abs(x @ a @ x - vs @ mj @ vs) < 1e-12 * abs(vs @ mj @ vs)
        assert np.array_equal(np.abs(vs), np.full(inst.d_s, 0.5))


@pytest.mark.parametrize("n_s,n_b,seed", [(1, 6, 3), (2, 5, 41)])
def test_lanczos_equals_dense_at_convergence(n_s, n_b, seed):
    inst = random_dense_terms(n_s, n_b, seed)
    betas = [0.3, 1.0, 2.5]
    ex = product.exact_samples(inst, betas, 4, 99)
    lz = product.lanczos_estimate(inst, betas, 4, 60, 99)
    assert np.abs(lz["log_z_t_samples"] - ex["log_z_t_samples"]).max() < 1e-9
    assert np.abs(lz["log_z_t"] - ex["log_z_t"]).max() < 1e-9
    # the bath part is the partial-trace estimator's (same vectors, same quadrature)
    inst.n_v, inst.k, inst.seed = 4, 60, 99
    o3 = olz.solve(inst, betas)
    assert np.abs(lz["log_z_b"] - np.array([r["log_z_b"] for r in o3["results"]])).max() < 1e-10
