"""Pins of the Hamiltonian convention (eqn:Ht, the site operators and the
system/bath split) in the oracle."""
import itertools

import numpy as np
import pytest

from oracle import spin
from oracle.exact import partial_trace_bath
from workloads import random_dense_terms, xx_chain


def test_two_site_heisenberg_spectrum():
    # sigma.sigma on two spins: triplet +1 (x3), singlet -3 (textbook)
    h = spin.dense_hamiltonian(2, [(0, 1, 1.0, 1.0, 1.0)], [0, 0], [0, 0])
    assert np.allclose(np.sort(np.linalg.eigvalsh(h)), [-3, 1, 1, 1], atol=1e-14)


def test_site_order_and_sz_sign():
    # site 0 is the most significant bit; sz|0> = +|0>
    h = spin.dense_hamiltonian(3, [], [0, 0, 0], [1.0, 0, 0])
    assert np.allclose(np.diag(h), [1, 1, 1, 1, -1, -1, -1, -1])
    h = spin.dense_hamiltonian(3, [], [0, 0, 0], [0, 0, 1.0])
    assert np.allclose(np.diag(h), [1, -1] * 4)


def test_yy_sign_pattern():
    # sy sy: <11|.|00> = -1, <10|.|01> = +1
    h = spin.dense_hamiltonian(2, [(0, 1, 0.0, 1.0, 0.0)], [0, 0], [0, 0])
    assert h[3, 0] == -1 and h[0, 3] == -1 and h[2, 1] == 1 and h[1, 2] == 1


@pytest.mark.parametrize("n,J,h", [(6, 1.0, 0.3), (7, 0.7, -1.1)])
def test_xx_chain_free_fermion_spectrum(n, J, h):
    # H = -(J/2) sum (sx sx + sy sy) + (h/2) sum sz maps to free fermions with
    # lambda_k = h - 2J cos(k pi/(N+1)) and a constant -N h/2: the many-body
    # spectrum is -N h/2 + sum over occupied k of lambda_k
    inst = xx_chain(n, 2, J, h)
    H = spin.dense_hamiltonian(n, inst.couplings, inst.hx, inst.hz)
    lam = h - 2 * J * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    many = [-n * h / 2 + sum(lam[list(s)]) for r in range(n + 1)
            for s in itertools.combinations(range(n), r)]
    assert np.allclose(np.sort(np.linalg.eigvalsh(H)), np.sort(many), atol=1e-12)


@pytest.mark.parametrize("n_s,n_b,seed", [(1, 4, 1), (2, 4, 2), (3, 3, 3), (4, 3, 4)])
def test_matrix_free_equals_dense(n_s, n_b, seed):
    inst = random_dense_terms(n_s, n_b, seed)
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    assert np.abs(H - H.T).max() == 0.0
    op = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    x = np.random.default_rng(seed).normal(size=(inst.dim, 3))
    assert np.abs(op.apply(x) - H @ x).max() < 1e-13
    rows = np.array([0, 5, inst.dim - 1])
    assert np.abs(op.rows(rows, x) - (H @ x)[rows]).max() < 1e-13


def test_split_sums_to_total_and_hsb_traceless_over_bath():
    inst = random_dense_terms(2, 3, 11)
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    hs, hb, hsb = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    assert np.abs(np.kron(hs, np.eye(8)) + np.kron(np.eye(4), hb) + hsb - H).max() < 1e-13
    # tr_b(H_sb) = 0 (appendix on the high-temperature limit)
    assert np.abs(partial_trace_bath(hsb, 4, 8)).max() < 1e-13
    # the matrix-free bath operator equals the dense H_b
    opb = spin.sparse_bath_hamiltonian(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    x = np.random.default_rng(0).normal(size=8)
    assert np.abs(opb.apply(x) - hb @ x).max() < 1e-13


@pytest.mark.parametrize("n_s,n_b,seed", [(1, 6, 41), (2, 5, 42), (3, 6, 43)])
def test_merged_apply_equals_dense_and_matrix_free(n_s, n_b, seed):
    # the merged form (strings grouped by flip mask, partners by axis reversal)
    # against the Kronecker H and the scatter form, every term type, both the
    # total and the bath operator, one and several columns
    inst = random_dense_terms(n_s, n_b, seed)
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    m = spin.merged_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    sp = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    x = np.random.default_rng(seed).normal(size=(inst.dim, 3))
    assert np.abs(m.apply(x) - H @ x).max() < 1e-13
    assert np.abs(m.apply(x[:, 1]) - sp.apply(x[:, 1])).max() < 1e-13
    _, hb, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    mb = spin.merged_bath_hamiltonian(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    xb = x[:inst.d_b]
    assert np.abs(mb.apply(xb) - hb @ xb).max() < 1e-13


def test_merged_apply_at_16_bits_equals_matrix_free():
    inst = random_dense_terms(2, 14, 44, density=0.15)
    m = spin.merged_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    sp = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    x = np.random.default_rng(44).normal(size=inst.dim)
    assert np.abs(m.apply(x) - sp.apply(x)).max() < 1e-12 * np.abs(x).max() * len(sp.terms)
