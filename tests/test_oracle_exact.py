"""Pins of O1 (dense exact rho*, H*, ln Z*, S) against closed forms and the
paper's limits."""
import numpy as np
import pytest

from oracle import closed_form, exact, spin
from workloads import Instance, random_dense_terms, xx_chain


@pytest.mark.parametrize("n,J,h,beta", [(6, 1.0, 0.3, 1.3), (8, 1.0, 0.3, 0.4),
                                        (8, 0.8, 1.7, 3.0), (10, 1.0, 2.5, 2.0)])
def test_xx_chain_closed_form(n, J, h, beta):
    inst = xx_chain(n, 2, J, h)
    ex = exact.exact_rdm(inst, beta)
    cf = closed_form.xx_chain_rdm(n, J, h, beta)
    assert np.allclose(np.sort(np.linalg.eigvalsh(ex["rho"])), np.sort(cf["p"]), atol=1e-13)
    assert abs(ex["log_z"] - cf["log_z"]) < 1e-12
    assert abs(ex["log_z_t"] - cf["log_z_n"]) < 1e-11
    assert np.allclose(np.sort(np.linalg.eigvalsh(ex["h_star"])), np.sort(cf["h_eig"]), atol=1e-11)
    assert abs(ex["entropy"] - cf["entropy"]) < 1e-12


@pytest.mark.parametrize("J,Jz,h1,h2,beta", [(0.7, -0.4, 0.3, -0.9, 1.1), (1.0, 1.0, 0.0, 0.5, 3.0)])
def test_two_spin_closed_form(J, Jz, h1, h2, beta):
    inst = Instance(1, 1, [(0, 1, J, J, Jz)], np.zeros(2), np.array([h1, h2]),
                    np.array([beta]), 1, 1, 0)
    ex = exact.exact_rdm(inst, beta)
    cf = closed_form.two_spin_rdm(J, Jz, h1, h2, beta)
    assert np.abs(ex["rho"] - cf["rho"]).max() < 1e-14
    assert abs(ex["log_z_t"] - cf["log_z_t"]) < 1e-13
    assert abs(ex["log_z"] - cf["log_z"]) < 1e-13


def _decoupled(inst):
    """Same instance with every system-bath coupling removed."""
    cps = [c for c in inst.couplings if (c[0] < inst.n_s) == (c[1] < inst.n_s)]
    return Instance(inst.n_s, inst.n_b, cps, inst.hx, inst.hz, inst.betas, inst.n_v, inst.k,
                    inst.seed)


def _expm_sym(a, beta):
    e, u = np.linalg.eigh(a)
    return (u * np.exp(-beta * e)) @ u.T


def test_no_coupling_gives_bare_system():
    inst = _decoupled(random_dense_terms(2, 4, 21))
    hs, _, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    beta = 0.9
    ex = exact.exact_rdm(inst, beta)
    rho_s = _expm_sym(hs, beta)
    rho_s /= np.trace(rho_s)
    assert np.abs(ex["rho"] - rho_s).max() < 1e-13
    assert np.abs(ex["h_star"] - hs).max() < 1e-12


def test_high_temperature_limit():
    inst = random_dense_terms(2, 4, 22)
    hs, _, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    for beta in (1e-3, 1e-4):
        ex = exact.exact_rdm(inst, beta)
        assert np.abs(ex["rho"] - np.eye(4) / 4).max() < 10 * beta * np.abs(hs).max() + 1e-12
        # H*(beta) = H_s + tr_b(H_sb)/d_b + O(beta) and tr_b(H_sb) = 0
        assert np.abs(ex["h_star"] - hs).max() < 2000 * beta


def test_low_temperature_limit():
    inst = random_dense_terms(1, 5, 23)
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    e, u = np.linalg.eigh(H)
    assert e[1] - e[0] > 1e-3  # nondegenerate ground state for this seed
    g = np.outer(u[:, 0], u[:, 0])
    rho_inf = exact.partial_trace_bath(g, 2, 32)
    ex = exact.exact_rdm(inst, 200.0)
    assert np.abs(ex["rho"] - rho_inf).max() < 1e-8
    # H* -> (E_t - E_b) I: the spread of H* eigenvalues shrinks like 1/beta
    prev = None
    for beta in (20.0, 40.0, 80.0):
        he = np.linalg.eigvalsh(exact.exact_rdm(inst, beta)["h_star"])
        dev = np.abs(he - (ex["e_t"] - ex["e_b"])).max()
        if prev is not None:
            assert dev < 0.6 * prev
        prev = dev


def test_density_matrix_invariants():
    inst = random_dense_terms(3, 3, 24)
    ex = exact.exact_rdm(inst, 1.7)
    rho = ex["rho"]
    assert np.abs(rho - rho.T).max() < 1e-15
    assert abs(np.trace(rho) - 1) < 1e-14
    assert np.linalg.eigvalsh(rho).min() > -1e-15
    # rho* = exp(-beta H*)/Z*  (eqn:density_from_H)
    back = _expm_sym(ex["h_star"], 1.7) / np.exp(ex["log_z"])
    assert np.abs(back - rho).max() < 1e-12
