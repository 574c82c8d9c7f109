"""Pins of O8, the low-temperature limit (Section "High and low temperature
limits"): closed forms, the large-beta limit of O1, and the step-by-step
Lanczos version against the dense ground space."""
import numpy as np
import pytest

from oracle import exact, ground
from workloads import Instance, cfg_small_chain, random_dense_terms


def _z():
    return np.zeros(2)


def test_two_spin_singlet():
    # antiferromagnetic Heisenberg pair, no fields: the singlet (E = -3J) is
    # the unique ground state, maximally entangled, so rho_s(inf) = I/2; the
    # lone bath spin has H_b = 0
    J = 0.8
    inst = Instance(1, 1, [(0, 1, J, J, J)], _z(), _z(), np.array([1.0]), 1, 4, 0)
    g = ground.exact(inst)
    assert g["degeneracy"] == 1
    assert abs(g["e_total"] + 3 * J) < 1e-12 and abs(g["e_bath"]) < 1e-12
    assert np.abs(g["rho"] - 0.5 * np.eye(2)).max() < 1e-12
    assert np.abs(g["h_star"] + 3 * J * np.eye(2)).max() < 1e-12
    assert abs(g["entropy"] - np.log(2)) < 1e-12


def test_ising_ferromagnet_degenerate():
    # zz chain without fields: |0...0> and |1...1> are degenerate ground states,
    # rho_s(inf) = diag(1/2, 1/2) for one system spin
    n = 6
    inst = Instance(1, n - 1, [(i, i + 1, 0.0, 0.0, -1.0) for i in range(n - 1)], np.zeros(n), np.zeros(n),
                    np.array([1.0]), 4, 20, 0)
    g = ground.exact(inst)
    assert g["degeneracy"] == 2
    assert abs(g["e_total"] + (n - 1)) < 1e-12 and abs(g["e_bath"] + (n - 2)) < 1e-12
    assert np.abs(g["rho"] - 0.5 * np.eye(2)).max() < 1e-12


@pytest.mark.parametrize("make", [cfg_small_chain, lambda: random_dense_terms(2, 5, 91)])
def test_exact_is_the_large_beta_limit(make):
    # O1 at large beta converges to the ground-space partial trace (gap > 0)
    inst = make()
    g = ground.exact(inst)
    assert g["degeneracy"] == 1
    o1 = exact.exact_rdm(inst, 200.0)
    assert np.abs(o1["rho"] - g["rho"]).max() < 1e-8


@pytest.mark.parametrize("make,r", [(cfg_small_chain, 1),
                                    (lambda: Instance(1, 5, [(i, i + 1, 0.0, 0.0, -1.0) for i in range(5)],
                                                      np.zeros(6), np.zeros(6), np.array([1.0]), 4, 64, 0), 2)])
def test_lanczos_ritz_equals_exact(make, r):
    inst = make()
    g = ground.exact(inst)
    lz = ground.lanczos_ritz(inst, 4, 64, 11)
    assert lz["degeneracy"] == r == g["degeneracy"]
    assert abs(lz["e_total"] - g["e_total"]) < 1e-10
    assert abs(lz["e_bath"] - g["e_bath"]) < 1e-10
    assert np.abs(lz["rho"] - g["rho"]).max() < 1e-8
