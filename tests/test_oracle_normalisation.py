"""Pins of the estimator's normalisation in ``oracle.exact.finalize``:
ln Z_t = ln tr M - beta E0 + ln d_b and ln Z_b = ln m_b - beta E0b + ln d_b
(eqn:trace_est with unit bath vectors, eqn:HMF, eqn:H_est).

Two facts fixed by the mathematics, not by the oracle's own formulas:

* with every bath vector of {+-2^(-n_b/2)}^(d_b) (the full Rademacher
  enumeration), sum_v v v^T / 2^(d_b) = I / d_b exactly, so the sample mean of
  the estimator IS the partial trace: rho*, ln Z_t, ln Z_b, ln Z* and H* equal
  the exact values, for O2 and for O3 run to the full Krylov dimension;
* with H_sb = 0, exp(-beta H_t) factorises, so ln Z* = ln tr exp(-beta H_s)
  for any single bath vector.

The exact side is a matrix exponential (scipy's Pade ``expm``) of the
Kronecker H, traced directly -- no eigendecomposition, no shift.  A dropped
ln d_b, a flipped sign of beta E0 or a shift that is not undone moves ln Z_t
by at least ln 2 or beta |E0| and fails these checks.
"""
import itertools

import numpy as np
import pytest
from scipy.linalg import expm

import oracle.exact as oexact
import oracle.lanczos as olz
from oracle import spin
from workloads import Instance, random_dense_terms


def _all_sign_vectors(n_b):
    d_b = 1 << n_b
    signs = np.array(list(itertools.product((1.0, -1.0), repeat=d_b))).T  # d_b x 2^d_b
    return signs * 2.0 ** (-n_b / 2)


def _exact_by_expm(inst, beta):
    h = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    a = expm(-beta * h)
    r = np.einsum("ibjb->ij", a.reshape(inst.d_s, inst.d_b, inst.d_s, inst.d_b))
    _, hb, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    z_b = float(np.trace(expm(-beta * hb)))
    return {"rho": r / np.trace(r), "log_z_t": float(np.log(np.trace(r))),
            "log_z_b": float(np.log(z_b)), "log_z": float(np.log(np.trace(r) / z_b)),
            "r": r, "z_b": z_b}


@pytest.fixture
def every_sign_vector(monkeypatch):
    """Bath vectors: the sign vectors of {+-2^(-n_b/2)}^(d_b) in a fixed
    order (vectors 0 .. n_v-1 are the first n_v, as with the seeded rule);
    n_v = 2^(d_b) takes all of them."""
    def fake(seed, n_v, n_b):
        v = _all_sign_vectors(n_b)
        assert n_v <= v.shape[1]
        return v[:, :n_v]
    monkeypatch.setattr(oexact, "bath_vectors", fake)
    monkeypatch.setattr(olz, "bath_vectors", fake)


@pytest.mark.parametrize("n_s,seed", [(1, 91), (2, 92)])
def test_full_enumeration_is_the_exact_partial_trace(every_sign_vector, n_s, seed):
    # n_b = 3: d_b = 8 bath states, 256 sign vectors
    base = random_dense_terms(n_s, 3, seed)
    inst = Instance(n_s, 3, base.couplings, base.hx, base.hz, np.array([0.4, 1.7]), 256,
                    1 << (n_s + 3), seed)
    for beta, o2 in zip(inst.betas, oexact.exact_typicality(inst)):
        ex = _exact_by_expm(inst, beta)
        assert np.abs(o2["rho"] - ex["rho"]).max() < 1e-13
        assert abs(o2["log_z_t"] - ex["log_z_t"]) < 1e-12
        assert abs(o2["log_z_b"] - ex["log_z_b"]) < 1e-12
        assert abs(o2["log_z"] - ex["log_z"]) < 1e-12
        # H* = -(1/beta) ln(tr_b exp(-beta H_t) / Z_b), through the eigenvalues
        mu, u = np.linalg.eigh(0.5 * (ex["r"] + ex["r"].T))
        h_star = (u * (-np.log(mu / ex["z_b"]) / beta)) @ u.T
        assert np.abs(o2["h_star"] - h_star).max() < 1e-11
    # the algorithm itself (O3) with the full Krylov space: the same answers
    o3 = olz.solve(inst)["results"]
    for beta, r in zip(inst.betas, o3):
        ex = _exact_by_expm(inst, beta)
        assert np.abs(r["rho"] - ex["rho"]).max() < 1e-11
        assert abs(r["log_z_t"] - ex["log_z_t"]) < 1e-10
        assert abs(r["log_z_b"] - ex["log_z_b"]) < 1e-10


def test_single_sample_mean_of_z_t(every_sign_vector):
    # one sample per sign vector (n_v = 1): the mean of exp(ln Z_t) is Z_t;
    # finalize is called on each single-sample M with its own arbitrary shift
    base = random_dense_terms(1, 3, 93)
    inst = Instance(1, 3, base.couplings, base.hx, base.hz, np.array([1.3]), 256, 16, 93)
    beta = 1.3
    h = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    _, hb, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    v = _all_sign_vectors(3)
    rng = np.random.default_rng(5)
    zt = zb = 0.0
    for j in range(v.shape[1]):
        e0, e0b = rng.uniform(-4, 1), rng.uniform(-4, 1)
        vj = np.kron(np.eye(inst.d_s), v[:, j:j + 1])            # I_s (x) |v_j>
        m = vj.T @ expm(-beta * (h - e0 * np.eye(inst.dim))) @ vj
        m_b = float(v[:, j] @ expm(-beta * (hb - e0b * np.eye(inst.d_b))) @ v[:, j])
        out = oexact.finalize(m, m_b, e0, e0b, beta, inst.d_b)
        zt += np.exp(out["log_z_t"])
        zb += np.exp(out["log_z_b"])
    zt /= v.shape[1]
    zb /= v.shape[1]
    assert abs(zt / np.trace(expm(-beta * h)) - 1) < 1e-12
    assert abs(zb / np.trace(expm(-beta * hb)) - 1) < 1e-12


@pytest.mark.parametrize("seed", [94, 95, 96])
def test_no_system_bath_coupling_gives_ln_tr_exp_hs(seed):
    # H_sb = 0: exp(-beta H_t) = exp(-beta H_s) (x) exp(-beta H_b), so for any
    # single bath vector ln Z* = ln tr exp(-beta H_s); both shifts (E0 from
    # H_t, E0b from H_b, which differ) must be undone for this to hold
    base = random_dense_terms(2, 5, seed)
    cps = [c for c in base.couplings if (c[0] < 2) == (c[1] < 2)]
    inst = Instance(2, 5, cps, base.hx, base.hz, np.array([0.3, 2.0, 6.0]), 1, 60, seed)
    hs, _, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    for res in (oexact.exact_typicality(inst), olz.solve(inst)["results"]):
        for beta, r in zip(inst.betas, res):
            want = float(np.log(np.trace(expm(-beta * hs))))
            assert abs(r["log_z"] - want) < 1e-10 * max(1.0, abs(want)), (beta, r["log_z"], want)
