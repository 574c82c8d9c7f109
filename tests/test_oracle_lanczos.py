"""Pins of O3 (per-column Lanczos, function approximation, Gram, bath
quadrature, finalize) and O4 (block Lanczos, Algorithm 1)."""
import numpy as np
import pytest

from oracle import block, exact, lanczos, spin
from oracle.rng import bath_vectors
from workloads import Instance, cfg_small_chain, long_range_xx_zz, random_dense_terms


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _scaled_op(inst):
    H = spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    s = np.abs(np.linalg.eigvalsh(H)).max()
    return H / s


def test_quadrature_moments_exact():
    # e_1^T T^p e_1 = x^T H^p x / |x|^2 for p <= 2k-1 (Gauss quadrature)
    inst = random_dense_terms(1, 6, 31)
    H = _scaled_op(inst)
    x = np.random.default_rng(1).normal(size=inst.dim)
    k = 8
    a, b, q, nx = lanczos.lanczos(lambda v: H @ v, x, k)
    T = lanczos.tridiag(a, b)
    xn = x / nx
    hp = xn.copy()
    tp = np.eye(k)[:, 0]
    for p in range(0, 2 * k):
        assert abs(xn @ hp - np.eye(k)[:, 0] @ tp) < 1e-12, p
        hp = H @ hp
        tp = T @ tp
    # degree 2k is no longer exact
    assert abs(xn @ hp - np.eye(k)[:, 0] @ tp) > 1e-10


def test_function_approximation_exact_for_low_degree():
    # |x| Q T^p e_1 = H^p x for p <= k-1
    inst = random_dense_terms(2, 4, 32)
    H = _scaled_op(inst)
    x = np.random.default_rng(2).normal(size=inst.dim)
    k = 7
    a, b, q, nx = lanczos.lanczos(lambda v: H @ v, x, k)
    T = lanczos.tridiag(a, b)
    hp, tp = x.copy(), np.eye(k)[:, 0]
    for p in range(k):
        assert np.abs(nx * q @ tp - hp).max() < 1e-12 * max(1, np.abs(hp).max()), p
        hp, tp = H @ hp, T @ tp
    assert np.abs(nx * q @ tp - hp).max() > 1e-10


@pytest.mark.parametrize("make", [cfg_small_chain,
                                  lambda: random_dense_terms(2, 5, 33, betas=(0.3, 1.0, 2.5), k=40),
                                  lambda: long_range_xx_zz(2, 6, 1.0, 34, n_v=3, k=40),
                                  # four system spins (d_s = 16), the Krylov space the whole space
                                  lambda: random_dense_terms(4, 3, 35, betas=(0.5, 2.0), n_v=2, k=128)])
def test_lanczos_path_equals_exact_typicality(make):
    inst = make()
    o2 = exact.exact_typicality(inst)
    o3 = lanczos.solve(inst)
    o4 = block.solve(inst)
    for r2, r3, r4 in zip(o2, o3["results"], o4["results"]):
        assert _rel(r3["rho"], r2["rho"]) < 1e-12
        assert _rel(r3["h_star"], r2["h_star"]) < 1e-11
        assert abs(r3["log_z"] - r2["log_z"]) < 1e-11
        assert abs(r3["entropy"] - r2["entropy"]) < 1e-12
        assert _rel(r4["rho"], r2["rho"]) < 1e-12
        assert _rel(r4["h_star"], r2["h_star"]) < 1e-11


def test_block_converges_faster_than_per_column():
    # the block quadrature is exact to degree 2k-1, the per-column Gram only for
    # f = g^2 with deg g <= k-1 (Section "Block Gauss quadrature")
    inst = cfg_small_chain()
    o2 = exact.exact_typicality(inst)[0]
    inst.k = 12
    e3 = _rel(lanczos.solve(inst)["results"][0]["rho"], o2["rho"])
    e4 = _rel(block.solve(inst)["results"][0]["rho"], o2["rho"])
    assert e4 < e3


def test_breakdown_small_space():
    # dim 8 < k: the recurrence stops on an invariant subspace and is exact
    inst = random_dense_terms(1, 2, 35, k=20, n_v=2)
    o3 = lanczos.solve(inst)
    assert all(len(a) <= 8 for a in o3["alpha"])
    o2 = exact.exact_typicality(inst)[0]
    assert _rel(o3["results"][0]["rho"], o2["rho"]) < 1e-10


def test_no_coupling_exact_with_one_sample():
    # H_sb = 0: (I (x) <v|) exp(-bH) (I (x) |v>) = exp(-b H_s) <v|exp(-b H_b)|v>,
    # so rho* = rho_s and H* = H_s for any single v
    base = random_dense_terms(2, 5, 36, k=60, n_v=1)
    cps = [c for c in base.couplings if (c[0] < 2) == (c[1] < 2)]
    inst = Instance(2, 5, cps, base.hx, base.hz, np.array([0.8]), 1, 60, 5)
    hs, _, _ = spin.split_dense(2, 5, cps, base.hx, base.hz)
    e, u = np.linalg.eigh(hs)
    rho_s = (u * np.exp(-0.8 * e)) @ u.T
    rho_s /= np.trace(rho_s)
    r = lanczos.solve(inst)["results"][0]
    assert np.abs(r["rho"] - rho_s).max() < 1e-13
    assert np.abs(r["h_star"] - hs).max() < 1e-12


def test_high_temperature_note():
    # beta -> 0: H*_est = H_s + avg_j (I (x) <v_j|) H_sb (I (x) |v_j>) + O(beta)
    inst = random_dense_terms(2, 4, 37, k=20, n_v=2)
    hs, _, hsb = spin.split_dense(2, 4, inst.couplings, inst.hx, inst.hz)
    v = bath_vectors(inst.seed, inst.n_v, inst.n_b)
    corr = np.zeros((4, 4))
    for j in range(inst.n_v):
        vj = np.kron(np.eye(4), v[:, j:j + 1])
        corr += vj.T @ hsb @ vj
    corr /= inst.n_v
    beta = 1e-5
    r = lanczos.solve(inst, betas=[beta])["results"][0]
    assert np.abs(r["h_star"] - (hs + corr)).max() < 1e-3
    assert np.abs(r["h_star"] - hs).max() > 10 * np.abs(r["h_star"] - (hs + corr)).max()
    assert np.abs(r["rho"] - np.eye(4) / 4).max() < 1e-3


TRUNCATION_CASES = [lambda b: random_dense_terms(1, 7, 38, betas=(b,), n_v=3, k=2),
                    lambda b: random_dense_terms(2, 6, 39, betas=(b,), n_v=2, k=2)]


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("beta", [0.5, 2.0])
def test_truncation_within_polynomial_bound(case, beta):
    # Section "Error analysis", "Block Gauss quadrature": after k steps the
    # block quadrature differs from the exact quadratic form by at most
    # 2 E_{2k-1}(f) on the spectral interval; the per-column Gram by the
    # bound derived from E_{k-1}(exp(-beta x / 2)).  Both are measured here
    # against O2 (same bath vectors, no Krylov error) for k = 2 .. 29.
    from oracle import bounds
    inst = TRUNCATION_CASES[case](beta)
    ev = np.linalg.eigvalsh(spin.dense_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz))
    lo, hi = ev[0], ev[-1]
    m_ex = exact.exact_typicality(inst)[0]["m"]          # shifted by lambda_min
    tight = []
    for k in range(2, 30, 3):
        inst.k = k
        o4 = block.solve(inst)
        ref = m_ex * np.exp(beta * (o4["e0"] - lo))
        err = np.linalg.norm(o4["results"][0]["m"] - ref, 2)
        bound = bounds.block_quadrature_bound(beta, lo, hi, o4["e0"], k)
        assert err <= bound + 1e-13 * np.linalg.norm(ref, 2), ("block", k, err, bound)
        o3 = lanczos.solve(inst)
        ref = m_ex * np.exp(beta * (o3["e0"] - lo))
        err3 = np.linalg.norm(o3["results"][0]["m"] - ref, 2)
        bound3 = bounds.per_column_gram_bound(beta, lo, hi, o3["e0"], k, inst.d_s)
        assert err3 <= bound3 + 1e-13 * np.linalg.norm(ref, 2), ("per-column", k, err3, bound3)
        tight.append(bound3 < 1e-3 * np.linalg.norm(ref, 2))
    # the bound is not vacuous: it falls far below |M| within the sweep
    assert any(tight)


def test_chebyshev_interpolation_error_closed_form():
    # for f = exp(-beta x) the interpolation error obeys the classical bound
    # ((hi-lo)/2)^{n+1} max|f^{(n+1)}| / (2^n (n+1)!) and exceeds the best
    # approximation error, which for degree 0 is (max f - min f)/2
    from math import exp, factorial
    from oracle import bounds
    for beta, lo, hi, n in [(1.0, -3.0, 2.0, 5), (0.3, 0.0, 10.0, 9), (2.0, -1.0, 1.0, 12)]:
        e = bounds.chebyshev_interpolation_error(beta, lo, hi, 0.0, n)
        cap = ((hi - lo) / 2) ** (n + 1) * beta ** (n + 1) * exp(-beta * lo) / (2 ** n * factorial(n + 1))
        assert e <= cap * (1 + 1e-12)
        assert e > 0.05 * cap
    e0 = bounds.chebyshev_interpolation_error(1.0, 0.0, 2.0, 0.0, 0)
    assert e0 >= 0.5 * (1.0 - exp(-2.0)) * (1 - 1e-12)


def test_pooled_merged_run_equals_serial_matrix_free():
    # the reference runs at full size use the merged operator and a process
    # pool over the columns; they must give the plain serial run's results
    import multiprocessing as mp
    inst = long_range_xx_zz(2, 7, 1.0, 35, betas=(0.5, 2.0), n_v=3, k=30)
    a = lanczos.solve(inst)
    with mp.get_context("spawn").Pool(2) as pool:
        b = lanczos.solve(inst, merged=True, mapper=pool.map)
    for x, y in zip(a["results"], b["results"]):
        assert _rel(y["rho"], x["rho"]) < 1e-13
        assert _rel(y["h_star"], x["h_star"]) < 1e-12
        assert abs(y["log_z"] - x["log_z"]) < 1e-12
    for ca, cb in zip(a["alpha"], b["alpha"]):
        assert np.abs(ca[:10] - cb[:10]).max() < 1e-12
