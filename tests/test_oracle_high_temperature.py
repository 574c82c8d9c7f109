"""Pins of O9, the estimator's high-temperature offset (Section "A note on
high temperatures"; the appendix deriving the high-temperature limit): the
small-beta limit of the sampled estimate (O2, dense exponentials), the exact
limit H_s (O1), zero mean over all sign vectors, and special cases."""
import itertools

import numpy as np
import pytest

from oracle import exact, high_temperature as ht
from oracle.rng import bath_vectors
from oracle.spin import split_dense
from workloads import Instance, random_dense_terms


def _hs(inst):
    return split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)[0]


@pytest.mark.parametrize("n_s,n_b,seed,n_v", [(1, 6, 3, 1), (2, 5, 17, 3), (2, 6, 29, 2)])
def test_offset_is_the_small_beta_limit_of_the_estimate(n_s, n_b, seed, n_v):
    inst = random_dense_terms(n_s, n_b, seed, n_v=n_v)
    hs = _hs(inst)
    c = ht.offset(inst)
    assert np.abs(c).max() > 1e-2                      # the offset is not trivially zero here
    errs = []
    for beta in (1e-4, 1e-5):
        est = exact.exact_typicality(inst, [beta])[0]["h_star"]
        errs.append(np.abs(est - hs - c).max())
        # without the offset the sampled estimate misses H_s by about |C|
        assert np.abs(est - hs).max() > 0.5 * np.abs(c).max()
        # the exact H*(beta) tends to H_s itself: tr_b(H_sb) = 0
        assert np.abs(exact.exact_rdm(inst, beta)["h_star"] - hs).max() < 50 * beta
    assert errs[1] < 50 * 1e-5
    assert errs[1] < 0.2 * errs[0]                     # the remainder is O(beta)


def test_mean_over_all_sign_vectors_is_zero():
    # E[v v^T] = I/d_b over all 2^d_b unit sign vectors, so the mean of C is
    # tr_b(H_sb)/d_b, which is zero for Pauli couplings
    inst = random_dense_terms(1, 2, 5, density=1.0)
    d_b = inst.d_b
    vs = [np.array(s, float) / np.sqrt(d_b) for s in itertools.product((1.0, -1.0), repeat=d_b)]
    cs = [ht.offset_from_vectors(1, 2, inst.couplings, v[:, None]) for v in vs]
    assert max(np.abs(c).max() for c in cs) > 1e-2
    assert np.abs(np.mean(cs, axis=0)).max() < 1e-15


def test_zz_and_yy_cross_couplings_give_zero():
    # equal-magnitude real entries: <v|sz|v> = 0 and <v|sy|v> = 0 exactly
    n_s, n_b = 2, 6
    n = n_s + n_b
    rng = np.random.default_rng(7)
    cps = [(a, c, 0.0, float(rng.normal()), float(rng.normal())) for a in range(n_s) for c in range(n_s, n)]
    cps += [(0, 1, 0.7, 0.2, 0.3), (3, 5, 1.1, 0.0, 0.4)]
    inst = Instance(n_s, n_b, cps, rng.normal(size=n), rng.normal(size=n), np.array([1.0]), 4, 10, 21)
    assert np.abs(ht.offset(inst)).max() < 1e-15          # zero up to rounding
    cps.append((1, 4, 0.5, 0.0, 0.0))
    inst.couplings = cps
    assert np.abs(ht.offset(inst)).max() > 1e-3


def test_single_xx_coupling_closed_form():
    # one coupling jx sx_0 sx_c: C = jx <v|sx_c|v> sx on the one system spin,
    # <v|sx_c|v> = sum_b v_b v_(b xor bit of c) with site c at bath bit n_b-1-(c-n_s)
    n_s, n_b, jx, site = 1, 5, -0.8, 3
    inst = Instance(n_s, n_b, [(0, site, jx, 0.0, 0.0)], np.zeros(6), np.zeros(6), np.array([1.0]), 3, 10, 99)
    v = bath_vectors(inst.seed, inst.n_v, n_b)
    flip = 1 << (n_b - 1 - (site - n_s))
    perm = np.arange(inst.d_b) ^ flip
    e = float(np.mean([v[:, j] @ v[perm, j] for j in range(inst.n_v)]))
    assert abs(e) > 1e-3
    want = jx * e * np.array([[0.0, 1.0], [1.0, 0.0]])
    assert np.abs(ht.offset(inst) - want).max() < 1e-15
    sx = ht.bath_sx(inst)
    assert abs(sx[site - n_s] - e) < 1e-15
