"""Pins of the oracle's SplitMix64 and bath-vector rule."""
import os

import numpy as np

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def test_splitmix64_published_sequence():
    want = [int(l) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert rng.sm64_stream(1234567, len(want)) == want


def test_vectorised_matches_scalar():
    xs = np.array([0, 1, 2 ** 63, 2 ** 64 - 1, 12345678901234567], dtype=np.uint64)
    got = rng._sm64_np(xs)
    assert [int(g) for g in got] == [rng.sm64(int(x)) for x in xs]


def test_bath_vector_rule_bits():
    # the rule: bit b of vector j is bit (b & 63) of sm64(key_j ^ (b >> 6))
    seed, j, n_b = 99, 3, 8
    key = rng.sm64(seed ^ rng.sm64(j))
    signs = rng.rademacher_signs(seed, j, n_b)
    for b in (0, 1, 63, 64, 100, 255):
        bit = (rng.sm64(key ^ (b >> 6)) >> (b & 63)) & 1
        assert signs[b] == 1 - 2 * bit


def test_bath_vector_unit_norm_and_balance():
    v = rng.bath_vectors(7, 8, 12)
    assert np.allclose((v * v).sum(axis=0), 1.0, atol=1e-14)
    assert set(np.unique(np.sign(v))) == {-1.0, 1.0}
    frac = (v > 0).mean()
    assert abs(frac - 0.5) < 0.01  # 32768 fair signs: sd 0.003
    # distinct samples are (nearly) orthogonal: |<v_i, v_j>| ~ 1/sqrt(d_b)
    g = v.T @ v
    off = np.abs(g - np.diag(np.diag(g))).max()
    assert off < 6.0 / np.sqrt(4096)
