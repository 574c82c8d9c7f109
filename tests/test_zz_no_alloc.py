"""The allocation-free solve entry point (rdm_solve_noalloc) against the
entry point whose workspace it replaces (rdm_solve_ws), through the C ABI:
two calls in a row, the second on a smaller instance, each equal to the
ordinary solve with the same plan (hbm_budget = the scratch size), and both
within the parity bar of the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
rdm = pytest.importorskip("paper_2204_08147_amd")

from oracle import lanczos as olz  # noqa: E402
from paper_2204_08147_amd import _lib  # noqa: E402
from workloads import cfg_small_chain, long_range_xx_zz, random_dense_terms  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("rho", "h_star", "log_z", "entropy")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_noalloc_equals_solve_ws_twice(prec, tol):
    big = long_range_xx_zz(2, 12, 1.0, 401, betas=(0.5, 2.0), n_v=4, k=40)   # two-pass in 64 MiB
    small = random_dense_terms(2, 6, 402, betas=(0.3, 1.0, 3.0), n_v=3, k=30)
    cap = _lib.NOALLOC_MAX_BYTES
    for inst in (big, small):
        h = rdm.Hamiltonian.from_instance(inst)
        # the ordinary entry point with the same plan (and it builds the tables)
        want = rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision=prec, hbm_budget=cap)
        got = rdm.solve_noalloc(h, inst.betas, inst.n_v, inst.k, inst.seed, precision=prec)
        assert got["two_pass"] == want["two_pass"]
        for key in KEYS:
            assert np.array_equal(got[key], want[key]), (inst.name, key)
        ref = olz.solve(inst)["results"]
        for b, r in enumerate(ref):
            assert _rel(got["rho"][b], r["rho"]) < tol
            assert abs(got["log_z"][b] - r["log_z"]) < tol * max(1.0, abs(r["log_z"]))
    assert rdm.solve_noalloc(h, small.betas, small.n_v, small.k, small.seed, precision=prec)["two_pass"] is False


def test_noalloc_refuses_what_does_not_fit_or_is_not_resident():
    # tables not built yet on this device in this precision: refused
    fresh = random_dense_terms(1, 7, 404, n_v=2, k=10)
    hf = rdm.Hamiltonian.from_instance(fresh)
    with pytest.raises(rdm.RdmError) as e:
        rdm.solve_noalloc(hf, fresh.betas, fresh.n_v, fresh.k, fresh.seed, precision="mixed")
    assert e.value.status == -1
    # 2^20 rows x 64 columns: beyond the array even with two passes
    inst = long_range_xx_zz(2, 18, 1.0, 403, betas=(1.0,), n_v=16, k=60)
    h = rdm.Hamiltonian.from_instance(inst)
    rdm.solve(h, inst.betas, 1, 2, 1, precision="mixed")
    with pytest.raises(rdm.RdmError) as e:
        rdm.solve_noalloc(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed")
    assert e.value.status == -2
    # the array still serves the next call
    small = cfg_small_chain()
    hs = rdm.Hamiltonian.from_instance(small)
    w = rdm.solve(hs, small.betas, small.n_v, small.k, small.seed, precision="fp64",
                  hbm_budget=_lib.NOALLOC_MAX_BYTES)
    r = rdm.solve_noalloc(hs, small.betas, small.n_v, small.k, small.seed, precision="fp64")
    for key in KEYS:
        assert np.array_equal(r[key], w[key])
