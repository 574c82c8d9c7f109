"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, validates arguments, compiles the Hamiltonian tables, and its
host routine for the tridiagonal step matches the oracle.  No GPU work."""
import os
import re

import numpy as np
import pytest

from oracle import lanczos as olz
from workloads import (long_range_xxz, cfg_long_range, cfg_small_chain, nn_xxz_chain, random_dense_terms,
                       random_sparse_xxz, tfim_request)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
rdm = pytest.importorskip("paper_2204_08147_amd")


def _declared():
    src = open(os.path.join(ROOT, "include", "rdm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rdm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(rdm.LIB, n), n
    # and the binding declares a signature for each of them
    from paper_2204_08147_amd import _lib
    assert sorted(s[0] for s in _lib.SIGNATURES) == names


def test_hamiltonian_tables():
    inst = cfg_long_range(0, n_b=8)
    h = rdm.Hamiltonian.from_instance(inst)
    info = h.info()
    n = inst.n
    # XX with J^y = 0 gives a state-independent hop per pair, plus one x-field hop per site
    assert info["hops_uniform"] == n * (n - 1) // 2 + n
    assert info["hops_parity"] == 0
    assert info["diag_terms"] == n * (n - 1) // 2
    nb = inst.n_b
    assert info["bath_hops_uniform"] == nb * (nb - 1) // 2 + nb
    # partner tiles (flip bits above a 256-row tile): the own tile and one per
    # single high bit (8 pair hops + 1 field each) are staged in LDS; a pair of
    # high bits is used by a single hop, which is gathered directly
    hi = n - 8
    assert info["tile_groups"] == 1 + hi
    assert info["direct_hops"] == hi * (hi - 1) // 2
    full = rdm.Hamiltonian.from_instance(cfg_long_range(0)).info()
    assert full["tile_groups"] == 13 and full["direct_hops"] == 66
    # XXZ with J^x = J^y: parity-dependent hops
    h2 = rdm.Hamiltonian.from_instance(cfg_small_chain())
    i2 = h2.info()
    assert i2["hops_parity"] == 9 and i2["hops_uniform"] == 0 and i2["diag_terms"] == 9 + 10


def test_transform_apply_selection():
    # operators on 16..28 bits are applied as D_Z + W D_X W (+ T W D_Y W T);
    # smaller ones keep the hop tables
    full = rdm.Hamiltonian.from_instance(cfg_long_range(0)).info()      # 2 + 18
    assert full["transform"] == 1 and full["bath_transform"] == 1
    small = rdm.Hamiltonian.from_instance(cfg_long_range(0, n_b=8)).info()  # 2 + 8
    assert small["transform"] == 0 and small["bath_transform"] == 0
    mid = rdm.Hamiltonian.from_instance(cfg_long_range(0, n_b=15)).info()   # 2 + 15: bath 15 bits
    assert mid["transform"] == 1 and mid["bath_transform"] == 0
    big = rdm.Hamiltonian.from_instance(cfg_long_range(0, n_b=20)).info()   # 22 bits
    assert big["transform"] == 1 and big["bath_transform"] == 1
    # above 22 bits the strided passes split the high bits in two groups
    over = rdm.Hamiltonian.from_instance(cfg_long_range(0, n_b=21)).info()  # 23 bits, bath 21
    assert over["transform"] == 1 and over["bath_transform"] == 1
    over = rdm.Hamiltonian.from_instance(cfg_long_range(0, n_b=23)).info()  # 25 bits, bath 23
    assert over["transform"] == 1 and over["bath_transform"] == 1
    big = rdm.Hamiltonian.from_instance(cfg_long_range(2, n_b=26)).info()   # 28 bits
    assert big["transform"] == 1
    # YY couplings (J^x = J^y): the transform with a YY part when the hop
    # tables would gather many partner rows (all pairs), hop tables for a
    # sparse chain; either kind on request
    xxz = rdm.Hamiltonian.from_instance(long_range_xxz(2, 16, 1)).info()
    assert xxz["transform"] == 1 and xxz["transform_yy"] == 1   # its 16-bit bath has fewer partners
    # two XXZ bonds on the last four sites (the low index bits): every hop
    # stays inside a 256-row tile
    few = [(12, 13, 0.5, 0.5, 1.0), (14, 15, 0.7, 0.7, -1.0)]
    sparse = rdm.Hamiltonian(2, 14, few).info()
    assert sparse["transform"] == 0 and sparse["bath_transform"] == 0
    forced = rdm.Hamiltonian(2, 14, few, apply="transform").info()
    assert forced["transform"] == 1 and forced["transform_yy"] == 1
    chain = rdm.Hamiltonian.from_instance(nn_xxz_chain(2, 14, 5)).info()   # 8 partner rows per row
    assert chain["transform"] == 0
    chain = rdm.Hamiltonian.from_instance(nn_xxz_chain(2, 14, 5), apply="transform").info()
    assert chain["transform"] == 1 and chain["transform_yy"] == 1
    hops = rdm.Hamiltonian.from_instance(cfg_long_range(0), apply="hops").info()
    assert hops["transform"] == 0 and hops["bath_transform"] == 0
    xonly = rdm.Hamiltonian.from_instance(cfg_long_range(0)).info()
    assert xonly["transform_yy"] == 0
    out = rdm.C.c_void_p()
    assert rdm.LIB.rdm_hamiltonian_create_ex(1, 3, None, 0, None, None, 7, rdm.C.byref(out)) == -1
    assert rdm.LIB.rdm_hamiltonian_create_ex(1, 3, None, 0, None, None, 4, rdm.C.byref(out)) == -1


def test_bitset_tile_selection():
    # hop-table operators on 12 sites and more: the Lanczos steps take tiles of
    # 4096 rows over 12 chosen row bits when those read fewer partner tiles
    # per tile than the 256-row tiles read partner rows per row
    sparse = random_sparse_xxz(3001, n_range=(22, 22), n_v=1, k=30)    # degree 4, 22 sites
    i = rdm.Hamiltonian.from_instance(sparse).info()
    assert i["transform"] == 0 and i["bitset_tiles"] == 1 and i["bath_bitset_tiles"] == 1
    assert 0 < i["bitset_partners"] < (i["tile_groups"] - 1 + i["direct_hops"]) / 2
    rows = rdm.Hamiltonian.from_instance(sparse, apply="hops_rows").info()
    assert rows["transform"] == 0 and rows["bitset_tiles"] == 0 and rows["bath_bitset_tiles"] == 0
    assert rows["tile_groups"] == i["tile_groups"] and rows["direct_hops"] == i["direct_hops"]
    # a transverse-field chain: one partner tile per site outside the tile bits
    tfim = rdm.Hamiltonian.from_instance(tfim_request(3, n_range=(24, 24))).info()
    assert tfim["bitset_tiles"] == 1 and tfim["bitset_partners"] == 24 - 12
    # exactly 12 sites: one tile holds the whole vector
    twelve = rdm.Hamiltonian.from_instance(random_sparse_xxz(3011, n_range=(12, 12))).info()
    assert twelve["n"] == 12 and twelve["bitset_tiles"] == 1 and twelve["bitset_partners"] == 0
    # under 12 sites, and for operators on the transform apply: no bit-set tiles
    small = rdm.Hamiltonian.from_instance(cfg_small_chain()).info()
    assert small["bitset_tiles"] == 0 and small["bitset_partners"] == 0
    xz = rdm.Hamiltonian.from_instance(cfg_long_range(0)).info()
    assert xz["transform"] == 1 and xz["bitset_tiles"] == 0 and xz["bath_bitset_tiles"] == 0


def _tile_bit_rule(flips, nbits, tile_bits=12, low_bits=4):
    # the documented choice: the low bits, then greedily the bit leaving the
    # fewest distinct partner offsets f & ~B (lowest bit on ties); returns the
    # partner tiles one tile reads (offsets used by two or more hops are one
    # staged tile each, the others one gathered hop each)
    B = (1 << low_bits) - 1
    while bin(B).count("1") < tile_bits:
        best = None
        for b in range(low_bits, nbits):
            if B >> b & 1:
                continue
            n = len({f & ~(B | 1 << b) for f in flips} - {0})
            if best is None or n < best[0]:
                best = (n, b)
        B |= 1 << best[1]
    uses = {}
    for f in flips:
        if f & ~B:
            uses[f & ~B] = uses.get(f & ~B, 0) + 1
    return sum(1 if u >= 2 else u for u in uses.values())


@pytest.mark.parametrize("make", [lambda: random_sparse_xxz(3001, n_range=(22, 22)),
                                  lambda: random_sparse_xxz(3021, n_range=(16, 16)),
                                  lambda: nn_xxz_chain(2, 13, 96),
                                  lambda: random_dense_terms(2, 13, 97, density=0.3),
                                  lambda: tfim_request(17, n_range=(23, 23))])
def test_bitset_partner_count_follows_the_tile_bit_rule(make):
    inst = make()
    n = inst.n
    flips = [(1 << (n - 1 - i)) | (1 << (n - 1 - j)) for (i, j, jx, jy, jz) in inst.couplings if jx or jy]
    flips += [1 << (n - 1 - s) for s in range(n) if inst.hx[s] != 0.0]
    i = rdm.Hamiltonian.from_instance(inst, apply="hops").info()
    assert i["bitset_partners"] == _tile_bit_rule(flips, n)


@pytest.mark.parametrize("bad", [
    dict(n_s=0, n_b=4, couplings=[]),
    dict(n_s=5, n_b=4, couplings=[]),
    dict(n_s=2, n_b=27, couplings=[]),
    dict(n_s=1, n_b=3, couplings=[(0, 0, 1.0, 0, 0)]),
    dict(n_s=1, n_b=3, couplings=[(0, 4, 1.0, 0, 0)]),
    dict(n_s=1, n_b=3, couplings=[(0, 1, float("nan"), 0, 0)]),
    dict(n_s=1, n_b=3, couplings=[], hx=np.array([0, 0, float("inf"), 0])),
])
def test_create_rejects_invalid(bad):
    with pytest.raises(rdm.RdmError) as e:
        rdm.Hamiltonian(**bad)
    assert e.value.status == -1
    assert "rdm_hamiltonian_create" in str(e.value)


def test_tridiag_fa_matches_oracle():
    rng = np.random.default_rng(3)
    for kk in (1, 2, 7, 40, 90):
        a = rng.normal(size=kk) * 3
        b = np.abs(rng.normal(size=kk - 1)) + 0.1
        bt = np.array([0.3, 1.0, 4.0])
        e0 = olz.min_ritz(a, b) - 0.5
        theta, y, quad = rdm.tridiag_fa(a, b, bt, e0)
        assert np.allclose(np.sort(theta), np.linalg.eigvalsh(olz.tridiag(a, b)), atol=1e-12, rtol=0)
        for i, beta in enumerate(bt):
            assert np.allclose(y[i], olz.fa_weights(a, b, beta, e0), atol=1e-13, rtol=1e-12)
            assert abs(quad[i] - olz.quad_weight(a, b, beta, e0)) < 1e-13 * max(1, quad[i])


def test_tridiag_fa_clustered_and_degenerate():
    # Lanczos matrices after loss of orthogonality have near-duplicate Ritz values
    a = np.array([1.0, 1.0, 1.0, 2.0, 1.0, 1.0])
    b = np.array([1e-9, 0.5, 1e-14, 0.3, 0.0])
    theta, y, quad = rdm.tridiag_fa(a, b, [1.0], 0.0)
    assert np.allclose(np.sort(theta), np.linalg.eigvalsh(olz.tridiag(a, b)), atol=1e-13)
    assert np.allclose(y[0], olz.fa_weights(a, b, 1.0, 0.0), atol=1e-13)


def test_solve_rejects_bad_arguments_without_touching_device():
    h = rdm.Hamiltonian.from_instance(random_dense_terms(1, 3, 1))
    for betas, n_v, k in (([0.0], 2, 5), ([float("nan")], 2, 5), ([1.0], 0, 5), ([1.0], 2, 0)):
        with pytest.raises(rdm.RdmError) as e:
            rdm.solve(h, betas, n_v, k, 1, library_alloc=True)
        assert e.value.status == -1


def test_block_quadrature_matches_oracle():
    # E_1^T exp(-beta (T - e0)) E_1 of the block variant (eqn:fT), host routine,
    # on random symmetric matrices and on a projected operator from O4
    from oracle import block, spin
    rng = np.random.default_rng(0)
    cases = []
    for n, b in [(1, 1), (4, 4), (12, 2), (40, 4), (96, 8)]:
        a = rng.normal(size=(n, n))
        cases.append(((a + a.T) / 2, b))
    inst = cfg_small_chain()
    op = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    v = np.zeros((inst.dim, inst.d_s))
    for m in range(inst.d_s):
        v[m * inst.d_b:(m + 1) * inst.d_b, m] = 1.0 / np.sqrt(inst.d_b)
    cases.append((block.krylov_projection(op.apply, v, 12), inst.d_s))
    for t, b in cases:
        e0 = float(np.linalg.eigvalsh(t)[0])
        f, mn = rdm.block_quadrature(t, b, [0.3, 1.7], e0)
        assert abs(mn - e0) < 1e-12 * max(1.0, abs(e0))
        for q, bt in enumerate([0.3, 1.7]):
            want = block.block_quadrature(t, b, bt, e0)
            assert np.abs(f[q] - want).max() < 1e-12 * np.abs(want).max(), (t.shape, b, bt)


def test_four_system_spins_take_the_per_column_path():
    # d_s = 16: the per-column solve (its Gram in three column blocks); the
    # block variant and the ground-state path keep d_s <= 8
    inst = random_dense_terms(4, 6, 93, n_v=2, k=30)
    h = rdm.Hamiltonian.from_instance(inst)
    with pytest.raises(rdm.RdmError) as e:
        rdm.workspace_size(h, 1, 2, 30, precision="fp64", method="block", hbm_budget=1 << 40)
    assert e.value.status == -1
    auto = rdm.workspace_size(h, 1, 2, 30, precision="fp64", method="auto", hbm_budget=1 << 40)
    assert auto == rdm.workspace_size(h, 1, 2, 30, precision="fp64", mode="stored", hbm_budget=1 << 40)


def test_block_method_validation():
    h = rdm.Hamiltonian.from_instance(cfg_small_chain())
    with pytest.raises(rdm.RdmError) as e:
        rdm.workspace_size(h, 1, 4, 30, precision="fp64", method=3, hbm_budget=1 << 40)
    assert e.value.status == -1
    # profile: 0 off, 1 event-timed kernels, 2 timed graph replays
    with pytest.raises(rdm.RdmError) as e:
        rdm.workspace_size(h, 1, 4, 30, precision="fp64", profile=3, hbm_budget=1 << 40)
    assert e.value.status == -1
    assert rdm.make_options(profile="replay").profile == 2 and rdm.make_options(profile=True).profile == 1
    # the block method plans a few vector blocks, no Lanczos basis (an explicit
    # budget keeps the planner off the device)
    wb = rdm.workspace_size(h, 1, 4, 30, precision="fp64", method="block", hbm_budget=1 << 40)
    wc = rdm.workspace_size(h, 1, 4, 30, precision="fp64", mode="stored", hbm_budget=1 << 40)
    assert 0 < wb < wc


def test_system_hamiltonian_matches_oracle_split():
    # H_s of the split H_t = H_s (x) I + I (x) H_b + H_sb (Section "Spin systems")
    from oracle import spin
    for args in [(1, 4, 11), (2, 5, 12), (3, 4, 13)]:
        inst = random_dense_terms(*args)
        h = rdm.Hamiltonian.from_instance(inst)
        hs, _, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
        assert np.abs(h.system_matrix() - hs).max() < 1e-14



def test_new_entry_points_validate_before_touching_the_device():
    # argument checks come first, so these run without a GPU
    h = rdm.Hamiltonian.from_instance(cfg_small_chain())
    for kw in (dict(n_v=0, k=10), dict(n_v=4, k=0), dict(n_v=5000, k=10)):
        with pytest.raises(rdm.RdmError) as e:
            rdm.product_trace(h, [1.0], kw["n_v"], kw["k"], 1)
        assert e.value.status == -1, kw
    with pytest.raises(rdm.RdmError) as e:
        rdm.product_trace(h, [-1.0], 2, 10, 1)
    assert e.value.status == -1
    with pytest.raises(rdm.RdmError) as e:
        rdm.product_trace(h, [float("nan")], 2, 10, 1)
    assert e.value.status == -1
    with pytest.raises(rdm.RdmError) as e:
        rdm.high_temperature_term(h, 0, 1)
    assert e.value.status == -1
    import ctypes as C
    g = C.c_double(0.0)
    assert rdm.LIB.rdm_stream_probe(7, 1 << 20, 1, None, C.byref(g)) == -1     # pattern
    assert rdm.LIB.rdm_stream_probe(1, 1000, 1, None, C.byref(g)) == -1        # not a multiple of 4096
    assert rdm.LIB.rdm_stream_probe(1, 1 << 20, 0, None, C.byref(g)) == -1     # reps
    assert rdm.LIB.rdm_stream_probe(1, 1 << 20, 1, None, None) == -1           # output
    # start block: which = 2 (product vectors) accepted, 3 rejected
    assert rdm.LIB.rdm_start_block(h.handle, 3, 0, 1, 1, C.c_void_p(1), None) == -1


def test_auto_method_picks_block_when_the_basis_does_not_fit():
    # per-column with a stored basis when it fits the budget, the block
    # variant otherwise (explicit budgets keep the planner off the device)
    h = rdm.Hamiltonian.from_instance(cfg_small_chain())
    stored = rdm.workspace_size(h, 1, 4, 30, precision="fp64", mode="stored", hbm_budget=1 << 40)
    block = rdm.workspace_size(h, 1, 4, 30, precision="fp64", method="block", hbm_budget=1 << 40)
    assert rdm.workspace_size(h, 1, 4, 30, precision="fp64", method="auto", hbm_budget=1 << 40) == stored
    assert block < stored
    assert rdm.workspace_size(h, 1, 4, 30, precision="fp64", method="auto",
                              hbm_budget=(block + stored) // 2) == block
    # a forced mode keeps the per-column path
    two = rdm.workspace_size(h, 1, 4, 30, precision="fp64", mode="two_pass", hbm_budget=1 << 40)
    assert rdm.workspace_size(h, 1, 4, 30, precision="fp64", method="auto", mode="two_pass",
                              hbm_budget=1 << 40) == two


def test_energy_deviation_host_routine():
    # tr(H* rho*) - tr(H_s rho_s) from given rho*, H* (Section "Deviation in
    # internal energy"): against the same formula written with eigh here, on
    # random density matrices; zero when H* = H_s and rho* = rho_s
    from oracle import spin
    inst = random_dense_terms(3, 4, 27)
    h = rdm.Hamiltonian.from_instance(inst)
    hs, _, _ = spin.split_dense(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz)
    rng = np.random.default_rng(4)
    betas = np.array([0.3, 1.0, 5.0])
    rho, hst = [], []
    for _ in betas:
        a = rng.normal(size=(8, 8))
        r = a @ a.T
        rho.append(r / np.trace(r))
        b = rng.normal(size=(8, 8))
        hst.append(b + b.T)
    rho, hst = np.array(rho), np.array(hst)
    got = h.energy_deviation(betas, rho, hst)
    w, v = np.linalg.eigh(hs)
    for t, beta in enumerate(betas):
        p = np.exp(-beta * (w - w.min()))
        rho_s = (v * (p / p.sum())) @ v.T
        want = np.trace(hst[t] @ rho[t]) - np.trace(hs @ rho_s)
        assert abs(got[t] - want) < 1e-12 * max(1.0, abs(want))
        assert abs(h.energy_deviation([beta], rho_s[None], hs[None])[0]) < 1e-12
    with pytest.raises(rdm.RdmError):
        h.energy_deviation([0.0], rho[:1], hst[:1])
