"""MI355X (gfx950) solver for the equilibrium reduced density matrix of a
strongly coupled spin system by partial-trace typicality (Chen & Cheng,
arXiv:2204.08147).

This module is a thin binding over the C ABI of ``librdm.so`` (declared in
``include/rdm.h``): it only marshals arguments.  Every step of the hot path
(Hamiltonian apply, Lanczos recurrences, recombination, Gram) runs in the
library's HIP kernels; PyTorch only provides device memory (workspaces) and
streams.  Importing fails when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (DIAG_FIXED, RDM_AUTO, RDM_FP64, RDM_MIXED, RDM_STORED_Q, RDM_TWO_PASS,
                   STATUS_NAMES)

LIB = _lib.load()

PRECISIONS = {"fp64": RDM_FP64, "mixed": RDM_MIXED}
MODES = {"auto": RDM_AUTO, "stored": RDM_STORED_Q, "two_pass": RDM_TWO_PASS}


class RdmError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = LIB.rdm_last_error()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: "
                         f"{msg.decode() if msg else ''}")
        self.status = status


def _check(status: int, where: str):
    if status != 0:
        raise RdmError(status, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


METHODS = {"per_column": 0, "block": 1, "auto": 2}


def make_options(precision="fp64", mode="auto", hbm_budget=0, slab=0, rows_per_lane=0, tau=0.0,
                 profile=False, eager=False, method="per_column") -> _lib.Options:
    o = _lib.Options()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.hbm_budget = int(hbm_budget)
    o.slab = int(slab)
    o.rows_per_lane = int(rows_per_lane)
    o.tau = float(tau)
    # profile: False, True (event-timed kernels, launched one by one) or
    # "replay" (the graph replay kept and each replayed phase timed)
    o.profile = 2 if profile == "replay" else int(profile)
    o.eager = 1 if eager else 0
    o.method = METHODS[method] if isinstance(method, str) else int(method)
    return o


APPLY_KINDS = {"auto": 0, "hops": 1, "transform": 2, "hops_rows": 3}


class Hamiltonian:
    """H_t of eqn:Ht (and its bath part) on n_s system + n_b bath spins.

    couplings: iterable of (i, j, jx, jy, jz); hx, hz: coefficients of the
    one-site Pauli terms (length n_s + n_b).  apply: how products with H are
    computed -- "auto", "hops" (hop-table gathers; 4096-row tiles of chosen
    row bits where those read fewer partner tiles),
    "hops_rows" (hop tables with 256-row tiles only) or "transform" (the
    Walsh-Hadamard form on 16..28 sites)."""

    def __init__(self, n_s: int, n_b: int, couplings: Iterable, hx=None, hz=None, apply: str = "auto"):
        cps = list(couplings)
        arr = (_lib.Coupling * max(len(cps), 1))()
        for t, (i, j, jx, jy, jz) in enumerate(cps):
            arr[t] = _lib.Coupling(int(i), int(j), float(jx), float(jy), float(jz))
        n = n_s + n_b
        self._hx = None if hx is None else np.ascontiguousarray(hx, dtype=np.float64)
        self._hz = None if hz is None else np.ascontiguousarray(hz, dtype=np.float64)
        for f in (self._hx, self._hz):
            if f is not None and f.shape != (n,):
                raise ValueError("fields must have length n_s + n_b")
        out = C.c_void_p()
        _check(LIB.rdm_hamiltonian_create_ex(n_s, n_b, arr, len(cps),
                                             None if self._hx is None else _dptr(self._hx),
                                             None if self._hz is None else _dptr(self._hz),
                                             APPLY_KINDS[apply], C.byref(out)), "rdm_hamiltonian_create_ex")
        self.handle = out.value
        self.n_s, self.n_b, self.n = n_s, n_b, n

    @classmethod
    def from_instance(cls, inst, apply: str = "auto") -> "Hamiltonian":
        return cls(inst.n_s, inst.n_b, inst.couplings, inst.hx, inst.hz, apply=apply)

    def info(self) -> dict:
        out = (C.c_int64 * 21)()
        _check(LIB.rdm_hamiltonian_info(self.handle, out), "rdm_hamiltonian_info")
        keys = ["n", "n_s", "n_b", "hops_uniform", "hops_parity", "diag_terms",
                "bath_hops_uniform", "bath_hops_parity", "bath_diag_terms", "tile_groups",
                "bath_tile_groups", "direct_hops", "bath_direct_hops", "transform", "bath_transform",
                "transform_yy", "bath_transform_yy", "bitset_tiles", "bath_bitset_tiles",
                "bitset_partners", "bath_bitset_partners"]
        return dict(zip(keys, list(out)))

    def system_matrix(self) -> np.ndarray:
        """H_s (d_s x d_s): the couplings and fields of the system sites."""
        d = 1 << self.n_s
        out = np.zeros((d, d))
        _check(LIB.rdm_system_hamiltonian(self.handle, _dptr(out)), "rdm_system_hamiltonian")
        return out

    def energy_deviation(self, betas, rho, h_star) -> np.ndarray:
        """tr(H* rho*) - tr(H_s rho_s) per temperature from a solve's rho* and
        H* (Section "Deviation in internal energy"), computed by the library."""
        bt = np.ascontiguousarray(np.atleast_1d(betas), dtype=np.float64)
        r = np.ascontiguousarray(rho, dtype=np.float64)
        hh = np.ascontiguousarray(h_star, dtype=np.float64)
        out = np.zeros(len(bt))
        _check(LIB.rdm_energy_deviation(self.handle, len(bt), _dptr(bt), _dptr(r), _dptr(hh), _dptr(out)),
               "rdm_energy_deviation")
        return out

    def close(self):
        if getattr(self, "handle", None):
            LIB.rdm_hamiltonian_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _ResultBuffers:
    def __init__(self, n_beta: int, d_s: int):
        self.rho = np.zeros((n_beta, d_s, d_s))
        self.h_star = np.zeros((n_beta, d_s, d_s))
        self.log_z = np.zeros(n_beta)
        self.entropy = np.zeros(n_beta)
        self.diag = np.zeros(DIAG_FIXED + 2 * n_beta)
        self.c = _lib.Result(_dptr(self.rho), _dptr(self.h_star), _dptr(self.log_z),
                             _dptr(self.entropy), _dptr(self.diag))

    def as_dict(self) -> dict:
        d = self.diag
        nb = len(self.log_z)
        return {"rho": self.rho, "h_star": self.h_star, "log_z": self.log_z,
                "entropy": self.entropy, "e0": d[0], "e0b": d[1],
                "breakdown_total": int(d[2]), "breakdown_bath": int(d[3]),
                "two_pass": bool(d[4]), "device_bytes": int(d[5]), "mu_ratio": d[6],
                "t_apply_ms": d[7], "t_norm_ms": d[8], "t_gram_ms": d[9], "t_xz1_ms": d[10],
                "t_replay_step_ms": d[11], "replay_steps": int(d[12]),
                "log_z_t": d[DIAG_FIXED::2][:nb].copy(), "log_z_b": d[DIAG_FIXED + 1::2][:nb].copy()}


def workspace_size(h: Hamiltonian, n_beta: int, n_v: int, k: int, **opts) -> int:
    o = make_options(**opts)
    out = C.c_uint64()
    _check(LIB.rdm_workspace_size(h.handle, n_beta, n_v, k, C.byref(o), C.byref(out)),
           "rdm_workspace_size")
    return out.value


def solve(h: Hamiltonian, betas: Sequence[float], n_v: int, k: int, seed: int, *, stream=None,
          workspace=None, library_alloc: bool = False, **opts) -> dict:
    """Full solve.  By default the device workspace is a torch tensor on the
    current device (torch owns the memory) and the work runs on torch's current
    stream; ``library_alloc=True`` lets the library allocate instead."""
    import torch
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    o = make_options(**opts)
    res = _ResultBuffers(len(betas), 1 << h.n_s)
    st = _stream_handle(stream)
    if library_alloc:
        _check(LIB.rdm_solve(h.handle, _dptr(betas), len(betas), n_v, k, seed, C.byref(o), st,
                             C.byref(res.c)), "rdm_solve")
    else:
        if workspace is None:
            wopts = dict(opts)
            if not wopts.get("hbm_budget"):
                # torch allocates the workspace and may reuse its cached
                # blocks: the budget is the free memory plus that cache, less
                # the library's 2 GiB reserve
                free, _ = torch.cuda.mem_get_info()
                cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
                wopts["hbm_budget"] = max(1, free + cached - (2 << 30))
            nbytes = workspace_size(h, len(betas), n_v, k, **wopts)
            workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(LIB.rdm_solve_ws(h.handle, _dptr(betas), len(betas), n_v, k, seed, C.byref(o), st,
                                C.byref(res.c), C.c_void_p(workspace.data_ptr()),
                                workspace.numel() * workspace.element_size()), "rdm_solve_ws")
    return res.as_dict()


def solve_noalloc(h: Hamiltonian, betas: Sequence[float], n_v: int, k: int, seed: int, *, stream=None,
                  **opts) -> dict:
    """As ``solve`` (per-column method), with the device workspace in the
    library's fixed scratch array (``_lib.NOALLOC_MAX_BYTES`` per device): the
    call allocates no device memory.  The Hamiltonian's device tables must be
    resident already (any earlier solve with it in this precision)."""
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    o = make_options(**opts)
    res = _ResultBuffers(len(betas), 1 << h.n_s)
    _check(LIB.rdm_solve_noalloc(h.handle, _dptr(betas), len(betas), n_v, k, seed, C.byref(o),
                                 _stream_handle(stream), C.byref(res.c)), "rdm_solve_noalloc")
    return res.as_dict()


def solve_batch(items: List[dict], *, stream=None, library_alloc: bool = False,
                reserve_bytes: int = 8 << 30, workspace=None, **opts) -> List[dict]:
    """items: dicts with keys h, betas, n_v, k, seed.  Returns per-item result
    dicts (each with a 'status' entry).  By default the workspace is a torch
    tensor sized to run every instance in one wave when device memory allows
    (less memory means more waves, never an error); ``workspace`` passes a
    caller-owned uint8 device tensor instead.  A failure of one item is
    reported in its 'status'; a failure of the call itself raises."""
    o = make_options(**opts)
    n = len(items)
    arr = (_lib.BatchItem * max(n, 1))()
    keep = []
    for t, it in enumerate(items):
        b = np.ascontiguousarray(it["betas"], dtype=np.float64)
        rb = _ResultBuffers(len(b), 1 << it["h"].n_s)
        keep.append((b, rb))
        arr[t].h = it["h"].handle
        arr[t].beta = _dptr(b)
        arr[t].n_beta = len(b)
        arr[t].n_v = it["n_v"]
        arr[t].k = it["k"]
        arr[t].seed = it["seed"]
        arr[t].out = rb.c
    st = _stream_handle(stream)

    def _batch_check(status: int, where: str):
        # the call returns the first failing item's status; any other
        # failure belongs to the call, not to an item
        if status != 0 and not any(int(arr[t].status) == status for t in range(n)):
            raise RdmError(status, where)

    if library_alloc:
        _batch_check(LIB.rdm_solve_batch(n, arr, C.byref(o), st), "rdm_solve_batch")
    else:
        import torch
        lo, hi = C.c_uint64(), C.c_uint64()
        _check(LIB.rdm_batch_workspace_size(n, arr, C.byref(o), C.byref(lo), C.byref(hi)),
               "rdm_batch_workspace_size")
        if workspace is not None:
            size = workspace.numel() * workspace.element_size()
            _batch_check(LIB.rdm_solve_batch_ws(n, arr, C.byref(o), st, C.c_void_p(workspace.data_ptr()),
                                                size), "rdm_solve_batch_ws")
        elif hi.value:
            free, _ = torch.cuda.mem_get_info()
            cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
            size = int(max(lo.value, min(hi.value, free + cached - reserve_bytes)))
            ws = torch.empty(size, dtype=torch.uint8, device="cuda")
            _batch_check(LIB.rdm_solve_batch_ws(n, arr, C.byref(o), st, C.c_void_p(ws.data_ptr()), size),
                         "rdm_solve_batch_ws")
            del ws
        else:
            _batch_check(LIB.rdm_solve_batch(n, arr, C.byref(o), st), "rdm_solve_batch")
    out = []
    for t in range(n):
        d = keep[t][1].as_dict()
        d["status"] = int(arr[t].status)
        out.append(d)
    return out


def apply(h: Hamiltonian, x, y, *, which: int = 0, precision="fp64", n_cols: int, stream=None,
          **opts):
    """Y = H X on device tensors in the library's panel layout (blocking)."""
    o = make_options(precision=precision, **opts)
    _check(LIB.rdm_apply(h.handle, which, o.precision, n_cols, C.c_void_p(x.data_ptr()),
                         C.c_void_p(y.data_ptr()), C.byref(o), _stream_handle(stream)), "rdm_apply")


def start_block(h: Hamiltonian, out, *, which: int, precision="fp64", n_v: int, seed: int,
                stream=None):
    p = PRECISIONS[precision] if isinstance(precision, str) else precision
    _check(LIB.rdm_start_block(h.handle, which, p, n_v, seed, C.c_void_p(out.data_ptr()),
                               _stream_handle(stream)), "rdm_start_block")


def lanczos(h: Hamiltonian, *, which: int, n_v: int, k: int, seed: int, stream=None, **opts):
    """Lanczos coefficients of every start column: (alpha[k, C], beta[k, C], kc[C])."""
    o = make_options(**opts)
    ncols = (1 << h.n_s) * n_v if which == 0 else n_v
    a = np.zeros((k, ncols))
    b = np.zeros((k, ncols))
    kc = np.zeros(ncols, dtype=np.int32)
    _check(LIB.rdm_lanczos(h.handle, which, n_v, k, seed, C.byref(o), _stream_handle(stream),
                           _dptr(a), _dptr(b), kc.ctypes.data_as(C.POINTER(C.c_int32))),
           "rdm_lanczos")
    return a, b, kc


def ground_state(h: Hamiltonian, n_v: int, k: int, seed: int, *, stream=None, **opts) -> dict:
    """Low-temperature limit: rho*(inf) over the ground space, E_t, E_b,
    H*(inf) = (E_t - E_b) I, the T = 0 entropy and the ground-space dimension."""
    o = make_options(**opts)
    d = 1 << h.n_s
    rho = np.zeros((d, d))
    et, eb, ent, resid = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    r = C.c_int32()
    res = _lib.GroundResult(_dptr(rho), C.pointer(et), C.pointer(eb), C.pointer(ent), C.pointer(r),
                            C.pointer(resid))
    _check(LIB.rdm_ground_state(h.handle, n_v, k, seed, C.byref(o), _stream_handle(stream), C.byref(res)),
           "rdm_ground_state")
    return {"rho": rho, "e_total": et.value, "e_bath": eb.value, "entropy": ent.value,
            "degeneracy": int(r.value), "h_star": (et.value - eb.value) * np.eye(d),
            "residual": resid.value}


def product_trace(h: Hamiltonian, betas, n_v: int, k: int, seed: int, *, stream=None, **opts) -> dict:
    """Product-state estimator: ln Z*, ln Z_t, ln Z_b per beta and the
    per-sample ln Z_t estimates ([n_beta, n_v]) from n_v columns
    |v_s^(j)> (x) |v_j>."""
    o = make_options(**opts)
    bt = np.ascontiguousarray(np.atleast_1d(betas), dtype=np.float64)
    nb = len(bt)
    lz, lzt, lzb = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    smp = np.zeros((nb, n_v))
    res = _lib.ProductResult(_dptr(lz), _dptr(lzt), _dptr(lzb), _dptr(smp))
    _check(LIB.rdm_product_trace(h.handle, _dptr(bt), nb, n_v, k, seed, C.byref(o), _stream_handle(stream),
                                 C.byref(res)), "rdm_product_trace")
    return {"log_z": lz, "log_z_t": lzt, "log_z_b": lzb, "samples": smp}


STREAM_PATTERNS = {"read": 0, "copy": 1, "r3w1": 2, "r2w2": 3}


def stream_probe(pattern: str, nbytes: int = 2 << 30, reps: int = 10, *, stream=None) -> float:
    """Device bandwidth (GB/s of bytes moved) of a nontemporal streaming
    kernel: 'read', 'copy', 'r3w1' (three reads, one write) or 'r2w2'."""
    g = C.c_double(0.0)
    _check(LIB.rdm_stream_probe(STREAM_PATTERNS[pattern], nbytes, reps, _stream_handle(stream), C.byref(g)),
           "rdm_stream_probe")
    return g.value


def high_temperature_term(h: Hamiltonian, n_v: int, seed: int, *, stream=None) -> dict:
    """The estimator's high-temperature offset C (d_s x d_s) for the bath
    vectors of a solve with this n_v and seed: the estimated H* tends to
    H_s + C as beta -> 0, the exact one to H_s.  Also returns the averaged
    bath expectations <v|sx_c|v> per bath site and the spectral norm of C."""
    d = 1 << h.n_s
    c = np.zeros((d, d))
    sx = np.zeros(h.n_b)
    _check(LIB.rdm_high_temperature_term(h.handle, n_v, seed, _stream_handle(stream), _dptr(c), _dptr(sx)),
           "rdm_high_temperature_term")
    return {"c": c, "sx": sx, "norm": float(np.abs(np.linalg.eigvalsh(c)).max())}


def block_quadrature(t, b: int, betas, e0: float):
    """Host routine: E_1^T exp(-beta (T - e0)) E_1 (b x b) for a symmetric T and
    each beta, and the smallest eigenvalue of T."""
    tt = np.ascontiguousarray(t, dtype=np.float64)
    bt = np.ascontiguousarray(betas, dtype=np.float64)
    n = tt.shape[0]
    f = np.zeros((len(bt), b, b))
    mn = C.c_double(0.0)
    _check(LIB.rdm_block_quadrature(n, b, _dptr(tt), len(bt), _dptr(bt), float(e0), C.byref(mn), _dptr(f)),
           "rdm_block_quadrature")
    return f, mn.value


def tridiag_fa(alpha, beta, betas, e0: float):
    """Host routine: eigenvalues of T, exp(-b (T - e0)/2) e_1 and the Gauss
    quadrature e_1^T exp(-b (T - e0)) e_1 for each b."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    bt = np.ascontiguousarray(betas, dtype=np.float64)
    kk = len(a)
    theta = np.zeros(kk)
    y = np.zeros((len(bt), kk))
    quad = np.zeros(len(bt))
    _check(LIB.rdm_tridiag_fa(kk, _dptr(a), _dptr(b) if len(b) else None, len(bt), _dptr(bt),
                              float(e0), _dptr(theta), _dptr(y), _dptr(quad)), "rdm_tridiag_fa")
    return theta, y, quad


def panel_width(precision) -> int:
    p = PRECISIONS[precision] if isinstance(precision, str) else precision
    return 2 if p == RDM_FP64 else 4


def to_panels(x, precision):
    """(dim, C) tensor -> the library's panel layout (flat tensor)."""
    import torch
    w = panel_width(precision)
    dim, c = x.shape
    cp = (c + w - 1) // w * w
    if cp != c:
        x = torch.cat([x, x.new_zeros(dim, cp - c)], dim=1)
    return x.reshape(dim, cp // w, w).permute(1, 0, 2).contiguous().reshape(-1)


def from_panels(p, dim: int, n_cols: int, precision):
    w = panel_width(precision)
    cp = (n_cols + w - 1) // w * w
    return p.reshape(cp // w, dim, w).permute(1, 0, 2).reshape(dim, cp)[:, :n_cols]


class Server:
    """Continuous-batching serving engine (a worker thread in the library)."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0, precision="mixed"):
        out = C.c_void_p()
        p = PRECISIONS[precision] if isinstance(precision, str) else precision
        _check(LIB.rdm_server_create(hbm_budget, max_active, p, C.byref(out)), "rdm_server_create")
        self.handle = out.value
        self._pending = {}

    def submit(self, h: Hamiltonian, betas, n_v: int, k: int, seed: int) -> int:
        b = np.ascontiguousarray(betas, dtype=np.float64)
        rb = _ResultBuffers(len(b), 1 << h.n_s)
        t = C.c_uint64()
        _check(LIB.rdm_server_submit(self.handle, h.handle, _dptr(b), len(b), n_v, k, seed, rb.c,
                                     C.byref(t)), "rdm_server_submit")
        self._pending[t.value] = (rb, h, b)
        return t.value

    def poll(self, ticket: int):
        done = C.c_int32()
        st = C.c_int32()
        _check(LIB.rdm_server_poll(self.handle, ticket, C.byref(done), C.byref(st)), "rdm_server_poll")
        if not done.value:
            return None
        return self._finish(ticket, st.value)

    def wait(self, ticket: int) -> dict:
        st = C.c_int32()
        _check(LIB.rdm_server_wait(self.handle, ticket, C.byref(st)), "rdm_server_wait")
        return self._finish(ticket, st.value)

    def cancel(self, ticket: int) -> None:
        """Cancel a request (it completes with status RDM_E_CANCELLED unless
        it had completed already); its result is still retrieved with wait
        or poll."""
        _check(LIB.rdm_server_cancel(self.handle, ticket), "rdm_server_cancel")

    def _finish(self, ticket, status):
        rb, _, _ = self._pending.pop(ticket)
        d = rb.as_dict()
        d["status"] = status
        return d

    def stats(self) -> dict:
        out = (C.c_int64 * 7)()
        _check(LIB.rdm_server_stats(self.handle, out), "rdm_server_stats")
        return dict(zip(["submitted", "completed", "active", "queued", "steps", "peak_active",
                         "peak_bytes"], list(out)))

    def close(self):
        if getattr(self, "handle", None):
            LIB.rdm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
