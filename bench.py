"""Benchmark: reduced-density-matrix solves per second on one MI355X.

Workload (the metric's configuration): 2 system + 18 bath spins (dim 2^20),
long-range XX+ZZ couplings J_ij = |i-j|^-1.5, transverse x-field
h in {0.5, 1.0, 1.5}, beta in {0.5, 1, 2, 4} from one Lanczos run per h,
n_v = 16 Rademacher bath vectors (64 start columns), k = 60 Lanczos steps.
One step = the whole hot path for the three fields (three solves, four
temperatures each), mixed precision (FP32 vectors, FP64 reductions); the FP64
plain path is timed the same way and reported beside it.

Prints one JSON line.  ``value`` = mixed-precision solves per second with the
Hamiltonian tables and workspaces resident on the device.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published vector peaks of MI355X: FP32 157.3 TFLOP/s (256 CUs x 4 SIMD x 16
# lanes x 2 flop x 2.4 GHz x 2 for packed FP32 FMA), FP64 78.6 TFLOP/s.  The
# library is compiled without packed FP32 instructions, so half of the FP32
# figure is what its kernels can issue; the published figure is the peak the
# roofline fraction is taken against.
VALU_PEAK_TFLOPS = {4: 157.3, 8: 78.6}

METRIC = ("ρ_s solves/s & spin-H apply GB/s, mixed vs FP64 plain; p50/p99 solve latency")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-b", type=int, default=18, help="bath spins (18 = the metric's workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-block", action="store_true", help="skip the block-Lanczos comparison")
    ap.add_argument("--no-truncation", action="store_true", help="skip the k against k + 20 check")
    ap.add_argument("--workload", default="lr",
                    choices=["lr", "small", "batch", "large", "serve", "scan", "estimators"],
                    help="lr: the metric's workload (default); small: the 1+9-spin FP64 instance; "
                         "batch: 64 heterogeneous sparse XXZ "
                         "instances in one batched solve; large: 3+23 spins (dim 2^26) two-pass; "
                         "serve: Poisson arrivals of transverse-field requests; scan: the paper's "
                         "entropy / internal-energy scans; estimators: product-state estimate, "
                         "high-temperature offset and low-temperature limit on the 2+18 instance")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests at the offered rate")
    ap.add_argument("--steady-requests", type=int, default=300,
                    help="serve: requests at 0.7x the measured capacity")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (reference kernel for HBM counters)")
    return ap.parse_args()


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of kernels.hip's code: comments,
    blank lines and surrounding white space removed, so that only a change
    of the code itself marks counter summaries as stale."""
    import re
    src = open(os.path.join(ROOT, "paper_2204_08147_amd", "csrc", "kernels.hip")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*$", "", line).strip() for line in src.splitlines()]
    code = "\n".join(line for line in lines if line)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def read_traffic(name):
    """HBM bytes per Lanczos step from the committed rocprofv3 counter
    summary, or None if absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def _oracle_worker(h_index, n_b, column, steps):
    """One host process: the oracle's FP64 Lanczos on one start column of the
    long-range instance; returns the seconds the steps took."""
    from threadpoolctl import threadpool_limits
    from oracle import exact, lanczos as olz, spin
    from workloads import cfg_long_range
    inst = cfg_long_range(h_index, n_b=n_b)
    op = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    x0 = exact.start_columns(inst)[:, column]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        olz.lanczos(op.apply, x0, steps, keep_q=False)
        return time.perf_counter() - t0


def _make_instance(kind, arg):
    from workloads import cfg_large, random_sparse_xxz, tfim_request
    if kind == "batch":
        return random_sparse_xxz(arg)
    if kind == "serve":
        return tfim_request(arg)
    return cfg_large()


def _oracle_step_worker(kind, arg, n_rows):
    """One host process: the oracle's FP64 work on one start column of the
    named instance.  n_rows = 0: one Lanczos step (apply, recurrence, dots);
    returns its seconds.  n_rows > 0 (instances whose full apply takes many
    minutes): the oracle's apply restricted to n_rows random rows; returns
    its seconds scaled to all rows."""
    from threadpoolctl import threadpool_limits
    from oracle import exact, lanczos as olz, spin
    inst = _make_instance(kind, arg)
    op = spin.sparse_hamiltonian(inst.n, inst.couplings, inst.hx, inst.hz)
    with threadpool_limits(limits=1):
        if n_rows == 0:
            x0 = exact.start_columns(inst)[:, 0]
            t0 = time.perf_counter()
            olz.lanczos(op.apply, x0, 1, keep_q=False)
            return time.perf_counter() - t0
        rng = np.random.default_rng(arg)
        x = rng.standard_normal(inst.dim)
        rows = rng.integers(0, inst.dim, n_rows)
        t0 = time.perf_counter()
        op.rows(rows, x)
        return (time.perf_counter() - t0) * inst.dim / n_rows


def _pool_starmap(nproc, fn, args):
    """starmap over a pool of fresh interpreters (the parent holds a GPU
    context), closed and joined so that no worker is killed mid-exit."""
    import multiprocessing as mp
    pool = mp.get_context("spawn").Pool(nproc)
    try:
        out = pool.starmap(fn, args)
        pool.close()
        return out
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()


def cpu_baseline_sample(kind, args_list, n_rows=0):
    """Oracle seconds per column step for each listed instance, one host
    process each (at most 16 at a time, BLAS one thread per process)."""
    nproc = max(1, min(16, os.cpu_count() or 1, len(args_list)))
    return nproc, _pool_starmap(nproc, _oracle_step_worker, [(kind, a, n_rows) for a in args_list])


def _solve_seconds(inst, t_col_step, applies_per_step=1):
    """A whole solve from one column step: every column (bath columns count
    by their size) for k steps."""
    cols = inst.n_cols + inst.n_v * (inst.d_b / inst.dim)
    return inst.k * cols * t_col_step * applies_per_step


def cpu_baseline(inst, h_index, n_b, steps=2):
    """The oracle's FP64 Lanczos path (as it stands), parallel over start
    columns with one process per host core (at most 16), on a bounded sample:
    `steps` Lanczos steps of one column per process.  Throughput = processes x
    steps / slowest process, scaled to a whole solve (every column, k steps,
    plus the bath run)."""
    nproc = max(1, min(16, os.cpu_count() or 1))
    times = _pool_starmap(nproc, _oracle_worker, [(h_index, n_b, c % inst.n_cols, steps) for c in range(nproc)])
    col_steps_per_s = nproc * steps / max(times)
    cols = inst.n_cols + inst.n_v * (inst.d_b / inst.dim)  # bath columns are 1/d_s the size
    t_solve = inst.k * cols / col_steps_per_s
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": nproc, "kind": "oracle",
            "extrapolated": True,
            "sample": f"{steps} FP64 Lanczos steps of one start column in each of {nproc} processes "
                      f"(dim 2^{inst.n}), slowest {max(times):.1f} s, extrapolated to {inst.k} steps x "
                      f"{cols:.2f} columns (a whole solve would take hours on the host; NumPy, BLAS one "
                      f"thread per process)"}


def operator_work(nbits, cols, nnz, transform, s, k):
    """Algorithmic bytes and flops of one Lanczos step (norm step + apply) on
    one operator: 2^nbits rows, cols columns padded to whole 16-byte panels,
    s bytes per scalar, averaged over k steps (p = (k-1)/k: r and u_(j-1)
    are absent at the first step).

    Hop tables: norm reads r and u_(j-1) and writes u_j, apply reads u_j and
    u_(j-1), writes r and reads the diagonal: (3 + 3p) vectors + dim*s;
    2*nnz flops per element.
    Transform (D_Z + W D_X W, basis kept in the low-bit Hadamard basis):
    pass 1 reads R and u~_(j-1), writes u~_j and R and reads D_X; pass 2
    reads u~_j, R, u~_(j-1) and D_Z and writes R: (6 + 2p) vectors + the two
    diagonals (once: every panel reads the same ones); 2*nbits + 8 flops per
    element."""
    dim = 1 << nbits
    w = 16 // s
    cp = (cols + w - 1) // w * w
    vec = dim * cp * s
    p = (k - 1) / k
    if transform:
        return vec * (6 + 2 * p) + 2 * dim * s, (2.0 * nbits + 8) * dim * cp
    return vec * (3 + 3 * p) + dim * s, 2.0 * nnz * dim * cols


def step_work(insts, prec_bytes):
    """Algorithmic bytes and flops of one Lanczos step over the H_t and H_b
    segments of the given instances, as the implementation computes it
    (transform operators: the transform's own streams and flops)."""
    import paper_2204_08147_amd as rdm
    by = fl = 0.0
    for inst in insts:
        info = rdm.Hamiltonian.from_instance(inst).info()
        nnz = 1 + info["hops_uniform"] + 0.5 * info["hops_parity"]
        nnz_b = 1 + info["bath_hops_uniform"] + 0.5 * info["bath_hops_parity"]
        b1, f1 = operator_work(inst.n, inst.n_cols, nnz, info["transform"], prec_bytes, inst.k)
        b2, f2 = operator_work(inst.n_b, inst.n_v, nnz_b, info["bath_transform"], prec_bytes, inst.k)
        by += b1 + b2
        fl += f1 + f2
    return by, fl


def plan_work(insts, prec_bytes):
    """The measurement plan's per-step work, independent of how the product
    is computed: flops = 2 C nnz per row (nnz = diagonal + non-zero hops per
    row) and the minimum bytes of a Lanczos step, three vector passes (read
    q_j and q_(j-1), write q_(j+1)), over the H_t and H_b segments."""
    import paper_2204_08147_amd as rdm
    by = fl = 0.0
    for inst in insts:
        info = rdm.Hamiltonian.from_instance(inst).info()
        nnz = 1 + info["hops_uniform"] + 0.5 * info["hops_parity"]
        nnz_b = 1 + info["bath_hops_uniform"] + 0.5 * info["bath_hops_parity"]
        fl += 2.0 * inst.n_cols * nnz * inst.dim + 2.0 * inst.n_v * nnz_b * inst.d_b
        by += 3.0 * prec_bytes * (inst.n_cols * inst.dim + inst.n_v * inst.d_b)
    return by, fl


def step_ms(res):
    """Mean device time of one Lanczos step's vector kernels (norm step and
    apply, either kind) from the library's event timing."""
    return res["t_norm_ms"] + res["t_xz1_ms"] + res["t_apply_ms"]


def roofline(bytes_, flops, t_s, traffic=None, prec_bytes=4):
    """Roofline object of one kernel (or step): bound by whichever of VALU
    and HBM takes longer at peak for this work."""
    peak_tf = VALU_PEAK_TFLOPS[prec_bytes]
    gbs = bytes_ / t_s / 1e9
    tf = flops / t_s / 1e12
    if flops / (peak_tf * 1e12) >= bytes_ / (HBM_PEAK_GBS * 1e9):
        return {"bound": "alu", "achieved": round(tf, 3), "peak": peak_tf, "unit": "TFLOP/s",
                "frac": round(tf / peak_tf, 4), "traffic": traffic}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}


def result_errors(a, b):
    """Largest differences of a's rho*, H* (relative Frobenius), ln Z* and S
    (absolute) from b's over the temperatures of one solve."""
    nb = len(b["log_z"])
    rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))  # noqa: E731
    return {"rho_rel": max(rel(a["rho"][t], b["rho"][t]) for t in range(nb)),
            "h_star_rel": max(rel(a["h_star"][t], b["h_star"][t]) for t in range(nb)),
            "log_z_abs": max(abs(float(a["log_z"][t] - b["log_z"][t])) for t in range(nb)),
            "entropy_abs": max(abs(float(a["entropy"][t] - b["entropy"][t])) for t in range(nb))}


def bench_batch(args):
    """64 independent random-sparse XXZ instances (N in [12, 22], N_s in
    {1,2,3}, average degree 4, beta log-uniform in [0.1, 10], n_v = 8, k = 50)
    solved together by one batched call, mixed precision."""
    import torch
    import paper_2204_08147_amd as rdm
    from workloads import cfg_batch
    insts = cfg_batch()
    hs = [rdm.Hamiltonian.from_instance(i) for i in insts]
    items = [dict(h=h, betas=i.betas, n_v=i.n_v, k=i.k, seed=i.seed) for h, i in zip(hs, insts)]
    for _ in range(args.warmup):
        rdm.solve_batch(items, precision="mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = rdm.solve_batch(items, precision="mixed")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = rdm.solve_batch(items, precision="mixed", profile=True)  # kernel timing, untimed
    assert all(o["status"] == 0 for o in out), [o["status"] for o in out]
    by, fl = step_work(insts, 4)
    # one launch covers every instance resident in a wave, and each instance
    # reports its wave's mean step time: the instances of one wave share the
    # value, so a step over the whole batch takes the sum over the waves
    wave_ms = sorted({(o["t_norm_ms"], o["t_xz1_ms"], o["t_apply_ms"]) for o in prof})
    t_step = sum(sum(w) for w in wave_ms) * 1e-3
    n = len(insts) * args.steps
    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle on the host (every fourth instance)")
        sample = list(range(0, len(insts), 4))
        cores, secs = cpu_baseline_sample("batch", [insts[i].seed for i in sample])
        t_all = 4 * sum(_solve_seconds(insts[i], t) for i, t in zip(sample, secs))
        cpu = {"value": len(insts) / t_all * cores, "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": f"one FP64 Lanczos step of one start column of every fourth instance "
                         f"({len(sample)} instances, one process each), scaled to k steps x all columns "
                         f"per instance and x4 for the other instances; throughput with one solve per core"}
    return {"metric": "batched solves/s (64 heterogeneous instances)", "value": round(n / wall, 3), "cpu_baseline": cpu,
            "unit": "solves/s", "ms_per_step": round(1e3 * wall / args.steps, 2), "steps": args.steps,
            "warmup": args.warmup, "dtype": "f32 vectors + f64 reductions",
            "config": {"workload": "64 random sparse XXZ instances, N in [12,22], N_s in {1,2,3}, "
                                   "degree 4, beta log-U[0.1,10], n_v=8, k=50",
                       "dims": sorted(int(i.n) for i in insts)},
            "step_kernels_ms_all_waves": round(1e3 * t_step, 4), "waves": len(wave_ms),
            "roofline_step": roofline(*plan_work(insts, 4), t_step),
            "two_pass_instances": int(sum(o["two_pass"] for o in out))}


def bench_large(args):
    """3 system + 23 bath spins (dim 2^26), long-range XXZ alpha = 1.2,
    Delta = 0.8, x-field 1.0, beta = 2, n_v = 4 (32 columns), k = 80,
    two-pass, mixed precision."""
    import torch
    import paper_2204_08147_amd as rdm
    from workloads import cfg_large
    inst = cfg_large()
    h = rdm.Hamiltonian.from_instance(inst)
    # a warm-up solve (device tables, workspace, the slab choice), the timed
    # solve on the default launch path (graph replay), then, untimed, one with
    # HIP-event timing of the kernels (launched one by one)
    stage("large instance: warm-up solve")
    rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed", mode="two_pass")
    torch.cuda.synchronize()
    stage("large instance: timed solve")
    t0 = time.perf_counter()
    rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed", mode="two_pass")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage("large instance: profiled solve")
    res = rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed", mode="two_pass",
                    profile=True)
    by, fl = step_work([inst], 4)
    t_step = step_ms(res) * 1e-3
    # the paper's block variant keeps three blocks instead of the basis, so it
    # needs no regeneration pass: one apply per step instead of two
    block = None
    if not args.no_block:
        stage("large instance: block variant")
        rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed", method="block")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rb = rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed", method="block")
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        block = {"s_per_solve": round(tb, 3),
                 "rho_rel_diff_vs_two_pass": float(np.linalg.norm(rb["rho"][0] - res["rho"][0]) /
                                                   np.linalg.norm(res["rho"][0])),
                 "entropy": float(rb["entropy"][0])}
    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle on the host (row sample of one apply)")
        cores, secs = cpu_baseline_sample("large", list(range(16)), n_rows=1 << 16)
        # two-pass: the regeneration pass applies H again; one column-apply per
        # process, the solve's columns spread over the cores
        t_solve = _solve_seconds(inst, float(np.mean(secs)), applies_per_step=2) / cores
        cpu = {"value": t_solve, "unit": "s/solve", "cores": cores, "kind": "oracle",
               "sample": f"the oracle's apply restricted to 65536 random rows of the 2^26-row operator, "
                         f"{len(secs)} processes, scaled to all rows (extrapolated), then to k steps x "
                         f"2 passes x all columns spread over {cores} cores"}
    return {"metric": "large-instance solve time", "value": round(wall, 3), "unit": "s/solve", "cpu_baseline": cpu,
            "higher_is_better": False, "dtype": "f32 vectors + f64 reductions",
            "config": {"workload": "long-range XXZ 3+23 spins (dim 2^26), alpha=1.2, Delta=0.8, "
                                   "x-field 1.0, beta=2, n_v=4 (32 columns), k=80, two-pass"},
            "step_kernels_ms": round(t_step * 1e3, 3), "apply_kernel_ms": round(res["t_apply_ms"], 3),
            "norm_kernel_ms": round(res["t_norm_ms"], 3),
            "roofline_step": roofline(*plan_work([inst], 4), t_step),
            "roofline_step_implementation": roofline(by, fl, t_step), "two_pass": res["two_pass"],
            "device_bytes": res["device_bytes"],
            "rho": res["rho"][0].round(6).tolist(), "entropy": float(res["entropy"][0]), "block_method": block,
            "h_star_eigs": np.linalg.eigvalsh(res["h_star"][0]).round(6).tolist()}


def bench_serve(args):
    """Serving: requests with N ~ U{14..24}, d_s in {2,4}, ZZ chain J = 1 with
    x-field h ~ U(0,2), beta log-uniform in [0.1,10], n_v = 8, k = 60, mixed
    precision, submitted to the continuous-batching engine.  Three runs:
    closed loop (200 requests submitted at once: saturated capacity), Poisson
    arrivals at the offered rate (args.requests requests; above capacity the
    queue, and so the latency, grows with the run's length), and Poisson
    arrivals at 0.7x the measured capacity (steady state)."""
    import threading
    import torch
    import paper_2204_08147_amd as rdm
    from workloads import poisson_arrivals, tfim_request
    # the engine's arena: the device's free memory less 16 GiB for the
    # Hamiltonians' own tables (at most max_active requests' worth resident)
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - (16 << 30))
    srv = rdm.Server(hbm_budget=budget, max_active=64, precision="mixed")
    next_req = [0]
    keep = []  # Hamiltonians of requests not yet finished (released as they finish)

    def new_request():
        inst = tfim_request(next_req[0])
        next_req[0] += 1
        return inst, rdm.Hamiltonian.from_instance(inst)

    def open_loop(n, rate):
        """n Poisson arrivals at rate/s; returns (solves/s, latencies in s,
        spin counts of the requests)."""
        arr = poisson_arrivals(n, rate, seed=int(rate * 1000) + n)
        done, pending, hams, sizes = {}, {}, {}, {}
        lock = threading.Lock()
        stop = [False]

        def poller():
            while not stop[0] or pending:
                with lock:
                    items = list(pending.items())
                for t, i in items:
                    r = srv.poll(t)
                    if r is not None:
                        done[i] = (time.perf_counter(), r["status"])
                        with lock:
                            del pending[t]
                        hams.pop(i).close()
                time.sleep(0.0005)

        th = threading.Thread(target=poller)
        th.start()
        start = time.perf_counter()
        sub = {}
        for i in range(n):
            now = time.perf_counter() - start
            if arr[i] > now:
                time.sleep(arr[i] - now)
            if i % 200 == 0:
                print(f"[serve] rate {rate:.1f}/s: submitted {i} of {n}, {len(done)} done", file=sys.stderr,
                      flush=True)
            inst, h = new_request()
            sizes[i] = inst.n
            hams[i] = h
            sub[i] = time.perf_counter()
            t = srv.submit(h, inst.betas, inst.n_v, inst.k, inst.seed)
            with lock:
                pending[t] = i
        last = time.perf_counter()
        while True:
            with lock:
                if not pending:
                    break
            time.sleep(0.01)
            if time.perf_counter() - last > 20:
                last = time.perf_counter()
                print(f"[serve] draining: {len(pending)} pending", file=sys.stderr, flush=True)
        stop[0] = True
        th.join()
        total = time.perf_counter() - start
        assert all(done[i][1] == 0 for i in range(n))
        return (n / total, np.array([done[i][0] - sub[i] for i in range(n)]),
                np.array([sizes[i] for i in range(n)]))

    try:
        # closed loop: everything submitted at once -> saturated capacity
        batch = [new_request() for _ in range(200)]
        t0 = time.perf_counter()
        keep.extend(h for _, h in batch)
        tk = [srv.submit(h, i.betas, i.n_v, i.k, i.seed) for i, h in batch]
        for t in tk:
            assert srv.wait(t)["status"] == 0
        capacity = 200 / (time.perf_counter() - t0)
        for h in keep:
            h.close()
        keep.clear()
        print(f"[serve] closed-loop capacity {capacity:.2f} solves/s", file=sys.stderr, flush=True)
        rate_a, lat_a, _ = open_loop(args.requests, args.rate)
        steady = 0.7 * capacity
        rate_b, lat_b, n_b = open_loop(args.steady_requests, steady)
        # the same number of arrivals at a fixed 12.6/s (0.7 x the capacity of
        # an earlier engine), for comparisons at equal offered load
        rate_c, lat_c, _ = open_loop(args.steady_requests, 12.6)
        stats = srv.stats()
    finally:
        srv.close()
        for h in keep:
            h.close()
    pct = lambda lat, q: round(1e3 * float(np.percentile(lat, q)), 2)  # noqa: E731
    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle on the host (16 requests)")
        from workloads import tfim_request
        cores, secs = cpu_baseline_sample("serve", list(range(16)))
        t_mean = float(np.mean([_solve_seconds(tfim_request(r), t) for r, t in zip(range(16), secs)]))
        cpu = {"value": cores / t_mean, "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": "one FP64 Lanczos step of one start column of each of the first 16 requests "
                         "(one process each), scaled to k steps x all columns; capacity with one "
                         "request per core"}
    return {"metric": "serving: solves/s and p50/p99 latency", "value": round(rate_a, 3), "cpu_baseline": cpu,
            "unit": "solves/s", "dtype": "f32 vectors + f64 reductions",
            "config": {"workload": f"Poisson arrivals {args.rate}/s of transverse-field ZZ-chain "
                                   "requests, N in [14,24], d_s in {2,4}, beta log-U[0.1,10], n_v=8, k=60",
                       "requests": args.requests},
            "capacity_closed_loop": round(capacity, 3),
            "p50_ms": pct(lat_a, 50), "p99_ms": pct(lat_a, 99), "offered_rate": args.rate,
            "steady": {"offered_rate": round(steady, 3), "requests": args.steady_requests,
                       "solves_per_s": round(rate_b, 3), "p50_ms": pct(lat_b, 50), "p99_ms": pct(lat_b, 99)},
            "steady_by_spins": {f"{lo}-{hi}": {"requests": int(((n_b >= lo) & (n_b <= hi)).sum()),
                                               "p50_ms": pct(lat_b[(n_b >= lo) & (n_b <= hi)], 50),
                                               "p99_ms": pct(lat_b[(n_b >= lo) & (n_b <= hi)], 99)}
                                for lo, hi in ((14, 20), (21, 22), (23, 24))},
            "fixed_12_6": {"offered_rate": 12.6, "requests": args.steady_requests, "solves_per_s": round(rate_c, 3),
                           "p50_ms": pct(lat_c, 50), "p99_ms": pct(lat_c, 99)},
            "peak_active": stats["peak_active"], "engine_steps": stats["steps"],
            "peak_device_bytes": stats["peak_bytes"], "arena_bytes": budget}


def bench_scan(args):
    """The paper's long-range experiments on 2 + 14 spins (isotropic XY,
    J_ij = |i-j|^-alpha, z-field h), mixed precision, one batched solve per
    scan: entropy over (field, temperature) at alpha = 1 with n_v = 400;
    internal-energy deviation over alpha at h = 0 and over the coupling scale
    eps at alpha = 1, n_v = 100; k = 60."""
    import paper_2204_08147_amd  # noqa: F401
    from paper_2204_08147_amd import scans
    from workloads import xy_power_law
    temps = np.array([0.1, 0.2, 0.3, 0.5, 0.7, 1.0, 1.5, 2.0])
    betas = tuple(1.0 / temps)
    fields = np.linspace(0.0, 2.2, 12)
    alphas = [0.0, 0.1, 0.3, 0.5, 1.0, 2.0, float("inf")]
    epss = np.linspace(0.0, 1.0, 11)
    out = {"metric": "scan solves/s (paper's long-range experiments)", "unit": "solves/s",
           "dtype": "f32 vectors + f64 reductions",
           "config": {"workload": "isotropic XY 2+14 spins, J_ij=|i-j|^-alpha, z-field h; entropy grid "
                                  "alpha=1, 12 fields in [0,2.2] x 8 temperatures, n_v=400; deviation over "
                                  "alpha (h=0) and eps (alpha=1, h=0), n_v=100; k=60"}}
    t0 = time.perf_counter()
    grid = scans.entropy_grid(lambda h: xy_power_law(2, 14, 1.0, h, 6100, betas=betas, n_v=400, k=60),
                              fields, precision="mixed")
    t_grid = time.perf_counter() - t0
    t0 = time.perf_counter()
    dev_a = scans.deviation_scan(lambda a: xy_power_law(2, 14, a, 0.0, 6200, betas=betas, n_v=100, k=60),
                                 alphas, precision="mixed")
    t_a = time.perf_counter() - t0
    t0 = time.perf_counter()
    dev_e = scans.deviation_scan(lambda e: xy_power_law(2, 14, 1.0, 0.0, 6300, eps=e, betas=betas, n_v=100,
                                                        k=60), epss, precision="mixed")
    t_e = time.perf_counter() - t0
    n = len(fields) + len(alphas) + len(epss)
    out.update({"value": round(n / (t_grid + t_a + t_e), 3),
                "entropy_grid_s": round(t_grid, 3), "alpha_scan_s": round(t_a, 3), "eps_scan_s": round(t_e, 3),
                "temperatures": temps.tolist(), "fields": fields.round(3).tolist(),
                "entropy": grid.round(4).tolist(),
                "alphas": ["inf" if np.isinf(a) else a for a in alphas],
                "deviation_vs_alpha": dev_a.round(5).tolist(),
                "eps": epss.round(2).tolist(), "deviation_vs_eps": dev_e.round(5).tolist(),
                "max_abs_deviation_at_eps0": float(np.abs(dev_e[0]).max())})
    return out


def _time_oracle_small(reps):
    """Host process: the oracle's O3 path and the dense O1 answer on the
    1 + 9 chain, each timed over whole calls (best of reps)."""
    from threadpoolctl import threadpool_limits
    from oracle import exact, lanczos as olz
    from workloads import cfg_small_chain
    inst = cfg_small_chain()
    with threadpool_limits(limits=1):
        t3, t1 = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            olz.solve(inst)
            t3.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            exact.exact_rdm(inst, float(inst.betas[0]))
            t1.append(time.perf_counter() - t0)
    return min(t3), min(t1)


def bench_small(args):
    """The CPU-checkable configuration: 1 system + 9 bath spins (dim 1024),
    nearest-neighbour XXZ chain, z-field h = 0.5, beta = 1, n_v = 4, k = 30,
    FP64, solves one after another on one stream (latency-bound: the whole
    solve is a few launches of small kernels)."""
    import torch
    import paper_2204_08147_amd as rdm
    from oracle import exact
    from workloads import cfg_small_chain
    inst = cfg_small_chain()
    h = rdm.Hamiltonian.from_instance(inst)
    ws = torch.empty(rdm.workspace_size(h, 1, inst.n_v, inst.k, precision="fp64"), dtype=torch.uint8,
                     device="cuda")
    for _ in range(max(1, args.warmup)):
        rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="fp64", workspace=ws)
    torch.cuda.synchronize()
    n = 50 * args.steps
    lat = []
    t0 = time.perf_counter()
    for _ in range(n):
        t1 = time.perf_counter()
        r = rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="fp64", workspace=ws)
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ex = exact.exact_rdm(inst, float(inst.betas[0]))
    err = float(np.linalg.norm(r["rho"][0] - ex["rho"]) / np.linalg.norm(ex["rho"]))
    # the same solves as one batched call per step (50 bath-vector seeds):
    # every kernel of a step launches once for all of them
    items = [dict(h=h, betas=inst.betas, n_v=inst.n_v, k=inst.k, seed=inst.seed + s_) for s_ in range(50)]
    rdm.solve_batch(items, precision="fp64")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(args.steps):
        outs = rdm.solve_batch(items, precision="fp64")
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    assert all(o["status"] == 0 for o in outs)
    batched = {"solves_per_s": round(50 * args.steps / tb, 3), "ms_per_call": round(1e3 * tb / args.steps, 3),
               "solves_per_call": 50}
    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle on the host (whole O3 solves and the dense answer)")
        t3, t1 = _pool_starmap(1, _time_oracle_small, [(3,)])[0]
        cpu = {"value": round(1.0 / t3, 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"whole O3 solves (FP64 Lanczos path), best of 3, one process, BLAS one thread; "
                         f"dense O1 exact answer {1e3 * t1:.1f} ms"}
    return {"metric": "small-instance solves/s (FP64)", "value": round(n / wall, 3), "unit": "solves/s",
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
            "dtype": "f64", "cpu_baseline": cpu,
            "config": {"workload": "XXZ chain 1+9 spins (dim 1024), J ~ U(-1,1), system-bath bond 1, "
                                   "z-field h=0.5, beta=1, n_v=4, k=30, FP64; 50 solves per step"},
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "rho_rel_err_vs_exact": err, "batched": batched,
            "note": "the estimate's error against the exact partial trace is the stochastic error of "
                    "n_v = 4 bath vectors, not a parity figure"}


def bench_estimators(args):
    """The estimator variants and limits on the long-range 2 + 18 workload
    (h = 0.5, n_v = 16, k = 60, beta in {0.5, 1, 2, 4}), mixed precision:
    the product-state estimate of ln Z* (n_v single columns), the
    high-temperature offset, and the low-temperature limit (n_v = 4 full-space
    Lanczos runs, k = 60).  Best of three timed calls after one warm-up, next
    to the partial-trace solve of the same instance."""
    import torch
    import paper_2204_08147_amd as rdm
    from workloads import cfg_long_range
    inst = cfg_long_range(0, n_b=args.n_b)
    h = rdm.Hamiltonian.from_instance(inst)

    def best(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return min(t), out

    t_solve, sv = best(lambda: rdm.solve(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed"))
    t_prod, pr = best(lambda: rdm.product_trace(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="mixed"))
    t_prod64, pr64 = best(lambda: rdm.product_trace(h, inst.betas, inst.n_v, inst.k, inst.seed, precision="fp64"))
    t_ht, ht = best(lambda: rdm.high_temperature_term(h, inst.n_v, inst.seed))
    t_gs, gs = best(lambda: rdm.ground_state(h, 4, inst.k, inst.seed, precision="mixed"))
    # algorithmic bytes of the product run's Lanczos steps: n_v columns on
    # H_t and on H_b, k steps (the whole call's time, host work included)
    info = h.info()
    b_t, _ = operator_work(inst.n, inst.n_v, 0, info["transform"], 4, inst.k)
    b_b, _ = operator_work(inst.n_b, inst.n_v, 0, info["bath_transform"], 4, inst.k)
    return {"metric": "estimator variants: calls/s of the product-state estimate (n_v = 16)",
            "value": round(1.0 / t_prod, 3), "unit": "calls/s", "dtype": "f32 vectors + f64 reductions",
            "config": {"workload": "long-range XX+ZZ 2+18 spins, h=0.5, n_v=16, k=60, beta in {0.5,1,2,4}"},
            "partial_trace_solve_ms": round(1e3 * t_solve, 2),
            "product_trace_ms": round(1e3 * t_prod, 2), "product_trace_fp64_ms": round(1e3 * t_prod64, 2),
            "product_whole_call_gbs_algorithmic": round(inst.k * (b_t + b_b) / t_prod / 1e9, 1),
            "log_z_partial_trace": np.round(sv["log_z"], 6).tolist(),
            "log_z_product": np.round(pr["log_z"], 6).tolist(),
            "log_z_product_fp64": np.round(pr64["log_z"], 6).tolist(),
            "high_temperature_term_ms": round(1e3 * t_ht, 3), "high_temperature_offset_norm": round(ht["norm"], 6),
            "ground_state_ms": round(1e3 * t_gs, 2), "ground_energy": round(gs["e_total"], 6),
            "ground_bath_energy": round(gs["e_bath"], 6), "ground_degeneracy": gs["degeneracy"],
            "ground_entropy": round(gs["entropy"], 6)}


def stage(msg: str) -> None:
    """Progress of a long run on stderr (the JSON line alone goes to stdout)."""
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for --gpus {args.gpus}): the bath-vector groups are "
              "independent and would be sharded across GPUs with one final reduce of the d_s x d_s sums, "
              "which is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2204_08147_amd as rdm
    from workloads import LR_FIELDS, cfg_long_range

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "lr":
        fn = {"small": bench_small, "batch": bench_batch, "large": bench_large, "serve": bench_serve,
              "scan": bench_scan, "estimators": bench_estimators}[args.workload]
        out = fn(args)
        out.update({"n_gpus": 1, "data": "synthetic", "scaling": "weak"})
        print(json.dumps(out))
        return
    insts = [cfg_long_range(i, n_b=args.n_b) for i in range(len(LR_FIELDS))]
    hs = [rdm.Hamiltonian.from_instance(i) for i in insts]
    inst0 = insts[0]
    stream = torch.cuda.current_stream()

    def make_ws(prec):
        return [torch.empty(rdm.workspace_size(h, len(i.betas), i.n_v, i.k, precision=prec, mode="stored"),
                            dtype=torch.uint8, device="cuda") for h, i in zip(hs, insts)]

    # one HIP stream (default priority) and one host thread per field: the
    # three solves of a step are independent, so one solve's host phase (the
    # tridiagonal eigenproblems between its Lanczos run and its Gram) overlaps
    # the others' device work
    streams = [torch.cuda.Stream() for _ in insts]

    def run(prec, steps, warmup, ws, profile, concurrent=True):
        """warmup + timed steps (the default launch path: each solve's Lanczos
        steps replayed as a hipGraph), then, outside the timed region, one
        step with HIP-event timing of the kernels (launched one by one).
        concurrent: the step's solves run on their own streams and threads;
        otherwise one after another on one stream."""
        import threading
        lat, apply_ms, norm_ms, gram_ms = [], [], [], []
        xz1_ms = []
        replay = []  # mean replayed Lanczos step (ms) of every timed solve
        res = [None] * len(insts)

        def solve_one(t, st):
            # profile="replay": the graph replay of the steps is kept and
            # timed with HIP events on the stream it runs on
            i = insts[t]
            return rdm.solve(hs[t], i.betas, i.n_v, i.k, i.seed, precision=prec, mode="stored",
                             workspace=ws[t], stream=st, profile="replay")

        for _ in range(warmup):
            for t in range(len(insts)):
                solve_one(t, streams[t] if concurrent else stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if concurrent:
            lats = [[] for _ in insts]
            errors = []

            def worker(t):
                try:
                    with torch.cuda.stream(streams[t]):
                        for _ in range(steps):
                            t1 = time.perf_counter()
                            res[t] = solve_one(t, streams[t])
                            lats[t].append(time.perf_counter() - t1)
                            replay.append(res[t]["t_replay_step_ms"])
                except BaseException as e:  # re-raised below, in the main thread
                    errors.append(e)

            th = [threading.Thread(target=worker, args=(t,)) for t in range(len(insts))]
            for x in th:
                x.start()
            for x in th:
                x.join()
            if errors:
                raise errors[0]
            lat = [v for l_ in lats for v in l_]
        else:
            for _ in range(steps):
                for t in range(len(insts)):
                    t1 = time.perf_counter()
                    res[t] = solve_one(t, stream)
                    lat.append(time.perf_counter() - t1)
                    replay.append(res[t]["t_replay_step_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if profile:
            for h, i, w in zip(hs, insts, ws):
                r = rdm.solve(h, i.betas, i.n_v, i.k, i.seed, precision=prec, mode="stored",
                              workspace=w, stream=stream, profile=True)
                apply_ms.append(r["t_apply_ms"])
                norm_ms.append(r["t_norm_ms"])
                xz1_ms.append(r["t_xz1_ms"])
                gram_ms.append(r["t_gram_ms"])
        return wall, lat, apply_ms, norm_ms, gram_ms, res, xz1_ms, replay

    stage("mixed-precision solves")
    ws_m = make_ws("mixed")
    wall_m, lat_m, ap_m, no_m, gr_m, res_m, x0_m, rep_m = run("mixed", args.steps, args.warmup, ws_m, True)
    # the same solves one after another on one stream (latency of a solve alone)
    wall_s, lat_s, _, _, _, _, _, _ = run("mixed", args.steps, 0, ws_m, False, concurrent=False)
    sequential = {"solves_per_s": round(len(lat_s) / wall_s, 3),
                  "p50_ms": round(1e3 * float(np.percentile(lat_s, 50)), 3),
                  "p99_ms": round(1e3 * float(np.percentile(lat_s, 99)), 3)}
    # the paper's block variant (Algorithm 1 + block Gauss quadrature) on the
    # same instances, mixed precision: time per solve and agreement with the
    # per-column path (same bath vectors)
    block = None
    if not args.no_block:
        stage("block variant")
        ws_b = [torch.empty(rdm.workspace_size(h, len(i.betas), i.n_v, i.k, precision="mixed", method="block"),
                            dtype=torch.uint8, device="cuda") for h, i in zip(hs, insts)]
        for h, i, w in zip(hs, insts, ws_b):
            rdm.solve(h, i.betas, i.n_v, i.k, i.seed, precision="mixed", method="block", workspace=w, stream=stream)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        outs = [rdm.solve(h, i.betas, i.n_v, i.k, i.seed, precision="mixed", method="block", workspace=w,
                          stream=stream) for h, i, w in zip(hs, insts, ws_b)]
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb
        ref = [rdm.solve(h, i.betas, i.n_v, i.k, i.seed, precision="mixed", mode="stored", workspace=w,
                         stream=stream) for h, i, w in zip(hs, insts, ws_m)]
        diff = max(float(np.linalg.norm(o["rho"][b] - r["rho"][b]) / np.linalg.norm(r["rho"][b]))
                   for o, r in zip(outs, ref) for b in range(len(o["rho"])))
        # accuracy at a short Krylov length: both methods at k = 20 against the
        # converged (k = 60) per-column result, same bath vectors
        kk = 20
        err_b = err_c = 0.0
        for h, i, r in zip(hs, insts, ref):
            ob = rdm.solve(h, i.betas, i.n_v, kk, i.seed, precision="mixed", method="block", stream=stream)
            oc = rdm.solve(h, i.betas, i.n_v, kk, i.seed, precision="mixed", stream=stream)
            for b in range(len(r["rho"])):
                nr = np.linalg.norm(r["rho"][b])
                err_b = max(err_b, float(np.linalg.norm(ob["rho"][b] - r["rho"][b]) / nr))
                err_c = max(err_c, float(np.linalg.norm(oc["rho"][b] - r["rho"][b]) / nr))
        block = {"solves_per_s": round(len(insts) / tb, 3), "ms_per_solve": round(1e3 * tb / len(insts), 2),
                 "rho_rel_diff_vs_per_column": diff, "workspace_bytes": int(ws_b[0].numel()),
                 "k20_rho_err_block": err_b, "k20_rho_err_per_column": err_c}
        del ws_b
    del ws_m
    torch.cuda.empty_cache()

    fp64 = None
    mixed_vs_fp64 = None
    if not args.no_fp64:
        stage("FP64 solves")
        ws_d = make_ws("fp64")
        wall_d, lat_d, ap_d, no_d, gr_d, res_d, x0_d, _ = run("fp64", max(1, args.steps // 2), args.warmup,
                                                              ws_d, True)
        del ws_d
        torch.cuda.empty_cache()
        n_d = len(lat_d)
        fp64 = {"solves_per_s": n_d / wall_d, "p50_ms": 1e3 * float(np.percentile(lat_d, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat_d, 99)),
                "step_kernels_ms": float(np.mean(ap_d) + np.mean(no_d) + np.mean(x0_d)),
                "transform_pass1_ms": round(float(np.mean(x0_d)), 4),
                "apply_kernel_ms": round(float(np.mean(ap_d)), 4)}
        # error of the mixed path against the FP64 path, same instances and
        # bath vectors (the largest over the fields and temperatures)
        errs = [result_errors(a, b) for a, b in zip(res_m, res_d)]
        mixed_vs_fp64 = {key: max(e[key] for e in errs) for key in errs[0]}

    # Krylov truncation (Section "Error analysis"): the FP64 result at k
    # against k + 20 steps with the same bath vectors, outside the timed region
    trunc = None
    if not args.no_truncation:
        stage("k against k + 20")
        d_rho = d_h = d_lz = 0.0
        for h, i in zip(hs, insts):
            a = rdm.solve(h, i.betas, i.n_v, i.k, i.seed, precision="fp64", stream=stream)
            b = rdm.solve(h, i.betas, i.n_v, i.k + 20, i.seed, precision="fp64", stream=stream)
            for t in range(len(i.betas)):
                d_rho = max(d_rho, float(np.linalg.norm(a["rho"][t] - b["rho"][t]) / np.linalg.norm(b["rho"][t])))
                d_h = max(d_h, float(np.linalg.norm(a["h_star"][t] - b["h_star"][t]) /
                                     np.linalg.norm(b["h_star"][t])))
                d_lz = max(d_lz, abs(float(a["log_z"][t] - b["log_z"][t])))
        torch.cuda.empty_cache()
        trunc = {"k": inst0.k, "k_ref": inst0.k + 20, "precision": "fp64", "rho_rel_diff": d_rho,
                 "h_star_rel_diff": d_h, "log_z_abs_diff": d_lz}

    n_solves = len(lat_m)
    value = n_solves / wall_m
    ms_per_step = 1e3 * wall_m / args.steps

    # measured streaming reference points (library probe: nontemporal loads and
    # stores, one 4 KiB chunk per workgroup and array, 2 GiB arrays, best of 10)
    stage("streaming probe")
    probe = {p: rdm.stream_probe(p, 1 << 31, 10) for p in ("read", "copy", "r3w1", "r2w2")}
    torch.cuda.empty_cache()

    # roofline of the dominant work, one Lanczos step (the two transform
    # passes over the H_t and H_b segments), on the measurement plan's count:
    # 2 C nnz flops per row against the FP32 vector peak (nnz = 211 makes the
    # product VALU-bound by that count); beside it the plan's minimum bytes
    # (three vector passes) and the transform's own streams against HBM
    info = hs[0].info()
    nnz = 1 + info["hops_uniform"] + 0.5 * info["hops_parity"]
    bytes_alg, flops = step_work([inst0], 4)
    min_bytes, nnz_flops = plan_work([inst0], 4)
    # the step as it ran in the timed region (HIP events around each solve's
    # replayed steps on the replay stream: both passes and the two step
    # reductions, with the other solves' work sharing the device) ...
    t_live = float(np.mean(rep_m)) * 1e-3
    # ... and the two passes of one step of a solve run alone (events around
    # each kernel, outside the timed region)
    t_step = float(np.mean(ap_m) + np.mean(no_m) + np.mean(x0_m)) * 1e-3
    achieved_gbs = bytes_alg / t_step / 1e9
    mix_gbs = 2.0 / (1.0 / probe["r2w2"] + 1.0 / probe["r3w1"])
    traffic = read_traffic("lanczos_step_lr_xxzz_2+18_mixed_counters.txt")
    roof = roofline(min_bytes, nnz_flops, t_live, traffic)
    roof_transform = roofline(bytes_alg, 0.0, t_live, traffic)
    roof_min_bytes = roofline(min_bytes, 0.0, t_live)
    roof_isolated = roofline(min_bytes, nnz_flops, t_step, traffic)

    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle on the host")
        cpu = cpu_baseline(inst0, 0, args.n_b)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 vectors + f64 reductions", "data": "synthetic",
        "config": {"workload": f"long-range XX+ZZ, N_s=2 + N_b={args.n_b} (dim 2^{2 + args.n_b}), "
                               "J_ij=|i-j|^-1.5, x-field h in {0.5,1.0,1.5}, beta in {0.5,1,2,4}, "
                               "n_v=16 Rademacher, k=60; one step = the three fields, solved concurrently "
                               "(one HIP stream and host thread each)",
                   "solves_per_step": len(insts), "n_columns": inst0.n_cols, "nnz_per_row": nnz,
                   "apply": "transform (D_Z + W D_X W, 2 passes per step)" if info["transform"] else "hop tables"},
        # per-solve latency with the step's three solves running concurrently
        "p50_ms": round(1e3 * float(np.percentile(lat_m, 50)), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat_m, 99)), 3),
        "sequential": sequential,
        "step_gbs_algorithmic": round(achieved_gbs, 1),
        "step_ms_timed_region": round(1e3 * t_live, 4),
        "step_kernels_ms": round(1e3 * t_step, 4),
        "apply_kernel_ms": round(float(np.mean(ap_m)), 4),
        "norm_kernel_ms": round(float(np.mean(no_m)), 4),
        "transform_pass1_ms": round(float(np.mean(x0_m)), 4),
        "gram_kernel_ms": round(float(np.mean(gr_m)), 4),
        # recombination + Gram: one read of the k stored FP32 vectors per solve
        # (all four temperatures in one pass)
        "gram_gbs_algorithmic": round(inst0.k * inst0.dim * inst0.n_cols * 4 / (float(np.mean(gr_m)) * 1e-3) / 1e9,
                                      1),
        "fp64": None if fp64 is None else {k2: round(v, 4) for k2, v in fp64.items()},
        "mixed_over_fp64": None if fp64 is None else round(value / fp64["solves_per_s"], 3),
        "mixed_vs_fp64": mixed_vs_fp64,
        "block_method": block,
        "truncation_k_vs_k20": trunc,
        "roofline": roof,
        "roofline_note": "one Lanczos step; achieved = 2*C*nnz flops per row (H_t and H_b) / the mean "
                         "step time of the timed region's solves (HIP events around the replayed steps) "
                         "against the published FP32 vector peak; the transform apply reaches the same "
                         "product with (2N+8) flops per element, so this is an effective rate",
        "roofline_step_alone": roof_isolated,
        "roofline_transform_bytes": roof_transform,
        "roofline_min_bytes": roof_min_bytes,
        "scope_notes": {"gram": "recombination + Gram on the vector units (C <= 64 columns, intensity "
                                "<= C/2 flop/B: bound by HBM, see gram_gbs_algorithmic)",
                        "cpu_baseline": "extrapolated from a timed sample of Lanczos steps"},
        # a transform step is half two-read-two-write (pass 1), half
        # three-read-one-write (pass 2): the probe's matching mix
        "stream_probe": {**{k: round(v, 1) for k, v in probe.items()},
                         "step_mix_gbs": round(mix_gbs, 1), "step_frac_of_mix": round(achieved_gbs / mix_gbs, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
