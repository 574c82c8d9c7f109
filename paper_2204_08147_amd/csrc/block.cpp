// Block Lanczos with block Gauss quadrature (Algorithm 1, eqn:fT,
// eqn:trB_est): the paper's own estimator, on the same apply kernels.
//
// For each bath vector j the start block V_j = [|m> (x) |v_j>]_m (d_s
// orthonormal columns) runs the block Lanczos recurrence of Algorithm 1,
// whose block QR is done here as two Cholesky passes on an FP64 Gram
// (Cholesky QR twice); only three blocks of vectors are kept.
// The block tridiagonal T_j (A_i on the diagonal, B_i below) gives
// E_1^T exp(-beta (T_j - E0)) E_1 directly, so there is no recombination and
// no Gram pass; E0 is the smallest eigenvalue over all T_j.  The bath
// quadrature (Z_b) is the per-column scalar Lanczos of the hot path.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"
#include "solve.h"

namespace rdm {

namespace {
int pw(int prec) { return prec == RDM_FP64 ? 2 : 4; }
size_t sbytes(int prec) { return prec == RDM_FP64 ? 8 : 4; }
}  // namespace

rdm_status block_plan(BlockPlan& bp, const rdm_hamiltonian* h, int n_beta, int n_v, int k, int prec,
                      uint64_t budget) {
  bp = BlockPlan{};
  if (h->n_s > 3) {
    set_error("the block variant takes n_s <= 3 (d_s <= 8)");
    return RDM_E_INVALID;
  }
  bp.h = h;
  bp.prec = prec;
  bp.n_beta = n_beta;
  bp.n_v = n_v;
  bp.ds_log = h->n_s;
  bp.ds = 1 << h->n_s;
  bp.dim = 1ull << h->n;
  // the block Krylov space of d_s columns has at most dim / d_s blocks
  bp.k = (int)std::min<uint64_t>((uint64_t)k, bp.dim / bp.ds);
  bp.kb = (int)std::min<uint64_t>((uint64_t)k, 1ull << h->n_b);
  const int W = pw(prec);
  const size_t sb = sbytes(prec);
  bp.C = bp.ds * n_v;
  bp.cpad = (bp.C + W - 1) / W * W;
  bp.CB = std::max(bp.ds, W);
  bp.cpad = (bp.cpad + bp.CB - 1) / bp.CB * bp.CB;
  bp.G = bp.cpad / bp.ds;
  bp.n_cb = bp.cpad / bp.CB;
  bp.blk = bp.dim * bp.cpad;
  // rows per lane so that at most ~1024 row tiles feed each reduction
  const uint64_t rows_per_tile = std::max<uint64_t>(kBlock, (bp.dim + 1023) / 1024);
  bp.rpl = (int)((rows_per_tile + kBlock - 1) / kBlock);
  bp.n_rt = (int)((bp.dim + (uint64_t)kBlock * bp.rpl - 1) / ((uint64_t)kBlock * bp.rpl));
  const int NE = bp.ds * bp.ds;
  // header: three apply segments (one per ring slot), the bath segment, BSeg
  bp.header = align_up(4 * sizeof(Seg)) + align_up(sizeof(BSeg));
  size_t off = 0;
  bp.o_Q = off; off = align_up(off + 3 * bp.blk * sb);
  bp.o_R = off; off = align_up(off + bp.blk * sb);
  // scratch block of the YY part of a transform apply
  bp.o_Y = off;
  if (needs_ybuf(h, 0)) off = align_up(off + bp.blk * sb);
  bp.o_part = off; off = align_up(off + (size_t)bp.n_rt * bp.G * NE * 8);
  bp.o_mats = off; off = align_up(off + (size_t)BM_COUNT * bp.G * NE * 8);
  bp.o_ah = off; off = align_up(off + (size_t)bp.k * bp.G * NE * 8);
  bp.o_bh = off; off = align_up(off + (size_t)bp.k * bp.G * NE * 8);
  bp.o_kc = off; off = align_up(off + (size_t)bp.G * 4);
  // geometry of the plain apply segments (no storage of their own)
  size_t dummy = 0;
  plan_seg(bp.apply, h->n, bp.cpad, 1, prec, 1, 0, 1, dummy);
  plan_seg(bp.bath, h->n_b, n_v, bp.kb, prec, 0, 0, 2, off, lanczos_needs_ybuf(h, 1, prec));
  bp.bytes = bp.header + off;
  if (budget != 0 && bp.bytes > budget) {
    set_error("block solve needs " + std::to_string(bp.bytes) + " device bytes, budget " +
              std::to_string(budget));
    return RDM_E_NOMEM;
  }
  return RDM_OK;
}

namespace {

template <typename T>
rdm_status run_block(const BlockPlan& bp, const OpDevice* op_t, char* ws, char* base, uint64_t seed, double tau,
                     hipStream_t st, StepTimers* tm) {
  const int NE = bp.ds * bp.ds;
  const size_t sb = sbytes(bp.prec);
  Seg* dsegs = (Seg*)ws;
  BSeg* dbs = (BSeg*)(ws + align_up(4 * sizeof(Seg)));
  // plain apply segments: Q = ring slot, R = scratch
  std::vector<Seg> ap(3);
  Launch L;
  for (int r = 0; r < 3; ++r) {
    Seg& sg = ap[r];
    sg = Seg{};
    sg.nbits = bp.h->n;
    sg.n_row_tiles = bp.apply.n_row_tiles;
    bind_apply(sg, op_t);
    sg.P = bp.apply.P;
    sg.S = 1;
    sg.rpl = 1;
    sg.C = bp.cpad;
    sg.cpad = bp.cpad;
    sg.k = 1;
    sg.mode = MODE_PLAIN;
    sg.blk = bp.blk;
    sg.Q = base + bp.o_Q + (size_t)r * bp.blk * sb;
    sg.R = base + bp.o_R;
    sg.Y = sg.xy ? base + bp.o_Y : nullptr;
    std::vector<Seg> one{sg};
    L = assign_tiles(one);
    sg = one[0];
  }
  BSeg bs{};
  bs.Q = base + bp.o_Q;
  bs.R = base + bp.o_R;
  bs.part = (double*)(base + bp.o_part);
  bs.mats = (double*)(base + bp.o_mats);
  bs.a_hist = (double*)(base + bp.o_ah);
  bs.b_hist = (double*)(base + bp.o_bh);
  bs.kc = (int32_t*)(base + bp.o_kc);
  bs.blk = bp.blk;
  bs.nbits = bp.h->n;
  bs.cpad = bp.cpad;
  bs.C = bp.C;
  bs.G = bp.G;
  bs.k = bp.k;
  bs.rpl = bp.rpl;
  bs.n_rt = bp.n_rt;
  bs.n_cb = bp.n_cb;
  bs.tau = tau;
  RDM_HIP(hipMemcpyAsync(dsegs, ap.data(), 3 * sizeof(Seg), hipMemcpyHostToDevice, st));
  RDM_HIP(hipMemcpyAsync(dbs, &bs, sizeof(BSeg), hipMemcpyHostToDevice, st));
  RDM_HIP(hipMemsetAsync(bs.mats, 0, (size_t)BM_COUNT * bp.G * NE * 8, st));
  RDM_HIP(hipMemsetAsync(bs.a_hist, 0, (size_t)bp.k * bp.G * NE * 8, st));
  RDM_HIP(hipMemsetAsync(bs.b_hist, 0, (size_t)bp.k * bp.G * NE * 8, st));
  std::vector<int32_t> kc0(bp.G, bp.k);
  RDM_HIP(hipMemcpyAsync(bs.kc, kc0.data(), bp.G * 4, hipMemcpyHostToDevice, st));
  // Q_1: the start block |m> (x) |v_j> (exactly orthonormal per group)
  RDM_HIP(launch_start_block<T>(bp.ds_log, bp.h->n_b, bp.C, seed, START_SYSBATH, (T*)ap[0].Q, bp.h->n, bp.cpad,
                                st));
  // transform operators: the blocks live in the orthogonal basis W_lo Q / 64
  // (inner products unchanged, so A_j, B_j and the quadrature are too), and
  // each product H Q_j takes two streaming passes instead of three
  const int deep = xz_geom(bp.h->n);
  if (op_t->xz) RDM_HIP(launch_xz_pass<T>(3, dsegs, 1, L.xz, st, deep));
  for (int j = 1; j <= bp.k; ++j) {
    const Seg* sj = dsegs + (j - 1) % 3;
    if (tm) RDM_HIP(tm->apply.mark(st));
    RDM_HIP(launch_apply<T>(sj, 1, L.apply, 1, st));
    RDM_HIP(launch_apply_wide<T>(sj, 1, L.wide, st));
    if (op_t->xz)
      for (int pass = 4; pass <= 5; ++pass) RDM_HIP(launch_xz_pass<T>(pass, sj, 1, L.xz, st, deep));
    if (op_t->xz && op_t->xy)
      for (int pass : {9, 7, 10}) RDM_HIP(launch_xz_pass<T>(pass, sj, 1, L.xz, st, deep));
    if (tm) RDM_HIP(tm->apply.mark(st));
    if (tm) RDM_HIP(tm->norm.mark(st));
    RDM_HIP(launch_block_update<T>(dbs, bp.ds, BLK_A, j, bp.n_rt, bp.n_cb, st));
    RDM_HIP(launch_block_reduce(dbs, bp.ds, bp.G, BLK_A, j, st));
    if (j < bp.k) {
      RDM_HIP(launch_block_update<T>(dbs, bp.ds, BLK_G, j, bp.n_rt, bp.n_cb, st));
      RDM_HIP(launch_block_reduce(dbs, bp.ds, bp.G, BLK_G, j, st));
      RDM_HIP(launch_block_update<T>(dbs, bp.ds, BLK_G2, j, bp.n_rt, bp.n_cb, st));
      RDM_HIP(launch_block_reduce(dbs, bp.ds, bp.G, BLK_G2, j, st));
      RDM_HIP(launch_block_update<T>(dbs, bp.ds, BLK_G2 + 1, j, bp.n_rt, bp.n_cb, st));
    }
    if (tm) RDM_HIP(tm->norm.mark(st));
  }
  return RDM_OK;
}

}  // namespace

rdm_status block_solve(const BlockPlan& bp, const double* betas, uint64_t seed, double tau, char* ws,
                       hipStream_t st, bool profile, rdm_result* out) {
  Range range("rdm block solve");
  const OpDevice *op_t = nullptr, *op_b = nullptr;
  rdm_status s = get_device_op(bp.h, 0, bp.prec, st, &op_t);
  if (s == RDM_OK) s = get_device_op(bp.h, 1, bp.prec, st, &op_b);
  if (s != RDM_OK) return s;
  char* base = ws + bp.header;
  StepTimers tm;
  tm.apply.on = tm.norm.on = profile;
  s = bp.prec == RDM_FP64 ? run_block<double>(bp, op_t, ws, base, seed, tau, st, profile ? &tm : nullptr)
                          : run_block<float>(bp, op_t, ws, base, seed, tau, st, profile ? &tm : nullptr);
  if (s != RDM_OK) return s;
  // bath: per-column Lanczos (A8), as in the hot path
  Seg* dbath = (Seg*)ws + 3;
  std::vector<Seg> segs{make_plain_seg(bp.bath, op_b, base, MODE_LANCZOS, START_BATH, 0, bp.h->n_b, seed, tau)};
  if ((s = run_phase(segs, dbath, bp.prec, 0, st, nullptr, false, false)) != RDM_OK) return s;
  const int NE = bp.ds * bp.ds;
  std::vector<double> ah((size_t)bp.k * bp.G * NE), bh((size_t)bp.k * bp.G * NE);
  std::vector<int32_t> kc(bp.G);
  RDM_HIP(hipMemcpyAsync(ah.data(), base + bp.o_ah, ah.size() * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipMemcpyAsync(bh.data(), base + bp.o_bh, bh.size() * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipMemcpyAsync(kc.data(), base + bp.o_kc, bp.G * 4, hipMemcpyDeviceToHost, st));
  std::vector<double> ba, bb, bsc;
  std::vector<int32_t> bkc;
  if ((s = fetch_history(bp.bath, base, ba, bb, bsc, bkc, st)) != RDM_OK) return s;
  RDM_HIP(hipStreamSynchronize(st));
  for (double x : ah)
    if (!std::isfinite(x)) {
      set_error("non-finite block Lanczos coefficients");
      return RDM_E_NONFINITE;
    }
  for (double x : bh)
    if (!std::isfinite(x)) {
      set_error("non-finite block Lanczos coefficients");
      return RDM_E_NONFINITE;
    }
  // block tridiagonal T_g of every bath vector, its eigensystem, E0
  const int ds = bp.ds, n_v = bp.n_v;
  std::vector<DenseSymEig> eig(n_v);
  parallel_jobs(n_v, [&](int g) {
    const int nb = kc[g];
    const int n = nb * ds;
    std::vector<double> t((size_t)n * n, 0.0);
    for (int i = 0; i < nb; ++i) {
      const double* a = ah.data() + ((size_t)i * bp.G + g) * NE;
      for (int x = 0; x < ds; ++x)
        for (int y = 0; y < ds; ++y) t[(size_t)(i * ds + x) * n + i * ds + y] = a[x * ds + y];
      if (i + 1 < nb) {
        const double* b = bh.data() + ((size_t)i * bp.G + g) * NE;
        for (int x = 0; x < ds; ++x)
          for (int y = 0; y < ds; ++y) {
            t[(size_t)((i + 1) * ds + x) * n + i * ds + y] = b[x * ds + y];
            t[(size_t)(i * ds + y) * n + (i + 1) * ds + x] = b[x * ds + y];
          }
      }
    }
    eig[g].solve(t.data(), n, std::min(ds, n));
  });
  InstPlan p;
  p.h = bp.h;
  p.prec = bp.prec;
  p.n_beta = bp.n_beta;
  p.n_v = n_v;
  p.k = bp.k;
  p.kb = bp.kb;
  p.ds = ds;
  p.ds_log = bp.ds_log;
  p.bytes = bp.bytes;
  InstRun r;
  r.plan = &p;
  r.betas.assign(betas, betas + bp.n_beta);
  double e0 = INFINITY;
  for (int g = 0; g < n_v; ++g) {
    if (!eig[g].ok) {
      set_error("block tridiagonal eigenproblem failed");
      return RDM_E_NONFINITE;
    }
    e0 = std::min(e0, eig[g].min_eig());
  }
  r.e0 = e0;
  r.gsum.assign((size_t)bp.n_beta * n_v * NE, 0.0);
  parallel_jobs(n_v, [&](int g) {
    for (int b = 0; b < bp.n_beta; ++b) eig[g].quad(betas[b], e0, r.gsum.data() + ((size_t)b * n_v + g) * NE);
  });
  r.n_break_t = 0;
  for (int g = 0; g < n_v; ++g) r.n_break_t += kc[g] < bp.k;
  // bath quadrature m_b = (1/n_v) sum_c e_1^T exp(-beta (T_c - E0b)) e_1 |v_c|^2
  std::vector<TridiagEig> eb(n_v);
  const int bcp = bp.bath.cpad;
  parallel_jobs(n_v, [&](int c) {
    const int kk = bkc[c];
    std::vector<double> a(kk), b(kk > 0 ? kk - 1 : 0);
    for (int j = 0; j < kk; ++j) a[j] = ba[(size_t)j * bcp + c];
    for (int j = 0; j + 1 < kk; ++j) b[j] = bb[(size_t)j * bcp + c];
    eb[c].solve(a.data(), b.data(), kk);
  });
  double e0b = INFINITY;
  for (auto& e : eb) {
    if (!e.ok || e.n == 0) {
      set_error("tridiagonal eigenproblem failed");
      return RDM_E_NONFINITE;
    }
    for (double x : e.theta) e0b = std::min(e0b, x);
  }
  r.e0b = e0b;
  r.n_break_b = 0;
  for (int c = 0; c < n_v; ++c) r.n_break_b += bkc[c] < bp.kb;
  r.mb.assign(bp.n_beta, 0.0);
  for (int b = 0; b < bp.n_beta; ++b) {
    double acc = 0.0;
    for (int c = 0; c < n_v; ++c) {
      const TridiagEig& e = eb[c];
      const double s1 = bsc[c];
      double q = 0.0;
      for (int t = 0; t < e.n; ++t) q += e.zrow[t] * e.zrow[t] * std::exp(-betas[b] * (e.theta[t] - e0b));
      acc += q / (s1 * s1);
    }
    r.mb[b] = acc / n_v;
  }
  if (profile) {
    r.t_apply_ms = tm.apply.avg_ms();
    r.t_norm_ms = tm.norm.avg_ms();
  }
  return finalize(r, out);
}

}  // namespace rdm
