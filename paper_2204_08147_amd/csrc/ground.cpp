// Low-temperature limit (Section "High and low temperature limits" and the
// appendix deriving them): rho*(inf) = (1/r) sum_i tr_b |psi_i><psi_i| over the
// r ground states of H_t, H*(inf) = (E_t - E_b) I with E_t, E_b the ground
// energies of H_t and H_b.
//
// n_v Lanczos runs on seeded full-space Rademacher vectors (the same kernels
// as the hot path, stored basis) give each column's lowest Ritz pair.  The
// columns whose lowest Ritz value reached E_t (the smallest of them) span the
// ground space: their Ritz vectors psi_c = sum_j y_c[j] q_j have the Gram
// matrix M (Gram kernel of the hot path, one group), M = U diag(l) U^T, and
// the r eigenvalues above a threshold give the orthonormal basis
// phi_i = sum_c psi_c U_ci / sqrt(l_i).  One more pass over the stored basis
// forms tr_b sum_i |phi_i><phi_i| on the device.  E_b comes from the bath
// runs of the hot path.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"
#include "solve.h"

namespace rdm {

namespace {

int pw(int prec) { return prec == RDM_FP64 ? 2 : 4; }
size_t sbytes(int prec) { return prec == RDM_FP64 ? 8 : 4; }
constexpr int kGroundMaxR = 4;  // ground-space dimension the partial-trace kernel holds

struct GroundPlan {
  int prec = RDM_FP64, n_v = 0, k = 0, kb = 0, dsg = 2, n_cblocks = 0, g_rpl = 1, g_rtiles = 0;
  int pt_rpl = 1, pt_tiles = 0, ds = 2;
  SegPlan tot, bath;
  size_t o_y = 0, o_gpart = 0, o_gsum = 0, o_gseg = 0, o_gtiles = 0, o_w = 0, o_gp = 0, o_ppart = 0;
  size_t o_psum = 0, header = 0, bytes = 0;
};

rdm_status ground_plan(GroundPlan& gp, const rdm_hamiltonian* h, int n_v, int k, int prec, uint64_t budget) {
  gp = GroundPlan{};
  if (h->n_s > 3) {
    set_error("rdm_ground_state takes n_s <= 3 (d_s <= 8)");
    return RDM_E_INVALID;
  }
  gp.prec = prec;
  gp.n_v = n_v;
  gp.ds = 1 << h->n_s;
  const uint64_t dim = 1ull << h->n;
  gp.k = (int)std::min<uint64_t>((uint64_t)k, dim);
  gp.kb = (int)std::min<uint64_t>((uint64_t)k, 1ull << h->n_b);
  const int W = pw(prec);
  const size_t sb = sbytes(prec);
  gp.dsg = 2;
  while (gp.dsg < n_v) gp.dsg <<= 1;
  const int cb = std::max(gp.dsg, W);
  const int cpad = (n_v + cb - 1) / cb * cb;
  // the Gram kernel keeps the k weights of a column block in LDS
  if ((size_t)gp.k * cb * sb + 4 * 144 * 8 > 60 * 1024) {
    set_error("k too large for the Gram kernel's LDS tile");
    return RDM_E_INVALID;
  }
  gp.header = align_up(2 * sizeof(Seg));
  size_t off = 0;
  plan_seg(gp.tot, h->n, cpad, gp.k, prec, 0, 0, gp.k, off, lanczos_needs_ybuf(h, 0, prec));
  plan_seg(gp.bath, h->n_b, n_v, gp.kb, prec, 0, 0, 2, off, lanczos_needs_ybuf(h, 1, prec));
  gp.n_cblocks = cpad / cb;
  const uint64_t r = (dim * gp.n_cblocks) / (kBlock * 4096ull);
  gp.g_rpl = (int)std::max<uint64_t>(1, std::min<uint64_t>(r, 16));
  gp.g_rtiles = (int)((dim + (uint64_t)kBlock * gp.g_rpl - 1) / ((uint64_t)kBlock * gp.g_rpl));
  const int groups = cpad / gp.dsg;
  gp.o_y = off; off = align_up(off + (size_t)gp.k * cpad * sb);
  gp.o_gpart = off; off = align_up(off + (size_t)gp.g_rtiles * groups * gp.dsg * gp.dsg * 8);
  gp.o_gsum = off; off = align_up(off + (size_t)groups * gp.dsg * gp.dsg * 8);
  gp.o_gseg = off; off = align_up(off + sizeof(GSeg));
  gp.o_gtiles = off; off = align_up(off + sizeof(GTile) * (size_t)gp.g_rtiles * gp.n_cblocks);
  gp.o_w = off; off = align_up(off + (size_t)gp.k * kGroundMaxR * cpad * sb);
  gp.o_gp = off; off = align_up(off + sizeof(GPSeg));
  const uint64_t db = 1ull << h->n_b;
  gp.pt_rpl = (int)std::max<uint64_t>(1, db / ((uint64_t)kBlock * 1024));
  gp.pt_tiles = (int)((db + (uint64_t)kBlock * gp.pt_rpl - 1) / ((uint64_t)kBlock * gp.pt_rpl));
  gp.o_ppart = off; off = align_up(off + (size_t)gp.pt_tiles * gp.ds * gp.ds * 8);
  gp.o_psum = off; off = align_up(off + (size_t)gp.ds * gp.ds * 8);
  gp.bytes = gp.header + off;
  if (budget != 0 && gp.bytes > budget) {
    set_error("ground-state solve needs " + std::to_string(gp.bytes) + " device bytes, budget " +
              std::to_string(budget));
    return RDM_E_NOMEM;
  }
  return RDM_OK;
}

template <typename T>
rdm_status ground_run(const GroundPlan& gp, const rdm_hamiltonian* h, uint64_t seed, double tau, bool graph,
                      char* ws, hipStream_t st, rdm_ground_result* out) {
  const OpDevice *op_t = nullptr, *op_b = nullptr;
  rdm_status s = get_device_op(h, 0, gp.prec, st, &op_t);
  if (s == RDM_OK) s = get_device_op(h, 1, gp.prec, st, &op_b);
  if (s != RDM_OK) return s;
  char* base = ws + gp.header;
  SegPlan tp = gp.tot;
  tp.C = gp.n_v;  // the padding columns start at zero and stay frozen
  std::vector<Seg> segs{make_plain_seg(tp, op_t, base, MODE_LANCZOS, START_BATH, 0, h->n, seed, tau),
                        make_plain_seg(gp.bath, op_b, base, MODE_LANCZOS, START_BATH, 0, h->n_b, seed, tau)};
  if ((s = run_phase(segs, (Seg*)ws, gp.prec, 0, st, nullptr, true, graph)) != RDM_OK) return s;
  std::vector<double> ta, tb, tsc, ba, bb, bsc;
  std::vector<int32_t> tkc, bkc;
  if ((s = fetch_history(gp.tot, base, ta, tb, tsc, tkc, st)) != RDM_OK) return s;
  if ((s = fetch_history(gp.bath, base, ba, bb, bsc, bkc, st)) != RDM_OK) return s;
  RDM_HIP(hipStreamSynchronize(st));
  const int cp = gp.tot.cpad, bcp = gp.bath.cpad, n_v = gp.n_v;
  std::vector<TridiagEig> et(n_v), eb(n_v);
  parallel_jobs(2 * n_v, [&](int t) {
    const bool bath = t >= n_v;
    const int c = bath ? t - n_v : t;
    const std::vector<double>& a = bath ? ba : ta;
    const std::vector<double>& b = bath ? bb : tb;
    const int kk = bath ? bkc[c] : tkc[c];
    const int stride = bath ? bcp : cp;
    std::vector<double> al(kk), be(kk > 0 ? kk - 1 : 0);
    for (int j = 0; j < kk; ++j) al[j] = a[(size_t)j * stride + c];
    for (int j = 0; j + 1 < kk; ++j) be[j] = b[(size_t)j * stride + c];
    (bath ? eb : et)[c].solve(al.data(), be.data(), kk);
  });
  double et_min = INFINITY, eb_min = INFINITY, scale = 0.0;
  std::vector<int> i0(n_v, 0);
  for (int c = 0; c < n_v; ++c) {
    if (!et[c].ok || !eb[c].ok || et[c].n == 0 || eb[c].n == 0) {
      set_error("tridiagonal eigenproblem failed");
      return RDM_E_NONFINITE;
    }
    for (int q = 0; q < et[c].n; ++q) {
      scale = std::max(scale, std::fabs(et[c].theta[q]));
      if (et[c].theta[q] < et[c].theta[i0[c]]) i0[c] = q;
    }
    et_min = std::min(et_min, et[c].theta[i0[c]]);
    for (double x : eb[c].theta) eb_min = std::min(eb_min, x);
  }
  // columns whose lowest Ritz value reached the ground energy
  const double e_tol = (gp.prec == RDM_FP64 ? 1e-9 : 1e-4) * std::max(1.0, scale);
  // convergence measure: the residual norm |H y - theta y| = beta_{k-1} |s_{k-1}|
  // of the lowest Ritz pair of the first k-1 steps (its last eigenvector
  // component times the coupling to step k), largest over the columns that
  // contribute; 0 for a column that reached an invariant subspace (it broke
  // down, or its Krylov space is the whole space), whose Ritz pairs are exact
  double resid = 0.0;
  const bool whole = (uint64_t)gp.k >= (1ull << h->n);
  for (int c = 0; c < n_v; ++c) {
    if (et[c].theta[i0[c]] > et_min + e_tol) continue;
    const int kk = tkc[c];
    if (kk < 2 || kk < gp.k || whole) continue;
    std::vector<double> al(kk - 1), be(kk > 2 ? kk - 2 : 0), sv(kk - 1);
    for (int j = 0; j + 1 < kk; ++j) al[j] = ta[(size_t)j * cp + c];
    for (int j = 0; j + 2 < kk; ++j) be[j] = tb[(size_t)j * cp + c];
    TridiagEig e;
    e.solve(al.data(), be.data(), kk - 1);
    if (!e.ok || e.n == 0) continue;
    int lo = 0;
    for (int q = 1; q < e.n; ++q)
      if (e.theta[q] < e.theta[lo]) lo = q;
    e.eigvec(lo, sv.data());
    resid = std::max(resid, std::fabs(tb[(size_t)(kk - 2) * cp + c] * sv[kk - 2]));
  }
  // Ritz vector weights (times L^-1/2 when the basis is kept as W_lo u)
  const double bscale = op_t->xz ? kXzBasisScale : 1.0;
  std::vector<double> y((size_t)gp.k * cp, 0.0);
  std::vector<std::vector<double>> yc(n_v);
  for (int c = 0; c < n_v; ++c) {
    if (et[c].theta[i0[c]] > et_min + e_tol) continue;
    yc[c].resize(et[c].n);
    et[c].eigvec(i0[c], yc[c].data());
    for (int j = 0; j < et[c].n; ++j) y[(size_t)j * cp + c] = bscale * yc[c][j] * tsc[(size_t)j * cp + c];
  }
  // Gram of the Ritz vectors (hot-path Gram kernel, one group of dsg columns)
  std::vector<T> yt(y.size());
  for (size_t i = 0; i < y.size(); ++i) yt[i] = (T)y[i];
  RDM_HIP(hipMemcpyAsync(base + gp.o_y, yt.data(), yt.size() * sizeof(T), hipMemcpyHostToDevice, st));
  GSeg g{};
  g.Q = base + gp.tot.o_Q;
  g.ytab = base + gp.o_y;
  g.gpart = (double*)(base + gp.o_gpart);
  g.blk = gp.tot.blk;
  g.nbits = gp.tot.nbits;
  g.cpad = cp;
  g.k = gp.k;
  g.n_beta = 1;
  int lg = 0;
  while ((1 << lg) < gp.dsg) ++lg;
  g.n_v = cp / gp.dsg;
  g.ds_log = lg;
  g.rpl = gp.g_rpl;
  g.from_psi = 0;
  g.n_row_tiles = gp.g_rtiles;
  std::vector<GTile> gt;
  for (int rt = 0; rt < gp.g_rtiles; ++rt)
    for (int cb = 0; cb < gp.n_cblocks; ++cb)
      gt.push_back(GTile{0, (uint32_t)((uint64_t)rt * kBlock * gp.g_rpl), cb, rt});
  RDM_HIP(hipMemcpyAsync(base + gp.o_gseg, &g, sizeof(GSeg), hipMemcpyHostToDevice, st));
  RDM_HIP(hipMemcpyAsync(base + gp.o_gtiles, gt.data(), gt.size() * sizeof(GTile), hipMemcpyHostToDevice, st));
  RDM_HIP(launch_gram<T>((GSeg*)(base + gp.o_gseg), (GTile*)(base + gp.o_gtiles), (int)gt.size(), gp.dsg, 1, 0,
                         gp.k, st));
  const int width = g.n_v * gp.dsg * gp.dsg;
  RDM_HIP(launch_colsum((double*)(base + gp.o_gpart), gp.g_rtiles, width, (double*)(base + gp.o_gsum), st));
  std::vector<double> gs(width);
  RDM_HIP(hipMemcpyAsync(gs.data(), base + gp.o_gsum, width * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipStreamSynchronize(st));
  // M (n_v x n_v, the first group) -> orthonormal ground-space basis
  const int D = gp.dsg;
  std::vector<double> m((size_t)D * D, 0.0), lam(D), u((size_t)D * D);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) m[a * D + b] = 0.5 * (gs[a * D + b] + gs[b * D + a]);
  sym_eig_small(D, m.data(), lam.data(), u.data());
  const double lmax = lam[D - 1];
  const double thr = (gp.prec == RDM_FP64 ? 1e-6 : 1e-3) * lmax;
  std::vector<int> keep;
  for (int i = D - 1; i >= 0; --i)
    if (lam[i] > thr) keep.push_back(i);
  const int r = (int)keep.size();
  if (!(lmax > 0.0) || r == 0) {
    set_error("no converged ground-state Ritz vector");
    return RDM_E_NONFINITE;
  }
  if (r > kGroundMaxR) {
    set_error("ground space of dimension " + std::to_string(r) + " exceeds " + std::to_string(kGroundMaxR));
    return RDM_E_INVALID;
  }
  std::vector<T> w((size_t)gp.k * kGroundMaxR * cp, T(0));
  for (int ii = 0; ii < r; ++ii) {
    const int i = keep[ii];
    const double f = 1.0 / std::sqrt(lam[i]);
    for (int c = 0; c < n_v; ++c)
      for (int j = 0; j < gp.k; ++j)
        w[((size_t)j * kGroundMaxR + ii) * cp + c] = (T)(y[(size_t)j * cp + c] * u[c * D + i] * f);
  }
  // the w table is laid out [k][R][cpad] with R = r
  std::vector<T> wr((size_t)gp.k * r * cp);
  for (int j = 0; j < gp.k; ++j)
    for (int ii = 0; ii < r; ++ii)
      for (int c = 0; c < cp; ++c) wr[((size_t)j * r + ii) * cp + c] = w[((size_t)j * kGroundMaxR + ii) * cp + c];
  RDM_HIP(hipMemcpyAsync(base + gp.o_w, wr.data(), wr.size() * sizeof(T), hipMemcpyHostToDevice, st));
  GPSeg p{};
  p.Q = base + gp.tot.o_Q;
  p.w = base + gp.o_w;
  p.part = (double*)(base + gp.o_ppart);
  p.blk = gp.tot.blk;
  p.nbits = h->n;
  p.nb = h->n_b;
  p.cpad = cp;
  p.k = gp.k;
  p.R = r;
  p.rpl = gp.pt_rpl;
  p.n_tiles = gp.pt_tiles;
  RDM_HIP(hipMemcpyAsync(base + gp.o_gp, &p, sizeof(GPSeg), hipMemcpyHostToDevice, st));
  RDM_HIP(launch_ground_ptrace<T>((GPSeg*)(base + gp.o_gp), gp.ds, gp.pt_tiles, st));
  const int ne = gp.ds * gp.ds;
  RDM_HIP(launch_colsum((double*)(base + gp.o_ppart), gp.pt_tiles, ne, (double*)(base + gp.o_psum), st));
  std::vector<double> rho(ne);
  RDM_HIP(hipMemcpyAsync(rho.data(), base + gp.o_psum, ne * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipStreamSynchronize(st));
  const int ds = gp.ds;
  double tr = 0.0;
  for (int a = 0; a < ds; ++a) tr += rho[a * ds + a];
  if (!(tr > 0.0) || !std::isfinite(tr)) {
    set_error("non-finite ground-state partial trace");
    return RDM_E_NONFINITE;
  }
  for (int a = 0; a < ds; ++a)
    for (int b = a; b < ds; ++b) {
      const double v = 0.5 * (rho[a * ds + b] + rho[b * ds + a]) / tr;
      rho[a * ds + b] = rho[b * ds + a] = v;
    }
  if (out->rho) std::memcpy(out->rho, rho.data(), ne * sizeof(double));
  if (out->e_total) *out->e_total = et_min;
  if (out->e_bath) *out->e_bath = eb_min;
  if (out->degeneracy) *out->degeneracy = r;
  if (out->residual) *out->residual = resid;
  if (out->entropy) {
    std::vector<double> ev(ds), vv((size_t)ds * ds);
    sym_eig_small(ds, rho.data(), ev.data(), vv.data());
    double sum = 0.0;
    for (double pr : ev)
      if (pr > 0.0) sum -= pr * std::log(pr);
    *out->entropy = sum;
  }
  return RDM_OK;
}

}  // namespace

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_ground_state(const rdm_hamiltonian* h, int32_t n_v, int32_t k, uint64_t seed,
                                       const rdm_options* opt, void* hip_stream, rdm_ground_result* out) {
  if (!h || !out || n_v < 1 || n_v > 8 || k < 1 || k > 4096) {
    set_error("rdm_ground_state: need a Hamiltonian, a result, 1 <= n_v <= 8 and 1 <= k <= 4096");
    return RDM_E_INVALID;
  }
  const int prec = opt ? opt->precision : RDM_FP64;
  if (prec != RDM_FP64 && prec != RDM_MIXED) {
    set_error("options: precision must be RDM_FP64 or RDM_MIXED");
    return RDM_E_INVALID;
  }
  double tau = opt && opt->tau > 0.0 ? opt->tau : (prec == RDM_FP64 ? 1e-12 : 1e-5);
  uint64_t budget = opt ? opt->hbm_budget : 0;
  if (!budget) {
    size_t fr = 0, tot = 0;
    RDM_HIP(hipMemGetInfo(&fr, &tot));
    budget = fr > (2ull << 30) ? fr - (2ull << 30) : fr / 2;
  }
  GroundPlan gp;
  rdm_status s = ground_plan(gp, h, n_v, k, prec, budget);
  if (s != RDM_OK) return s;
  char* ws = nullptr;
  RDM_HIP(hipMalloc(&ws, gp.bytes));
  hipStream_t st = (hipStream_t)hip_stream;
  const bool graph = !(opt && opt->eager);
  s = prec == RDM_FP64 ? ground_run<double>(gp, h, seed, tau, graph, ws, st, out)
                       : ground_run<float>(gp, h, seed, tau, graph, ws, st, out);
  (void)hipFree(ws);
  return s;
}
