// Product-state (rank-one) estimator of the total partition function
// (appendix "A consistent partial trace estimator").
//
// Sample j is the unit product vector x_j = |v_s^(j)> (x) |v_j>: v_j is bath
// vector j of the partial-trace estimator and v_s^(j) the same sign rule on
// the system bits with a fixed seed offset.  With E[x x^T] = I / 2^N,
// 2^N <x_j| exp(-beta H_t) |x_j> is unbiased for Z_t, and its conditional
// means over either factor are the quadratic forms of the two partial traces,
// so the trace estimate is the trace of the partial-trace estimates.  One
// column per sample instead of d_s.
//
// The hot-path kernels run Lanczos on the n_v product columns (H_t) and the
// n_v bath vectors (H_b) in one launch sequence; each column's T gives the
// Gauss quadrature e_1^T exp(-beta (T - E0)) e_1 (eqn:fT with block size one),
// with E0 the smallest Ritz value over the columns (overflow shift), on the
// host.
#include <algorithm>
#include <cmath>

#include "host.h"
#include "solve.h"

namespace rdm {

namespace {

struct ProductPlan {
  int prec = RDM_FP64, n_v = 0, k = 0, kb = 0;
  SegPlan tot, bath;
  size_t header = 0, bytes = 0;
};

rdm_status product_plan(ProductPlan& pp, const rdm_hamiltonian* h, int n_v, int k, int prec, uint64_t budget) {
  pp = ProductPlan{};
  pp.prec = prec;
  pp.n_v = n_v;
  pp.k = (int)std::min<uint64_t>((uint64_t)k, 1ull << h->n);
  pp.kb = (int)std::min<uint64_t>((uint64_t)k, 1ull << h->n_b);
  pp.header = align_up(2 * sizeof(Seg));
  size_t off = 0;
  // only the coefficients are needed: two basis slots per segment
  plan_seg(pp.tot, h->n, n_v, pp.k, prec, 0, 0, 2, off, lanczos_needs_ybuf(h, 0, prec));
  plan_seg(pp.bath, h->n_b, n_v, pp.kb, prec, 0, 0, 2, off, lanczos_needs_ybuf(h, 1, prec));
  pp.bytes = pp.header + off;
  if (budget != 0 && pp.bytes > budget) {
    set_error("product-state estimate needs " + std::to_string(pp.bytes) + " device bytes, budget " +
              std::to_string(budget));
    return RDM_E_NOMEM;
  }
  return RDM_OK;
}

double log_mean_exp(const double* x, int n) {
  double m = -INFINITY;
  for (int i = 0; i < n; ++i) m = std::max(m, x[i]);
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += std::exp(x[i] - m);
  return m + std::log(s / n);
}

rdm_status product_run(const ProductPlan& pp, const rdm_hamiltonian* h, const double* betas, int n_beta,
                       uint64_t seed, double tau, bool graph, char* ws, hipStream_t st,
                       rdm_product_result* out) {
  const OpDevice *op_t = nullptr, *op_b = nullptr;
  rdm_status s = get_device_op(h, 0, pp.prec, st, &op_t);
  if (s == RDM_OK) s = get_device_op(h, 1, pp.prec, st, &op_b);
  if (s != RDM_OK) return s;
  char* base = ws + pp.header;
  std::vector<Seg> segs{make_plain_seg(pp.tot, op_t, base, MODE_LANCZOS, START_PRODUCT, h->n_s, h->n_b, seed, tau),
                        make_plain_seg(pp.bath, op_b, base, MODE_LANCZOS, START_BATH, 0, h->n_b, seed, tau)};
  if ((s = run_phase(segs, (Seg*)ws, pp.prec, 0, st, nullptr, true, graph)) != RDM_OK) return s;
  std::vector<double> ta, tb, tsc, ba, bb, bsc;
  std::vector<int32_t> tkc, bkc;
  if ((s = fetch_history(pp.tot, base, ta, tb, tsc, tkc, st)) != RDM_OK) return s;
  if ((s = fetch_history(pp.bath, base, ba, bb, bsc, bkc, st)) != RDM_OK) return s;
  RDM_HIP(hipStreamSynchronize(st));
  const int n_v = pp.n_v;
  std::vector<TridiagEig> et(n_v), eb(n_v);
  parallel_jobs(2 * n_v, [&](int t) {
    const bool bath = t >= n_v;
    const int c = bath ? t - n_v : t;
    const std::vector<double>& a = bath ? ba : ta;
    const std::vector<double>& b = bath ? bb : tb;
    const int kk = bath ? bkc[c] : tkc[c];
    const int stride = bath ? pp.bath.cpad : pp.tot.cpad;
    std::vector<double> al(kk), be(kk > 0 ? kk - 1 : 0);
    for (int j = 0; j < kk; ++j) al[j] = a[(size_t)j * stride + c];
    for (int j = 0; j + 1 < kk; ++j) be[j] = b[(size_t)j * stride + c];
    (bath ? eb : et)[c].solve(al.data(), be.data(), kk);
  });
  double e0 = INFINITY, e0b = INFINITY;
  for (int c = 0; c < n_v; ++c) {
    if (!et[c].ok || !eb[c].ok || et[c].n == 0 || eb[c].n == 0) {
      set_error("tridiagonal eigenproblem failed");
      return RDM_E_NONFINITE;
    }
    for (double x : et[c].theta) e0 = std::min(e0, x);
    for (double x : eb[c].theta) e0b = std::min(e0b, x);
  }
  const double ln2 = std::log(2.0);
  std::vector<double> lt(n_v), lb(n_v);
  for (int bi = 0; bi < n_beta; ++bi) {
    const double beta = betas[bi];
    for (int c = 0; c < n_v; ++c) {
      double wt = 0.0, wb = 0.0;
      for (int q = 0; q < et[c].n; ++q) wt += et[c].zrow[q] * et[c].zrow[q] * std::exp(-beta * (et[c].theta[q] - e0));
      for (int q = 0; q < eb[c].n; ++q) wb += eb[c].zrow[q] * eb[c].zrow[q] * std::exp(-beta * (eb[c].theta[q] - e0b));
      // x^T f(H) x = |x|^2 e_1^T f(T) e_1, |x| = 1 / s_1 (unit up to rounding)
      const double st1 = tsc[c], sb1 = bsc[c];
      lt[c] = std::log(wt / (st1 * st1)) - beta * e0 + h->n * ln2;
      lb[c] = std::log(wb / (sb1 * sb1)) - beta * e0b + h->n_b * ln2;
      if (!std::isfinite(lt[c]) || !std::isfinite(lb[c])) {
        set_error("non-finite quadrature value");
        return RDM_E_NONFINITE;
      }
      if (out->samples) out->samples[(size_t)bi * n_v + c] = lt[c];
    }
    const double zt = log_mean_exp(lt.data(), n_v), zb = log_mean_exp(lb.data(), n_v);
    if (out->log_z) out->log_z[bi] = zt - zb;
    if (out->log_z_t) out->log_z_t[bi] = zt;
    if (out->log_z_b) out->log_z_b[bi] = zb;
  }
  return RDM_OK;
}

}  // namespace

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_product_trace(const rdm_hamiltonian* h, const double* betas, int32_t n_beta, int32_t n_v,
                                        int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                                        rdm_product_result* out) {
  if (!h || !betas || !out || n_beta < 1 || n_v < 1 || n_v > 4096 || k < 1 || k > 4096) {
    set_error("rdm_product_trace: need a Hamiltonian, betas, a result, 1 <= n_v <= 4096 and 1 <= k <= 4096");
    return RDM_E_INVALID;
  }
  for (int i = 0; i < n_beta; ++i)
    if (!(betas[i] >= 0.0) || !std::isfinite(betas[i])) {
      set_error("rdm_product_trace: every beta must be finite and >= 0");
      return RDM_E_INVALID;
    }
  const int prec = opt ? opt->precision : RDM_FP64;
  if (prec != RDM_FP64 && prec != RDM_MIXED) {
    set_error("options: precision must be RDM_FP64 or RDM_MIXED");
    return RDM_E_INVALID;
  }
  const double tau = opt && opt->tau > 0.0 ? opt->tau : (prec == RDM_FP64 ? 1e-12 : 1e-5);
  uint64_t budget = opt ? opt->hbm_budget : 0;
  if (!budget) {
    size_t fr = 0, tot = 0;
    RDM_HIP(hipMemGetInfo(&fr, &tot));
    budget = fr > (2ull << 30) ? fr - (2ull << 30) : fr / 2;
  }
  ProductPlan pp;
  rdm_status s = product_plan(pp, h, n_v, k, prec, budget);
  if (s != RDM_OK) return s;
  char* ws = nullptr;
  RDM_HIP(hipMalloc(&ws, pp.bytes));
  const bool graph = !(opt && opt->eager);
  s = product_run(pp, h, betas, n_beta, seed, tau, graph, ws, (hipStream_t)hip_stream, out);
  (void)hipFree(ws);
  return s;
}
