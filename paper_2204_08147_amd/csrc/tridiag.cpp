// Small dense eigenproblems on the host: the tridiagonal Lanczos matrices T_k
// (function-approximation weights and Gauss quadrature, eqn:fT) and the
// averaged d_s x d_s matrix of the finalisation (eigenvalue route of the
// paper's estimator section, no matrix logarithm).
#include <algorithm>
#include <cmath>

#include "host.h"

namespace rdm {

// Implicit symmetric QR on a tridiagonal matrix with Wilkinson shifts
// (Golub & Van Loan, "Matrix Computations", the implicit symmetric QR step).
// Each step chases a bulge with Givens rotations G acting on rows/columns
// (i, i+1); T <- G^T T G.  The eigenvector matrix would be Z = G_1 G_2 ... ;
// it is never formed: its first row is accumulated directly, and products
// Z w are formed later by replaying the rotations backwards.
void TridiagEig::solve(const double* alpha, const double* beta, int nn) {
  n = nn;
  theta.assign(alpha, alpha + n);
  std::vector<double> e(n > 1 ? n - 1 : 0);
  for (int i = 0; i + 1 < n; ++i) e[i] = beta[i];
  zrow.assign(n, 0.0);
  if (n > 0) zrow[0] = 1.0;
  rot_i.clear();
  rot_c.clear();
  rot_s.clear();
  ok = true;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iters = 0;
  const int max_iters = 60 * std::max(n, 1);
  while (hi > 0) {
    // deflate negligible off-diagonals at the bottom
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(theta[hi - 1]) + std::fabs(theta[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    // find the top of the unreduced block ending at hi
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(theta[lo - 1]) + std::fabs(theta[lo])))
      --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    if (++iters > max_iters) {
      ok = false;
      return;
    }
    // Wilkinson shift from the trailing 2x2 of the block
    const double d = 0.5 * (theta[hi - 1] - theta[hi]);
    const double b2 = e[hi - 1] * e[hi - 1];
    const double den = d + (d >= 0.0 ? 1.0 : -1.0) * std::hypot(d, e[hi - 1]);
    const double mu = theta[hi] - b2 / den;
    double x = theta[lo] - mu;
    double z = e[lo];
    double bulge = 0.0;
    for (int i = lo; i < hi; ++i) {
      // rotation zeroing z against x: c x - s z = r, s x + c z = 0
      const double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -z / r;
      }
      if (i > lo) e[i - 1] = r;  // T[i, i-1] after eliminating the bulge T[i+1, i-1]
      const double a0 = theta[i], a1 = theta[i + 1], b = e[i];
      theta[i] = c * c * a0 - 2.0 * c * s * b + s * s * a1;
      theta[i + 1] = s * s * a0 + 2.0 * c * s * b + c * c * a1;
      e[i] = c * s * (a0 - a1) + (c * c - s * s) * b;
      if (i + 1 < hi) {
        bulge = -s * e[i + 1];
        e[i + 1] = c * e[i + 1];
        x = e[i];
        z = bulge;
      }
      // first row of Z <- Z G
      const double z0 = zrow[i], z1 = zrow[i + 1];
      zrow[i] = c * z0 - s * z1;
      zrow[i + 1] = s * z0 + c * z1;
      rot_i.push_back(i);
      rot_c.push_back(c);
      rot_s.push_back(s);
    }
  }
}

void TridiagEig::apply_fn(const double* g, double* y) const {
  for (int i = 0; i < n; ++i) y[i] = g[i] * zrow[i];
  // Z w = G_1 (G_2 (... (G_M w)))
  for (size_t t = rot_i.size(); t-- > 0;) {
    const int i = rot_i[t];
    const double c = rot_c[t], s = rot_s[t];
    const double w0 = y[i], w1 = y[i + 1];
    y[i] = c * w0 + s * w1;
    y[i + 1] = -s * w0 + c * w1;
  }
}

void sym_eig_small(int n, const double* a_in, double* w, double* v) {
  double a[16 * 16];
  for (int i = 0; i < n * n; ++i) a[i] = a_in[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        // rotation annihilating a[p][q]
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  // sort ascending
  int idx[16];
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx, idx + n, [&](int x, int y) { return a[x * n + x] < a[y * n + y]; });
  double vv[16 * 16];
  for (int j = 0; j < n; ++j) {
    w[j] = a[idx[j] * n + idx[j]];
    for (int i = 0; i < n; ++i) vv[i * n + j] = v[i * n + idx[j]];
  }
  for (int i = 0; i < n * n; ++i) v[i] = vv[i];
}

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_tridiag_fa(int32_t kk, const double* alpha, const double* beta,
                                     int32_t n_beta, const double* betas, double e0, double* theta,
                                     double* y, double* quad) {
  if (kk < 1 || !alpha || (kk > 1 && !beta) || n_beta < 0 || (n_beta > 0 && !betas)) {
    set_error("rdm_tridiag_fa: bad arguments");
    return RDM_E_INVALID;
  }
  TridiagEig te;
  te.solve(alpha, beta, kk);
  if (!te.ok) {
    set_error("rdm_tridiag_fa: QR iteration did not converge");
    return RDM_E_NONFINITE;
  }
  if (theta)
    for (int i = 0; i < kk; ++i) theta[i] = te.theta[i];
  std::vector<double> g(kk);
  for (int b = 0; b < n_beta; ++b) {
    for (int i = 0; i < kk; ++i) g[i] = std::exp(-0.5 * betas[b] * (te.theta[i] - e0));
    if (y) te.apply_fn(g.data(), y + (size_t)b * kk);
    if (quad) {
      double q = 0.0;
      for (int i = 0; i < kk; ++i) q += te.zrow[i] * te.zrow[i] * g[i] * g[i];
      quad[b] = q;
    }
  }
  return RDM_OK;
}
