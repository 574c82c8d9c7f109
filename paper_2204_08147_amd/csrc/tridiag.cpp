// Small dense eigenproblems on the host: the tridiagonal Lanczos matrices T_k
// (function-approximation weights and Gauss quadrature, eqn:fT) and the
// averaged d_s x d_s matrix of the finalisation (eigenvalue route of the
// paper's estimator section, no matrix logarithm).
#include <algorithm>
#include <cmath>

#include "host.h"

namespace rdm {

namespace {

// sqrt(x^2 + z^2): the plain form (the entries are bounded by the norm of H),
// library hypot only where the squares would overflow or lose precision
inline double norm2(double x, double z) {
  const double q = x * x + z * z;
  if (q > 1e-280 && q < 1e280) return std::sqrt(q);
  return std::hypot(x, z);
}

}  // namespace

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
  const size_t guess = (size_t)3 * n * n + 16;
  rot_i.reserve(guess);
  rot_c.reserve(guess);
  rot_s.reserve(guess);
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
    const double den = d + (d >= 0.0 ? 1.0 : -1.0) * norm2(d, e[hi - 1]);
    const double mu = theta[hi] - b2 / den;
    double x = theta[lo] - mu;
    double z = e[lo];
    double bulge = 0.0;
    for (int i = lo; i < hi; ++i) {
      // rotation zeroing z against x: c x - s z = r, s x + c z = 0
      const double r = norm2(x, z);
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

void TridiagEig::apply_fn_multi(int nf, const double* g, double* y) const {
  // the same replay as apply_fn for nf vectors at once, interleaved so that
  // the updates of one rotation are independent of each other
  std::vector<double> w((size_t)n * nf);
  for (int i = 0; i < n; ++i)
    for (int f = 0; f < nf; ++f) w[(size_t)i * nf + f] = g[(size_t)f * n + i] * zrow[i];
  for (size_t t = rot_i.size(); t-- > 0;) {
    double* w0 = w.data() + (size_t)rot_i[t] * nf;
    double* w1 = w0 + nf;
    const double c = rot_c[t], s = rot_s[t];
    for (int f = 0; f < nf; ++f) {
      const double a0 = w0[f], a1 = w1[f];
      w0[f] = c * a0 + s * a1;
      w1[f] = -s * a0 + c * a1;
    }
  }
  for (int f = 0; f < nf; ++f)
    for (int i = 0; i < n; ++i) y[(size_t)f * n + i] = w[(size_t)i * nf + f];
}

void TridiagEig::apply_st_multi(int nf, double* w) const {
  // S^T = G_M^T ... G_1^T: the rotations in recorded order, transposed
  for (size_t t = 0; t < rot_i.size(); ++t) {
    double* w0 = w + (size_t)rot_i[t] * nf;
    double* w1 = w0 + nf;
    const double c = rot_c[t], s = rot_s[t];
    for (int f = 0; f < nf; ++f) {
      const double a0 = w0[f], a1 = w1[f];
      w0[f] = c * a0 - s * a1;
      w1[f] = s * a0 + c * a1;
    }
  }
}

void TridiagEig::apply_fn_vec(const double* g, const double* x, double* y) const {
  // S^T x = G_M^T (... (G_1^T x)): the rotations in recorded order, transposed
  for (int i = 0; i < n; ++i) y[i] = x[i];
  for (size_t t = 0; t < rot_i.size(); ++t) {
    const int i = rot_i[t];
    const double c = rot_c[t], s = rot_s[t];
    const double w0 = y[i], w1 = y[i + 1];
    y[i] = c * w0 - s * w1;
    y[i + 1] = s * w0 + c * w1;
  }
  for (int i = 0; i < n; ++i) y[i] *= g[i];
  for (size_t t = rot_i.size(); t-- > 0;) {
    const int i = rot_i[t];
    const double c = rot_c[t], s = rot_s[t];
    const double w0 = y[i], w1 = y[i + 1];
    y[i] = c * w0 + s * w1;
    y[i + 1] = -s * w0 + c * w1;
  }
}

void TridiagEig::eigvec(int i0, double* y) const {
  for (int i = 0; i < n; ++i) y[i] = i == i0 ? 1.0 : 0.0;
  for (size_t t = rot_i.size(); t-- > 0;) {
    const int i = rot_i[t];
    const double c = rot_c[t], s = rot_s[t];
    const double w0 = y[i], w1 = y[i + 1];
    y[i] = c * w0 + s * w1;
    y[i + 1] = -s * w0 + c * w1;
  }
}

// Householder tridiagonalisation (Golub & Van Loan, symmetric Householder
// reduction): for k = 0..n-3 the reflector H = I - tau v v^T on rows/columns
// k+1.. maps column k below the diagonal onto a multiple of e_1; the trailing
// block B becomes H B H = B - v w^T - w v^T with p = tau B v and
// w = p - (tau/2)(v^T p) v.  P accumulates H_0 H_1 ..., so A = P T P^T.
void DenseSymEig::solve(const double* a_in, int nn, int bb) {
  n = nn;
  b = bb;
  std::vector<double> a(a_in, a_in + (size_t)n * n);
  // only the first b rows of P are needed (the leading block of f(A))
  std::vector<double> p((size_t)b * n, 0.0);
  for (int i = 0; i < b; ++i) p[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), pv(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double xn = 0.0;
    for (int i = 0; i < m; ++i) xn += a[(size_t)(k + 1 + i) * n + k] * a[(size_t)(k + 1 + i) * n + k];
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double x0 = a[(size_t)(k + 1) * n + k];
    const double alpha = x0 >= 0.0 ? -xn : xn;
    for (int i = 0; i < m; ++i) v[i] = a[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    double vp = 0.0;
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int jj = 0; jj < m; ++jj) acc += a[(size_t)(k + 1 + i) * n + (k + 1 + jj)] * v[jj];
      pv[i] = tau * acc;
      vp += v[i] * pv[i];
    }
    for (int i = 0; i < m; ++i) w[i] = pv[i] - 0.5 * tau * vp * v[i];
    for (int i = 0; i < m; ++i)
      for (int jj = 0; jj < m; ++jj)
        a[(size_t)(k + 1 + i) * n + (k + 1 + jj)] -= v[i] * w[jj] + w[i] * v[jj];
    a[(size_t)(k + 1) * n + k] = a[(size_t)k * n + (k + 1)] = alpha;
    for (int i = 1; i < m; ++i) a[(size_t)(k + 1 + i) * n + k] = a[(size_t)k * n + (k + 1 + i)] = 0.0;
    // P <- P H on columns k+1.. (rows 0..b-1)
    for (int r = 0; r < b; ++r) {
      double acc = 0.0;
      for (int i = 0; i < m; ++i) acc += p[(size_t)r * n + (k + 1 + i)] * v[i];
      acc *= tau;
      for (int i = 0; i < m; ++i) p[(size_t)r * n + (k + 1 + i)] -= acc * v[i];
    }
  }
  std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];
  te.solve(d.data(), e.data(), n);
  ok = te.ok;
  // Z = S^T P_b^T: one replay of the rotations over the b columns
  z.assign((size_t)n * b, 0.0);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < b; ++m) z[(size_t)i * b + m] = p[(size_t)m * n + i];
  if (ok) te.apply_st_multi(b, z.data());
}

double DenseSymEig::min_eig() const {
  double m = INFINITY;
  for (double t : te.theta) m = std::min(m, t);
  return m;
}

void DenseSymEig::quad(double beta, double e0, double* f) const {
  for (int q = 0; q < b * b; ++q) f[q] = 0.0;
  for (int i = 0; i < n; ++i) {
    const double g = std::exp(-beta * (te.theta[i] - e0));
    const double* zi = z.data() + (size_t)i * b;
    for (int r = 0; r < b; ++r)
      for (int m = 0; m < b; ++m) f[r * b + m] += zi[r] * g * zi[m];
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
  std::vector<double> g((size_t)n_beta * kk);
  for (int b = 0; b < n_beta; ++b) {
    double* gb = g.data() + (size_t)b * kk;
    for (int i = 0; i < kk; ++i) gb[i] = std::exp(-0.5 * betas[b] * (te.theta[i] - e0));
    if (quad) {
      double q = 0.0;
      for (int i = 0; i < kk; ++i) q += te.zrow[i] * te.zrow[i] * gb[i] * gb[i];
      quad[b] = q;
    }
  }
  if (y && n_beta > 0) te.apply_fn_multi(n_beta, g.data(), y);
  return RDM_OK;
}

extern "C" rdm_status rdm_block_quadrature(int32_t n, int32_t b, const double* t, int32_t n_beta,
                                           const double* betas, double e0, double* min_eig, double* f) {
  if (n < 1 || b < 1 || b > n || !t || n_beta < 0 || (n_beta > 0 && (!betas || !f))) {
    set_error("rdm_block_quadrature: bad arguments");
    return RDM_E_INVALID;
  }
  DenseSymEig de;
  de.solve(t, n, b);
  if (!de.ok) {
    set_error("rdm_block_quadrature: QR iteration did not converge");
    return RDM_E_NONFINITE;
  }
  if (min_eig) *min_eig = de.min_eig();
  for (int q = 0; q < n_beta; ++q) de.quad(betas[q], e0, f + (size_t)q * b * b);
  return RDM_OK;
}
