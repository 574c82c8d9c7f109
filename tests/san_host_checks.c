/* Host-side entry points of librdm under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_san_host.py): every call
 * here runs on the host only (Hamiltonian compilation and validation, the
 * tridiagonal and block quadratures, the energy deviation), so no GPU is
 * needed.  Exits 0 when every check holds; a sanitizer report aborts. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rdm.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);    \
      return 1;                                                         \
    }                                                                   \
  } while (0)

static int hamiltonians(void) {
  /* every term type, duplicates summed, every apply kind, several sizes */
  for (int n = 4; n <= 20; n += 4) {
    int n_s = n < 8 ? 1 : 2, n_b = n - n_s, nc = 0;
    rdm_coupling cps[256];
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n && nc < 250; j += 1 + (i % 3)) {
        rdm_coupling c = {i, j, 0.3 * (i + 1), (i + j) % 3 ? 0.2 : 0.0, -0.1 * j};
        cps[nc++] = c;
      }
    rdm_coupling dup = {1, 0, 0.5, 0.5, 0.0};
    cps[nc++] = dup;
    double* hx = malloc(sizeof(double) * n);
    double* hz = malloc(sizeof(double) * n);
    for (int s = 0; s < n; ++s) {
      hx[s] = 0.1 * s;
      hz[s] = -0.05 * s;
    }
    for (int kind = RDM_APPLY_AUTO; kind <= RDM_APPLY_HOPS_ROWS; ++kind) {
      rdm_hamiltonian* h = NULL;
      CHECK(rdm_hamiltonian_create_ex(n_s, n_b, cps, nc, hx, hz, kind, &h) == RDM_OK);
      int64_t info[21];
      CHECK(rdm_hamiltonian_info(h, info) == RDM_OK && info[0] == n);
      /* bit-set tiles only from 12 sites on, never with the transform or on request of row tiles */
      CHECK(info[17] == 0 || (n >= 12 && info[13] == 0 && kind != RDM_APPLY_HOPS_ROWS));
      CHECK(info[19] >= 0 && (n >= 12 || info[19] == 0));
      int ds = 1 << n_s;
      double* m = malloc(sizeof(double) * ds * ds);
      CHECK(rdm_system_hamiltonian(h, m) == RDM_OK);
      for (int a = 0; a < ds; ++a)
        for (int b = 0; b < ds; ++b) CHECK(fabs(m[a * ds + b] - m[b * ds + a]) < 1e-14);
      /* deviation: zero for H* = H_s and rho* = the bare thermal state's
         diagonal case is not needed here, only that it runs and is finite */
      double rho[64] = {0}, hs[64] = {0}, beta = 0.7, dev = 0;
      for (int a = 0; a < ds; ++a) rho[a * ds + a] = 1.0 / ds;
      for (int a = 0; a < ds * ds; ++a) hs[a] = m[a];
      CHECK(rdm_energy_deviation(h, 1, &beta, rho, hs, &dev) == RDM_OK && isfinite(dev));
      free(m);
      rdm_hamiltonian_destroy(h);
    }
    free(hx);
    free(hz);
  }
  /* invalid arguments are rejected with a message */
  rdm_hamiltonian* h = NULL;
  rdm_coupling bad = {0, 0, 1.0, 0.0, 0.0};
  CHECK(rdm_hamiltonian_create(1, 3, &bad, 1, NULL, NULL, &h) == RDM_E_INVALID && h == NULL);
  CHECK(rdm_last_error()[0] != '\0');
  CHECK(rdm_hamiltonian_create(0, 3, NULL, 0, NULL, NULL, &h) == RDM_E_INVALID);
  CHECK(rdm_hamiltonian_create_ex(1, 3, NULL, 0, NULL, NULL, 9, &h) == RDM_E_INVALID);
  return 0;
}

static int quadratures(void) {
  /* tridiagonal eigenproblems of several orders; block quadratures */
  for (int kk = 1; kk <= 80; kk += 13) {
    double* a = malloc(sizeof(double) * kk);
    double* b = malloc(sizeof(double) * kk);
    for (int j = 0; j < kk; ++j) {
      a[j] = sin(1.0 + j);
      b[j] = 0.5 + 0.3 * cos(2.0 * j);
    }
    double betas[3] = {0.1, 1.0, 5.0}, quad[3];
    double* theta = malloc(sizeof(double) * kk);
    double* y = malloc(sizeof(double) * 3 * kk);
    CHECK(rdm_tridiag_fa(kk, a, kk > 1 ? b : NULL, 3, betas, -3.0, theta, y, quad) == RDM_OK);
    for (int q = 0; q < 3; ++q) CHECK(isfinite(quad[q]) && quad[q] > 0);
    free(a);
    free(b);
    free(theta);
    free(y);
  }
  for (int n = 2; n <= 64; n *= 2) {
    int bsz = n >= 8 ? 4 : 1;
    double* t = malloc(sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) t[i * n + j] = cos(i + j) + (i == j ? 2.0 : 0.0);
    double betas[2] = {0.5, 2.0}, mn = 0;
    double* f = malloc(sizeof(double) * 2 * bsz * bsz);
    CHECK(rdm_block_quadrature(n, bsz, t, 2, betas, -5.0, &mn, f) == RDM_OK);
    for (int i = 0; i < 2 * bsz * bsz; ++i) CHECK(isfinite(f[i]));
    free(t);
    free(f);
  }
  return 0;
}

int main(void) {
  if (hamiltonians() || quadratures()) return 1;
  printf("host checks passed\n");
  return 0;
}
