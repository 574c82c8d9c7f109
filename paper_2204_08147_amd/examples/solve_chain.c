/* Minimal C client of librdm: rho*, ln Z* and the entropy of one spin
 * coupled to a three-spin Heisenberg chain (nearest-neighbour XX + YY + ZZ,
 * J = 1, z-fields 0.2 per site), beta in {0.5, 2}, n_v = 4 bath vectors,
 * k = 16 Lanczos steps, FP64, default stream.  Uses only include/rdm.h.
 *
 *   gcc -std=c99 -I<repo>/include solve_chain.c -L<repo>/paper_2204_08147_amd \
 *       -lrdm -Wl,-rpath,<repo>/paper_2204_08147_amd -o solve_chain
 *
 * Prints one "name beta_index values..." line per output (rho* and H*
 * row-major); exits 1 with the library's
 * error message when a call fails (for instance without a GPU). */
#include <stdio.h>
#include <stdlib.h>

#include "rdm.h"

static int check(rdm_status s, const char* what) {
  if (s != RDM_OK) {
    fprintf(stderr, "%s failed (%d): %s\n", what, (int)s, rdm_last_error());
    return 1;
  }
  return 0;
}

int main(void) {
  enum { N_S = 1, N_B = 3, N = N_S + N_B, N_BETA = 2, D_S = 1 << N_S };
  rdm_coupling cp[N - 1];
  double hx[N], hz[N];
  for (int i = 0; i < N - 1; ++i) {
    cp[i].i = i;
    cp[i].j = i + 1;
    cp[i].jx = cp[i].jy = cp[i].jz = 1.0;
  }
  for (int i = 0; i < N; ++i) {
    hx[i] = 0.0;
    hz[i] = 0.2;
  }
  rdm_hamiltonian* h = NULL;
  if (check(rdm_hamiltonian_create(N_S, N_B, cp, N - 1, hx, hz, &h), "rdm_hamiltonian_create")) return 1;
  const double beta[N_BETA] = {0.5, 2.0};
  double rho[N_BETA * D_S * D_S], h_star[N_BETA * D_S * D_S], log_z[N_BETA], entropy[N_BETA];
  rdm_result out = {rho, h_star, log_z, entropy, NULL};
  const int bad = check(rdm_solve(h, beta, N_BETA, 4, 16, 7, NULL, NULL, &out), "rdm_solve");
  rdm_hamiltonian_destroy(h);
  if (bad) return 1;
  for (int b = 0; b < N_BETA; ++b) {
    printf("rho %d", b);
    for (int q = 0; q < D_S * D_S; ++q) printf(" %.17g", rho[b * D_S * D_S + q]);
    printf("\nh_star %d", b);
    for (int q = 0; q < D_S * D_S; ++q) printf(" %.17g", h_star[b * D_S * D_S + q]);
    printf("\nlog_z %d %.17g\nentropy %d %.17g\n", b, log_z[b], b, entropy[b]);
  }
  return 0;
}
