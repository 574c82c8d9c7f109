// Observables of a solve's outputs on the host (d_s x d_s work): the
// internal-energy deviation of Section "Deviation in internal energy"
// (formula:deviation_of_Hamiltonian).
#include <cmath>
#include <vector>

#include "host.h"

using namespace rdm;

extern "C" rdm_status rdm_energy_deviation(const rdm_hamiltonian* h, int32_t n_beta, const double* beta,
                                           const double* rho, const double* h_star, double* out) {
  if (!h || n_beta < 1 || !beta || !rho || !h_star || !out) {
    set_error("rdm_energy_deviation: bad arguments");
    return RDM_E_INVALID;
  }
  for (int b = 0; b < n_beta; ++b)
    if (!(beta[b] > 0.0) || !std::isfinite(beta[b])) {
      set_error("rdm_energy_deviation: every beta must be finite and > 0");
      return RDM_E_INVALID;
    }
  const int ds = 1 << h->n_s;
  std::vector<double> hs((size_t)ds * ds), w(ds), v((size_t)ds * ds);
  rdm_status s = rdm_system_hamiltonian(h, hs.data());
  if (s != RDM_OK) return s;
  // the bare system's thermal state rho_s = exp(-beta H_s) / tr, through the
  // eigenvalues of H_s (shifted by the smallest)
  sym_eig_small(ds, hs.data(), w.data(), v.data());
  for (int b = 0; b < n_beta; ++b) {
    const double* r = rho + (size_t)b * ds * ds;
    const double* hb = h_star + (size_t)b * ds * ds;
    double after = 0.0;  // tr(H* rho*)
    for (int x = 0; x < ds; ++x)
      for (int y = 0; y < ds; ++y) after += hb[x * ds + y] * r[y * ds + x];
    double z = 0.0, e = 0.0;  // tr(H_s rho_s) = sum_i E_i p_i
    for (int i = 0; i < ds; ++i) {
      const double p = std::exp(-beta[b] * (w[i] - w[0]));
      z += p;
      e += p * w[i];
    }
    if (!std::isfinite(after)) {
      set_error("rdm_energy_deviation: non-finite input");
      return RDM_E_NONFINITE;
    }
    out[b] = after - e / z;
  }
  return RDM_OK;
}
