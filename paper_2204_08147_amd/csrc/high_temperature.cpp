// High-temperature offset of the estimated mean force Hamiltonian (Section "A
// note on high temperatures", and the appendix deriving the high-temperature
// limit).
//
// With H_t = H_s (x) I + I (x) H_b + H_sb and unit bath vectors v_j, the
// estimate of H*(beta) built from the n_v bath vectors tends, as beta -> 0,
// to H_s + C with
//     C = (1/n_v) sum_j (I_s (x) <v_j|) H_sb (I_s (x) |v_j>),
// while the exact H*(beta) tends to H_s (every term of H_sb has a traceless
// bath factor).  For a coupling  jx sx_a sx_c + jy sy_a sy_c + jz sz_a sz_c
// between system site a and bath site c the bath factors reduce to the
// expectations <v_j| s_c |v_j>: the sy one vanishes for real v_j (sy is
// antisymmetric), and the sz one vanishes because every entry of v_j has the
// same magnitude (half the diagonal of sz_c is +1, half -1).  Only the sx
// expectations remain; they come from the device as exact integer sums.
#include <cmath>
#include <vector>

#include "host.h"

using namespace rdm;

extern "C" rdm_status rdm_high_temperature_term(const rdm_hamiltonian* h, int32_t n_v, uint64_t seed,
                                                void* hip_stream, double* c_out, double* sx_out) {
  if (!h || !c_out || n_v < 1 || n_v > 65535) {
    set_error("rdm_high_temperature_term: need a Hamiltonian, an output and 1 <= n_v <= 65535");
    return RDM_E_INVALID;
  }
  const int ns = h->n_s, nb = h->n_b, ds = 1 << ns;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nblk = bath_sx_blocks(nb);
  const size_t nent = (size_t)n_v * nblk * nb;
  long long* part = nullptr;
  RDM_HIP(hipMalloc(&part, nent * sizeof(long long)));
  std::vector<long long> hp(nent);
  hipError_t e = launch_bath_sx(seed, nb, n_v, part, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, nent * sizeof(long long), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  if (e != hipSuccess) {
    set_error(std::string("rdm_high_temperature_term: ") + hipGetErrorString(e));
    return RDM_E_DEVICE;
  }
  // (1/n_v) sum_j <v_j| sx |v_j> per bath bit p: total count / (n_v 2^nb)
  std::vector<double> sx_bit(nb);
  for (int p = 0; p < nb; ++p) {
    long long tot = 0;
    for (size_t r = 0; r < (size_t)n_v * nblk; ++r) tot += hp[r * nb + p];
    sx_bit[p] = std::ldexp((double)tot, -nb) / n_v;
  }
  // bath site c (n_s <= c < N) is bath bit n_b - 1 - (c - n_s)
  auto sx_site = [&](int c) { return sx_bit[nb - 1 - (c - ns)]; };
  if (sx_out)
    for (int c = ns; c < ns + nb; ++c) sx_out[c - ns] = sx_site(c);
  for (int i = 0; i < ds * ds; ++i) c_out[i] = 0.0;
  for (const auto& cp : h->couplings) {
    const bool si = cp.i < ns, sj = cp.j < ns;
    if (si == sj) continue;  // H_s or H_b term
    const int a = si ? cp.i : cp.j, c = si ? cp.j : cp.i;
    const double w = cp.jx * sx_site(c);
    const uint32_t f = 1u << (ns - 1 - a);  // system site a is bit n_s-1-a
    for (uint32_t m = 0; m < (uint32_t)ds; ++m) c_out[m * ds + (m ^ f)] += w;
  }
  return RDM_OK;
}
