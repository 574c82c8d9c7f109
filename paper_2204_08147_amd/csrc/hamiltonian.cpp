// Hamiltonian construction: validation and compilation of eqn:Ht into the
// apply kernel's term tables.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>

#include "host.h"

namespace rdm {

namespace {

thread_local std::string g_err;

bool is_fin(double x) { return std::isfinite(x); }

// Compile the terms acting only on sites >= first_site (bath: first_site =
// n_s) or all sites (first_site = 0).  Site s is bit (n-1-s) of the full
// index; the bath operator uses the same bits (they are the low n_b bits).
void compile(const rdm_hamiltonian& h, int first_site, OpTables& t) {
  const int n = h.n;
  t = OpTables{};
  t.nbits = n - first_site;
  std::map<std::pair<int, int>, rdm_coupling> pairs;  // duplicates summed in input order
  for (const auto& c : h.couplings) {
    int i = c.i, j = c.j;
    if (i > j) std::swap(i, j);
    if (i < first_site) continue;
    auto it = pairs.find({i, j});
    if (it == pairs.end()) {
      pairs[{i, j}] = rdm_coupling{i, j, c.jx, c.jy, c.jz};
    } else {
      it->second.jx += c.jx;
      it->second.jy += c.jy;
      it->second.jz += c.jz;
    }
  }
  for (const auto& kv : pairs) {
    const rdm_coupling& c = kv.second;
    const uint32_t bi = 1u << (n - 1 - c.i), bj = 1u << (n - 1 - c.j);
    const uint32_t f = bi | bj;
    if (c.jz != 0.0) t.diag.push_back(DiagTerm{f, 0, c.jz});
    // sx sx + sy sy on (i, j): flips both bits with coefficient jx - jy when
    // the bits agree and jx + jy when they differ
    const double cs = c.jx - c.jy, cd = c.jx + c.jy;
    if (cs == 0.0 && cd == 0.0) continue;
    if (cs == cd) {
      t.uf.push_back(f);
      t.uc.push_back(cs);
    } else {
      t.pf.push_back(f);
      t.pm.push_back(f);
      t.pcs.push_back(cs);
      t.pcd.push_back(cd);
    }
  }
  for (int s = first_site; s < n; ++s) {
    const uint32_t b = 1u << (n - 1 - s);
    if (h.hz[s] != 0.0) t.diag.push_back(DiagTerm{b, 0, h.hz[s]});
    if (h.hx[s] != 0.0) {
      t.uf.push_back(b);
      t.uc.push_back(h.hx[s]);
    }
  }
  // parity hops whose tested bits are all >= 6 first: within a wave of 64
  // consecutive rows their coefficient is uniform
  std::vector<size_t> order(t.pf.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return ((t.pm[a] & 63u) == 0u) > ((t.pm[b] & 63u) == 0u);
  });
  OpTables s2 = t;
  for (size_t i = 0; i < order.size(); ++i) {
    t.pf[i] = s2.pf[order[i]];
    t.pm[i] = s2.pm[order[i]];
    t.pcs[i] = s2.pcs[order[i]];
    t.pcd[i] = s2.pcd[order[i]];
  }
  t.nPh = 0;
  for (size_t i = 0; i < t.pm.size(); ++i) t.nPh += (t.pm[i] & 63u) == 0u;
}

template <typename T>
rdm_status upload(const OpTables& t, OpDevice& d, hipStream_t st) {
  std::vector<HopU<T>> hu(t.uf.size());
  for (size_t i = 0; i < hu.size(); ++i) hu[i] = HopU<T>{t.uf[i], 0, (T)t.uc[i]};
  std::vector<HopP<T>> hp(t.pf.size());
  for (size_t i = 0; i < hp.size(); ++i) hp[i] = HopP<T>{t.pf[i], t.pm[i], (T)t.pcs[i], (T)t.pcd[i]};
  const size_t dim = size_t(1) << t.nbits;
  RDM_HIP(hipMalloc(&d.hopU, std::max<size_t>(16, hu.size() * sizeof(HopU<T>))));
  RDM_HIP(hipMalloc(&d.hopP, std::max<size_t>(16, hp.size() * sizeof(HopP<T>))));
  RDM_HIP(hipMalloc(&d.dterms, std::max<size_t>(16, t.diag.size() * sizeof(DiagTerm))));
  RDM_HIP(hipMalloc(&d.diag, dim * sizeof(T)));
  if (!hu.empty())
    RDM_HIP(hipMemcpyAsync(d.hopU, hu.data(), hu.size() * sizeof(HopU<T>), hipMemcpyHostToDevice, st));
  if (!hp.empty())
    RDM_HIP(hipMemcpyAsync(d.hopP, hp.data(), hp.size() * sizeof(HopP<T>), hipMemcpyHostToDevice, st));
  if (!t.diag.empty())
    RDM_HIP(hipMemcpyAsync(d.dterms, t.diag.data(), t.diag.size() * sizeof(DiagTerm),
                           hipMemcpyHostToDevice, st));
  RDM_HIP(launch_diag<T>((const DiagTerm*)d.dterms, (int)t.diag.size(), (T*)d.diag, t.nbits, st));
  RDM_HIP(hipStreamSynchronize(st));
  d.nU = (int)hu.size();
  d.nP = (int)hp.size();
  d.nPh = t.nPh;
  d.ready = true;
  return RDM_OK;
}

void free_dev(rdm::OpDevice& d) {
  if (d.hopU) (void)hipFree(d.hopU);
  if (d.hopP) (void)hipFree(d.hopP);
  if (d.diag) (void)hipFree(d.diag);
  if (d.dterms) (void)hipFree(d.dterms);
  d = rdm::OpDevice{};
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

rdm_status get_device_op(const rdm_hamiltonian* h, int which, int precision, hipStream_t st,
                         const OpDevice** out) {
  std::lock_guard<std::mutex> lk(h->mu);
  int dev = 0;
  RDM_HIP(hipGetDevice(&dev));
  OpDevice& d = h->dev[which][precision];
  if (d.ready && d.device != dev) free_dev(d);
  if (!d.ready) {
    d.device = dev;
    rdm_status s = precision == RDM_FP64 ? upload<double>(h->op[which], d, st)
                                         : upload<float>(h->op[which], d, st);
    if (s != RDM_OK) {
      free_dev(d);
      return s;
    }
  }
  *out = &d;
  return RDM_OK;
}

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_hamiltonian_create(int32_t n_s, int32_t n_b, const rdm_coupling* couplings,
                                             int64_t n_couplings, const double* hx, const double* hz,
                                             rdm_hamiltonian** out) {
  if (!out) {
    set_error("rdm_hamiltonian_create: out is NULL");
    return RDM_E_INVALID;
  }
  *out = nullptr;
  if (n_s < 1 || n_s > 3 || n_b < 1 || n_s + n_b > 28) {
    set_error("rdm_hamiltonian_create: need 1 <= n_s <= 3, n_b >= 1, n_s + n_b <= 28");
    return RDM_E_INVALID;
  }
  if (n_couplings < 0 || (n_couplings > 0 && !couplings)) {
    set_error("rdm_hamiltonian_create: bad coupling list");
    return RDM_E_INVALID;
  }
  const int n = n_s + n_b;
  for (int64_t t = 0; t < n_couplings; ++t) {
    const rdm_coupling& c = couplings[t];
    if (c.i < 0 || c.j < 0 || c.i >= n || c.j >= n || c.i == c.j) {
      set_error("rdm_hamiltonian_create: coupling " + std::to_string(t) + " has bad sites");
      return RDM_E_INVALID;
    }
    if (!is_fin(c.jx) || !is_fin(c.jy) || !is_fin(c.jz)) {
      set_error("rdm_hamiltonian_create: coupling " + std::to_string(t) + " is not finite");
      return RDM_E_INVALID;
    }
  }
  for (int s = 0; s < n; ++s) {
    if ((hx && !is_fin(hx[s])) || (hz && !is_fin(hz[s]))) {
      set_error("rdm_hamiltonian_create: field on site " + std::to_string(s) + " is not finite");
      return RDM_E_INVALID;
    }
  }
  auto* h = new rdm_hamiltonian();
  h->n_s = n_s;
  h->n_b = n_b;
  h->n = n;
  h->couplings.assign(couplings, couplings + n_couplings);
  h->hx.assign(n, 0.0);
  h->hz.assign(n, 0.0);
  for (int s = 0; s < n; ++s) {
    if (hx) h->hx[s] = hx[s];
    if (hz) h->hz[s] = hz[s];
  }
  compile(*h, 0, h->op[0]);
  compile(*h, n_s, h->op[1]);
  *out = h;
  return RDM_OK;
}

extern "C" void rdm_hamiltonian_destroy(rdm_hamiltonian* h) {
  if (!h) return;
  for (auto& w : h->dev)
    for (auto& d : w) free_dev(d);
  delete h;
}

extern "C" rdm_status rdm_hamiltonian_info(const rdm_hamiltonian* h, int64_t* out) {
  if (!h || !out) {
    set_error("rdm_hamiltonian_info: NULL argument");
    return RDM_E_INVALID;
  }
  out[0] = h->n;
  out[1] = h->n_s;
  out[2] = h->n_b;
  for (int w = 0; w < 2; ++w) {
    out[3 + 3 * w] = (int64_t)h->op[w].uf.size();
    out[4 + 3 * w] = (int64_t)h->op[w].pf.size();
    out[5 + 3 * w] = (int64_t)h->op[w].diag.size();
  }
  return RDM_OK;
}

extern "C" const char* rdm_last_error(void) { return last_error(); }
