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

// the bits of x at the set bits of mask, packed to the low end (lowest first)
uint32_t compress_bits(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  int k = 0;
  for (int b = 0; b < 32; ++b)
    if ((mask >> b) & 1u) {
      if ((x >> b) & 1u) r |= 1u << k;
      ++k;
    }
  return r;
}

// distinct nonzero partner-tile offsets f & ~B over the flip masks
int distinct_partners(const std::vector<uint32_t>& flips, uint32_t B) {
  std::vector<uint32_t> o;
  for (uint32_t f : flips)
    if (f & ~B) o.push_back(f & ~B);
  std::sort(o.begin(), o.end());
  return (int)(std::unique(o.begin(), o.end()) - o.begin());
}

// Tile bits B of the bit-set tiles: the kWideLowBits lowest row bits (256-byte
// runs per 16 lanes), then one bit at a time the one that leaves the fewest
// distinct partner tiles (the lowest such bit on ties), kWideBits in all.
uint32_t choose_tile_bits(const std::vector<uint32_t>& flips, int nbits) {
  uint32_t B = (1u << kWideLowBits) - 1u;
  while (__builtin_popcount(B) < kWideBits) {
    int best = -1, best_n = 0;
    for (int b = kWideLowBits; b < nbits; ++b) {
      if ((B >> b) & 1u) continue;
      const int n = distinct_partners(flips, B | (1u << b));
      if (best < 0 || n < best_n) {
        best = b;
        best_n = n;
      }
    }
    if (best < 0) break;  // fewer than kWideBits bits: callers need nbits >= kWideBits
    B |= 1u << best;
  }
  return B;
}

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
  // grouped form: sort every hop by the partner tile it reads (flip bits above
  // the 256-row tile), then by kind, keeping the input order otherwise
  struct H {
    uint32_t f, m;
    double cs, cd;
    int kind;
  };
  std::vector<H> all;
  for (size_t i = 0; i < t.uf.size(); ++i) all.push_back(H{t.uf[i], 0u, t.uc[i], t.uc[i], 0});
  for (size_t i = 0; i < t.pf.size(); ++i)
    all.push_back(H{t.pf[i], t.pm[i], t.pcs[i], t.pcd[i], (t.pm[i] & 63u) == 0u ? 1 : 2});
  const uint32_t lo_mask = (1u << kTileBits) - 1u;
  std::stable_sort(all.begin(), all.end(), [&](const H& a, const H& b) {
    const uint32_t ha = a.f & ~lo_mask, hb = b.f & ~lo_mask;
    if (ha != hb) return ha < hb;
    return a.kind < b.kind;
  });
  // count the hops per partner tile; tiles used at least kFatGroup times (and
  // the own tile) are staged in LDS, the other hops are gathered directly
  std::map<uint32_t, int> uses;
  for (const H& x : all) uses[x.f & ~lo_mask] += 1;
  t.groups.clear();
  t.groups.push_back(HopGroup{0u, 0, 0, 0, 0, 0, {0, 0}});  // the own tile always comes first
  std::vector<H> thin[3];
  for (size_t i = 0; i < all.size(); ++i) {
    const uint32_t fhi = all[i].f & ~lo_mask;
    if (fhi != 0u && uses[fhi] < kFatGroup) {
      thin[all[i].kind].push_back(all[i]);
      continue;
    }
    if (fhi != t.groups.back().fhi)
      t.groups.push_back(HopGroup{fhi, (int32_t)t.g_flo.size(), 0, 0, 0, 0, {0, 0}});
    HopGroup& g = t.groups.back();
    (all[i].kind == 0 ? g.n0 : all[i].kind == 1 ? g.n1 : g.n2) += 1;
    t.g_flo.push_back(all[i].f & lo_mask);
    t.g_m.push_back(all[i].m);
    t.g_cs.push_back(all[i].cs);
    t.g_cd.push_back(all[i].cd);
  }
  for (size_t g = 1; g < t.groups.size(); ++g) {
    HopGroup& gr = t.groups[g];
    bool uni = gr.n0 == 0 && gr.n2 == 0 && gr.n1 > 0;
    for (int h = gr.start; uni && h < gr.start + gr.n1; ++h) uni = (t.g_m[h] & lo_mask) == 0u;
    gr.tile_uniform = uni ? 1 : 0;
  }
  // Transform form (Section "Spin systems": products of site Paulis).  With
  // W the unnormalised Walsh-Hadamard transform on all nbits bits (W W =
  // 2^N I), W Z_i Z_j W = 2^N X_i X_j and W Z_i W = 2^N X_i, so the XX
  // couplings and x-fields are W D_X W with D_X(s) = 2^-N sum c (1 - 2
  // parity(s & f)).  For a pair, Y_i Y_j = T X_i X_j T with
  // T = diag((-1)^floor(popcount(idx)/2)) (flipping two equal bits moves the
  // popcount by 2, two different bits leave it), so the YY couplings are
  // T W D_Y W T with D_Y built the same way from J^y.
  bool any_x = false, any_y = false;
  std::vector<DiagTerm> xt, yt;
  for (const auto& kv : pairs) {
    const rdm_coupling& c = kv.second;
    const uint32_t f = (1u << (n - 1 - c.i)) | (1u << (n - 1 - c.j));
    if (c.jx != 0.0) xt.push_back(DiagTerm{f, 0, std::ldexp(c.jx, -t.nbits)});
    if (c.jy != 0.0) yt.push_back(DiagTerm{f, 0, std::ldexp(c.jy, -t.nbits)});
  }
  for (int s = first_site; s < n; ++s)
    if (h.hx[s] != 0.0) xt.push_back(DiagTerm{1u << (n - 1 - s), 0, std::ldexp(h.hx[s], -t.nbits)});
  any_x = !xt.empty();
  any_y = !yt.empty();
  const bool in_range = t.nbits >= kXzMinBits && t.nbits <= kXzMaxBits && (any_x || any_y);
  // A transform step streams 8 vectors, 15 with a YY part and 4 more with
  // split strided passes (above 22 bits); a hop-table step streams about 6
  // and reads one partner row per staged partner tile and per gathered hop,
  // from cache for the most part.  Measured: with YY terms the hop tables win
  // at 28 partner rows per row (random graphs of degree 4, 22 bits) and lose
  // from 78 on (all pairs, 20-26 bits); with split passes the transverse-field
  // chain (16 partner rows) runs 3-4 % faster from hop tables.  So operators
  // with YY terms, and all operators above 22 bits, take the transform from
  // 40 partner rows on; X-type operators up to 22 bits always.
  const int partners = (int)(t.groups.size() - 1 + thin[0].size() + thin[1].size() + thin[2].size());
  const bool dense_enough = partners >= 40;
  bool use = false;
  if (h.apply == RDM_APPLY_TRANSFORM) use = in_range;
  else if (h.apply == RDM_APPLY_AUTO)
    use = in_range && (any_y || xz_geom(t.nbits) == XG_SPLIT ? dense_enough : true);
  t.xz = use;
  t.xy = use && any_y;
  // Bit-set tile form of the same hops (kWideBits sites and more): grouped by
  // partner tile f & ~B; tiles read by at least kWideFat hops (and the own
  // tile) are staged in LDS, the other hops gathered directly.  Products use
  // it when it reads fewer partner tiles per tile than the 256-row form reads
  // partner rows per row.
  if (t.nbits >= kWideBits) {
    std::vector<uint32_t> flips;
    for (const H& x : all) flips.push_back(x.f);
    const uint32_t B = choose_tile_bits(flips, t.nbits);
    t.wbits = B;
    std::vector<H> w = all;
    for (H& x : w) x.kind = x.m == 0u ? 0 : ((x.m & B) == 0u ? 1 : 2);
    std::stable_sort(w.begin(), w.end(), [&](const H& a, const H& b) {
      const uint32_t ha = a.f & ~B, hb = b.f & ~B;
      if (ha != hb) return ha < hb;
      return a.kind < b.kind;
    });
    std::map<uint32_t, int> wuses;
    for (const H& x : w) wuses[x.f & ~B] += 1;
    t.wgroups.clear();
    t.wgroups.push_back(HopGroup{0u, 0, 0, 0, 0, 0, {0, 0}});
    std::vector<H> wthin[3];
    for (const H& x : w) {
      const uint32_t fo = x.f & ~B;
      if (fo != 0u && wuses[fo] < kWideFat) {
        wthin[x.kind].push_back(x);
        continue;
      }
      if (fo != t.wgroups.back().fhi)
        t.wgroups.push_back(HopGroup{fo, (int32_t)t.w_flo.size(), 0, 0, 0, 0, {0, 0}});
      HopGroup& g = t.wgroups.back();
      (x.kind == 0 ? g.n0 : x.kind == 1 ? g.n1 : g.n2) += 1;
      t.w_flo.push_back(compress_bits(x.f & B, B));
      t.w_m.push_back(x.m);
      t.w_cs.push_back(x.cs);
      t.w_cd.push_back(x.cd);
    }
    for (size_t g = 1; g < t.wgroups.size(); ++g) {
      HopGroup& gr = t.wgroups[g];
      gr.tile_uniform = gr.n0 == 0 && gr.n2 == 0 && gr.n1 > 0 ? 1 : 0;
    }
    for (int k = 0; k < 3; ++k) {
      t.wnt[k] = (int)wthin[k].size();
      for (const H& x : wthin[k]) {
        t.wt_f.push_back(x.f);
        t.wt_m.push_back(x.m);
        t.wt_cs.push_back(x.cs);
        t.wt_cd.push_back(x.cd);
      }
    }
    const int wpartners = (int)(t.wgroups.size() - 1 + t.wt_f.size());
    t.wide = !use && h.apply != RDM_APPLY_HOPS_ROWS && wpartners < partners;
  }
  if (use) {
    t.xterms = xt;
    t.yterms = yt;
  }
  for (int k = 0; k < 3; ++k) {
    t.nt[k] = (int)thin[k].size();
    for (const H& x : thin[k]) {
      t.t_f.push_back(x.f);
      t.t_m.push_back(x.m);
      t.t_cs.push_back(x.cs);
      t.t_cd.push_back(x.cd);
    }
  }
}

template <typename T>
rdm_status upload(const OpTables& t, OpDevice& d, hipStream_t st) {
  std::vector<GHop<T>> hops(t.g_flo.size());
  for (size_t i = 0; i < hops.size(); ++i)
    hops[i] = GHop<T>{t.g_flo[i], t.g_m[i], (T)t.g_cs[i], (T)t.g_cd[i]};
  const size_t dim = size_t(1) << t.nbits;
  RDM_HIP(hipMalloc(&d.hops, std::max<size_t>(16, hops.size() * sizeof(GHop<T>))));
  RDM_HIP(hipMalloc(&d.groups, std::max<size_t>(16, t.groups.size() * sizeof(HopGroup))));
  std::vector<GHop<T>> thin(t.t_f.size());
  for (size_t i = 0; i < thin.size(); ++i) thin[i] = GHop<T>{t.t_f[i], t.t_m[i], (T)t.t_cs[i], (T)t.t_cd[i]};
  RDM_HIP(hipMalloc(&d.thin, std::max<size_t>(16, thin.size() * sizeof(GHop<T>))));
  if (!thin.empty())
    RDM_HIP(hipMemcpyAsync(d.thin, thin.data(), thin.size() * sizeof(GHop<T>), hipMemcpyHostToDevice, st));
  for (int k = 0; k < 3; ++k) d.nt[k] = t.nt[k];
  RDM_HIP(hipMalloc(&d.dterms, std::max<size_t>(16, t.diag.size() * sizeof(DiagTerm))));
  RDM_HIP(hipMalloc(&d.diag, dim * sizeof(T)));
  if (!hops.empty())
    RDM_HIP(hipMemcpyAsync(d.hops, hops.data(), hops.size() * sizeof(GHop<T>), hipMemcpyHostToDevice, st));
  RDM_HIP(hipMemcpyAsync(d.groups, t.groups.data(), t.groups.size() * sizeof(HopGroup),
                         hipMemcpyHostToDevice, st));
  if (!t.diag.empty())
    RDM_HIP(hipMemcpyAsync(d.dterms, t.diag.data(), t.diag.size() * sizeof(DiagTerm),
                           hipMemcpyHostToDevice, st));
  RDM_HIP(launch_diag<T>((const DiagTerm*)d.dterms, (int)t.diag.size(), (T*)d.diag, t.nbits, st));
  d.xz = t.xz;
  d.xy = t.xy;
  if (t.xz) {
    // D_X and D_Y of deep operators (21, 22 bits) in the order of the strided tiles that
    // read them (an operator without XX / x terms gets D_X = 0)
    RDM_HIP(hipMalloc(&d.xterms, std::max<size_t>(16, t.xterms.size() * sizeof(DiagTerm))));
    RDM_HIP(hipMalloc(&d.dx, dim * sizeof(T)));
    if (!t.xterms.empty())
      RDM_HIP(hipMemcpyAsync(d.xterms, t.xterms.data(), t.xterms.size() * sizeof(DiagTerm),
                             hipMemcpyHostToDevice, st));
    RDM_HIP(launch_diag<T>((const DiagTerm*)d.xterms, (int)t.xterms.size(), (T*)d.dx, t.nbits, st,
                           xz_geom(t.nbits) == XG_DEEP));
  }
  if (t.xy) {
    RDM_HIP(hipMalloc(&d.yterms, t.yterms.size() * sizeof(DiagTerm)));
    RDM_HIP(hipMalloc(&d.dy, dim * sizeof(T)));
    RDM_HIP(hipMemcpyAsync(d.yterms, t.yterms.data(), t.yterms.size() * sizeof(DiagTerm),
                           hipMemcpyHostToDevice, st));
    RDM_HIP(launch_diag<T>((const DiagTerm*)d.yterms, (int)t.yterms.size(), (T*)d.dy, t.nbits, st,
                           xz_geom(t.nbits) == XG_DEEP));
  }
  if (t.wide) {
    std::vector<GHop<T>> wh(t.w_flo.size()), wt(t.wt_f.size());
    for (size_t i = 0; i < wh.size(); ++i) wh[i] = GHop<T>{t.w_flo[i], t.w_m[i], (T)t.w_cs[i], (T)t.w_cd[i]};
    for (size_t i = 0; i < wt.size(); ++i) wt[i] = GHop<T>{t.wt_f[i], t.wt_m[i], (T)t.wt_cs[i], (T)t.wt_cd[i]};
    RDM_HIP(hipMalloc(&d.whops, std::max<size_t>(16, wh.size() * sizeof(GHop<T>))));
    RDM_HIP(hipMalloc(&d.wgroups, std::max<size_t>(16, t.wgroups.size() * sizeof(HopGroup))));
    RDM_HIP(hipMalloc(&d.wthin, std::max<size_t>(16, wt.size() * sizeof(GHop<T>))));
    if (!wh.empty())
      RDM_HIP(hipMemcpyAsync(d.whops, wh.data(), wh.size() * sizeof(GHop<T>), hipMemcpyHostToDevice, st));
    RDM_HIP(hipMemcpyAsync(d.wgroups, t.wgroups.data(), t.wgroups.size() * sizeof(HopGroup),
                           hipMemcpyHostToDevice, st));
    if (!wt.empty())
      RDM_HIP(hipMemcpyAsync(d.wthin, wt.data(), wt.size() * sizeof(GHop<T>), hipMemcpyHostToDevice, st));
    // the host vectors above must outlive the copies
    RDM_HIP(hipStreamSynchronize(st));
    d.wngroups = (int)t.wgroups.size();
    for (int k = 0; k < 3; ++k) d.wnt[k] = t.wnt[k];
  }
  d.wide = t.wide;
  d.wbits = t.wbits;
  RDM_HIP(hipStreamSynchronize(st));
  d.ngroups = (int)t.groups.size();
  d.ready = true;
  return RDM_OK;
}

void free_dev(rdm::OpDevice& d) {
  if (d.hops) (void)hipFree(d.hops);
  if (d.groups) (void)hipFree(d.groups);
  if (d.thin) (void)hipFree(d.thin);
  if (d.whops) (void)hipFree(d.whops);
  if (d.wgroups) (void)hipFree(d.wgroups);
  if (d.wthin) (void)hipFree(d.wthin);
  if (d.diag) (void)hipFree(d.diag);
  if (d.dx) (void)hipFree(d.dx);
  if (d.xterms) (void)hipFree(d.xterms);
  if (d.dy) (void)hipFree(d.dy);
  if (d.yterms) (void)hipFree(d.yterms);
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

rdm_status find_device_op(const rdm_hamiltonian* h, int which, int precision, const OpDevice** out) {
  std::lock_guard<std::mutex> lk(h->mu);
  int dev = 0;
  RDM_HIP(hipGetDevice(&dev));
  const OpDevice& d = h->dev[which][precision];
  if (!d.ready || d.device != dev) {
    set_error("the Hamiltonian's device tables are not resident on this device in this precision "
              "(any earlier solve or apply with it builds them)");
    return RDM_E_INVALID;
  }
  *out = &d;
  return RDM_OK;
}

}  // namespace rdm

using namespace rdm;

extern "C" rdm_status rdm_hamiltonian_create(int32_t n_s, int32_t n_b, const rdm_coupling* couplings,
                                             int64_t n_couplings, const double* hx, const double* hz,
                                             rdm_hamiltonian** out) {
  return rdm_hamiltonian_create_ex(n_s, n_b, couplings, n_couplings, hx, hz, RDM_APPLY_AUTO, out);
}

extern "C" rdm_status rdm_hamiltonian_create_ex(int32_t n_s, int32_t n_b, const rdm_coupling* couplings,
                                                int64_t n_couplings, const double* hx, const double* hz,
                                                int32_t apply, rdm_hamiltonian** out) {
  if (!out) {
    set_error("rdm_hamiltonian_create: out is NULL");
    return RDM_E_INVALID;
  }
  *out = nullptr;
  if (apply != RDM_APPLY_AUTO && apply != RDM_APPLY_HOPS && apply != RDM_APPLY_TRANSFORM &&
      apply != RDM_APPLY_HOPS_ROWS) {
    set_error("rdm_hamiltonian_create_ex: apply must be RDM_APPLY_AUTO, RDM_APPLY_HOPS, RDM_APPLY_TRANSFORM "
              "or RDM_APPLY_HOPS_ROWS");
    return RDM_E_INVALID;
  }
  if (n_s < 1 || n_s > 4 || n_b < 1 || n_s + n_b > 28) {
    set_error("rdm_hamiltonian_create: need 1 <= n_s <= 4, n_b >= 1, n_s + n_b <= 28");
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
  h->apply = apply;
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
    out[9 + w] = (int64_t)h->op[w].groups.size();
    out[11 + w] = (int64_t)h->op[w].t_f.size();
    out[13 + w] = h->op[w].xz ? 1 : 0;
    out[15 + w] = h->op[w].xy ? 1 : 0;
    out[17 + w] = h->op[w].wide ? 1 : 0;
    out[19 + w] = h->op[w].wgroups.empty() ? 0
                                            : (int64_t)(h->op[w].wgroups.size() - 1 + h->op[w].wt_f.size());
  }
  return RDM_OK;
}

extern "C" const char* rdm_last_error(void) { return last_error(); }

extern "C" rdm_status rdm_system_hamiltonian(const rdm_hamiltonian* h, double* out) {
  if (!h || !out) {
    set_error("rdm_system_hamiltonian: NULL argument");
    return RDM_E_INVALID;
  }
  // H_s on the 2^n_s system states: the couplings and fields of system sites
  // only (site s < n_s is bit n_s-1-s of the system index)
  const int ns = h->n_s, ds = 1 << ns;
  for (int i = 0; i < ds * ds; ++i) out[i] = 0.0;
  auto bit = [&](int site) { return 1u << (ns - 1 - site); };
  for (const auto& c : h->couplings) {
    if (c.i >= ns || c.j >= ns) continue;
    const uint32_t f = bit(c.i) | bit(c.j);
    for (uint32_t r = 0; r < (uint32_t)ds; ++r) {
      const bool differ = (__builtin_popcount(r & f) & 1u) != 0;
      out[r * ds + r] += differ ? -c.jz : c.jz;
      // sx sx + sy sy: jx - jy when the two bits agree, jx + jy when they differ
      out[r * ds + (r ^ f)] += differ ? c.jx + c.jy : c.jx - c.jy;
    }
  }
  for (int s = 0; s < ns; ++s) {
    const uint32_t b = bit(s);
    for (uint32_t r = 0; r < (uint32_t)ds; ++r) {
      out[r * ds + r] += (r & b) ? -h->hz[s] : h->hz[s];
      out[r * ds + (r ^ b)] += h->hx[s];
    }
  }
  return RDM_OK;
}
