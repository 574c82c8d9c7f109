// Solve driver: planning, workspace layout, the Lanczos step loop over a
// batch of segments, host eigen-work, recombination + Gram, finalisation.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <thread>

#include "host.h"
#include "solve.h"

namespace rdm {

namespace {

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int panel_width(int prec) { return prec == RDM_FP64 ? 2 : 4; }
size_t scalar_bytes(int prec) { return prec == RDM_FP64 ? 8 : 4; }

int ilog2(uint64_t x) {
  int r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}

// Worker threads for the host eigen-work, created on first use and kept for
// the life of the process (the pool is never destroyed, so no thread is
// joined during static destruction).  One job at a time; a caller that finds
// the pool busy runs its loop itself.
class Pool {
 public:
  explicit Pool(int nworkers) {
    for (int t = 0; t < nworkers; ++t) std::thread([this] { work(); }).detach();
    nworkers_ = nworkers;
  }
  void run(int n, const std::function<void(int)>& fn) {
    std::unique_lock<std::mutex> busy(job_mu_, std::try_to_lock);
    if (!busy.owns_lock() || nworkers_ == 0) {
      for (int i = 0; i < n; ++i) fn(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_ = 0;
      active_ = nworkers_;
      ++gen_;
    }
    cv_.notify_all();
    for (int i = next_++; i < n; i = next_++) fn(i);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return active_ == 0; });
    fn_ = nullptr;
  }

 private:
  void work() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* fn;
      int n;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        fn = fn_;
        n = n_;
      }
      for (int i = next_++; i < n; i = next_++) (*fn)(i);
      std::lock_guard<std::mutex> lk(mu_);
      if (--active_ == 0) done_cv_.notify_one();
    }
  }
  std::mutex job_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0, active_ = 0, nworkers_ = 0;
  uint64_t gen_ = 0;
  std::atomic<int> next_{0};
};

void parallel_for(int n, const std::function<void(int)>& fn) {
  static Pool* pool = new Pool(std::min(16, (int)std::max(1u, std::thread::hardware_concurrency())) - 1);
  if (n <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  pool->run(n, fn);
}

}  // namespace

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
bool needs_ybuf(const rdm_hamiltonian* h, int which) { return h->op[which].xz && h->op[which].xy; }
bool lanczos_needs_ybuf(const rdm_hamiltonian* h, int which, int prec) {
  return h->op[which].xz && (h->op[which].xy || prec == RDM_FP64);
}

void plan_seg(SegPlan& g, int nbits, int C, int k, int prec, int slab_opt, int rpl_opt, int nslots,
              size_t& off, bool ybuf) {
  const int W = panel_width(prec);
  const size_t sb = scalar_bytes(prec);
  g.nbits = nbits;
  g.prec = prec;
  g.dim = 1ull << nbits;
  g.C = C;
  g.P = (C + W - 1) / W;
  g.cpad = g.P * W;
  g.k = k;
  int S = slab_opt > 0 ? slab_opt : kMaxSlab;
  S = std::min(S, kMaxSlab);
  while (S > 1 && (g.P % S) != 0) S >>= 1;
  g.S = std::max(S, 1);
  // the apply stages one partner tile of kBlock rows per workgroup, one row
  // per lane; the norm kernel uses the same tiles
  (void)rpl_opt;
  const int rpl = 1;
  g.rpl = rpl;
  g.n_row_tiles = (int)((g.dim + (uint64_t)kBlock * rpl - 1) / ((uint64_t)kBlock * rpl));
  g.blk = g.dim * g.cpad;
  g.nslots = nslots;
  g.o_Q = off; off = al(off + (size_t)nslots * g.blk * sb);
  g.o_R = off; off = al(off + g.blk * sb);
  g.o_st = off; off = al(off + (size_t)ST_COUNT * g.cpad * 8);
  g.o_ha = off; off = al(off + (size_t)k * g.cpad * 8);
  g.o_hb = off; off = al(off + (size_t)k * g.cpad * 8);
  g.o_hs = off; off = al(off + (size_t)k * g.cpad * 8);
  g.o_part = off; off = al(off + (size_t)g.n_row_tiles * g.cpad * 8);
  g.o_step = off; off = al(off + (size_t)g.cpad * 4);
  g.o_kc = off; off = al(off + (size_t)g.cpad * 4);
  g.ybuf = ybuf;
  if (ybuf) {
    g.o_Y = off;
    off = al(off + g.blk * sb);
  }
}

int max_nb_chunk(int prec, int ds) {
  if (ds >= 16) return 1;  // the Gram in three column blocks, one temperature at a time
  if (ds >= 8) return prec == RDM_FP64 ? 1 : 2;
  return 4;
}

rdm_status plan_instance(InstPlan& p, const rdm_hamiltonian* h, int n_beta, int n_v, int k, int prec,
                         int mode_req, uint64_t budget, int slab_opt, int rpl_opt) {
  p.h = h;
  p.prec = prec;
  p.n_beta = n_beta;
  p.n_v = n_v;
  const uint64_t dim = 1ull << h->n;
  p.k = (int)std::min<uint64_t>((uint64_t)k, dim);
  p.kb = (int)std::min<uint64_t>((uint64_t)k, 1ull << h->n_b);
  p.ds_log = h->n_s;
  p.ds = 1 << h->n_s;
  const int W = panel_width(prec);
  const size_t sb = scalar_bytes(prec);
  p.cb = std::max(p.ds, W);
  p.groups_per_block = p.cb / p.ds;
  p.n_cblocks = (n_v + p.groups_per_block - 1) / p.groups_per_block;
  p.nb_chunk = std::min(max_nb_chunk(prec, p.ds), n_beta <= 1 ? 1 : (n_beta <= 2 ? 2 : 4));
  // LDS for the y slice of the Gram kernel
  while (p.nb_chunk > 1 &&
         (size_t)p.k * p.nb_chunk * p.cb * sb + 4 * 144 * 8 > 60 * 1024)
    p.nb_chunk >>= 1;
  if ((size_t)p.k * p.nb_chunk * p.cb * sb + 4 * 144 * 8 > 60 * 1024) {
    set_error("k too large for the Gram kernel's LDS tile");
    return RDM_E_INVALID;
  }
  auto layout = [&](bool two_pass) {
    size_t off = 0;
    plan_seg(p.tot, h->n, p.ds * n_v, p.k, prec, slab_opt, rpl_opt, two_pass ? 2 : p.k, off,
             lanczos_needs_ybuf(h, 0, prec));
    plan_seg(p.bath, h->n_b, n_v, p.kb, prec, slab_opt, rpl_opt, 2, off, lanczos_needs_ybuf(h, 1, prec));
    p.o_psi = off;
    if (two_pass) off = al(off + (size_t)n_beta * p.tot.blk * sb);
    p.o_y = off; off = al(off + (size_t)n_beta * p.k * p.tot.cpad * sb);
    // Gram tiling
    uint64_t r = (p.tot.dim * p.n_cblocks) / (kBlock * 4096ull);
    p.g_rpl = rpl_opt > 0 ? rpl_opt : (int)std::max<uint64_t>(1, std::min<uint64_t>(r, 16));
    p.g_rtiles = (int)((p.tot.dim + (uint64_t)kBlock * p.g_rpl - 1) / ((uint64_t)kBlock * p.g_rpl));
    p.o_gpart = off; off = al(off + (size_t)p.g_rtiles * n_beta * n_v * p.ds * p.ds * 8);
    p.o_gsum = off; off = al(off + (size_t)n_beta * n_v * p.ds * p.ds * 8);
    p.o_gseg = off; off = al(off + sizeof(GSeg));
    p.o_gtiles = off; off = al(off + sizeof(GTile) * (size_t)p.g_rtiles * p.n_cblocks);
    return off;
  };
  const size_t stored = layout(false);
  const size_t twop = layout(true);
  if (mode_req == RDM_STORED_Q) {
    p.two_pass = false;
  } else if (mode_req == RDM_TWO_PASS) {
    p.two_pass = true;
  } else {
    p.two_pass = budget != 0 && stored > budget;
  }
  p.bytes = layout(p.two_pass);
  (void)twop;
  if (budget != 0 && p.bytes > budget) {
    set_error("instance needs " + std::to_string(p.bytes) + " device bytes, budget " +
              std::to_string(budget));
    return RDM_E_NOMEM;
  }
  return RDM_OK;
}

// ---------------------------------------------------------------------------
// execution
// ---------------------------------------------------------------------------
namespace {

Seg make_seg(const SegPlan& g, const OpDevice* op, char* base, int mode, int start_kind, int ns_log,
             int nb, uint64_t seed, double tau) {
  Seg s{};
  s.nbits = g.nbits;
  s.n_row_tiles = g.n_row_tiles;
  bind_apply(s, op);
  // FP64 transform steps assemble <u_j, r_j> from XP_COUNT planes of x_tiles
  // rows each (n_row_tiles = dim / 256 rows leave room for them)
  static_assert(XP_COUNT * kBlock <= (1 << kXzTileBits), "partial-sum planes exceed the part buffer");
  s.xdots = op->xz && g.prec == RDM_FP64 ? 1 : 0;
  s.P = g.P;
  s.S = g.S;
  s.rpl = g.rpl;
  s.C = g.C;
  s.cpad = g.cpad;
  s.k = g.k;
  s.mode = mode;
  s.ring = g.nslots < g.k ? 1 : 0;
  s.start_kind = start_kind;
  s.ns_log = ns_log;
  s.nb = nb;
  s.n_beta = 0;
  s.seed = seed;
  s.blk = g.blk;
  s.Q = base + g.o_Q;
  s.R = base + g.o_R;
  s.Y = g.ybuf ? base + g.o_Y : nullptr;
  s.psi = nullptr;
  s.ytab = nullptr;
  s.st = (double*)(base + g.o_st);
  s.h_alpha = (double*)(base + g.o_ha);
  s.h_beta = (double*)(base + g.o_hb);
  s.h_s = (double*)(base + g.o_hs);
  s.part = (double*)(base + g.o_part);
  s.stepc = (int32_t*)(base + g.o_step);
  s.kc = (int32_t*)(base + g.o_kc);
  s.tau = tau;
  return s;
}

struct HostHist {
  std::vector<double> a, b, s;
  std::vector<int32_t> kc;
};

rdm_status fetch_hist(const SegPlan& g, char* base, HostHist& hh, hipStream_t st) {
  const size_t n = (size_t)g.k * g.cpad;
  hh.a.resize(n);
  hh.b.resize(n);
  hh.s.resize(n);
  hh.kc.resize(g.cpad);
  RDM_HIP(hipMemcpyAsync(hh.a.data(), base + g.o_ha, n * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipMemcpyAsync(hh.b.data(), base + g.o_hb, n * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipMemcpyAsync(hh.s.data(), base + g.o_hs, n * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipMemcpyAsync(hh.kc.data(), base + g.o_kc, g.cpad * 4, hipMemcpyDeviceToHost, st));
  return RDM_OK;
}

// Column c of a history as contiguous alpha[0..kc-1], beta[0..kc-2].
void column(const HostHist& hh, int cpad, int c, std::vector<double>& a, std::vector<double>& b) {
  const int kc = hh.kc[c];
  a.resize(kc);
  b.resize(kc > 0 ? kc - 1 : 0);
  for (int j = 0; j < kc; ++j) a[j] = hh.a[(size_t)j * cpad + c];
  for (int j = 0; j + 1 < kc; ++j) b[j] = hh.b[(size_t)j * cpad + c];
}

bool all_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// phases shared by single solves, batches and the serving engine
// ---------------------------------------------------------------------------
// exported helpers (solve.h) for the block-Lanczos driver
Seg make_plain_seg(const SegPlan& g, const OpDevice* op, char* base, int mode, int start_kind, int ns_log,
                   int nb, uint64_t seed, double tau) {
  return make_seg(g, op, base, mode, start_kind, ns_log, nb, seed, tau);
}
rdm_status fetch_history(const SegPlan& g, char* base, std::vector<double>& a, std::vector<double>& b,
                         std::vector<double>& s, std::vector<int32_t>& kc, hipStream_t st) {
  HostHist hh;
  rdm_status r = fetch_hist(g, base, hh, st);
  a.swap(hh.a);
  b.swap(hh.b);
  s.swap(hh.s);
  kc.swap(hh.kc);
  return r;
}
void parallel_jobs(int n, const std::function<void(int)>& fn) { parallel_for(n, fn); }
size_t align_up(size_t x) { return al(x); }

rdm_status bind_ops(InstRun& r, hipStream_t st, bool build_tables) {
  const InstPlan& p = *r.plan;
  if (!build_tables) {
    rdm_status s = find_device_op(p.h, 0, p.prec, &r.op_t);
    if (s != RDM_OK) return s;
    return find_device_op(p.h, 1, p.prec, &r.op_b);
  }
  rdm_status s = get_device_op(p.h, 0, p.prec, st, &r.op_t);
  if (s != RDM_OK) return s;
  return get_device_op(p.h, 1, p.prec, st, &r.op_b);
}

Seg seg_of(const InstRun& r, int which, int mode, double tau) {
  const InstPlan& p = *r.plan;
  if (which == 1)
    return make_seg(p.bath, r.op_b, r.base, MODE_LANCZOS, START_BATH, 0, p.h->n_b, r.seed, tau);
  Seg sg = make_seg(p.tot, r.op_t, r.base, mode, START_SYSBATH, p.ds_log, p.h->n_b, r.seed, tau);
  if (mode == MODE_REGEN) {
    sg.n_beta = p.n_beta;
    sg.psi = r.base + p.o_psi;
    sg.ytab = r.base + p.o_y;
  }
  return sg;
}

int common_slab(std::vector<Seg>& segs) {
  // one launch uses one panel count per lane; every segment's own choice is a
  // power of two dividing its panel count, so the smallest one divides all.
  // Results do not depend on it (it only splits columns across lanes).
  int slab = kMaxSlab;
  for (auto& sg : segs) slab = std::min(slab, sg.S);
  for (auto& sg : segs) sg.S = slab;
  return slab;
}

void bind_apply(Seg& s, const OpDevice* op) {
  s.hops = op->hops;
  s.groups = op->groups;
  s.thin = op->thin;
  s.diag = op->diag;
  s.ngroups = op->ngroups;
  s.nt0 = op->nt[0];
  s.nt1 = op->nt[1];
  s.nt2 = op->nt[2];
  s.xz = op->xz ? 1 : 0;
  s.xy = op->xz && op->xy ? 1 : 0;
  s.dx = op->dx;
  s.dy = op->dy;
  s.x_tiles = op->xz ? 1 << (s.nbits - kXzTileBits) : 0;
  s.ap_rows = op->xz ? s.x_tiles : s.n_row_tiles;
  s.nm_rows = s.ap_rows;
  s.wide = 0;
  s.wbits = 0;
  if (op->wide && !op->xz && s.nbits >= kWideBits) {
    // the apply on bit-set tiles: their tables, one partial-sum row per tile
    // (the norm step keeps its 256-row tiles)
    s.wide = 1;
    s.wbits = op->wbits;
    s.hops = op->whops;
    s.groups = op->wgroups;
    s.thin = op->wthin;
    s.ngroups = op->wngroups;
    s.nt0 = op->wnt[0];
    s.nt1 = op->wnt[1];
    s.nt2 = op->wnt[2];
    s.ap_rows = 1 << (s.nbits - kWideBits);
  }
}

Launch assign_tiles(std::vector<Seg>& segs) {
  // the norm launch covers the hop-table segments, the apply launch those of
  // them on 256-row tiles and the bit-set apply launch the others, the
  // transform passes the rest (pass 1 doing their norm step).  Segments
  // outside a launch get no workgroups in it (their base is the running
  // count, which the kernels' binary search never resolves to them).
  Launch L;
  for (auto& sg : segs) {
    sg.tile_base = L.norm;
    if (!sg.xz) L.norm += sg.n_row_tiles * (sg.P / sg.S);
    sg.ap_base = L.apply;
    if (!sg.xz && !sg.wide) L.apply += sg.n_row_tiles * (sg.P / sg.S);
    sg.wp_base = L.wide;
    if (sg.wide) L.wide += (1 << (sg.nbits - kWideBits)) * sg.P;
    sg.x_base = L.xz;
    if (sg.xz) {
      L.xz += sg.x_tiles * sg.P;
      (sg.mode == MODE_REGEN ? L.xz_regen : L.xz_lanczos)[xz_geom(sg.nbits)] = true;
      if (sg.xy) L.xy[xz_geom(sg.nbits)] = true;
    }
  }
  return L;
}

rdm_status init_run(int prec, const Seg* dsegs, int nseg, int cmax, int phase, int xz_tiles, int xz_boff,
                    hipStream_t st) {
  RDM_HIP(launch_init_state(dsegs, nseg, cmax, phase, st));
  RDM_HIP(prec == RDM_FP64 ? launch_xz_lanczos<double>(0, false, dsegs, nseg, xz_tiles, xz_boff, st)
                           : launch_xz_lanczos<float>(0, false, dsegs, nseg, xz_tiles, xz_boff, st));
  return RDM_OK;
}

rdm_status launch_step(int prec, const Seg* dsegs, int nseg, const Launch& L, int slab, int cmax, hipStream_t st,
                       StepTimers* tm) {
  Range range("rdm step launch");
  const bool d = prec == RDM_FP64;
  if (tm) RDM_HIP(tm->norm.mark(st));
  RDM_HIP(d ? launch_norm<double>(dsegs, nseg, L.norm, slab, st) : launch_norm<float>(dsegs, nseg, L.norm, slab, st));
  if (tm) RDM_HIP(tm->norm.mark(st));
  if (tm) RDM_HIP(tm->xz1.mark(st));
  for (int regen = 0; regen < 2; ++regen)
    for (int geo = 0; geo < 3; ++geo) {
      if (!(regen ? L.xz_regen : L.xz_lanczos)[geo]) continue;
      RDM_HIP(d ? launch_xz_lanczos<double>(1, regen, dsegs, nseg, L.xz, 0, st, geo)
                : launch_xz_lanczos<float>(1, regen, dsegs, nseg, L.xz, 0, st, geo));
    }
  // split segments: pass 1 did the norm step and W_A; then W_B D_X W_B, W_A
  if (L.any_split())
    for (int op : {1, 0})
      RDM_HIP(d ? launch_xz_split<double>(op, dsegs, nseg, L.xz, st) : launch_xz_split<float>(op, dsegs, nseg, L.xz, st));
  // the YY part of transform segments: Y = W_hi D_Y W_hi W_lo T W_lo u~ / L
  if (L.any_xy()) {
    RDM_HIP(d ? launch_xz_lanczos<double>(3, false, dsegs, nseg, L.xz, 0, st)
              : launch_xz_lanczos<float>(3, false, dsegs, nseg, L.xz, 0, st));
    for (int geo = 0; geo < 2; ++geo) {
      if (!L.xy[geo]) continue;
      RDM_HIP(d ? launch_xz_lanczos<double>(4, false, dsegs, nseg, L.xz, 0, st, geo)
                : launch_xz_lanczos<float>(4, false, dsegs, nseg, L.xz, 0, st, geo));
    }
    if (L.xy[XG_SPLIT])
      for (int op : {2, 3, 2})
        RDM_HIP(d ? launch_xz_split<double>(op, dsegs, nseg, L.xz, st)
                  : launch_xz_split<float>(op, dsegs, nseg, L.xz, st));
    RDM_HIP(d ? launch_xz_lanczos<double>(5, false, dsegs, nseg, L.xz, 0, st)
              : launch_xz_lanczos<float>(5, false, dsegs, nseg, L.xz, 0, st));
  }
  if (tm) RDM_HIP(tm->xz1.mark(st));
  RDM_HIP(launch_red_beta(dsegs, nseg, cmax, st));
  if (tm) RDM_HIP(tm->apply.mark(st));
  RDM_HIP(d ? launch_apply<double>(dsegs, nseg, L.apply, slab, st)
            : launch_apply<float>(dsegs, nseg, L.apply, slab, st));
  RDM_HIP(d ? launch_apply_wide<double>(dsegs, nseg, L.wide, st) : launch_apply_wide<float>(dsegs, nseg, L.wide, st));
  RDM_HIP(d ? launch_xz_lanczos<double>(2, false, dsegs, nseg, L.xz, 0, st)
            : launch_xz_lanczos<float>(2, false, dsegs, nseg, L.xz, 0, st));
  if (tm) RDM_HIP(tm->apply.mark(st));
  RDM_HIP(launch_red_alpha(dsegs, nseg, cmax, st));
  return RDM_OK;
}

namespace {

template <typename T>
rdm_status host_phase_t(InstRun& r, hipStream_t st) {
  const InstPlan& p = *r.plan;
  HostHist ht, hb;
  rdm_status s;
  if ((s = fetch_hist(p.tot, r.base, ht, st)) != RDM_OK) return s;
  if ((s = fetch_hist(p.bath, r.base, hb, st)) != RDM_OK) return s;
  RDM_HIP(hipStreamSynchronize(st));
  if (!all_finite(ht.a) || !all_finite(ht.b) || !all_finite(hb.a) || !all_finite(hb.b)) {
    set_error("non-finite Lanczos coefficients");
    return RDM_E_NONFINITE;
  }
  std::vector<TridiagEig> et(p.tot.C), eb(p.bath.C);
  parallel_for(p.tot.C + p.bath.C, [&](int t) {
    std::vector<double> a, b;
    if (t < p.tot.C) {
      column(ht, p.tot.cpad, t, a, b);
      et[t].solve(a.data(), b.data(), (int)a.size());
    } else {
      const int c = t - p.tot.C;
      column(hb, p.bath.cpad, c, a, b);
      eb[c].solve(a.data(), b.data(), (int)a.size());
    }
  });
  double e0 = INFINITY, e0b = INFINITY;
  bool ok = true;
  for (auto& e : et) {
    ok &= e.ok && e.n > 0;
    for (double x : e.theta) e0 = std::min(e0, x);
  }
  for (auto& e : eb) {
    ok &= e.ok && e.n > 0;
    for (double x : e.theta) e0b = std::min(e0b, x);
  }
  if (!ok || !std::isfinite(e0) || !std::isfinite(e0b)) {
    set_error("tridiagonal eigenproblem failed");
    return RDM_E_NONFINITE;
  }
  r.e0 = e0;
  r.e0b = e0b;
  r.n_break_t = r.n_break_b = 0;
  for (int c = 0; c < p.tot.C; ++c) r.n_break_t += ht.kc[c] < p.tot.k;
  for (int c = 0; c < p.bath.C; ++c) r.n_break_b += hb.kc[c] < p.bath.k;
  // weights y'_{b,j,c} = y_b[j] s_j / s_1: psi = |x| Q y and q_j = s_j u_j, |x| = 1/s_1
  // (times L^-1/2 when the basis is kept as W_lo u)
  const double bscale = r.op_t->xz ? kXzBasisScale : 1.0;
  std::vector<T> yt((size_t)p.n_beta * p.k * p.tot.cpad, T(0));
  parallel_for(p.tot.C, [&](int c) {
    const TridiagEig& e = et[c];
    std::vector<double> g((size_t)p.n_beta * e.n), y((size_t)p.n_beta * e.n);
    const double s1 = ht.s[c];
    for (int b = 0; b < p.n_beta; ++b)
      for (int q = 0; q < e.n; ++q) g[(size_t)b * e.n + q] = std::exp(-0.5 * r.betas[b] * (e.theta[q] - e0));
    e.apply_fn_multi(p.n_beta, g.data(), y.data());
    for (int b = 0; b < p.n_beta; ++b)
      for (int j = 0; j < e.n; ++j)
        yt[((size_t)b * p.k + j) * p.tot.cpad + c] =
            (T)(bscale * y[(size_t)b * e.n + j] * ht.s[(size_t)j * p.tot.cpad + c] / s1);
  });
  // bath: Gauss quadrature e_1^T exp(-b (T_b - E0b)) e_1 scaled by |v|^2 = 1/s_1^2
  r.mb.assign(p.n_beta, 0.0);
  for (int b = 0; b < p.n_beta; ++b) {
    double acc = 0.0;
    for (int c = 0; c < p.bath.C; ++c) {
      const TridiagEig& e = eb[c];
      const double s1 = hb.s[c];
      double q = 0.0;
      for (int t = 0; t < e.n; ++t) q += e.zrow[t] * e.zrow[t] * std::exp(-r.betas[b] * (e.theta[t] - e0b));
      acc += q / (s1 * s1);
    }
    r.mb[b] = acc / p.n_v;
  }
  RDM_HIP(hipMemcpyAsync(r.base + p.o_y, yt.data(), yt.size() * sizeof(T), hipMemcpyHostToDevice, st));
  RDM_HIP(hipStreamSynchronize(st));
  return RDM_OK;
}

}  // namespace

rdm_status host_phase(InstRun& r, hipStream_t st) {
  return r.plan->prec == RDM_FP64 ? host_phase_t<double>(r, st) : host_phase_t<float>(r, st);
}

rdm_status gram_phase(InstRun& r, hipStream_t st, Timers* tg) {
  const InstPlan& p = *r.plan;
  GSeg g{};
  g.Q = r.base + (p.two_pass ? p.o_psi : p.tot.o_Q);
  g.ytab = r.base + p.o_y;
  g.gpart = (double*)(r.base + p.o_gpart);
  g.blk = p.tot.blk;
  g.nbits = p.tot.nbits;
  g.cpad = p.tot.cpad;
  g.k = p.k;
  g.n_beta = p.n_beta;
  g.n_v = p.n_v;
  g.ds_log = p.ds_log;
  g.rpl = p.g_rpl;
  g.from_psi = p.two_pass ? 1 : 0;
  g.n_row_tiles = p.g_rtiles;
  std::vector<GTile> gt;
  for (int rt = 0; rt < p.g_rtiles; ++rt)
    for (int cb = 0; cb < p.n_cblocks; ++cb)
      gt.push_back(GTile{0, (uint32_t)((uint64_t)rt * kBlock * p.g_rpl), cb, rt});
  GSeg* dg = (GSeg*)(r.base + p.o_gseg);
  GTile* dgt = (GTile*)(r.base + p.o_gtiles);
  RDM_HIP(hipMemcpyAsync(dg, &g, sizeof(GSeg), hipMemcpyHostToDevice, st));
  RDM_HIP(hipMemcpyAsync(dgt, gt.data(), gt.size() * sizeof(GTile), hipMemcpyHostToDevice, st));
  for (int b0 = 0; b0 < p.n_beta; b0 += p.nb_chunk) {
    if (tg) RDM_HIP(tg->mark(st));
    RDM_HIP(p.prec == RDM_FP64 ? launch_gram<double>(dg, dgt, (int)gt.size(), p.ds, p.nb_chunk, b0, p.k, st)
                               : launch_gram<float>(dg, dgt, (int)gt.size(), p.ds, p.nb_chunk, b0, p.k, st));
    if (tg) RDM_HIP(tg->mark(st));
  }
  const int width = p.n_beta * p.n_v * p.ds * p.ds;
  RDM_HIP(launch_colsum((double*)(r.base + p.o_gpart), p.g_rtiles, width, (double*)(r.base + p.o_gsum), st));
  r.gsum.assign(width, 0.0);
  RDM_HIP(hipMemcpyAsync(r.gsum.data(), r.base + p.o_gsum, width * 8, hipMemcpyDeviceToHost, st));
  RDM_HIP(hipStreamSynchronize(st));
  return RDM_OK;
}

size_t batch_header_bytes(const std::vector<InstPlan>& plans) {
  return al(sizeof(Seg) * 2 * plans.size());
}

namespace {

// Panels per lane chosen by measurement, per shape of the largest segment of a
// launch (the slab never changes results, only speed).
struct SlabKey {
  int prec, nbits, cpad, ngroups, nthin;
  bool operator<(const SlabKey& o) const {
    return std::tie(prec, nbits, cpad, ngroups, nthin) < std::tie(o.prec, o.nbits, o.cpad, o.ngroups, o.nthin);
  }
};
std::mutex g_slab_mu;
std::map<SlabKey, int> g_slab_best;

SlabKey slab_key(int prec, const std::vector<Seg>& segs) {
  const Seg* big = &segs[0];
  for (const auto& sg : segs)
    if (((uint64_t)sg.cpad << sg.nbits) > ((uint64_t)big->cpad << big->nbits)) big = &sg;
  return SlabKey{prec, big->nbits, big->cpad, big->ngroups, big->nt0 + big->nt1 + big->nt2};
}

void set_slab(std::vector<Seg>& segs, int slab) {
  for (auto& sg : segs) sg.S = slab;
}

}  // namespace

int tuned_slab(int prec, std::vector<Seg>& segs) {
  const int smax = common_slab(segs);
  std::lock_guard<std::mutex> lk(g_slab_mu);
  auto it = g_slab_best.find(slab_key(prec, segs));
  const int s = it == g_slab_best.end() ? 1 : std::min(it->second, smax);
  set_slab(segs, s);
  return s;
}

namespace {

// The remaining Lanczos steps of a phase as one captured hipGraph.  Every
// step launches the same kernels with the same arguments (the step index and
// all per-column scalars live in device memory), so a graph captured once per
// (segment table address, launch shape, step count) is replayed by later
// solves that reuse the workspace; the segment table itself is uploaded
// before each phase.  Capture and replay run on a private stream per device
// that is ordered after / before the caller's stream with events, so the
// caller's stream may be the legacy default stream.
// The key holds every launch parameter a step depends on, including which
// variants of the strided transform pass it records (Lanczos or regeneration,
// by geometry, with or without a YY part): two tables at one address can
// agree on every count and still need different variants.
struct GraphKey {
  int device;
  const void* dsegs;
  int nseg, norm, apply, wide, xz, slab, cmax, prec, nsteps;
  int variants;  // bit (3 * regen + geometry) set when that strided variant runs, bit
                 // (6 + geometry) when that YY strided variant runs
  bool operator<(const GraphKey& o) const {
    return std::tie(device, dsegs, nseg, norm, apply, wide, xz, slab, cmax, prec, nsteps, variants) <
           std::tie(o.device, o.dsegs, o.nseg, o.norm, o.apply, o.wide, o.xz, o.slab, o.cmax, o.prec, o.nsteps,
                    o.variants);
  }
};
int launch_variants(const Launch& L) {
  int v = 0;
  for (int geo = 0; geo < 3; ++geo) {
    if (L.xz_lanczos[geo]) v |= 1 << geo;
    if (L.xz_regen[geo]) v |= 1 << (3 + geo);
    if (L.xy[geo]) v |= 1 << (6 + geo);
  }
  return v;
}
constexpr size_t kMaxGraphs = 64;
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
std::vector<GraphKey> g_graph_order;  // insertion order, for eviction
std::map<int, hipStream_t> g_graph_stream;

rdm_status graph_steps_locked(int prec, Seg* dsegs, int nseg, const Launch& L, int slab, int cmax, int nsteps,
                              hipStream_t st, int dev, hipEvent_t t0, hipEvent_t t1);

rdm_status graph_steps(int prec, Seg* dsegs, int nseg, const Launch& L, int slab, int cmax, int nsteps,
                       hipStream_t st, ReplayTimer* rt) {
  int dev = 0;
  RDM_HIP(hipGetDevice(&dev));
  // rt: timing events around the replay on the replay stream, read after
  // the lock is released
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (rt) {
    RDM_HIP(hipEventCreate(&t0));
    if (hipEventCreate(&t1) != hipSuccess) {
      (void)hipEventDestroy(t0);
      set_error("hipEventCreate failed");
      return RDM_E_DEVICE;
    }
  }
  auto drop_timers = [&]() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  rdm_status ls = graph_steps_locked(prec, dsegs, nseg, L, slab, cmax, nsteps, st, dev, t0, t1);
  if (ls == RDM_OK && rt) {
    float ms = 0.f;
    if (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
      drop_timers();
      set_error("replay timing failed");
      return RDM_E_DEVICE;
    }
    rt->ms += ms;
    rt->steps += nsteps;
  }
  drop_timers();
  return ls;
}

rdm_status graph_steps_locked(int prec, Seg* dsegs, int nseg, const Launch& L, int slab, int cmax, int nsteps,
                              hipStream_t st, int dev, hipEvent_t t0, hipEvent_t t1) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  hipStream_t gs;
  auto its = g_graph_stream.find(dev);
  if (its == g_graph_stream.end()) {
    RDM_HIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    g_graph_stream[dev] = gs;
  } else {
    gs = its->second;
  }
  const GraphKey key{dev, dsegs, nseg, L.norm, L.apply, L.wide, L.xz, slab, cmax, prec, nsteps, launch_variants(L)};
  hipGraphExec_t exec = nullptr;
  auto it = g_graphs.find(key);
  if (it != g_graphs.end()) {
    exec = it->second;
  } else {
    hipGraph_t graph = nullptr;
    RDM_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    rdm_status s = RDM_OK;
    for (int i = 0; i < nsteps && s == RDM_OK; ++i) s = launch_step(prec, dsegs, nseg, L, slab, cmax, gs, nullptr);
    const hipError_t e = hipStreamEndCapture(gs, &graph);
    if (s != RDM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    RDM_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    RDM_HIP(ei);
    if (g_graphs.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(g_graphs[g_graph_order.front()]);
      g_graphs.erase(g_graph_order.front());
      g_graph_order.erase(g_graph_order.begin());
    }
    g_graphs[key] = exec;
    g_graph_order.push_back(key);
  }
  hipEvent_t before, after;
  RDM_HIP(hipEventCreateWithFlags(&before, hipEventDisableTiming));
  const hipError_t e1 = hipEventCreateWithFlags(&after, hipEventDisableTiming);
  if (e1 != hipSuccess) {
    (void)hipEventDestroy(before);
    RDM_HIP(e1);
  }
  hipError_t e = hipEventRecord(before, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(gs, before, 0);
  if (e == hipSuccess && t0) e = hipEventRecord(t0, gs);
  if (e == hipSuccess) e = hipGraphLaunch(exec, gs);
  if (e == hipSuccess && t1) e = hipEventRecord(t1, gs);
  if (e == hipSuccess) e = hipEventRecord(after, gs);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, after, 0);
  (void)hipEventDestroy(before);
  (void)hipEventDestroy(after);
  RDM_HIP(e);
  return RDM_OK;
}

}  // namespace

rdm_status run_phase(std::vector<Seg>& hsegs, Seg* dsegs, int prec, int phase, hipStream_t st,
                     StepTimers* tm, bool tune, bool graph, ReplayTimer* rt) {
  if (hsegs.empty()) return RDM_OK;
  for (const auto& sg : hsegs)
    if ((sg.xy || (sg.xz && prec == RDM_FP64)) && !sg.Y) {
      set_error("internal: a transform segment that needs the Y block has none");
      return RDM_E_INVALID;
    }
  int kmax = 0, cmax = 0;
  for (const auto& sg : hsegs) {
    kmax = std::max(kmax, sg.k);
    cmax = std::max(cmax, sg.cpad);
  }
  const int nseg = (int)hsegs.size();
  int slab = common_slab(hsegs);
  int j = 1;
  if (tune) {
    const SlabKey key = slab_key(prec, hsegs);
    int cached = -1;
    {
      std::lock_guard<std::mutex> lk(g_slab_mu);
      auto it = g_slab_best.find(key);
      if (it != g_slab_best.end()) cached = it->second;
    }
    std::vector<int> cands;
    for (int c = 1; c <= slab; c *= 2) cands.push_back(c);
    const int reps = 2;
    if (cached > 0) {
      slab = std::min(cached, slab);
    } else if (cands.size() > 1 && kmax >= 2 + reps * (int)cands.size()) {
      // steps 2.. run each candidate `reps` times between events; the best
      // one is kept for the remaining steps and for later launches of the
      // same shape
      std::vector<std::vector<Seg>> tabs(cands.size(), hsegs);
      std::vector<Launch> nt(cands.size());
      for (size_t c = 0; c < cands.size(); ++c) {
        set_slab(tabs[c], cands[c]);
        nt[c] = assign_tiles(tabs[c]);
      }
      std::vector<hipEvent_t> ev(2 * cands.size());
      for (auto& e : ev) RDM_HIP(hipEventCreate(&e));
      rdm_status s = RDM_OK;
      RDM_HIP(hipMemcpyAsync(dsegs, tabs[0].data(), nseg * sizeof(Seg), hipMemcpyHostToDevice, st));
      if ((s = init_run(prec, dsegs, nseg, cmax, phase, nt[0].xz, 0, st)) != RDM_OK) return s;
      s = launch_step(prec, dsegs, nseg, nt[0], cands[0], cmax, st, tm);
      ++j;
      for (size_t c = 0; c < cands.size() && s == RDM_OK; ++c) {
        RDM_HIP(hipMemcpyAsync(dsegs, tabs[c].data(), nseg * sizeof(Seg), hipMemcpyHostToDevice, st));
        RDM_HIP(hipEventRecord(ev[2 * c], st));
        for (int r = 0; r < reps && s == RDM_OK; ++r, ++j) s = launch_step(prec, dsegs, nseg, nt[c], cands[c], cmax, st, tm);
        RDM_HIP(hipEventRecord(ev[2 * c + 1], st));
      }
      RDM_HIP(hipStreamSynchronize(st));
      int best = 0;
      float best_ms = 1e30f;
      for (size_t c = 0; c < cands.size(); ++c) {
        float ms = 0.f;
        RDM_HIP(hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]));
        if (ms < best_ms) {
          best_ms = ms;
          best = (int)c;
        }
      }
      for (auto& e : ev) (void)hipEventDestroy(e);
      if (s != RDM_OK) return s;
      slab = cands[best];
      std::lock_guard<std::mutex> lk(g_slab_mu);
      g_slab_best[key] = slab;
    } else {
      slab = 1;
    }
  }
  set_slab(hsegs, slab);
  const Launch ntiles = assign_tiles(hsegs);
  RDM_HIP(hipMemcpyAsync(dsegs, hsegs.data(), nseg * sizeof(Seg), hipMemcpyHostToDevice, st));
  if (j == 1) {
    rdm_status s = init_run(prec, dsegs, nseg, cmax, phase, ntiles.xz, 0, st);
    if (s != RDM_OK) return s;
  }
  if (graph && !tm && kmax - j + 1 >= 2) {
    rdm_status s = graph_steps(prec, dsegs, nseg, ntiles, slab, cmax, kmax - j + 1, st, rt);
    if (s != RDM_OK) return s;
    j = kmax + 1;
  }
  for (; j <= kmax; ++j) {
    rdm_status s = launch_step(prec, dsegs, nseg, ntiles, slab, cmax, st, tm);
    if (s != RDM_OK) return s;
  }
  // the host table above must outlive the asynchronous copy
  RDM_HIP(hipStreamSynchronize(st));
  return RDM_OK;
}

rdm_status execute(std::vector<InstRun>& runs, char* ws, hipStream_t st, double tau, bool profile,
                   bool tune, bool graph, bool build_tables, bool replay_timing) {
  Range range("rdm execute");
  const int ni = (int)runs.size();
  if (ni == 0) return RDM_OK;
  const int prec = runs[0].plan->prec;
  std::vector<InstPlan> plans;
  for (auto& r : runs) plans.push_back(*r.plan);
  const size_t header = batch_header_bytes(plans);
  Seg* dsegs = (Seg*)ws;
  size_t inst_off = header;
  for (auto& r : runs) {
    r.base = ws + inst_off;
    inst_off += r.plan->bytes;
    rdm_status s = bind_ops(r, st, build_tables);
    if (s != RDM_OK) return s;
  }
  StepTimers tm;
  tm.apply.on = tm.norm.on = tm.xz1.on = profile;
  ReplayTimer rt;
  // pass 1: every total and bath segment in the same launches
  std::vector<Seg> segs;
  for (auto& r : runs) {
    segs.push_back(seg_of(r, 0, MODE_LANCZOS, tau));
    segs.push_back(seg_of(r, 1, MODE_LANCZOS, tau));
  }
  rdm_status s;
  {
    Range lr("rdm lanczos");
    s = run_phase(segs, dsegs, prec, 0, st, profile ? &tm : nullptr, tune, graph, replay_timing ? &rt : nullptr);
  }
  if (s != RDM_OK) return s;
  {
    Range hr("rdm host phase");
    for (auto& r : runs) r.status = host_phase(r, st);
  }
  // pass 2 (two-pass plans): regenerate u_j from the stored coefficients
  segs.clear();
  for (auto& r : runs)
    if (r.plan->two_pass && r.status == RDM_OK) segs.push_back(seg_of(r, 0, MODE_REGEN, tau));
  {
    Range rr("rdm regeneration");
    if ((s = run_phase(segs, dsegs, prec, 1, st, nullptr, tune, graph, replay_timing ? &rt : nullptr)) != RDM_OK)
      return s;
  }
  Timers tg;
  tg.on = profile;
  {
    Range gr("rdm gram");
    for (auto& r : runs) {
      if (r.status != RDM_OK) continue;
      if ((s = gram_phase(r, st, profile ? &tg : nullptr)) != RDM_OK) return s;
    }
  }
  for (auto& r : runs) {
    r.replay_steps = rt.steps;
    r.t_replay_ms = rt.steps ? rt.ms / rt.steps : 0.0;
  }
  if (profile)
    for (auto& r : runs) {
      r.t_apply_ms = tm.apply.avg_ms();
      r.t_norm_ms = tm.norm.avg_ms();
      r.t_xz1_ms = tm.xz1.avg_ms();
      r.t_gram_ms = tg.avg_ms();
    }
  return RDM_OK;
}

// A9: rho*, H*, ln Z*, S from the averaged Gram and the bath scalar.
rdm_status finalize(const InstRun& r, rdm_result* out) {
  const InstPlan& p = *r.plan;
  const int ds = p.ds;
  const double ln_db = p.h->n_b * std::log(2.0);
  double ratio_last = 0.0;
  std::vector<double> m(ds * ds), w(ds), v(ds * ds);
  for (int b = 0; b < p.n_beta; ++b) {
    std::fill(m.begin(), m.end(), 0.0);
    for (int jv = 0; jv < p.n_v; ++jv)
      for (int t = 0; t < ds * ds; ++t) m[t] += r.gsum[((size_t)b * p.n_v + jv) * ds * ds + t];
    for (int t = 0; t < ds * ds; ++t) m[t] /= p.n_v;
    for (int x = 0; x < ds; ++x)
      for (int y = x + 1; y < ds; ++y) {
        const double a = 0.5 * (m[x * ds + y] + m[y * ds + x]);
        m[x * ds + y] = m[y * ds + x] = a;
      }
    double tr = 0.0;
    for (int x = 0; x < ds; ++x) tr += m[x * ds + x];
    const double beta = r.betas[b];
    const double mb = r.mb[b];
    if (!(tr > 0.0) || !(mb > 0.0) || !std::isfinite(tr) || !std::isfinite(mb)) {
      set_error("non-positive or non-finite trace in finalisation");
      return RDM_E_NONFINITE;
    }
    sym_eig_small(ds, m.data(), w.data(), v.data());
    const double mu_max = w[ds - 1];
    double mu_sum = 0.0;
    for (int x = 0; x < ds; ++x) mu_sum += w[x];
    const double ln_zt = std::log(tr) - beta * r.e0 + ln_db;
    const double ln_zb = std::log(mb) - beta * r.e0b + ln_db;
    if (out->rho)
      for (int t = 0; t < ds * ds; ++t) out->rho[(size_t)b * ds * ds + t] = m[t] / tr;
    if (out->h_star) {
      std::vector<double> he(ds);
      for (int x = 0; x < ds; ++x) {
        const double mu = std::max(w[x], mu_max * std::ldexp(1.0, -52));
        he[x] = -std::log(mu / mb) / beta + r.e0 - r.e0b;
      }
      for (int x = 0; x < ds; ++x)
        for (int y = 0; y < ds; ++y) {
          double acc = 0.0;
          for (int q = 0; q < ds; ++q) acc += v[x * ds + q] * he[q] * v[y * ds + q];
          out->h_star[(size_t)b * ds * ds + x * ds + y] = acc;
        }
    }
    if (out->log_z) out->log_z[b] = ln_zt - ln_zb;
    if (out->entropy) {
      double sum = 0.0;
      for (int x = 0; x < ds; ++x) {
        const double pp = w[x] / mu_sum;
        if (pp > 0.0) sum -= pp * std::log(pp);
      }
      out->entropy[b] = sum;
    }
    if (out->diag) {
      out->diag[kDiagFixed + 2 * b] = ln_zt;
      out->diag[kDiagFixed + 2 * b + 1] = ln_zb;
    }
    ratio_last = w[0] / mu_max;
  }
  if (out->diag) {
    double* d = out->diag;
    d[0] = r.e0;
    d[1] = r.e0b;
    d[2] = r.n_break_t;
    d[3] = r.n_break_b;
    d[4] = p.two_pass ? 1.0 : 0.0;
    d[5] = (double)p.bytes;
    d[6] = ratio_last;
    d[7] = r.t_apply_ms;
    d[8] = r.t_norm_ms;
    d[9] = r.t_gram_ms;
    d[10] = r.t_xz1_ms;
    d[11] = r.t_replay_ms;
    d[12] = r.replay_steps;
    for (int t = 13; t < kDiagFixed; ++t) d[t] = 0.0;
  }
  return RDM_OK;
}

rdm_status lanczos_only(const rdm_hamiltonian* h, int which, int n_v, int k, uint64_t seed, int prec,
                        int slab, int rpl, double tau, hipStream_t st, double* alpha, double* beta,
                        int32_t* kc) {
  SegPlan g;
  const int nbits = which == 0 ? h->n : h->n_b;
  const int C = which == 0 ? (1 << h->n_s) * n_v : n_v;
  const int kk = (int)std::min<uint64_t>((uint64_t)k, 1ull << nbits);
  const size_t base_off = al(sizeof(Seg));
  size_t off = base_off;
  plan_seg(g, nbits, C, kk, prec, slab, rpl, 2, off, lanczos_needs_ybuf(h, which, prec));
  char* ws = nullptr;
  RDM_HIP(hipMalloc(&ws, off));
  const OpDevice* op = nullptr;
  rdm_status s = get_device_op(h, which, prec, st, &op);
  if (s != RDM_OK) {
    (void)hipFree(ws);
    return s;
  }
  std::vector<Seg> segs;
  // plan_seg laid the segment out from offset base_off, so its offsets are
  // relative to ws itself
  segs.push_back(make_seg(g, op, ws, MODE_LANCZOS, which == 0 ? START_SYSBATH : START_BATH, h->n_s, h->n_b,
                          seed, tau));
  s = run_phase(segs, (Seg*)ws, prec, 0, st, nullptr, slab == 0, false);
  HostHist hh;
  if (s == RDM_OK) s = fetch_hist(g, ws, hh, st);
  if (s == RDM_OK && hipStreamSynchronize(st) != hipSuccess) {
    set_error("hipStreamSynchronize failed");
    s = RDM_E_DEVICE;
  }
  (void)hipFree(ws);
  if (s != RDM_OK) return s;
  for (int j = 0; j < k; ++j)
    for (int c = 0; c < C; ++c) {
      alpha[(size_t)j * C + c] = j < kk ? hh.a[(size_t)j * g.cpad + c] : 0.0;
      beta[(size_t)j * C + c] = j < kk ? hh.b[(size_t)j * g.cpad + c] : 0.0;
    }
  for (int c = 0; c < C; ++c) kc[c] = hh.kc[c];
  return RDM_OK;
}

}  // namespace rdm
