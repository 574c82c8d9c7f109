// extern "C" entry points of the solver (argument checks, planning, memory).
#include <cmath>
#include <cstring>

#include "host.h"
#include "solve.h"

using namespace rdm;

namespace {

struct Opts {
  int prec = RDM_FP64, mode = RDM_AUTO, slab = 0, rpl = 0;
  uint64_t budget = 0;
  double tau = 0;
  bool profile = false;
};

rdm_status read_opts(const rdm_options* o, Opts& r) {
  if (o) {
    r.prec = o->precision;
    r.mode = o->mode;
    r.budget = o->hbm_budget;
    r.slab = o->slab;
    r.rpl = o->rows_per_lane;
    r.tau = o->tau;
    r.profile = o->reserved[0] != 0;
  }
  if (r.prec != RDM_FP64 && r.prec != RDM_MIXED) {
    set_error("options: precision must be RDM_FP64 or RDM_MIXED");
    return RDM_E_INVALID;
  }
  if (r.mode < RDM_AUTO || r.mode > RDM_TWO_PASS) {
    set_error("options: bad mode");
    return RDM_E_INVALID;
  }
  if (r.slab < 0 || r.slab > kMaxSlab || (r.slab & (r.slab - 1)) || r.rpl < 0 || r.rpl > 64) {
    set_error("options: slab must be 0, 1, 2 or 4 and rows_per_lane in [0, 64]");
    return RDM_E_INVALID;
  }
  if (!(r.tau >= 0.0) || !std::isfinite(r.tau)) {
    set_error("options: tau must be finite and >= 0");
    return RDM_E_INVALID;
  }
  if (r.tau == 0.0) r.tau = r.prec == RDM_FP64 ? 1e-12 : 1e-5;
  return RDM_OK;
}

rdm_status check_solve_args(const rdm_hamiltonian* h, const double* beta, int32_t n_beta, int32_t n_v,
                            int32_t k) {
  if (!h) {
    set_error("NULL Hamiltonian");
    return RDM_E_INVALID;
  }
  if (n_beta < 1 || !beta) {
    set_error("need n_beta >= 1 inverse temperatures");
    return RDM_E_INVALID;
  }
  for (int b = 0; b < n_beta; ++b)
    if (!(beta[b] > 0.0) || !std::isfinite(beta[b])) {
      set_error("every beta must be finite and > 0");
      return RDM_E_INVALID;
    }
  if (n_v < 1 || k < 1 || k > 4096) {
    set_error("need n_v >= 1 and 1 <= k <= 4096");
    return RDM_E_INVALID;
  }
  return RDM_OK;
}

rdm_status default_budget(uint64_t& budget) {
  if (budget) return RDM_OK;
  size_t fr = 0, tot = 0;
  RDM_HIP(hipMemGetInfo(&fr, &tot));
  const uint64_t reserve = 2ull << 30;
  budget = fr > reserve ? fr - reserve : fr / 2;
  return RDM_OK;
}

}  // namespace

extern "C" rdm_status rdm_workspace_size(const rdm_hamiltonian* h, int32_t n_beta, int32_t n_v,
                                         int32_t k, const rdm_options* opt, uint64_t* bytes) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (!h || n_beta < 1 || n_v < 1 || k < 1 || !bytes) {
    set_error("rdm_workspace_size: bad arguments");
    return RDM_E_INVALID;
  }
  if ((s = default_budget(o.budget)) != RDM_OK) return s;
  std::vector<InstPlan> plans(1);
  s = plan_instance(plans[0], h, n_beta, n_v, k, o.prec, o.mode, o.budget, o.slab, o.rpl);
  if (s != RDM_OK) return s;
  *bytes = batch_header_bytes(plans) + plans[0].bytes;
  return RDM_OK;
}

static rdm_status solve_impl(const rdm_hamiltonian* h, const double* beta, int32_t n_beta, int32_t n_v,
                             int32_t k, uint64_t seed, const rdm_options* opt, void* hip_stream,
                             rdm_result* out, void* dev_ws, uint64_t ws_bytes) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if ((s = check_solve_args(h, beta, n_beta, n_v, k)) != RDM_OK) return s;
  if (!out) {
    set_error("NULL result");
    return RDM_E_INVALID;
  }
  if (dev_ws && !o.budget) o.budget = ws_bytes;
  if ((s = default_budget(o.budget)) != RDM_OK) return s;
  std::vector<InstPlan> plans(1);
  s = plan_instance(plans[0], h, n_beta, n_v, k, o.prec, o.mode, o.budget, o.slab, o.rpl);
  if (s != RDM_OK) return s;
  const size_t need = batch_header_bytes(plans) + plans[0].bytes;
  hipStream_t st = (hipStream_t)hip_stream;
  char* ws = (char*)dev_ws;
  bool owned = false;
  if (ws) {
    if (ws_bytes < need || ((uintptr_t)ws & 255)) {
      set_error("workspace too small or not 256-byte aligned: need " + std::to_string(need));
      return RDM_E_INVALID;
    }
  } else {
    RDM_HIP(hipMalloc(&ws, need));
    owned = true;
  }
  std::vector<InstRun> runs(1);
  runs[0].plan = &plans[0];
  runs[0].betas.assign(beta, beta + n_beta);
  runs[0].seed = seed;
  s = execute(runs, ws, st, o.tau, o.profile);
  if (s == RDM_OK) s = runs[0].status;
  if (s == RDM_OK) s = finalize(runs[0], out);
  if (owned) (void)hipFree(ws);
  return s;
}

extern "C" rdm_status rdm_solve(const rdm_hamiltonian* h, const double* beta, int32_t n_beta,
                                int32_t n_v, int32_t k, uint64_t seed, const rdm_options* opt,
                                void* hip_stream, rdm_result* out) {
  return solve_impl(h, beta, n_beta, n_v, k, seed, opt, hip_stream, out, nullptr, 0);
}

extern "C" rdm_status rdm_solve_ws(const rdm_hamiltonian* h, const double* beta, int32_t n_beta,
                                   int32_t n_v, int32_t k, uint64_t seed, const rdm_options* opt,
                                   void* hip_stream, rdm_result* out, void* dev_workspace,
                                   uint64_t ws_bytes) {
  if (!dev_workspace) {
    set_error("rdm_solve_ws: NULL workspace");
    return RDM_E_INVALID;
  }
  return solve_impl(h, beta, n_beta, n_v, k, seed, opt, hip_stream, out, dev_workspace, ws_bytes);
}

extern "C" rdm_status rdm_solve_batch(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                                      void* hip_stream) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (n_items < 0 || (n_items > 0 && !items)) {
    set_error("rdm_solve_batch: bad item list");
    return RDM_E_INVALID;
  }
  if ((s = default_budget(o.budget)) != RDM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<InstPlan> plans(n_items);
  rdm_status first = RDM_OK;
  std::vector<int> valid;
  for (int i = 0; i < n_items; ++i) {
    rdm_batch_item& it = items[i];
    it.status = check_solve_args(it.h, it.beta, it.n_beta, it.n_v, it.k);
    if (it.status == RDM_OK)
      it.status = plan_instance(plans[i], it.h, it.n_beta, it.n_v, it.k, o.prec, o.mode, o.budget,
                                o.slab, o.rpl);
    if (it.status == RDM_OK)
      valid.push_back(i);
    else if (first == RDM_OK)
      first = it.status;
  }
  // waves of instances that fit in the budget together (largest first)
  std::sort(valid.begin(), valid.end(), [&](int a, int b) { return plans[a].bytes > plans[b].bytes; });
  size_t pos = 0;
  while (pos < valid.size()) {
    std::vector<InstPlan> wave_plans;
    std::vector<int> wave;
    size_t used = 0;
    while (pos < valid.size()) {
      const InstPlan& p = plans[valid[pos]];
      std::vector<InstPlan> trial = wave_plans;
      trial.push_back(p);
      const size_t need = batch_header_bytes(trial) + used + p.bytes;
      if (!wave.empty() && need > o.budget) break;
      wave_plans.push_back(p);
      wave.push_back(valid[pos]);
      used += p.bytes;
      ++pos;
    }
    const size_t need = batch_header_bytes(wave_plans) + used;
    char* ws = nullptr;
    RDM_HIP(hipMalloc(&ws, need));
    std::vector<InstRun> runs(wave.size());
    for (size_t w = 0; w < wave.size(); ++w) {
      runs[w].plan = &wave_plans[w];
      runs[w].betas.assign(items[wave[w]].beta, items[wave[w]].beta + items[wave[w]].n_beta);
      runs[w].seed = items[wave[w]].seed;
    }
    s = execute(runs, ws, st, o.tau, o.profile);
    (void)hipFree(ws);
    for (size_t w = 0; w < wave.size(); ++w) {
      rdm_batch_item& it = items[wave[w]];
      it.status = s != RDM_OK ? s : runs[w].status;
      if (it.status == RDM_OK) it.status = finalize(runs[w], &it.out);
      if (it.status != RDM_OK && first == RDM_OK) first = it.status;
    }
  }
  return first;
}

extern "C" rdm_status rdm_apply(const rdm_hamiltonian* h, int32_t which, int32_t precision,
                                int32_t n_cols, const void* x, void* y, const rdm_options* opt,
                                void* hip_stream) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (!h || (which != 0 && which != 1) || (precision != RDM_FP64 && precision != RDM_MIXED) ||
      n_cols < 1 || !x || !y || x == y) {
    set_error("rdm_apply: bad arguments");
    return RDM_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const OpDevice* op = nullptr;
  if ((s = get_device_op(h, which, precision, st, &op)) != RDM_OK) return s;
  SegPlan g;
  size_t off = 0;
  const int nbits = which == 0 ? h->n : h->n_b;
  plan_seg(g, nbits, n_cols, 1, precision, o.slab, o.rpl, 1, off);
  Seg sg{};
  sg.hopU = op->hopU;
  sg.hopP = op->hopP;
  sg.diag = op->diag;
  sg.nU = op->nU;
  sg.nP = op->nP;
  sg.nPh = op->nPh;
  sg.nbits = nbits;
  sg.P = g.P;
  sg.S = g.S;
  sg.rpl = g.rpl;
  sg.C = n_cols;
  sg.cpad = g.cpad;
  sg.k = 1;
  sg.mode = MODE_PLAIN;
  sg.blk = g.blk;
  sg.Q = (void*)x;
  sg.R = y;
  std::vector<Tile> tiles;
  for (int rt = 0; rt < g.n_row_tiles; ++rt)
    for (int p0 = 0; p0 < g.P; p0 += g.S)
      tiles.push_back(Tile{0, (uint32_t)((uint64_t)rt * kBlock * g.rpl), p0, rt});
  char* d = nullptr;
  const size_t tb = tiles.size() * sizeof(Tile);
  RDM_HIP(hipMalloc(&d, 256 + tb));
  rdm_status r = RDM_OK;
  auto run = [&]() -> rdm_status {
    RDM_HIP(hipMemcpyAsync(d, &sg, sizeof(Seg), hipMemcpyHostToDevice, st));
    RDM_HIP(hipMemcpyAsync(d + 256, tiles.data(), tb, hipMemcpyHostToDevice, st));
    if (precision == RDM_FP64)
      RDM_HIP(launch_apply<double>((Seg*)d, (Tile*)(d + 256), (int)tiles.size(), g.S, st));
    else
      RDM_HIP(launch_apply<float>((Seg*)d, (Tile*)(d + 256), (int)tiles.size(), g.S, st));
    RDM_HIP(hipStreamSynchronize(st));
    return RDM_OK;
  };
  r = run();
  (void)hipFree(d);
  return r;
}

extern "C" rdm_status rdm_start_block(const rdm_hamiltonian* h, int32_t which, int32_t precision,
                                      int32_t n_v, uint64_t seed, void* out, void* hip_stream) {
  if (!h || (which != 0 && which != 1) || (precision != RDM_FP64 && precision != RDM_MIXED) || n_v < 1 ||
      !out) {
    set_error("rdm_start_block: bad arguments");
    return RDM_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const int nbits = which == 0 ? h->n : h->n_b;
  const int C = which == 0 ? (1 << h->n_s) * n_v : n_v;
  const int W = precision == RDM_FP64 ? 2 : 4;
  const int cpad = (C + W - 1) / W * W;
  const int kind = which == 0 ? START_SYSBATH : START_BATH;
  if (precision == RDM_FP64)
    RDM_HIP(launch_start_block<double>(h->n_s, h->n_b, C, seed, kind, (double*)out, nbits, cpad, st));
  else
    RDM_HIP(launch_start_block<float>(h->n_s, h->n_b, C, seed, kind, (float*)out, nbits, cpad, st));
  return RDM_OK;
}

extern "C" rdm_status rdm_lanczos(const rdm_hamiltonian* h, int32_t which, int32_t n_v, int32_t k,
                                  uint64_t seed, const rdm_options* opt, void* hip_stream,
                                  double* host_alpha, double* host_beta, int32_t* host_kc) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (!h || (which != 0 && which != 1) || n_v < 1 || k < 1 || k > 4096 || !host_alpha || !host_beta ||
      !host_kc) {
    set_error("rdm_lanczos: bad arguments");
    return RDM_E_INVALID;
  }
  return lanczos_only(h, which, n_v, k, seed, o.prec, o.slab, o.rpl, o.tau, (hipStream_t)hip_stream,
                      host_alpha, host_beta, host_kc);
}
