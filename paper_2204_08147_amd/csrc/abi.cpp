// extern "C" entry points of the solver (argument checks, planning, memory).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "host.h"
#include "solve.h"

using namespace rdm;

namespace {

struct Opts {
  int prec = RDM_FP64, mode = RDM_AUTO, slab = 0, rpl = 0;
  uint64_t budget = 0;
  double tau = 0;
  int profile = 0;     // 1: event-timed kernels (eager), 2: timed graph replays
  bool eager = false;  // no hipGraph replay of the Lanczos steps
  int method = RDM_PER_COLUMN;
};

rdm_status read_opts(const rdm_options* o, Opts& r) {
  if (o) {
    r.prec = o->precision;
    r.mode = o->mode;
    r.budget = o->hbm_budget;
    r.slab = o->slab;
    r.rpl = o->rows_per_lane;
    r.tau = o->tau;
    r.profile = o->profile;
    r.eager = o->eager != 0;
    r.method = o->method;
    if (o->reserved != 0) {
      set_error("options: reserved must be 0");
      return RDM_E_INVALID;
    }
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
  if (r.profile < 0 || r.profile > 2) {
    set_error("options: profile must be 0, 1 or 2");
    return RDM_E_INVALID;
  }
  if (r.method != RDM_PER_COLUMN && r.method != RDM_BLOCK && r.method != RDM_METHOD_AUTO) {
    set_error("options: method must be RDM_PER_COLUMN, RDM_BLOCK or RDM_METHOD_AUTO");
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

// RDM_METHOD_AUTO: the per-column path when its plan keeps the Lanczos basis
// within the budget, else the block variant, which keeps three blocks and
// needs no regeneration pass (a mode other than RDM_AUTO keeps the per-column
// path).  Call after the budget is known.
static rdm_status resolve_method(Opts& o, const rdm_hamiltonian* h, int n_beta, int n_v, int k) {
  if (o.method != RDM_METHOD_AUTO) return RDM_OK;
  o.method = RDM_PER_COLUMN;
  if (o.mode != RDM_AUTO || h->n_s > 3) return RDM_OK;  // the block variant takes d_s <= 8
  std::vector<InstPlan> plans(1);
  const rdm_status s = plan_instance(plans[0], h, n_beta, n_v, k, o.prec, o.mode, o.budget, o.slab, o.rpl);
  if (s == RDM_E_NOMEM || (s == RDM_OK && plans[0].two_pass)) o.method = RDM_BLOCK;
  else if (s != RDM_OK) return s;
  return RDM_OK;
}

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
  if ((s = resolve_method(o, h, n_beta, n_v, k)) != RDM_OK) return s;
  if (o.method == RDM_BLOCK) {
    BlockPlan bp;
    if ((s = block_plan(bp, h, n_beta, n_v, k, o.prec, o.budget)) != RDM_OK) return s;
    *bytes = bp.bytes;
    return RDM_OK;
  }
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
  if ((s = resolve_method(o, h, n_beta, n_v, k)) != RDM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  if (o.method == RDM_BLOCK) {
    BlockPlan bp;
    if ((s = block_plan(bp, h, n_beta, n_v, k, o.prec, o.budget)) != RDM_OK) return s;
    char* ws = (char*)dev_ws;
    bool owned = false;
    if (ws) {
      if (ws_bytes < bp.bytes || ((uintptr_t)ws & 255)) {
        set_error("workspace too small or not 256-byte aligned: need " + std::to_string(bp.bytes));
        return RDM_E_INVALID;
      }
    } else {
      RDM_HIP(hipMalloc(&ws, bp.bytes));
      owned = true;
    }
    s = block_solve(bp, beta, seed, o.tau, ws, st, o.profile == 1, out);
    if (owned) (void)hipFree(ws);
    return s;
  }
  std::vector<InstPlan> plans(1);
  s = plan_instance(plans[0], h, n_beta, n_v, k, o.prec, o.mode, o.budget, o.slab, o.rpl);
  if (s != RDM_OK) return s;
  const size_t need = batch_header_bytes(plans) + plans[0].bytes;
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
  s = execute(runs, ws, st, o.tau, o.profile == 1, o.slab == 0, !o.eager, true, o.profile == 2);
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

// ---------------------------------------------------------------------------
// rdm_solve_noalloc: the per-column solve with its workspace in a fixed
// device array of this library instead of memory it allocates.  The array is
// part of the code object: each device the library runs on holds its own copy
// until the process ends.  Host code must never pass the array's name to a
// kernel or a copy (in host code it names a host-side stand-in): the device
// address of this device's copy comes from hipGetSymbolAddress, once per
// device, and is kept below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[RDM_NOALLOC_MAX_BYTES];

namespace {

std::mutex g_noalloc_mu;             // serialises the calls: one array per device
std::map<int, char*> g_noalloc_ptr;  // device -> address of its copy of the array

rdm_status noalloc_workspace(char** out) {
  int dev = 0;
  RDM_HIP(hipGetDevice(&dev));
  auto it = g_noalloc_ptr.find(dev);
  if (it == g_noalloc_ptr.end()) {
    void* ptr = nullptr;
    RDM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) {
      set_error("rdm_solve_noalloc: bad device address of the scratch array");
      return RDM_E_DEVICE;
    }
    it = g_noalloc_ptr.emplace(dev, (char*)ptr).first;
  }
  *out = it->second;
  return RDM_OK;
}

}  // namespace

extern "C" rdm_status rdm_solve_noalloc(const rdm_hamiltonian* h, const double* beta, int32_t n_beta,
                                        int32_t n_v, int32_t k, uint64_t seed, const rdm_options* opt,
                                        void* hip_stream, rdm_result* out) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if ((s = check_solve_args(h, beta, n_beta, n_v, k)) != RDM_OK) return s;
  if (!out) {
    set_error("NULL result");
    return RDM_E_INVALID;
  }
  if (o.method == RDM_BLOCK || o.profile) {
    set_error("rdm_solve_noalloc: the per-column method only, without profiling");
    return RDM_E_INVALID;
  }
  // the plan must fit the array (two-pass if the stored basis does not)
  const uint64_t cap = RDM_NOALLOC_MAX_BYTES;
  o.budget = o.budget ? std::min<uint64_t>(o.budget, cap) : cap;
  std::vector<InstPlan> plans(1);
  s = plan_instance(plans[0], h, n_beta, n_v, k, o.prec, o.mode, o.budget, o.slab, o.rpl);
  if (s == RDM_E_NOMEM) {
    set_error("rdm_solve_noalloc: the instance needs more than the " + std::to_string(cap >> 20) +
              " MiB scratch array even with two passes");
    return RDM_E_NOMEM;
  }
  if (s != RDM_OK) return s;
  const size_t need = batch_header_bytes(plans) + plans[0].bytes;
  if (need > cap) {
    set_error("rdm_solve_noalloc: the instance needs " + std::to_string(need) + " bytes, the scratch array holds " +
              std::to_string(cap));
    return RDM_E_NOMEM;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  char* ws = nullptr;
  if ((s = noalloc_workspace(&ws)) != RDM_OK) return s;
  std::vector<InstRun> runs(1);
  runs[0].plan = &plans[0];
  runs[0].betas.assign(beta, beta + n_beta);
  runs[0].seed = seed;
  // eager launches (no graph capture, no slab timing events), resident
  // tables only: nothing below allocates device memory
  s = execute(runs, ws, (hipStream_t)hip_stream, o.tau, false, false, false, false);
  if (s == RDM_OK) s = runs[0].status;
  if (s == RDM_OK) s = finalize(runs[0], out);
  return s;
}

namespace {

// Plan every item; invalid ones get their status and are left out.
rdm_status plan_batch(int32_t n_items, rdm_batch_item* items, const Opts& o, std::vector<InstPlan>& plans,
                      std::vector<int>& valid) {
  rdm_status first = RDM_OK;
  plans.assign(n_items, InstPlan{});
  valid.clear();
  for (int i = 0; i < n_items; ++i) {
    rdm_batch_item& it = items[i];
    it.status = check_solve_args(it.h, it.beta, it.n_beta, it.n_v, it.k);
    if (it.status == RDM_OK)
      it.status = plan_instance(plans[i], it.h, it.n_beta, it.n_v, it.k, o.prec, o.mode, o.budget, o.slab,
                                o.rpl);
    if (it.status == RDM_OK)
      valid.push_back(i);
    else if (first == RDM_OK)
      first = it.status;
  }
  return first;
}

// Greedy waves, largest instances first, each fitting in `budget` bytes.
std::vector<std::vector<int>> make_waves(const std::vector<InstPlan>& plans, std::vector<int> valid,
                                         uint64_t budget, size_t* max_need) {
  std::sort(valid.begin(), valid.end(), [&](int a, int b) { return plans[a].bytes > plans[b].bytes; });
  std::vector<std::vector<int>> waves;
  *max_need = 0;
  size_t pos = 0;
  while (pos < valid.size()) {
    std::vector<int> wave;
    std::vector<InstPlan> wp;
    size_t used = 0;
    while (pos < valid.size()) {
      const InstPlan& p = plans[valid[pos]];
      wp.push_back(p);
      const size_t need = batch_header_bytes(wp) + used + p.bytes;
      if (!wave.empty() && need > budget) {
        wp.pop_back();
        break;
      }
      wave.push_back(valid[pos]);
      used += p.bytes;
      ++pos;
    }
    *max_need = std::max(*max_need, batch_header_bytes(wp) + used);
    waves.push_back(wave);
  }
  return waves;
}

rdm_status batch_impl(int32_t n_items, rdm_batch_item* items, const rdm_options* opt, void* hip_stream,
                      void* dev_ws, uint64_t ws_bytes) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (n_items < 0 || (n_items > 0 && !items)) {
    set_error("rdm_solve_batch: bad item list");
    return RDM_E_INVALID;
  }
  if (o.method == RDM_BLOCK) {
    set_error("batched solves use the per-column method");
    return RDM_E_INVALID;
  }
  if (dev_ws && !o.budget) o.budget = ws_bytes;
  if ((s = default_budget(o.budget)) != RDM_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<InstPlan> plans;
  std::vector<int> valid;
  rdm_status first = plan_batch(n_items, items, o, plans, valid);
  size_t need = 0;
  const auto waves = make_waves(plans, valid, o.budget, &need);
  if (valid.empty()) return first;
  char* ws = (char*)dev_ws;
  bool owned = false;
  if (ws) {
    if (ws_bytes < need || ((uintptr_t)ws & 255)) {
      set_error("batch workspace too small or not 256-byte aligned: need " + std::to_string(need));
      return RDM_E_INVALID;
    }
  } else {
    RDM_HIP(hipMalloc(&ws, need));  // one allocation reused by every wave
    owned = true;
  }
  for (const auto& wave : waves) {
    std::vector<InstPlan> wave_plans;
    for (int i : wave) wave_plans.push_back(plans[i]);
    std::vector<InstRun> runs(wave.size());
    for (size_t w = 0; w < wave.size(); ++w) {
      runs[w].plan = &wave_plans[w];
      runs[w].betas.assign(items[wave[w]].beta, items[wave[w]].beta + items[wave[w]].n_beta);
      runs[w].seed = items[wave[w]].seed;
    }
    s = execute(runs, ws, st, o.tau, o.profile == 1, o.slab == 0, !o.eager, true, o.profile == 2);
    for (size_t w = 0; w < wave.size(); ++w) {
      rdm_batch_item& it = items[wave[w]];
      it.status = s != RDM_OK ? s : runs[w].status;
      if (it.status == RDM_OK) it.status = finalize(runs[w], &it.out);
      if (it.status != RDM_OK && first == RDM_OK) first = it.status;
    }
  }
  if (owned) (void)hipFree(ws);
  return first;
}

}  // namespace

extern "C" rdm_status rdm_solve_batch(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                                      void* hip_stream) {
  return batch_impl(n_items, items, opt, hip_stream, nullptr, 0);
}

extern "C" rdm_status rdm_solve_batch_ws(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                                         void* hip_stream, void* dev_workspace, uint64_t ws_bytes) {
  if (!dev_workspace) {
    set_error("rdm_solve_batch_ws: NULL workspace");
    return RDM_E_INVALID;
  }
  return batch_impl(n_items, items, opt, hip_stream, dev_workspace, ws_bytes);
}

extern "C" rdm_status rdm_batch_workspace_size(int32_t n_items, rdm_batch_item* items, const rdm_options* opt,
                                               uint64_t* min_bytes, uint64_t* all_bytes) {
  Opts o;
  rdm_status s = read_opts(opt, o);
  if (s != RDM_OK) return s;
  if (n_items < 0 || (n_items > 0 && !items) || !min_bytes || !all_bytes) {
    set_error("rdm_batch_workspace_size: bad arguments");
    return RDM_E_INVALID;
  }
  if ((s = default_budget(o.budget)) != RDM_OK) return s;
  std::vector<InstPlan> plans;
  std::vector<int> valid;
  plan_batch(n_items, items, o, plans, valid);
  size_t mx = 0, sum = 0;
  std::vector<InstPlan> all;
  for (int i : valid) {
    mx = std::max(mx, plans[i].bytes);
    sum += plans[i].bytes;
    all.push_back(plans[i]);
  }
  std::vector<InstPlan> one(valid.empty() ? 0 : 1);
  *min_bytes = valid.empty() ? 0 : batch_header_bytes(one) + mx;
  *all_bytes = valid.empty() ? 0 : batch_header_bytes(all) + sum;
  return RDM_OK;
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
  sg.nbits = nbits;
  sg.n_row_tiles = g.n_row_tiles;
  bind_apply(sg, op);
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
  std::vector<Seg> one{sg};
  const Launch L = assign_tiles(one);
  sg = one[0];
  // the segment descriptor, then the scratch block of a YY transform part
  const size_t dbytes = align_up(sizeof(Seg));
  const size_t ybytes = sg.xy ? g.blk * (precision == RDM_FP64 ? 8 : 4) : 0;
  char* d = nullptr;
  RDM_HIP(hipMalloc(&d, dbytes + ybytes));
  if (sg.xy) sg.Y = d + dbytes;
  rdm_status r = RDM_OK;
  auto run = [&]() -> rdm_status {
    RDM_HIP(hipMemcpyAsync(d, &sg, sizeof(Seg), hipMemcpyHostToDevice, st));
    const int deep = xz_geom(sg.nbits);
    for (int pass = 0; pass <= 2; ++pass)
      RDM_HIP(precision == RDM_FP64 ? launch_xz_pass<double>(pass, (Seg*)d, 1, L.xz, st, deep)
                                    : launch_xz_pass<float>(pass, (Seg*)d, 1, L.xz, st, deep));
    if (sg.xy)
      for (int pass : {6, 7, 8})
        RDM_HIP(precision == RDM_FP64 ? launch_xz_pass<double>(pass, (Seg*)d, 1, L.xz, st, deep)
                                      : launch_xz_pass<float>(pass, (Seg*)d, 1, L.xz, st, deep));
    RDM_HIP(precision == RDM_FP64 ? launch_apply<double>((Seg*)d, 1, L.apply, g.S, st)
                                  : launch_apply<float>((Seg*)d, 1, L.apply, g.S, st));
    RDM_HIP(precision == RDM_FP64 ? launch_apply_wide<double>((Seg*)d, 1, L.wide, st)
                                  : launch_apply_wide<float>((Seg*)d, 1, L.wide, st));
    RDM_HIP(hipStreamSynchronize(st));
    return RDM_OK;
  };
  r = run();
  (void)hipFree(d);
  return r;
}

extern "C" rdm_status rdm_start_block(const rdm_hamiltonian* h, int32_t which, int32_t precision,
                                      int32_t n_v, uint64_t seed, void* out, void* hip_stream) {
  if (!h || which < 0 || which > 2 || (precision != RDM_FP64 && precision != RDM_MIXED) || n_v < 1 || !out) {
    set_error("rdm_start_block: bad arguments");
    return RDM_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const int nbits = which == 1 ? h->n_b : h->n;
  const int C = which == 0 ? (1 << h->n_s) * n_v : n_v;
  const int W = precision == RDM_FP64 ? 2 : 4;
  const int cpad = (C + W - 1) / W * W;
  const int kind = which == 0 ? START_SYSBATH : which == 1 ? START_BATH : START_PRODUCT;
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
