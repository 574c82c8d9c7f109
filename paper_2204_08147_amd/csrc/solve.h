// Planning and execution of (batched) solves.
#pragma once

#include <functional>
#include <vector>

#include "host.h"

namespace rdm {

constexpr int kDiagFixed = 16;  // fixed entries of rdm_result.diag before the per-beta pairs

// Geometry and workspace offsets of one Lanczos segment.
struct SegPlan {
  int nbits = 0, C = 0, cpad = 0, P = 0, S = 1, rpl = 1, n_row_tiles = 0, k = 0, nslots = 0;
  uint64_t dim = 0, blk = 0;
  size_t o_Q = 0, o_R = 0, o_st = 0, o_ha = 0, o_hb = 0, o_hs = 0, o_part = 0, o_step = 0, o_kc = 0;
  int prec = 0;       // RDM_FP64 / RDM_MIXED
  bool ybuf = false;  // one more block (the YY part of a transform operator) at o_Y
  size_t o_Y = 0;
};
// Whether operator `which` of h (0: H_t, 1: H_b) is applied by the transform
// with a YY part, which needs the scratch block Y.
bool needs_ybuf(const rdm_hamiltonian* h, int which);
// Whether a Lanczos segment of operator `which` in precision prec needs the
// block Y: the YY part, and every FP64 transform step (Z = W_lo D_Z u_j
// between the contiguous pass and the next strided pass; the YY part uses Y
// only between those two, so one block serves both).
bool lanczos_needs_ybuf(const rdm_hamiltonian* h, int which, int prec);

struct InstPlan {
  const rdm_hamiltonian* h = nullptr;
  int prec = RDM_FP64, n_beta = 0, n_v = 0, k = 0, kb = 0;
  int ds = 2, ds_log = 1, cb = 2, groups_per_block = 1, n_cblocks = 0, nb_chunk = 1;
  int g_rpl = 1, g_rtiles = 0;
  bool two_pass = false;
  SegPlan tot, bath;
  size_t o_psi = 0, o_y = 0, o_gpart = 0, o_gsum = 0, o_gseg = 0, o_gtiles = 0;
  size_t bytes = 0;
};

// Event pairs recorded around kernel launches on the solve's stream.
struct Timers {
  bool on = false;
  std::vector<hipEvent_t> ev;
  Timers() = default;
  Timers(const Timers&) = delete;
  Timers& operator=(const Timers&) = delete;
  ~Timers() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipError_t mark(hipStream_t st) {
    if (!on) return hipSuccess;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    return hipEventRecord(e, st);
  }
  // mean duration of the (start, stop) pairs in ms (after the stream synced)
  double avg_ms() const {
    if (!on || ev.size() < 2) return 0.0;
    double tot = 0.0;
    int n = 0;
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) {
        tot += ms;
        ++n;
      }
    }
    return n ? tot / n : 0.0;
  }
};
// apply: hop-table apply and transform pass 2; norm: the norm kernel;
// xz1: transform pass 1 (norm step + high-bit transform)
struct StepTimers {
  Timers apply, norm, xz1;
};
// Replayed Lanczos steps timed as they run (rdm_options.profile = 2): HIP
// events around each graph replay on the replay stream.
struct ReplayTimer {
  double ms = 0.0;
  int steps = 0;
};

struct InstRun {
  const InstPlan* plan = nullptr;
  const OpDevice* op_t = nullptr;
  const OpDevice* op_b = nullptr;
  std::vector<double> betas;
  uint64_t seed = 0;
  char* base = nullptr;
  rdm_status status = RDM_OK;
  double e0 = 0, e0b = 0;
  int n_break_t = 0, n_break_b = 0;
  std::vector<double> mb, gsum;
  double t_apply_ms = 0, t_norm_ms = 0, t_gram_ms = 0, t_xz1_ms = 0;
  double t_replay_ms = 0;  // mean replayed step (ms) and steps replayed (profile = 2)
  int replay_steps = 0;
};

void plan_seg(SegPlan& g, int nbits, int C, int k, int prec, int slab_opt, int rpl_opt, int nslots,
              size_t& off, bool ybuf = false);
rdm_status plan_instance(InstPlan& p, const rdm_hamiltonian* h, int n_beta, int n_v, int k, int prec,
                         int mode_req, uint64_t budget, int slab_opt, int rpl_opt);
size_t batch_header_bytes(const std::vector<InstPlan>& plans);
// graph: replay the Lanczos steps as a captured hipGraph (unless profiling)
// build_tables = false: the operators' device tables must be resident
// already (nothing is allocated)
// replay_timing: time the replayed steps with HIP events (graphs kept)
rdm_status execute(std::vector<InstRun>& runs, char* ws, hipStream_t st, double tau, bool profile,
                   bool tune, bool graph, bool build_tables = true, bool replay_timing = false);

// Phases (used by execute and by the serving engine).
rdm_status bind_ops(InstRun& r, hipStream_t st, bool build_tables = true);
Seg seg_of(const InstRun& r, int which, int mode, double tau);
int common_slab(std::vector<Seg>& segs);
// Operator tables of a segment's apply (hop tables or transform).  Needs
// nbits and n_row_tiles set.
// A wide operator's segment takes the bit-set tables (Seg::wide).
void bind_apply(Seg& s, const OpDevice* op);
// workgroups of the norm launch and of the three kinds of apply launch
struct Launch {
  int norm = 0, apply = 0, xz = 0;
  int wide = 0;  // workgroups of the apply on bit-set tiles
  // transform segments in each mode, by strided geometry (XG_SHALLOW,
  // XG_DEEP, XG_SPLIT); xy: those with a YY part
  bool xz_lanczos[3] = {false, false, false}, xz_regen[3] = {false, false, false};
  bool xy[3] = {false, false, false};
  bool any_xy() const { return xy[0] || xy[1] || xy[2]; }
  bool any_split() const { return xz_lanczos[XG_SPLIT] || xz_regen[XG_SPLIT]; }
};
// sets every segment's tile_base / ap_base / wp_base / x_base
Launch assign_tiles(std::vector<Seg>& segs);
rdm_status launch_step(int prec, const Seg* dsegs, int nseg, const Launch& L, int slab, int cmax, hipStream_t st,
                       StepTimers* tm);
// Runs every step of a phase.  tune: choose the panels per lane by timing the
// first steps (cached per shape); otherwise the segments' own value is used.
// graph: the steps after tuning run as one captured hipGraph (not with tm).
// State initialisation of a run (phase 0) or regeneration pass (phase 1):
// per-column state, and the start block of the transform segments in the
// low-bit Hadamard basis (xz_tiles tiles from tile xz_boff).
rdm_status init_run(int prec, const Seg* dsegs, int nseg, int cmax, int phase, int xz_tiles, int xz_boff,
                    hipStream_t st);
rdm_status run_phase(std::vector<Seg>& hsegs, Seg* dsegs, int prec, int phase, hipStream_t st,
                     StepTimers* tm, bool tune, bool graph, ReplayTimer* rt = nullptr);
// Panels per lane for a launch over these segments: the cached measurement
// for the shape of the largest one, else one panel.
int tuned_slab(int prec, std::vector<Seg>& segs);
rdm_status host_phase(InstRun& r, hipStream_t st);   // synchronous
rdm_status gram_phase(InstRun& r, hipStream_t st, Timers* tg);  // synchronous
rdm_status finalize(const InstRun& r, rdm_result* out);

// helpers shared with the block-Lanczos driver
Seg make_plain_seg(const SegPlan& g, const OpDevice* op, char* base, int mode, int start_kind, int ns_log,
                   int nb, uint64_t seed, double tau);
// alpha, beta, s histories ([k][cpad]) and Krylov sizes ([cpad]) of a segment
// (asynchronous: synchronise the stream before reading)
rdm_status fetch_history(const SegPlan& g, char* base, std::vector<double>& a, std::vector<double>& b,
                         std::vector<double>& s, std::vector<int32_t>& kc, hipStream_t st);
void parallel_jobs(int n, const std::function<void(int)>& fn);
size_t align_up(size_t x);

// Block Lanczos (Algorithm 1) with block Gauss quadrature: one solve.
struct BlockPlan {
  const rdm_hamiltonian* h = nullptr;
  int prec = RDM_FP64, n_beta = 0, n_v = 0, k = 0, kb = 0;
  int ds = 2, ds_log = 1, C = 0, cpad = 0, G = 0, CB = 0, n_cb = 0, rpl = 1, n_rt = 0;
  uint64_t dim = 0, blk = 0;
  SegPlan apply, bath;
  size_t o_Q = 0, o_R = 0, o_Y = 0, o_part = 0, o_mats = 0, o_ah = 0, o_bh = 0, o_kc = 0;
  size_t header = 0, bytes = 0;
};
rdm_status block_plan(BlockPlan& bp, const rdm_hamiltonian* h, int n_beta, int n_v, int k, int prec,
                      uint64_t budget);
rdm_status block_solve(const BlockPlan& bp, const double* betas, uint64_t seed, double tau, char* ws,
                       hipStream_t st, bool profile, rdm_result* out);

// Lanczos coefficients only (rdm_lanczos).
rdm_status lanczos_only(const rdm_hamiltonian* h, int which, int n_v, int k, uint64_t seed, int prec,
                        int slab, int rpl, double tau, hipStream_t st, double* alpha, double* beta,
                        int32_t* kc);

}  // namespace rdm
