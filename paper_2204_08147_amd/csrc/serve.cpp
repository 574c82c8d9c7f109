// Serving engine: continuous batching of solve requests on one device stream.
//
// A worker thread owns the stream.  Every engine step launches one Lanczos
// step (norm, beta reduction, apply, alpha reduction) for *all* resident
// requests at once, each at its own step index.  Requests waiting in the
// queue are admitted at step boundaries when a slot and enough arena memory
// are free (admission by device footprint); a request that finishes its
// recurrences leaves the batch for its host eigen-work, recombination and
// Gram, and its memory returns to the arena.  Each request's reductions run
// over its own tiles in a fixed order, so its result does not depend on what
// else is resident.
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "host.h"
#include "solve.h"

using namespace rdm;

namespace {

constexpr size_t kArenaAlign = 256;

// First-fit sub-allocator over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(char* b, size_t n) {
    base = b;
    size = n;
    free_.clear();
    free_[0] = n;
  }
  char* alloc(size_t n) {
    n = (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        return base + off;
      }
    }
    return nullptr;
  }
  void release(char* p, size_t n) {
    n = (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    size_t off = (size_t)(p - base);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
};

struct Req {
  uint64_t ticket = 0;
  const rdm_hamiltonian* h = nullptr;
  int n_v = 0, k = 0;
  rdm_result out{};
  rdm_status status = RDM_OK;
  bool done = false;
  bool claimed = false;  // a poll that saw it done, or a wait, owns the ticket
  InstPlan plan;
  InstRun run;
  char* mem = nullptr;
  int phase = 0;       // 0: pass 1 (H_t and H_b), 1: regeneration pass
  int steps = 0;       // steps run in the current phase
  bool need_init = true;
};

}  // namespace

struct rdm_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::vector<Req*> active;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  uint64_t budget = 0;
  int max_active = 64;
  int prec = RDM_MIXED;
  double tau = 1e-5;
  bool stop = false;
  int device = 0;
  std::thread worker;
  hipStream_t stream = nullptr;
  Arena arena;
  char* arena_mem = nullptr;
  Seg* dsegs = nullptr;
  size_t segs_cap = 0;
  int64_t n_submitted = 0, n_completed = 0, n_steps = 0, peak_active = 0, peak_bytes = 0, used = 0;

  void run();
  rdm_status ensure_tables(size_t nseg);
  void complete(Req* r, rdm_status s);
};

void rdm_server::complete(Req* r, rdm_status s) {
  if (r->mem) arena.release(r->mem, r->plan.bytes);
  r->mem = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  used -= (int64_t)r->plan.bytes;
  r->status = s;
  r->done = true;
  ++n_completed;
  cv_done.notify_all();
}

rdm_status rdm_server::ensure_tables(size_t nseg) {
  if (nseg > segs_cap) {
    if (dsegs) RDM_HIP(hipFree(dsegs));
    segs_cap = std::max<size_t>(nseg, 2 * segs_cap);
    RDM_HIP(hipMalloc(&dsegs, segs_cap * sizeof(Seg)));
  }
  return RDM_OK;
}

void rdm_server::run() {
  (void)hipSetDevice(device);
  std::vector<Seg> segs;
  while (true) {
    std::vector<Req*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
      if (stop && queue.empty() && active.empty()) break;
      // admission at a step boundary: FIFO, by slot and device footprint
      while (!queue.empty() && (int)active.size() + (int)admitted.size() < max_active) {
        Req* r = queue.front();
        char* m = arena.alloc(r->plan.bytes);
        if (!m) {
          if (active.empty() && admitted.empty()) {
            // cannot ever fit: fail it rather than block the queue
            queue.pop_front();
            r->status = RDM_E_NOMEM;
            r->done = true;
            ++n_completed;
            cv_done.notify_all();
            continue;
          }
          break;
        }
        queue.pop_front();
        r->mem = m;
        used += (int64_t)r->plan.bytes;
        peak_bytes = std::max(peak_bytes, used);
        admitted.push_back(r);
      }
    }
    for (Req* r : admitted) {
      r->run.plan = &r->plan;
      r->run.base = r->mem;
      r->phase = 0;
      r->steps = 0;
      r->need_init = true;
      const rdm_status s = bind_ops(r->run, stream);
      if (s != RDM_OK) {
        complete(r, s);
        continue;
      }
      std::lock_guard<std::mutex> lk(mu);
      active.push_back(r);
      peak_active = std::max<int64_t>(peak_active, (int64_t)active.size());
    }
    if (active.empty()) continue;

    // segment table of the resident batch
    segs.clear();
    std::vector<std::pair<int, int>> init_ranges;  // (first seg, phase) of segments to initialise
    int cmax = 0;
    for (Req* r : active) {
      const int first = (int)segs.size();
      if (r->phase == 0) {
        segs.push_back(seg_of(r->run, 0, MODE_LANCZOS, tau));
        segs.push_back(seg_of(r->run, 1, MODE_LANCZOS, tau));
      } else {
        segs.push_back(seg_of(r->run, 0, MODE_REGEN, tau));
      }
      if (r->need_init) {
        for (int q = first; q < (int)segs.size(); ++q) init_ranges.push_back({q, r->phase});
        r->need_init = false;
      }
    }
    const int slab = tuned_slab(prec, segs);
    const Launch ntiles = assign_tiles(segs);
    for (const auto& sg : segs) cmax = std::max(cmax, sg.cpad);
    rdm_status s = ensure_tables(segs.size());
    if (s == RDM_OK && hipMemcpyAsync(dsegs, segs.data(), segs.size() * sizeof(Seg),
                                      hipMemcpyHostToDevice, stream) != hipSuccess)
      s = RDM_E_DEVICE;
    for (auto& ir : init_ranges) {
      const Seg& sg = segs[ir.first];
      if (s == RDM_OK)
        s = init_run(prec, dsegs + ir.first, 1, cmax, ir.second, sg.xz ? sg.x_tiles * sg.P : 0, sg.x_base, stream);
    }
    if (s == RDM_OK) s = launch_step(prec, dsegs, (int)segs.size(), ntiles, slab, cmax, stream, nullptr);
    // the host tables must stay valid until the copies above completed
    if (s == RDM_OK && hipStreamSynchronize(stream) != hipSuccess) s = RDM_E_DEVICE;
    ++n_steps;
    if (s != RDM_OK) {
      std::vector<Req*> failed;
      {
        std::lock_guard<std::mutex> lk(mu);
        failed.swap(active);
      }
      for (Req* r : failed) complete(r, s);
      continue;
    }
    // advance and retire
    std::vector<Req*> keep;
    for (Req* r : active) {
      ++r->steps;
      const int need = r->phase == 0 ? std::max(r->plan.k, r->plan.kb) : r->plan.k;
      if (r->steps < need) {
        keep.push_back(r);
        continue;
      }
      if (r->phase == 0) {
        rdm_status q = host_phase(r->run, stream);
        if (q != RDM_OK) {
          complete(r, q);
          continue;
        }
        if (r->plan.two_pass) {
          r->phase = 1;
          r->steps = 0;
          r->need_init = true;
          keep.push_back(r);
          continue;
        }
      }
      rdm_status q = gram_phase(r->run, stream, nullptr);
      if (q == RDM_OK) q = finalize(r->run, &r->out);
      complete(r, q);
    }
    std::lock_guard<std::mutex> lk(mu);
    active.swap(keep);
  }
}

extern "C" rdm_status rdm_server_create(uint64_t hbm_budget, int32_t max_active, int32_t precision,
                                        rdm_server** out) {
  if (!out || max_active < 0 || (precision != RDM_FP64 && precision != RDM_MIXED)) {
    set_error("rdm_server_create: bad arguments");
    return RDM_E_INVALID;
  }
  *out = nullptr;
  auto* s = new rdm_server();
  s->max_active = max_active ? max_active : 64;
  s->prec = precision;
  s->tau = precision == RDM_FP64 ? 1e-12 : 1e-5;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    set_error("rdm_server_create: no device");
    return RDM_E_DEVICE;
  }
  if (!hbm_budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      set_error("rdm_server_create: hipMemGetInfo failed");
      return RDM_E_DEVICE;
    }
    hbm_budget = fr > (8ull << 30) ? fr - (8ull << 30) : fr / 2;
  }
  s->budget = hbm_budget;
  if (hipMalloc(&s->arena_mem, hbm_budget) != hipSuccess) {
    delete s;
    set_error("rdm_server_create: cannot allocate the arena");
    return RDM_E_NOMEM;
  }
  s->arena.init(s->arena_mem, hbm_budget);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(s->arena_mem);
    delete s;
    set_error("rdm_server_create: cannot create a stream");
    return RDM_E_DEVICE;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return RDM_OK;
}

extern "C" rdm_status rdm_server_submit(rdm_server* s, const rdm_hamiltonian* h, const double* beta,
                                        int32_t n_beta, int32_t n_v, int32_t k, uint64_t seed,
                                        rdm_result out, uint64_t* ticket) {
  if (!s || !h || !beta || n_beta < 1 || n_v < 1 || k < 1 || k > 4096 || !ticket) {
    set_error("rdm_server_submit: bad arguments");
    return RDM_E_INVALID;
  }
  for (int b = 0; b < n_beta; ++b)
    if (!(beta[b] > 0.0) || !std::isfinite(beta[b])) {
      set_error("rdm_server_submit: every beta must be finite and > 0");
      return RDM_E_INVALID;
    }
  auto* r = new Req();
  r->h = h;
  r->n_v = n_v;
  r->k = k;
  r->out = out;
  r->run.betas.assign(beta, beta + n_beta);
  r->run.seed = seed;
  // a request keeps all its Lanczos vectors if that takes at most half of
  // the arena (the regeneration pass of a two-pass plan costs as much as the
  // first one); larger ones run two-pass so that others stay resident too
  rdm_status ps = plan_instance(r->plan, h, n_beta, n_v, k, s->prec, RDM_AUTO, s->budget / 2, 0, 0);
  if (ps == RDM_E_NOMEM)
    ps = plan_instance(r->plan, h, n_beta, n_v, k, s->prec, RDM_TWO_PASS, s->budget, 0, 0);
  if (ps != RDM_OK) {
    delete r;
    return ps;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  ++s->n_submitted;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return RDM_OK;
}

extern "C" rdm_status rdm_server_poll(rdm_server* s, uint64_t ticket, int32_t* done, rdm_status* status) {
  if (!s || !done || !status) {
    set_error("rdm_server_poll: bad arguments");
    return RDM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->claimed) {
    set_error("rdm_server_poll: unknown ticket, or one already retrieved or being waited for");
    return RDM_E_INVALID;
  }
  *done = it->second->done ? 1 : 0;
  *status = it->second->status;
  if (it->second->done) {
    delete it->second;
    s->reqs.erase(it);
  }
  return RDM_OK;
}

extern "C" rdm_status rdm_server_wait(rdm_server* s, uint64_t ticket, rdm_status* status) {
  if (!s || !status) {
    set_error("rdm_server_wait: bad arguments");
    return RDM_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->claimed) {
    set_error("rdm_server_wait: unknown ticket, or one already retrieved or being waited for");
    return RDM_E_INVALID;
  }
  Req* r = it->second;
  r->claimed = true;
  s->cv_done.wait(lk, [&] { return r->done; });
  *status = r->status;
  delete r;
  s->reqs.erase(ticket);
  return RDM_OK;
}

extern "C" rdm_status rdm_server_stats(rdm_server* s, int64_t* out) {
  if (!s || !out) {
    set_error("rdm_server_stats: bad arguments");
    return RDM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  out[0] = s->n_submitted;
  out[1] = s->n_completed;
  out[2] = (int64_t)s->active.size();
  out[3] = (int64_t)s->queue.size();
  out[4] = s->n_steps;
  out[5] = s->peak_active;
  out[6] = s->peak_bytes;
  return RDM_OK;
}

extern "C" void rdm_server_destroy(rdm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->reqs) delete kv.second;
  if (s->dsegs) (void)hipFree(s->dsegs);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}
