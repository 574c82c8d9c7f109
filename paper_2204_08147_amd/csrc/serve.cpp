// Serving engine: continuous batching of solve requests on one device stream.
//
// A worker thread owns the stream.  Every engine step launches one Lanczos
// step (norm, beta reduction, apply, alpha reduction) for *all* resident
// requests at once, each at its own step index.  Requests waiting in the
// queue are admitted at step boundaries when a slot and enough arena memory
// are free (admission by device footprint).  A request that finishes its
// recurrences leaves the batch for a finisher thread, which runs its host
// eigen-work, recombination and Gram on a stream of its own while the worker
// goes on launching steps; its memory returns to the arena when it is done
// (or it comes back for its regeneration pass).  The worker does not wait for
// the device after each step: it waits only to stay a few steps ahead and
// before it rewrites a segment table (two alternate).  Each request's
// reductions run over its own tiles in a fixed order, so its result does not
// depend on what else is resident.
#include <algorithm>
#include <chrono>
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
  bool cancel = false;   // rdm_server_cancel asked to drop it
  InstPlan plan;
  InstRun run;
  char* mem = nullptr;
  int phase = 0;       // 0: pass 1 (H_t and H_b), 1: regeneration pass
  int steps = 0;       // steps launched in the current phase
  bool need_init = true;
  bool light = false;  // takes 1 + kExtra steps per engine step (see run())
  hipEvent_t last = nullptr;  // recorded after the request's last launched step
};

}  // namespace

// The engine.  The worker thread launches the steps on `stream` and never
// waits for them except to bound how far it runs ahead (kAhead steps) and to
// reuse a segment table; finisher threads take the requests whose recurrences
// are done, each on its own stream: host eigen-work, recombination + Gram and
// finalisation overlap the worker's next steps.
struct rdm_server {
  static constexpr int kAhead = 4;        // steps in flight at most
  static constexpr int kFinishers = 2;
  static constexpr int kExtra = 3;        // extra steps per engine step of a light request
  static constexpr int kScan = 64;        // queued requests looked at per admission
  static constexpr double kBypassSec = 0.5;  // longest a blocked head of the queue is passed
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_fin;
  std::deque<Req*> queue;        // submitted, not admitted
  std::deque<Req*> regen_ready;  // back from a finisher for their regeneration pass
  std::deque<Req*> finishing;    // recurrences done (or dropped), for a finisher
  std::vector<Req*> active;      // resident in the step loop (worker only)
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  uint64_t budget = 0;
  int max_active = 64;
  int prec = RDM_MIXED;
  double tau = 1e-5;
  bool stop = false;
  bool worker_done_ = false;
  int busy_finishers = 0;
  int device = 0;
  std::thread worker;
  std::vector<std::thread> finishers;
  hipStream_t stream = nullptr;
  Arena arena;                   // guarded by mu
  char* arena_mem = nullptr;
  // segment tables, each with the event after the last step that read it:
  // 0 and 1 alternate for all resident requests, 2 and 3 for the light ones
  Seg* dsegs[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t segs_cap[4] = {0, 0, 0, 0};
  std::vector<Seg> hsegs[4];
  hipEvent_t seg_done[4] = {nullptr, nullptr, nullptr, nullptr};
  std::deque<hipEvent_t> ahead, spare;  // events after the steps in flight
  int64_t n_submitted = 0, n_completed = 0, n_steps = 0, peak_active = 0, peak_bytes = 0, used = 0;
  int64_t n_active = 0;  // active.size() as last published by the worker (under mu)
  uint64_t blocked_ticket = 0;  // head of the queue that did not fit, and since when (worker, under mu)
  std::chrono::steady_clock::time_point blocked_since{};

  void run();
  bool cancelled(const Req* r) {
    std::lock_guard<std::mutex> lk(mu);
    return r->cancel;
  }
  void finish_loop();
  rdm_status upload_table(int b, const std::vector<Seg>& segs);
  void complete(Req* r, rdm_status s);
  void hand_over(Req* r);
};

void rdm_server::complete(Req* r, rdm_status s) {
  if (r->last) (void)hipEventDestroy(r->last);
  r->last = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (r->mem) arena.release(r->mem, r->plan.bytes);
  if (r->mem) used -= (int64_t)r->plan.bytes;
  r->mem = nullptr;
  r->status = s;
  r->done = true;
  ++n_completed;
  cv_done.notify_all();
  cv_work.notify_one();  // freed memory may admit a queued request
}

void rdm_server::hand_over(Req* r) {
  std::lock_guard<std::mutex> lk(mu);
  finishing.push_back(r);
  cv_fin.notify_one();
}

rdm_status rdm_server::upload_table(int b, const std::vector<Seg>& segs) {
  // every step that read table b has completed once seg_done[b] has
  RDM_HIP(hipEventSynchronize(seg_done[b]));
  if (segs.size() > segs_cap[b]) {
    if (dsegs[b]) RDM_HIP(hipFree(dsegs[b]));
    dsegs[b] = nullptr;
    segs_cap[b] = std::max<size_t>(segs.size(), 2 * segs_cap[b]);
    RDM_HIP(hipMalloc(&dsegs[b], segs_cap[b] * sizeof(Seg)));
  }
  hsegs[b] = segs;  // the host copy lives until the table is reused
  RDM_HIP(hipMemcpyAsync(dsegs[b], hsegs[b].data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, stream));
  return RDM_OK;
}

void rdm_server::finish_loop() {
  (void)hipSetDevice(device);
  hipStream_t fs = nullptr;
  if (hipStreamCreateWithFlags(&fs, hipStreamNonBlocking) != hipSuccess) fs = nullptr;
  while (true) {
    Req* r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_fin.wait(lk, [&] { return !finishing.empty() || (stop && worker_done_); });
      if (finishing.empty()) break;
      r = finishing.front();
      finishing.pop_front();
      ++busy_finishers;
    }
    Range range("rdm serve finish");
    rdm_status q = fs ? RDM_OK : RDM_E_DEVICE;
    if (q == RDM_OK && hipEventSynchronize(r->last) != hipSuccess) q = RDM_E_DEVICE;
    bool requeued = false;
    if (q == RDM_OK && cancelled(r)) q = RDM_E_CANCELLED;
    if (q == RDM_OK && r->phase == 0) {
      q = host_phase(r->run, fs);
      if (q == RDM_OK && r->plan.two_pass) {
        r->phase = 1;
        r->steps = 0;
        r->need_init = true;
        std::lock_guard<std::mutex> lk(mu);
        regen_ready.push_back(r);
        cv_work.notify_one();
        requeued = true;
      }
    }
    if (!requeued) {
      if (q == RDM_OK) q = gram_phase(r->run, fs, nullptr);
      if (q == RDM_OK) q = finalize(r->run, &r->out);
      complete(r, q);
    }
    std::lock_guard<std::mutex> lk(mu);
    --busy_finishers;
    cv_work.notify_one();
  }
  if (fs) (void)hipStreamDestroy(fs);
}

void rdm_server::run() {
  (void)hipSetDevice(device);
  std::vector<Seg> segs, lsegs;
  int cur = 0, lcur = 2;
  bool changed = true;
  Launch ntiles, ltiles;
  int slab = 1, cmax = 0, lslab = 1, lcmax = 0;
  while (true) {
    std::vector<Req*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return !queue.empty() || !active.empty() || !regen_ready.empty() ||
               (stop && finishing.empty() && busy_finishers == 0);
      });
      if (stop && queue.empty() && active.empty() && regen_ready.empty() && finishing.empty() &&
          busy_finishers == 0)
        break;
      // admission at a step boundary: regeneration passes first (they hold
      // their memory already), then the queue in order, by slot and footprint
      while (!regen_ready.empty()) {
        admitted.push_back(regen_ready.front());
        regen_ready.pop_front();
      }
      // In arrival order; a request that does not fit yet may be passed by
      // later ones that do (among the first kScan queued) for at most
      // kBypassSec after it first failed to fit at the head of the queue;
      // after that the queue waits until enough memory drains for it.
      const auto now = std::chrono::steady_clock::now();
      int scanned = 0;
      for (auto it = queue.begin(); it != queue.end() && scanned < kScan &&
                                    (int)active.size() + (int)admitted.size() < max_active;) {
        Req* r = *it;
        ++scanned;
        char* m = arena.alloc(r->plan.bytes);
        if (!m) {
          if (used == 0) {
            // cannot fit even in an empty arena: fail it rather than block the queue
            it = queue.erase(it);
            r->status = RDM_E_NOMEM;
            r->done = true;
            ++n_completed;
            cv_done.notify_all();
            continue;
          }
          if (it == queue.begin()) {
            if (blocked_ticket != r->ticket) {
              blocked_ticket = r->ticket;
              blocked_since = now;
            }
            if (std::chrono::duration<double>(now - blocked_since).count() > kBypassSec) break;
          }
          ++it;
          continue;
        }
        it = queue.erase(it);
        r->mem = m;
        used += (int64_t)r->plan.bytes;
        peak_bytes = std::max(peak_bytes, used);
        admitted.push_back(r);
      }
    }
    for (Req* r : admitted) {
      if (cancelled(r)) {
        hand_over(r);  // its last event (if any) has completed; nothing to wait for
        continue;
      }
      if (r->phase == 0) {
        r->run.plan = &r->plan;
        r->run.base = r->mem;
        const rdm_status s = bind_ops(r->run, stream);
        if (s != RDM_OK) {
          complete(r, s);
          continue;
        }
      }
      active.push_back(r);
      changed = true;
    }
    // requests cancelled while resident leave at this step boundary; their
    // memory is released once the steps already launched for them are done
    for (size_t i = 0; i < active.size();) {
      Req* r = active[i];
      if (cancelled(r) && hipEventRecord(r->last, stream) == hipSuccess) {
        active.erase(active.begin() + (long)i);
        hand_over(r);
        changed = true;
      } else {
        ++i;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      n_active = (int64_t)active.size();
      peak_active = std::max<int64_t>(peak_active, n_active);
    }
    if (active.empty()) continue;

    Range range("rdm serve step");
    rdm_status s = RDM_OK;
    if (changed) {
      // a new segment table (in the buffer not in use), and the state of the
      // requests that start a phase
      segs.clear();
      std::vector<std::pair<int, int>> init_ranges;  // (first seg, phase)
      auto add_segs = [&](std::vector<Seg>& v, Req* r) {
        if (r->phase == 0) {
          v.push_back(seg_of(r->run, 0, MODE_LANCZOS, tau));
          v.push_back(seg_of(r->run, 1, MODE_LANCZOS, tau));
        } else {
          v.push_back(seg_of(r->run, 0, MODE_REGEN, tau));
        }
      };
      for (Req* r : active) {
        const int first = (int)segs.size();
        add_segs(segs, r);
        if (r->need_init) {
          for (int q = first; q < (int)segs.size(); ++q) init_ranges.push_back({q, r->phase});
          r->need_init = false;
        }
      }
      slab = tuned_slab(prec, segs);
      ntiles = assign_tiles(segs);
      cmax = 0;
      for (const auto& sg : segs) cmax = std::max(cmax, sg.cpad);
      cur ^= 1;
      s = upload_table(cur, segs);
      for (auto& ir : init_ranges) {
        const Seg& sg = segs[ir.first];
        if (s == RDM_OK)
          s = init_run(prec, dsegs[cur] + ir.first, 1, cmax, ir.second, sg.xz ? sg.x_tiles * sg.P : 0,
                       sg.x_base, stream);
      }
      // Light requests take 1 + kExtra steps per engine step, so that a
      // small request is not held to the pace of the largest resident one
      // (every request otherwise advances one step per engine step): the
      // cheapest requests by rows x columns, as long as their extra steps add
      // at most a quarter of the engine step's work.  The extra launches run
      // on a table of their segments only; a segment past its last step is
      // left alone by every kernel, so a request may overrun its k there.
      std::vector<std::pair<double, Req*>> cost;
      double total = 0.0;
      for (Req* r : active) {
        double c = 0.0;
        for (int w = 0; w < (r->phase == 0 ? 2 : 1); ++w) {
          const SegPlan& g = w == 0 ? r->plan.tot : r->plan.bath;
          c += (double)g.dim * g.cpad * (r->phase == 0 ? 1.0 : 1.0 + r->run.betas.size());
        }
        total += c;
        cost.push_back({c, r});
        r->light = false;
      }
      std::sort(cost.begin(), cost.end(),
                [](const std::pair<double, Req*>& a, const std::pair<double, Req*>& b) { return a.first < b.first; });
      double extra = 0.0;
      for (auto& cr : cost) {
        if (extra + kExtra * cr.first > 0.25 * total) break;
        cr.second->light = true;
        extra += kExtra * cr.first;
      }
      lsegs.clear();
      for (Req* r : active)
        if (r->light) add_segs(lsegs, r);
      if (s == RDM_OK && !lsegs.empty()) {
        lslab = tuned_slab(prec, lsegs);
        ltiles = assign_tiles(lsegs);
        lcmax = 0;
        for (const auto& sg : lsegs) lcmax = std::max(lcmax, sg.cpad);
        lcur ^= 1;
        s = upload_table(lcur, lsegs);
      }
      changed = false;
    }
    if (s == RDM_OK) s = launch_step(prec, dsegs[cur], (int)segs.size(), ntiles, slab, cmax, stream, nullptr);
    if (s == RDM_OK && hipEventRecord(seg_done[cur], stream) != hipSuccess) s = RDM_E_DEVICE;
    if (!lsegs.empty()) {
      for (int e = 0; e < kExtra && s == RDM_OK; ++e)
        s = launch_step(prec, dsegs[lcur], (int)lsegs.size(), ltiles, lslab, lcmax, stream, nullptr);
      if (s == RDM_OK && hipEventRecord(seg_done[lcur], stream) != hipSuccess) s = RDM_E_DEVICE;
    }
    // bound how far the launches run ahead of the device
    if (s == RDM_OK) {
      hipEvent_t e = nullptr;
      if (!spare.empty()) {
        e = spare.front();
        spare.pop_front();
      } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        s = RDM_E_DEVICE;
      }
      if (s == RDM_OK && hipEventRecord(e, stream) != hipSuccess) s = RDM_E_DEVICE;
      if (e) ahead.push_back(e);
      while (s == RDM_OK && (int)ahead.size() > kAhead) {
        if (hipEventSynchronize(ahead.front()) != hipSuccess) s = RDM_E_DEVICE;
        spare.push_back(ahead.front());
        ahead.pop_front();
      }
    }
    ++n_steps;
    if (s != RDM_OK) {
      (void)hipStreamSynchronize(stream);
      std::vector<Req*> failed;
      failed.swap(active);
      for (Req* r : failed) complete(r, s);
      changed = true;
      continue;
    }
    // requests whose recurrences are complete leave for a finisher
    for (size_t i = 0; i < active.size();) {
      Req* r = active[i];
      r->steps += r->light ? 1 + kExtra : 1;
      const int need = r->phase == 0 ? std::max(r->plan.k, r->plan.kb) : r->plan.k;
      if (r->steps < need) {
        ++i;
        continue;
      }
      if (hipEventRecord(r->last, stream) != hipSuccess) {
        (void)hipStreamSynchronize(stream);
      }
      active.erase(active.begin() + (long)i);
      hand_over(r);
      changed = true;
    }
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    worker_done_ = true;
  }
  cv_fin.notify_all();
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
  bool ev_ok = true;
  for (auto& e : s->seg_done) ev_ok = ev_ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess || !ev_ok) {
    for (auto e : s->seg_done)
      if (e) (void)hipEventDestroy(e);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    (void)hipFree(s->arena_mem);
    delete s;
    set_error("rdm_server_create: cannot create a stream or events");
    return RDM_E_DEVICE;
  }
  s->worker = std::thread([s] { s->run(); });
  for (int f = 0; f < rdm_server::kFinishers; ++f) s->finishers.emplace_back([s] { s->finish_loop(); });
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
  if (hipEventCreateWithFlags(&r->last, hipEventDisableTiming) != hipSuccess) {
    delete r;
    set_error("rdm_server_submit: cannot create an event");
    return RDM_E_DEVICE;
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

extern "C" rdm_status rdm_server_cancel(rdm_server* s, uint64_t ticket) {
  if (!s) {
    set_error("rdm_server_cancel: NULL server");
    return RDM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->claimed) {
    set_error("rdm_server_cancel: unknown ticket, or one already retrieved or being waited for");
    return RDM_E_INVALID;
  }
  Req* r = it->second;
  if (r->done) return RDM_OK;
  auto q = std::find(s->queue.begin(), s->queue.end(), r);
  if (q != s->queue.end()) {
    // not admitted yet: done at once
    s->queue.erase(q);
    if (r->last) (void)hipEventDestroy(r->last);
    r->last = nullptr;
    r->status = RDM_E_CANCELLED;
    r->done = true;
    ++s->n_completed;
    s->cv_done.notify_all();
    return RDM_OK;
  }
  r->cancel = true;  // the engine drops it at its next step boundary
  s->cv_work.notify_one();
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
  out[2] = s->n_active;
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
  s->cv_fin.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& f : s->finishers)
    if (f.joinable()) f.join();
  (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) {
    if (kv.second->last) (void)hipEventDestroy(kv.second->last);
    delete kv.second;
  }
  for (auto e : s->ahead) (void)hipEventDestroy(e);
  for (auto e : s->spare) (void)hipEventDestroy(e);
  for (int b = 0; b < 4; ++b) {
    if (s->dsegs[b]) (void)hipFree(s->dsegs[b]);
    if (s->seg_done[b]) (void)hipEventDestroy(s->seg_done[b]);
  }
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}
