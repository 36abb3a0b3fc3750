// Request loop: FIFO queue, worker threads with their own streams, admission
// by the estimated device footprint of the admitted requests, and resident
// H^2 / HSS / factor state for requests that name the same matrix by a key.
#include "model.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace spd {
spd_status build_state(const spd_instance& I, hipStream_t s, spd_instance_result& R, spd_h2_t* A,
                       spd_hss_t* M, spd_ulv_t* F);
void solve_state(const spd_instance& I, spd_h2_t A, spd_ulv_t F, hipStream_t s, spd_instance_result& R);
}

using Clock = std::chrono::steady_clock;

// Device bytes of a request's PCG vectors (the part of the footprint that a
// request solving on resident state still needs).
static int64_t rows_of(const spd_instance* q) { return q->kernel.kind == SPD_K_RPY ? 3 * q->n : q->n; }

static int64_t pcg_bytes(const spd_instance* q) {
  return (int64_t)(8.0 * (double)rows_of(q) * 8.0 * std::max(q->nrhs, 1));
}

struct spd_server {
  struct Request {
    spd_instance inst{};
    uint64_t key = 0;
    int64_t bytes = 0;  // footprint estimate: state + PCG vectors
    int64_t held = 0;   // bytes counted in in_use while it runs
    int32_t phase = 0;  // 0 queued, 1 building, 2 solving, 3 finished
    bool done = false;
    spd_instance_result res{};
    Clock::time_point t_submit, t_admit, t_done;
  };
  // state of a keyed matrix kept on the device between its requests
  struct Resident {
    spd_h2_t A = nullptr;
    spd_hss_t M = nullptr;
    spd_ulv_t F = nullptr;
    int64_t bytes = 0;  // counted in in_use while resident
    bool ready = false; // built (false while its first request builds it)
    bool busy = false;  // a request is using it (one at a time)
    Clock::time_point last;
  };
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::map<int64_t, Request> reqs;
  std::map<uint64_t, Resident> resident;
  int64_t next_ticket = 1;
  int64_t budget = 0, in_use = 0;
  int running = 0;
  bool stop = false;
  int dev = 0;
  std::vector<std::thread> workers;

  // Bytes request r needs to start: the PCG vectors on a built resident state,
  // the whole footprint otherwise.
  int64_t need(const Request& r) const {
    if (r.key) {
      auto it = resident.find(r.key);
      if (it != resident.end() && it->second.ready) return pcg_bytes(&r.inst);
    }
    return r.bytes;
  }
  // Resident states that are idle and not r's, least recently used first,
  // released until r fits; their handles are handed back to be destroyed
  // outside the lock.
  bool make_room(const Request& r, int64_t want, std::vector<Resident>& freed) {
    auto idle = [&](const std::pair<const uint64_t, Resident>& kv) {
      return kv.first != r.key && kv.second.ready && !kv.second.busy;
    };
    int64_t can = 0;
    for (const auto& kv : resident)
      if (idle(kv)) can += kv.second.bytes;
    if (in_use - can + want > budget) return false;  // evicting everything idle would not do
    while (in_use + want > budget) {
      auto victim = resident.end();
      for (auto it = resident.begin(); it != resident.end(); ++it)
        if (idle(*it) && (victim == resident.end() || it->second.last < victim->second.last)) victim = it;
      in_use -= victim->second.bytes;
      freed.push_back(victim->second);
      resident.erase(victim);
    }
    return true;
  }
  // The request to admit next, or 0.  First come first served, except that a
  // request whose matrix state is in use (or being built) by another request
  // waits without holding up the requests behind it.  The first request that
  // may run is admitted once it fits, after idle resident states are
  // released, or when nothing else runs (a request above the budget then runs
  // alone).
  int64_t pick(std::vector<Resident>& freed) {
    for (auto qi = queue.begin(); qi != queue.end(); ++qi) {
      Request& r = reqs[*qi];
      if (r.key) {
        auto it = resident.find(r.key);
        if (it != resident.end() && (it->second.busy || !it->second.ready)) continue;
      }
      const int64_t want = need(r);
      bool go = in_use + want <= budget || make_room(r, want, freed);
      if (!go && running == 0) {
        // above the budget: it runs alone, with every idle resident state released
        for (auto it = resident.begin(); it != resident.end();) {
          if (it->first != r.key && it->second.ready && !it->second.busy) {
            in_use -= it->second.bytes;
            freed.push_back(it->second);
            it = resident.erase(it);
          } else {
            ++it;
          }
        }
        go = true;
      }
      if (go) {
        const int64_t t = *qi;
        queue.erase(qi);
        return t;
      }
      return 0;
    }
    return 0;
  }

  static void release(Resident& z) {
    if (z.F) ulv_destroy(z.F);
    if (z.M) spdhss_destroy(z.M);
    if (z.A) h2_destroy(z.A);
    z = Resident{};
  }

  void work() {
    // a worker that cannot set the device or make a stream still drains the
    // queue (the instance then reports the device error per request, or runs
    // on the null stream), so that no request waits forever
    (void)hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      s = nullptr;
    }
    for (;;) {
      int64_t t = 0;
      spd_instance inst{};
      uint64_t key = 0;
      Resident use{};
      bool reuse = false;
      std::vector<Resident> freed;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          if (queue.empty()) return stop;
          t = pick(freed);
          return t != 0;
        });
        if (t == 0) break;  // stopping with an empty queue
        Request& r = reqs[t];
        r.t_admit = Clock::now();
        key = r.key;
        if (key) {
          auto it = resident.find(key);
          if (it != resident.end()) {  // built and idle (pick checked)
            it->second.busy = true;
            use = it->second;
            reuse = true;
          } else {
            Resident& z = resident[key];  // placeholder while this request builds it
            z.busy = true;
            z.bytes = r.bytes - pcg_bytes(&r.inst);
          }
        }
        r.held = reuse ? pcg_bytes(&r.inst) : r.bytes;
        r.phase = reuse ? 2 : 1;
        in_use += r.held;
        ++running;
        inst = r.inst;
      }
      auto solving = [&]() {
        std::lock_guard<std::mutex> lk(mu);
        reqs[t].phase = 2;
      };
      for (Resident& z : freed) release(z);
      spd_instance_result res{};
      if (reuse) {
        spd::solve_state(inst, use.A, use.F, s, res);
      } else {
        const spd_status st = spd::build_state(inst, s, res, &use.A, &use.M, &use.F);
        if (st == SPD_OK) {
          solving();
          spd::solve_state(inst, use.A, use.F, s, res);
        } else {
          res.status = st;
        }
        if (!key) {  // nothing stays resident
          if (use.F) ulv_destroy(use.F);
          if (use.M) spdhss_destroy(use.M);
          if (use.A) h2_destroy(use.A);
          use = Resident{};
        }
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        Request& r = reqs[t];
        r.res = res;
        r.t_done = Clock::now();
        r.done = true;
        r.phase = 3;
        --running;
        if (!key) {
          in_use -= r.held;
        } else {
          Resident& z = resident[key];
          if (!reuse) {
            if (use.A && use.F) {  // built: keep it resident, counted in in_use
              z.A = use.A;
              z.M = use.M;
              z.F = use.F;
              z.ready = true;
              in_use -= pcg_bytes(&r.inst);
            } else {  // the build failed: nothing stays
              in_use -= r.held;
              resident.erase(key);
            }
          } else {
            in_use -= r.held;
          }
          auto it = resident.find(key);
          if (it != resident.end()) {
            it->second.busy = false;
            it->second.last = Clock::now();
          }
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

extern "C" {

int64_t spd_request_footprint(const spd_instance* q) {
  if (!q || q->n <= 0) return 0;
  const double n = (double)rows_of(q), leaf = std::max(q->h2.leaf_size, 1);
  const double s = std::max(q->hss.max_rank + q->hss.oversample, 1);
  // points; near blocks (about 27 neighbours a leaf); coupling blocks (taken
  // as 60 leaf-sized blocks a leaf); samples and their level stacks; HSS
  // factors and solve operators; PCG vectors
  const double bytes = 24.0 * n + 8.0 * n * leaf * (27.0 + 60.0) + 8.0 * n * s * 4.0 +
                       8.0 * n * (3.0 * leaf + 4.0 * q->hss.max_rank) + 8.0 * n * 8.0 * std::max(q->nrhs, 1);
  return (int64_t)bytes;
}

spd_status spd_server_create(int32_t workers, int64_t hbm_budget_bytes, spd_server_t* out) {
  if (out) *out = nullptr;
  if (!out || workers < 1 || hbm_budget_bytes <= 0) {
    spd::set_last_error("bad server arguments");
    return SPD_E_INVALID;
  }
  auto* S = new spd_server();
  if (hipGetDevice(&S->dev) != hipSuccess) {
    delete S;
    spd::set_last_error("no current device");
    return SPD_E_DEVICE;
  }
  S->budget = hbm_budget_bytes;
  for (int w = 0; w < workers; ++w) S->workers.emplace_back([S] { S->work(); });
  *out = S;
  return SPD_OK;
}

static spd_status submit(spd_server_t S, const spd_instance* q, uint64_t key, int64_t* ticket) {
  if (!S || !q || !ticket) {
    spd::set_last_error("null argument");
    return SPD_E_INVALID;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      spd::set_last_error("server is stopping");
      return SPD_E_INVALID;
    }
    const int64_t t = S->next_ticket++;
    spd_server::Request& r = S->reqs[t];
    r.inst = *q;
    r.key = key;
    r.bytes = spd_request_footprint(q);
    r.t_submit = Clock::now();
    S->queue.push_back(t);
    *ticket = t;
  }
  S->cv_work.notify_all();
  return SPD_OK;
}

spd_status spd_server_submit(spd_server_t S, const spd_instance* q, int64_t* ticket) {
  return submit(S, q, 0, ticket);
}

spd_status spd_server_submit_keyed(spd_server_t S, const spd_instance* q, uint64_t key, int64_t* ticket) {
  if (key == 0) {
    spd::set_last_error("key must be nonzero");
    return SPD_E_INVALID;
  }
  return submit(S, q, key, ticket);
}

spd_status spd_server_wait(spd_server_t S, int64_t ticket, int32_t block, spd_instance_result* result,
                           double* seconds_queued, double* seconds_total) {
  if (!S || !result) {
    spd::set_last_error("null argument");
    return SPD_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    spd::set_last_error("unknown or already collected ticket");
    return SPD_E_INVALID;
  }
  if (!it->second.done) {
    if (!block) return SPD_PENDING;
    // look the ticket up again after every wake-up: another thread waiting for
    // the same ticket may have collected (and erased) it meanwhile
    S->cv_done.wait(lk, [&] {
      it = S->reqs.find(ticket);
      return it == S->reqs.end() || it->second.done;
    });
    if (it == S->reqs.end()) {
      spd::set_last_error("ticket collected by another waiter");
      return SPD_E_INVALID;
    }
  }
  const spd_server::Request& r = it->second;
  *result = r.res;
  if (seconds_queued) *seconds_queued = std::chrono::duration<double>(r.t_admit - r.t_submit).count();
  if (seconds_total) *seconds_total = std::chrono::duration<double>(r.t_done - r.t_submit).count();
  S->reqs.erase(it);
  return SPD_OK;
}

spd_status spd_server_phase(spd_server_t S, int64_t ticket, int32_t* phase) {
  if (!S || !phase) {
    spd::set_last_error("null argument");
    return SPD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    spd::set_last_error("unknown or already collected ticket");
    return SPD_E_INVALID;
  }
  *phase = it->second.phase;
  return SPD_OK;
}

void spd_server_destroy(spd_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->resident) spd_server::release(kv.second);
  delete S;
}

}  // extern "C"
