// Request loop: FIFO queue, worker threads with their own streams, admission
// by the estimated device footprint of the admitted requests.
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
void run_instance(const spd_instance& I, hipStream_t s, spd_instance_result& R);
}

using Clock = std::chrono::steady_clock;

struct spd_server {
  struct Request {
    spd_instance inst{};
    int64_t bytes = 0;
    bool done = false;
    spd_instance_result res{};
    Clock::time_point t_submit, t_admit, t_done;
  };
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::map<int64_t, Request> reqs;
  int64_t next_ticket = 1;
  int64_t budget = 0, in_use = 0;
  int running = 0;
  bool stop = false;
  int dev = 0;
  std::vector<std::thread> workers;

  void work() {
    // a worker that cannot set the device or make a stream still drains the
    // queue (run_instance then reports the device error per request, or runs
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
      {
        std::unique_lock<std::mutex> lk(mu);
        // first come first served: the head is admitted once it fits, or when
        // nothing else runs (a request above the budget then runs alone)
        cv_work.wait(lk, [&] {
          if (queue.empty()) return stop;
          const Request& h = reqs[queue.front()];
          return running == 0 || in_use + h.bytes <= budget;
        });
        if (queue.empty()) break;
        t = queue.front();
        queue.pop_front();
        Request& r = reqs[t];
        r.t_admit = Clock::now();
        in_use += r.bytes;
        ++running;
        inst = r.inst;
      }
      spd_instance_result res{};
      spd::run_instance(inst, s, res);
      {
        std::lock_guard<std::mutex> lk(mu);
        Request& r = reqs[t];
        r.res = res;
        r.t_done = Clock::now();
        r.done = true;
        in_use -= r.bytes;
        --running;
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
  const double n = (double)q->n, leaf = std::max(q->h2.leaf_size, 1);
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

spd_status spd_server_submit(spd_server_t S, const spd_instance* q, int64_t* ticket) {
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
    r.bytes = spd_request_footprint(q);
    r.t_submit = Clock::now();
    S->queue.push_back(t);
    *ticket = t;
  }
  S->cv_work.notify_all();
  return SPD_OK;
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

void spd_server_destroy(spd_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  delete S;
}

}  // extern "C"
