// Many independent instances on a pool of worker threads.
//
// Each worker owns a non-blocking HIP stream (default priority) on the calling
// thread's device and runs its instances end to end through the public entry
// points, so an instance computes exactly what the same calls made alone
// compute; the instances of different workers overlap on the device.  Graph
// capture inside pcg_solve is thread-local, so captures on different workers
// do not interfere.
#include "model.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

namespace {

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

namespace spd {
// h2_build, spdhss_build and ulv_factor_ex of one instance; on failure the
// handles made so far are destroyed and left null
spd_status build_state(const spd_instance& I, hipStream_t s, spd_instance_result& R, spd_h2_t* A,
                       spd_hss_t* M, spd_ulv_t* F) {
  *A = nullptr;
  *M = nullptr;
  *F = nullptr;
  auto t0 = std::chrono::steady_clock::now();
  spd_status st = h2_build(I.points, I.n, I.kernel, &I.h2, s, A);
  R.seconds_h2 = seconds_since(t0);
  if (st == SPD_OK) {
    t0 = std::chrono::steady_clock::now();
    st = spdhss_build(*A, &I.hss, s, M);
    if (st == SPD_OK) st = ulv_factor_ex(*M, I.solve_precision, s, F);
    R.seconds_build = seconds_since(t0);
  }
  if (st != SPD_OK) {
    if (*F) ulv_destroy(*F);
    if (*M) spdhss_destroy(*M);
    if (*A) h2_destroy(*A);
    *A = nullptr;
    *M = nullptr;
    *F = nullptr;
  }
  return st;
}

// pcg_solve of the instance's right-hand sides on built state
void solve_state(const spd_instance& I, spd_h2_t A, spd_ulv_t F, hipStream_t s, spd_instance_result& R) {
  std::vector<int32_t> it(std::max(I.nrhs, 1));
  std::vector<double> rr(std::max(I.nrhs, 1));
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t rows = I.kernel.kind == SPD_K_RPY ? 3 * I.n : I.n;  // 3 rows a particle for the tensor
  const spd_status st = pcg_solve(A, F, I.b, I.x, I.nrhs, rows, I.rtol, I.maxit, s, it.data(), rr.data());
  R.seconds_solve = seconds_since(t0);
  if (st == SPD_OK || st == SPD_E_NOT_CONVERGED) {
    for (int c = 0; c < I.nrhs; ++c) {
      R.iters_max = std::max(R.iters_max, it[c]);
      R.relres_max = std::max(R.relres_max, rr[c]);
      if (I.iters) I.iters[c] = it[c];
      if (I.relres) I.relres[c] = rr[c];
    }
  }
  R.status = st;
}

void run_instance(const spd_instance& I, hipStream_t s, spd_instance_result& R) {
  R = spd_instance_result{};
  spd_h2_t A = nullptr;
  spd_hss_t M = nullptr;
  spd_ulv_t F = nullptr;
  const spd_status st = build_state(I, s, R, &A, &M, &F);
  if (st == SPD_OK) solve_state(I, A, F, s, R);
  else R.status = st;
  if (F) ulv_destroy(F);
  if (M) spdhss_destroy(M);
  if (A) h2_destroy(A);
}
}  // namespace spd

extern "C" spd_status spd_solve_batch(const spd_instance* instances, int32_t count, int32_t workers,
                                      spd_instance_result* results) {
  if (count < 0 || workers < 1 || (count > 0 && (!instances || !results))) {
    spd::set_last_error("bad batch arguments");
    return SPD_E_INVALID;
  }
  if (count == 0) return SPD_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    spd::set_last_error("no current device");
    return SPD_E_DEVICE;
  }
  // largest instances first (longest-processing-time order, with the rows
  // as the cost estimate): a large instance taken last would otherwise run
  // on after the others have finished
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto rows = [&](int i) {
    const spd_instance& q = instances[i];
    return (int64_t)(q.kernel.kind == SPD_K_RPY ? 3 : 1) * q.n;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rows(a) > rows(b); });
  std::atomic<int> next{0};
  std::atomic<int> setup_fail{0};
  auto worker = [&]() {
    if (hipSetDevice(dev) != hipSuccess) {
      setup_fail = 1;
      return;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      setup_fail = 1;
      return;
    }
    for (int j = next++; j < count; j = next++) spd::run_instance(instances[order[j]], s, results[order[j]]);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  };
  const int nw = std::min<int>(workers, count);
  std::vector<std::thread> pool;
  for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  if (setup_fail) {
    // instances a failed worker never took are run on this thread
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      spd::set_last_error("stream creation failed");
      return SPD_E_DEVICE;
    }
    for (int j = next++; j < count; j = next++) spd::run_instance(instances[order[j]], s, results[order[j]]);
    (void)hipStreamDestroy(s);
  }
  return SPD_OK;
}
