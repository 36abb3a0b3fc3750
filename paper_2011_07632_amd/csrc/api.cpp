// C ABI of the library (declared in include/spdhss.h).  Every entry point
// converts exceptions into status codes and records a thread-local message.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <cstring>

struct spd_h2 {
  spd::H2Model m;
};
struct spd_hss {
  spd::HSSModel m;
};
struct spd_ulv {
  spd::ULVModel m;
};

using namespace spd;

#define SPD_API_BEGIN try {
#define SPD_API_END                                \
  }                                                \
  catch (const spd::Error& e) {                    \
    spd::set_last_error(e.what());                 \
    return e.code;                                 \
  }                                                \
  catch (const std::bad_alloc&) {                  \
    spd::set_last_error("host allocation failed"); \
    return SPD_E_NOMEM;                            \
  }                                                \
  catch (const std::exception& e) {                \
    spd::set_last_error(e.what());                 \
    return SPD_E_DEVICE;                           \
  }                                                \
  spd::set_last_error("");                         \
  return SPD_OK;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <class T>
static void put(void* out, int64_t bytes, const T* src, size_t count) {
  SPD_REQUIRE(out != nullptr, SPD_E_INVALID, "null output buffer");
  SPD_REQUIRE((int64_t)(count * sizeof(T)) <= bytes, SPD_E_INVALID, "output buffer too small");
  if (count) std::memcpy(out, src, count * sizeof(T));
}

static void get_dev(void* out, int64_t bytes, const double* dev, size_t count) {
  SPD_REQUIRE(out != nullptr, SPD_E_INVALID, "null output buffer");
  SPD_REQUIRE((int64_t)(count * sizeof(double)) <= bytes, SPD_E_INVALID, "output buffer too small");
  if (count) SPD_HIP(hipMemcpy(out, dev, count * sizeof(double), hipMemcpyDeviceToHost));
}

extern "C" {

const char* spd_last_error(void) { return spd::last_error_cstr(); }

spd_status h2_build(const double* points, int64_t n, spd_kernel kernel, const spd_h2_opts* opts,
                    void* stream, spd_h2_t* out) {
  if (out) *out = nullptr;
  SPD_API_BEGIN
  SPD_REQUIRE(points && out && opts, SPD_E_INVALID, "null argument");
  SPD_REQUIRE(n >= 1, SPD_E_INVALID, "n must be positive");
  SPD_REQUIRE(n < (int64_t(1) << 31), SPD_E_INVALID, "n must be below 2^31");
  SPD_REQUIRE(kernel.kind >= 0 && kernel.kind <= 4, SPD_E_INVALID, "unknown kernel kind");
  SPD_REQUIRE(kernel.ell > 0 && std::isfinite(kernel.ell), SPD_E_INVALID, "ell must be positive");
  SPD_REQUIRE(std::isfinite(kernel.shift), SPD_E_INVALID, "shift must be finite");
  SPD_REQUIRE(opts->leaf_size >= 1 && opts->leaf_size <= 512, SPD_E_INVALID,
              "leaf_size must be in [1, 512]");
  SPD_REQUIRE(opts->tree == SPD_TREE_KD || opts->tree == SPD_TREE_BOX, SPD_E_INVALID,
              "unknown tree kind");
  SPD_REQUIRE(opts->eta > 0, SPD_E_INVALID, "eta must be positive");
  SPD_REQUIRE(opts->tol >= 0 && opts->tol < 1, SPD_E_INVALID, "tol must be in [0, 1)");
  SPD_REQUIRE(opts->proxy_shells >= 1 && opts->proxy_shells <= 64 && opts->proxy_per_shell >= 4,
              SPD_E_INVALID, "bad proxy counts");
  SPD_REQUIRE(opts->proxy_per_shell_max >= opts->proxy_per_shell, SPD_E_INVALID,
              "proxy_per_shell_max below proxy_per_shell");
  SPD_REQUIRE((int64_t)opts->proxy_shells * opts->proxy_per_shell_max <= 65536, SPD_E_INVALID,
              "at most 65536 proxy points");
  SPD_REQUIRE(opts->proxy_density >= 0 && std::isfinite(opts->proxy_density), SPD_E_INVALID,
              "proxy_density must be finite and non-negative");
  std::unique_ptr<spd_h2> h(new spd_h2());
  h->m.kern = kernel;
  h->m.opts = *opts;
  h->m.s = as_stream(stream);
  h2_build_impl(h->m, points, n);
  *out = h.release();
  SPD_API_END
}

spd_status spdhss_build(spd_h2_t A, const spd_hss_opts* opts, void* stream, spd_hss_t* out) {
  if (out) *out = nullptr;
  SPD_API_BEGIN
  SPD_REQUIRE(A && opts && out, SPD_E_INVALID, "null argument");
  std::unique_ptr<spd_hss> h(new spd_hss());
  hipStream_t s = as_stream(stream);
  A->m.s = s;
  spdhss_build_impl(A->m, *opts, h->m, s);
  *out = h.release();
  SPD_API_END
}

spd_status ulv_factor_ex(spd_hss_t M, int32_t precision, void* stream, spd_ulv_t* out) {
  if (out) *out = nullptr;
  SPD_API_BEGIN
  SPD_REQUIRE(M && out, SPD_E_INVALID, "null argument");
  SPD_REQUIRE(precision == SPD_SOLVE_F64 || precision == SPD_SOLVE_F32, SPD_E_INVALID,
              "unknown solve precision");
  std::unique_ptr<spd_ulv> u(new spd_ulv());
  u->m.precision = precision;
  ulv_factor_impl(M->m, u->m, as_stream(stream));
  *out = u.release();
  SPD_API_END
}

spd_status ulv_factor(spd_hss_t M, void* stream, spd_ulv_t* out) {
  return ulv_factor_ex(M, SPD_SOLVE_F64, stream, out);
}

spd_status ulv_apply(spd_ulv_t F, const double* b, double* x, int32_t nrhs, int64_t ld,
                     void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(F && b && x, SPD_E_INVALID, "null argument");
  const int64_t N = F->m.f->T.N;
  SPD_REQUIRE(nrhs >= 1 && ld >= N, SPD_E_INVALID, "bad nrhs or ld");
  hipStream_t s = as_stream(stream);
  F->m.s = s;
  double* in = ulv_plan_in(F->m, nrhs);
  double* out = ulv_plan_out(F->m, nrhs);
  launch_gather_rows(s, b, ld, in, N, F->m.f->perm_d, N, nrhs);
  ulv_apply_tree(F->m, in, out, nrhs);
  launch_scatter_rows(s, out, N, x, ld, F->m.f->perm_d, N, nrhs);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status ulv_apply_noalloc(spd_ulv_t F, const double* b, double* x, int32_t nrhs, int64_t ld,
                             void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(F && b && x, SPD_E_INVALID, "null argument");
  const int64_t N = F->m.f->T.N;
  SPD_REQUIRE(nrhs >= 1 && ld >= N, SPD_E_INVALID, "bad nrhs or ld");
  static_assert(SPD_NOALLOC_SCRATCH_BYTES == (long long)kNoAllocScratchBytes, "scratch size");
  F->m.s = as_stream(stream);
  ulv_apply_noalloc_impl(F->m, b, x, nrhs, ld);
  SPD_API_END
}

int64_t spd_noalloc_bytes(spd_ulv_t F, int32_t nrhs) {
  if (!F || nrhs < 1) return -1;
  return ulv_noalloc_bytes(F->m, nrhs);
}

spd_status h2_matvec_ex(spd_h2_t A, const double* x, double* y, int32_t nrhs, int64_t ld,
                        int32_t precision, void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && x && y, SPD_E_INVALID, "null argument");
  const int64_t N = A->m.T.N;
  SPD_REQUIRE(nrhs >= 1 && ld >= N, SPD_E_INVALID, "bad nrhs or ld");
  SPD_REQUIRE(x != y, SPD_E_INVALID, "x and y must not alias");
  SPD_REQUIRE(precision == SPD_SOLVE_F64 || precision == SPD_SOLVE_F32, SPD_E_INVALID,
              "unknown precision");
  SPD_REQUIRE(precision == SPD_SOLVE_F64 || nrhs <= 16, SPD_E_INVALID,
              "the FP32 product takes at most 16 columns");
  hipStream_t s = as_stream(stream);
  A->m.s = s;
  double* xt = h2_plan_x(A->m, nrhs);
  double* yt = h2_plan_y(A->m, nrhs);
  launch_gather_rows(s, x, ld, xt, N, A->m.perm_d, N, nrhs);
  if (precision == SPD_SOLVE_F32) h2_plan_run32(A->m, nrhs);
  else h2_plan_run(A->m);
  launch_scatter_rows(s, yt, N, y, ld, A->m.perm_d, N, nrhs);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status h2_matvec(spd_h2_t A, const double* x, double* y, int32_t nrhs, int64_t ld,
                     void* stream) {
  return h2_matvec_ex(A, x, y, nrhs, ld, SPD_SOLVE_F64, stream);
}

spd_status pcg_solve(spd_h2_t A, spd_ulv_t M, const double* b, double* x, int32_t nrhs, int64_t ld,
                     double rtol, int32_t maxit, void* stream, int32_t* iters, double* relres) {
  return pcg_solve_ex(A, M, b, x, nrhs, ld, rtol, maxit, SPD_SOLVE_F64, stream, iters, relres);
}

spd_status pcg_solve_ex(spd_h2_t A, spd_ulv_t M, const double* b, double* x, int32_t nrhs,
                        int64_t ld, double rtol, int32_t maxit, int32_t op_precision, void* stream,
                        int32_t* iters, double* relres) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && b && x, SPD_E_INVALID, "null argument");
  const int64_t N = A->m.T.N;
  SPD_REQUIRE(nrhs >= 1 && nrhs <= 4096 && ld >= N, SPD_E_INVALID, "bad nrhs or ld");
  SPD_REQUIRE(rtol >= 0 && maxit >= 0, SPD_E_INVALID, "bad rtol or maxit");
  SPD_REQUIRE(op_precision == SPD_SOLVE_F64 || op_precision == SPD_SOLVE_F32, SPD_E_INVALID,
              "unknown precision");
  SPD_REQUIRE(op_precision == SPD_SOLVE_F64 || nrhs <= 16, SPD_E_INVALID,
              "the FP32 product takes at most 16 columns");
  if (M) SPD_REQUIRE(M->m.f->T.N == N, SPD_E_INVALID, "preconditioner size mismatch");
  hipStream_t s = as_stream(stream);
  A->m.s = s;
  if (M) M->m.s = s;
  Arena a;
  double* bt = a.get_n<double>((size_t)N * nrhs);
  double* xt = a.get_n<double>((size_t)N * nrhs);
  launch_gather_rows(s, b, ld, bt, N, A->m.perm_d, N, nrhs);
  PcgResult r = pcg_tree(A->m, M ? &M->m : nullptr, bt, xt, nrhs, rtol, maxit,
                         op_precision == SPD_SOLVE_F32);
  launch_scatter_rows(s, xt, N, x, ld, A->m.perm_d, N, nrhs);
  SPD_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < nrhs; ++c) {
    if (iters) iters[c] = r.iters[c];
    if (relres) relres[c] = r.relres[c];
  }
  if (!r.converged) throw Error(SPD_E_NOT_CONVERGED, "PCG reached maxit before rtol");
  SPD_API_END
}

spd_status spd_h2_time_near(spd_h2_t A, int32_t nrhs, int32_t reps, void* stream, double* ms,
                            double* bytes) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && ms && bytes && nrhs >= 1 && reps >= 1, SPD_E_INVALID, "bad args");
  A->m.s = as_stream(stream);
  h2_time_near(A->m, nrhs, reps, ms, bytes);
  SPD_API_END
}

spd_status spd_h2_time_launches(spd_h2_t A, int32_t nrhs, int32_t reps, void* stream, double* ms,
                                double* bytes, int32_t* tags, int32_t cap, int32_t* count) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && ms && bytes && count && nrhs >= 1 && reps >= 1 && cap >= 1, SPD_E_INVALID,
              "bad args");
  A->m.s = as_stream(stream);
  *count = h2_time_launches(A->m, nrhs, reps, ms, bytes, tags, cap);
  SPD_API_END
}

void h2_destroy(spd_h2_t A) {
  try { delete A; } catch (...) {}
}
void spdhss_destroy(spd_hss_t M) {
  try { delete M; } catch (...) {}
}
void ulv_destroy(spd_ulv_t F) {
  try { delete F; } catch (...) {}
}

spd_status spd_h2_query_get(spd_h2_t A, int32_t what, void* out, int64_t bytes) {
  SPD_API_BEGIN
  SPD_REQUIRE(A, SPD_E_INVALID, "null handle");
  const H2Model& H = A->m;
  const TreeHost& T = H.T;
  switch (what) {
    case SPD_Q_N: { int64_t v = T.N; put(out, bytes, &v, 1); break; }
    case SPD_Q_LEVELS: { int64_t v = T.L; put(out, bytes, &v, 1); break; }
    case SPD_Q_NNODES: { int64_t v = T.nnodes; put(out, bytes, &v, 1); break; }
    case SPD_Q_PERM: put(out, bytes, T.perm.data(), T.perm.size()); break;
    case SPD_Q_NODE_START: {
      std::vector<int64_t> v(T.nnodes + 1);
      for (int i = 0; i < T.nnodes; ++i) v[i] = T.start[i];
      v[T.nnodes] = T.N;
      put(out, bytes, v.data(), v.size());
      break;
    }
    case SPD_Q_H2_RANK: put(out, bytes, H.k.data(), H.k.size()); break;
    case SPD_Q_SKELETON: {
      std::vector<int64_t> v;
      for (int i = 1; i < T.nnodes; ++i)
        for (int q = 0; q < H.k[i]; ++q) v.push_back(T.perm[H.skel_h[i][q]]);
      put(out, bytes, v.data(), v.size());
      break;
    }
    case SPD_Q_NEAR_PTR: put(out, bytes, T.near_ptr.data(), T.near_ptr.size()); break;
    case SPD_Q_NEAR_IDX: put(out, bytes, T.near_idx.data(), T.near_idx.size()); break;
    case SPD_Q_COUP_PTR: put(out, bytes, T.coup_ptr.data(), T.coup_ptr.size()); break;
    case SPD_Q_COUP_IDX: put(out, bytes, T.coup_idx.data(), T.coup_idx.size()); break;
    case SPD_Q_BYTES: { int64_t v = (int64_t)A->m.arena.bytes_used(); put(out, bytes, &v, 1); break; }
    case SPD_Q_H2_TIMES: put(out, bytes, H.times, 4); break;
    case SPD_Q_PROXY_COUNT: put(out, bytes, H.proxy_n.data(), H.proxy_n.size()); break;
    case SPD_Q_H2_STORAGE: {
      int64_t v[3] = {0, 0, 0};
      for (int i = T.first_at(1); i < T.first_at(1) + T.count_at(1); ++i)
        for (int64_t e = T.near_ptr[i]; e < T.near_ptr[i + 1]; ++e)
          v[0] += (int64_t)8 * std::max(H.near_ld(i), 16) * T.size(T.near_idx[e]);
      for (int i = 1; i < T.nnodes; ++i) {
        for (int64_t e = T.coup_ptr[i]; e < T.coup_ptr[i + 1]; ++e)
          if (H.Bh[e]) v[1] += (int64_t)8 * H.coup_ld(i) * H.k[T.coup_idx[e]];
        if (H.W[i]) v[2] += (int64_t)16 * H.cand[i] * H.k[i];
        if (H.E[i]) v[2] += (int64_t)16 * H.k[i] * (H.cand[i] - H.k[i]);
      }
      put(out, bytes, v, 3);
      break;
    }
    default: throw Error(SPD_E_INVALID, "unknown query");
  }
  SPD_API_END
}

spd_status spd_hss_query_get(spd_hss_t Mh, int32_t what, int32_t node, int32_t node2, void* out,
                             int64_t bytes) {
  SPD_API_BEGIN
  SPD_REQUIRE(Mh, SPD_E_INVALID, "null handle");
  const HSSModel& M = Mh->m;
  const Factors& F = *M.f;
  const TreeHost& T = F.T;
  const bool needs_node = what == SPD_HQ_PIVOTS || what == SPD_HQ_BASIS || what == SPD_HQ_TRANSFER ||
                          what == SPD_HQ_PHIU || what == SPD_HQ_COUPLING || what == SPD_HQ_FACTOR ||
                          what == SPD_HQ_ROWS;
  if (needs_node) SPD_REQUIRE(node >= 0 && node < T.nnodes, SPD_E_INVALID, "node out of range");
  switch (what) {
    case SPD_HQ_RANK: put(out, bytes, F.r.data(), F.r.size()); break;
    case SPD_HQ_ROWS: { int64_t v = F.rho[node]; put(out, bytes, &v, 1); break; }
    case SPD_HQ_PIVOTS: {
      std::vector<int> v(F.r[node]);
      if (!v.empty())
        SPD_HIP(hipMemcpy(v.data(), M.piv[node], v.size() * sizeof(int), hipMemcpyDeviceToHost));
      put(out, bytes, v.data(), v.size());
      break;
    }
    case SPD_HQ_BASIS:
      SPD_REQUIRE(node > 0 && F.V[node], SPD_E_INVALID, "no basis at this node");
      get_dev(out, bytes, F.V[node], (size_t)F.rho[node] * F.r[node]);
      break;
    case SPD_HQ_TRANSFER:
      SPD_REQUIRE(node > 0 && !T.is_leaf(node) && M.R[node], SPD_E_INVALID, "no transfer matrix");
      get_dev(out, bytes, M.R[node], (size_t)F.rho[node] * F.r[node]);
      break;
    case SPD_HQ_PHIU:
      SPD_REQUIRE(node > 0 && M.PhiU[node], SPD_E_INVALID, "no Phi U at this node");
      get_dev(out, bytes, M.PhiU[node], (size_t)F.r[node] * M.hk[node]);
      break;
    case SPD_HQ_COUPLING: {
      SPD_REQUIRE(node2 >= 0 && node2 < T.nnodes && node2 != node, SPD_E_INVALID, "bad pair");
      const int64_t e = M.lists.near_pos(node, node2);
      const double* B = nullptr;
      if (e >= 0) B = M.Bn[e];
      else {
        const int64_t f = M.lists.coup_pos(node, node2);
        SPD_REQUIRE(f >= 0, SPD_E_INVALID, "pair is neither near nor coupling");
        B = M.Bc[f];
      }
      SPD_REQUIRE(B, SPD_E_INVALID, "coupling not computed");
      get_dev(out, bytes, B, (size_t)F.r[node] * F.r[node2]);
      break;
    }
    case SPD_HQ_FACTOR: {
      const double* p = T.is_leaf(node) ? F.S[node] : F.F[node];
      SPD_REQUIRE(p, SPD_E_INVALID, "no factor at this node");
      get_dev(out, bytes, p, (size_t)F.rho[node] * F.rho[node]);
      break;
    }
    case SPD_HQ_BYTES: {
      int64_t v = (int64_t)(M.arena.bytes_used() + F.arena.bytes_used());
      put(out, bytes, &v, 1);
      break;
    }
    case SPD_HQ_TIMES: put(out, bytes, M.times, 8); break;
    case SPD_HQ_FLOPS: put(out, bytes, M.flops, 4); break;
    default: throw Error(SPD_E_INVALID, "unknown query");
  }
  SPD_API_END
}

// ---------------------------------------------------------- test hooks --
spd_status spd_test_gemm(const double* A, const double* B, double* C, int32_t batch, int32_t m,
                         int32_t n, int32_t k, int32_t transA, int32_t transB, double alpha,
                         double beta, void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && B && C && batch >= 1 && m >= 1 && n >= 1 && k >= 1, SPD_E_INVALID, "bad args");
  hipStream_t s = as_stream(stream);
  Stage st;
  GemmBatch g(transA, transB);
  const int lda = transA ? k : m, ldb = transB ? n : k;
  for (int b = 0; b < batch; ++b) {
    g.add(C + (size_t)b * m * n, m, n, m, beta, alpha);
    g.term(A + (size_t)b * m * k, lda, B + (size_t)b * k * n, ldb, k);
  }
  g.run(s, st);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status spd_test_symm(const double* A, const double* X, double* Y, int32_t nblk, int32_t m,
                         int32_t nterm, int32_t n, int32_t reps, void* stream, double* ms) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && X && Y && nblk >= 1 && m >= 1 && nterm >= 0 && n >= 1 && n <= 16 && reps >= 0,
              SPD_E_INVALID, "bad args");
  SPD_REQUIRE(nblk >= 2 * nterm + 1, SPD_E_INVALID, "nblk must be at least 2 nterm + 1");
  SPD_REQUIRE((int64_t)nblk * m <= (1ll << 30), SPD_E_INVALID, "nblk m above 2^30 rows");
  SPD_REQUIRE(reps == 0 || ms, SPD_E_INVALID, "null time output");
  hipStream_t s = as_stream(stream);
  const int ld = nblk * m;
  std::vector<SymRow> rows(nblk);
  for (int i = 0; i < nblk; ++i) {
    rows[i] = SymRow{Y + (size_t)i * m, ld, X + (size_t)i * m, ld, m, {}};
    for (int t = 0; t < nterm; ++t) {
      const int j = (i + 1 + t) % nblk;
      rows[i].terms.push_back({A + ((size_t)i * nterm + t) * m * m, m, X + (size_t)j * m, ld, m, j});
    }
  }
  Arena a;
  Recorder rec;
  rec.symv(a, s, rows, n, 0.0, false);
  rec.replay(s);
  if (reps > 0 && !rec.recs.empty()) {
    Recorder one;
    one.recs.push_back(rec.recs[0]);
    hipEvent_t e0, e1;
    SPD_HIP(hipEventCreate(&e0));
    SPD_HIP(hipEventCreate(&e1));
    SPD_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) one.replay(s);
    SPD_HIP(hipEventRecord(e1, s));
    SPD_HIP(hipEventSynchronize(e1));
    float t = 0;
    SPD_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
  }
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status spd_test_chol(double* A, int32_t batch, int32_t n, int32_t* fail, void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && fail && batch >= 1 && n >= 1 && n <= 1024, SPD_E_INVALID, "bad args");
  hipStream_t s = as_stream(stream);
  Stage st;
  std::vector<CholProblem> p(batch);
  for (int b = 0; b < batch; ++b) p[b] = {A + (size_t)b * n * n, n, n};
  auto* d = (const CholProblem*)st.push(s, p.data(), p.size() * sizeof(CholProblem));
  launch_chol(s, d, batch, n, fail);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status spd_test_trsm(const double* L, double* B, int32_t batch, int32_t n, int32_t nrhs,
                         int32_t trans, int32_t upper, void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(L && B && batch >= 1 && n >= 1 && n <= 2048 && nrhs >= 1, SPD_E_INVALID, "bad args");
  hipStream_t s = as_stream(stream);
  Stage st;
  TrsmBatch tb;
  for (int b = 0; b < batch; ++b) tb.add(L + (size_t)b * n * n, n, B + (size_t)b * n * nrhs, n, n, nrhs);
  tb.run(s, st, trans, upper);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

spd_status spd_test_cpqr(double* A, double* Q, int32_t* piv, int32_t* rank, double* diag,
                         int32_t batch, int32_t m, int32_t n, int32_t maxrank, double tol,
                         int32_t which, void* stream) {
  SPD_API_BEGIN
  SPD_REQUIRE(A && piv && rank && batch >= 1 && m >= 1 && n >= 1 && maxrank >= 0, SPD_E_INVALID,
              "bad args");
  if (which == 0) SPD_REQUIRE(cpqr_reg_fits(m, n) && Q, SPD_E_INVALID, "shape exceeds register kernel");
  if (which == 1) SPD_REQUIRE(m <= kCpqrWideRows && n <= 4096, SPD_E_INVALID, "shape too large");
  hipStream_t s = as_stream(stream);
  Stage st;
  Arena a;
  const int mr = std::min(std::min(m, n), maxrank);
  std::vector<CpqrProblem> p(batch);
  for (int b = 0; b < batch; ++b) {
    CpqrProblem& c = p[b];
    c = CpqrProblem{};
    c.A = A + (size_t)b * m * n;
    c.Q = which == 0 ? Q + (size_t)b * m * std::max(maxrank, 1) : nullptr;
    c.V = which == 0 ? a.get_n<double>((size_t)m * std::max(mr, 1)) : nullptr;
    c.R = which == 1 ? a.get_n<double>((size_t)std::max(mr, 1) * n) : nullptr;
    c.piv = piv + (size_t)b * (which == 1 ? n : std::max(maxrank, 1));
    c.rank = rank + b;
    c.diag = diag ? diag + (size_t)b * std::max(maxrank, 1) : nullptr;
    c.m = m;
    c.n = n;
    c.lda = m;
    c.ldq = m;
    c.maxrank = mr;
    c.tol = tol;
    c.nrm = which == 1 ? a.get_n<double>(2 * (size_t)n + mr + 2) : nullptr;
  }
  auto* d = (const CpqrProblem*)st.push(s, p.data(), p.size() * sizeof(CpqrProblem));
  if (which == 0) launch_cpqr_reg(s, d, batch, m, n);
  else cpqr_global(s, st, p, d, m, n);
  SPD_HIP(hipStreamSynchronize(s));
  SPD_API_END
}

}  // extern "C"

extern "C" void spd_release_cached_memory(void) { spd::release_cached_chunks(); }
