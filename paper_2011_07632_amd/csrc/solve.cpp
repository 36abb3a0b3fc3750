// Solves with the SPD HSS matrix and PCG.
//
// Nested-factor solve.  At the leaf level the HSS matrix is
// A = S (I + V M V^T) S^T with S = diag(S_i) and orthonormal V = diag(V_i)
// (eq. Aii0 applied to the whole matrix), so
// A^{-1} = S^{-T} (I + V((I + M)^{-1} - I) V^T) S^{-1}, and I + M has the same
// form one level up with the factors F_i of I + bold B_ii (eqs. Si0/Si) down
// to I + bold B_root at the root.  Unfolded this gives an upward sweep
// (z = S^{-1} b, t = V^T z, u = F^{-1}[t_c], t = V-bar^T u), a root solve and a
// downward sweep (u += V-bar (w - t), w_c = F^{-T} u; at the leaves
// z += V (w - t), x = S^{-T} z).  The paper calls this step a ULV solve and
// times it with the construction; the method is not spelled out there.
//
// PCG (Section 6): x0 = 0, one recurrence per right-hand side, a column stops
// once its recursively updated residual satisfies ||r|| <= rtol ||b||.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace spd {

struct ULVModel::ApplyPlan {
  int ncols = 0;
  Arena arena;
  Recorder rec;
  double* z = nullptr;   // tree-order work vector (input and output)
  double* ts = nullptr;  // stacked t blocks
  double* ws = nullptr;  // stacked w blocks
  std::vector<double*> u;
};

ULVModel::ULVModel() = default;
ULVModel::~ULVModel() = default;

// Explicit inverses of the triangular factors (S_v at the leaves, F_v above),
// formed once by triangular solves against the identity, so that every sweep
// of the solve is a batched product.
static void invert_factors(Factors& F, Stage& st, hipStream_t s) {
  if (F.inverted) return;
  const TreeHost& T = F.T;
  F.Sinv.assign(T.nnodes, nullptr);
  F.Finv.assign(T.nnodes, nullptr);
  BlockBatch eye;
  TrsmBatch tb;
  for (int v = 0; v < T.nnodes; ++v) {
    const bool leaf = T.is_leaf(v);
    const double* L = leaf ? F.S[v] : F.F[v];
    const int n = F.rho[v];
    if (!L || n <= 0) continue;
    double* X = F.arena.get_n<double>((size_t)n * n);
    (leaf ? F.Sinv : F.Finv)[v] = X;
    eye.add(X, n, n, n, 0.0, 1);
    tb.add(L, n, X, n, n, n);
  }
  eye.run(s, st);
  tb.run(s, st, 0);
  SPD_HIP(hipStreamSynchronize(s));
  st.reset();
  F.inverted = true;
}

void ulv_factor_impl(HSSModel& M, ULVModel& U, hipStream_t s) {
  U.f = M.f;
  U.s = s;
  Factors& F = *U.f;
  const TreeHost& T = F.T;
  if (T.L == 1 || F.root_factored) {
    F.root_factored = true;
    invert_factors(F, U.stage, s);
    return;
  }
  const int c1 = 1, c2 = 2, r1 = F.r[c1], r2 = F.r[c2], rv = r1 + r2;
  F.rho[0] = rv;
  F.F[0] = F.arena.get_n<double>((size_t)std::max(rv * rv, 1));
  if (rv > 0) {
    BlockBatch as;
    if (r1 > 0) as.add(F.F[0], r1, r1, rv, 0.0, 1);
    if (r2 > 0) as.add(F.F[0] + r1 + (size_t)r1 * rv, r2, r2, rv, 0.0, 1);
    if (r1 > 0 && r2 > 0) {
      const int64_t e12 = M.lists.near_pos(c1, c2), e21 = M.lists.near_pos(c2, c1);
      const double* B12 = e12 >= 0 ? M.Bn[e12] : M.Bc[M.lists.coup_pos(c1, c2)];
      const double* B21 = e21 >= 0 ? M.Bn[e21] : M.Bc[M.lists.coup_pos(c2, c1)];
      as.add(F.F[0] + (size_t)r1 * rv, r1, r2, rv);
      as.term(B12, r1);
      as.add(F.F[0] + r1, r2, r1, rv);
      as.term(B21, r2);
    }
    as.run(s, U.stage);
    int* fail = F.arena.get_n<int>(2);
    launch_fill(s, (double*)fail, 0.0, 1);
    std::vector<CholProblem> ch{{F.F[0], rv, rv}};
    auto* d = (const CholProblem*)U.stage.push(s, ch.data(), sizeof(CholProblem));
    launch_chol(s, d, 1, rv, fail);
    int hf = 0;
    SPD_HIP(hipMemcpyAsync(&hf, fail, sizeof(int), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    U.stage.reset();
    if (hf) throw Error(SPD_E_NOT_SPD, "I + B_root not positive definite (root, level " +
                                           std::to_string(T.L) + ")");
  }
  SPD_HIP(hipStreamSynchronize(s));
  F.root_factored = true;
  invert_factors(F, U.stage, s);
}

static void build_apply_plan(ULVModel& U, int m) {
  auto pl = std::make_unique<ULVModel::ApplyPlan>();
  pl->ncols = m;
  Factors& F = *U.f;
  const TreeHost& T = F.T;
  const int L = T.L, nn = T.nnodes;
  const int64_t N = T.N;
  hipStream_t s = U.s;
  Arena& a = pl->arena;
  Recorder& rec = pl->rec;
  pl->z = a.get_n<double>((size_t)N * m);
  double* z2 = a.get_n<double>((size_t)N * m);
  const int lf = T.first_at(1), lc = T.count_at(1);
  const int Ni = (int)N;
  if (L == 1) {
    GemmBatch g1(0, 0), g2(1, 0);
    g1.add(z2, Ni, m, Ni);
    g1.term(F.Sinv[0], Ni, pl->z, Ni, Ni);
    g2.add(pl->z, Ni, m, Ni);
    g2.term(F.Sinv[0], Ni, z2, Ni, Ni);
    rec.gemm(a, s, g1);
    rec.gemm(a, s, g2);
    SPD_HIP(hipStreamSynchronize(s));
    U.plan = std::move(pl);
    return;
  }
  const int64_t rows = std::max<int64_t>(F.stack_rows, 1);
  pl->ts = a.get_n<double>((size_t)rows * m);
  pl->ws = a.get_n<double>((size_t)rows * m);
  pl->u.assign(nn, nullptr);
  double* rt = a.get_n<double>((size_t)std::max(F.rho[0], 1) * m);
  // leaves: z2 = S^{-1} b ; t = V^T z2
  {
    GemmBatch g1(0, 0), g2(1, 0);
    for (int v = lf; v < lf + lc; ++v) {
      const int nv = F.rho[v];
      g1.add(z2 + T.start[v], nv, m, Ni);
      g1.term(F.Sinv[v], nv, pl->z + T.start[v], Ni, nv);
      if (F.r[v] == 0) continue;
      g2.add(F.blk(pl->ts, v, m), F.r[v], m, F.blk_ld(v));
      g2.term(F.V[v], nv, z2 + T.start[v], Ni, nv);
    }
    rec.gemm(a, s, g1);
    rec.gemm(a, s, g2);
  }
  // upward: u = F^{-1} [t_c] ; t = V-bar^T u
  for (int lev = 2; lev <= L - 1; ++lev) {
    GemmBatch g1(0, 0), g2(1, 0);
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      const int rv = F.rho[v];
      pl->u[v] = a.get_n<double>((size_t)std::max(rv, 1) * m);
      if (rv == 0) continue;
      g1.add(pl->u[v], rv, m, rv);
      g1.term(F.Finv[v], rv, pl->ts + F.par_off[v] * m, rv, rv);
      if (F.r[v] == 0) continue;
      g2.add(F.blk(pl->ts, v, m), F.r[v], m, F.blk_ld(v));
      g2.term(F.V[v], rv, pl->u[v], rv, rv);
    }
    rec.gemm(a, s, g1);
    rec.gemm(a, s, g2);
  }
  // root: w = F_root^{-T} F_root^{-1} [t_c]
  {
    const int rv = F.rho[0];
    if (rv > 0) {
      GemmBatch g1(0, 0), g2(1, 0);
      g1.add(rt, rv, m, rv);
      g1.term(F.Finv[0], rv, pl->ts + F.par_off[0] * m, rv, rv);
      g2.add(pl->ws + F.par_off[0] * m, rv, m, rv);
      g2.term(F.Finv[0], rv, rt, rv, rv);
      rec.gemm(a, s, g1);
      rec.gemm(a, s, g2);
    }
  }
  // downward: u += V-bar (w - t) ; [w_c] = F^{-T} u
  for (int lev = L - 1; lev >= 2; --lev) {
    GemmBatch g1(0, 0), g2(1, 0);
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      const int rv = F.rho[v];
      if (rv == 0) continue;
      if (F.r[v] > 0) {
        g1.add(pl->u[v], rv, m, rv, 1.0);
        g1.term(F.V[v], rv, F.blk(pl->ws, v, m), F.blk_ld(v), F.r[v], 1.0);
        g1.term(F.V[v], rv, F.blk(pl->ts, v, m), F.blk_ld(v), F.r[v], -1.0);
      }
      g2.add(pl->ws + F.par_off[v] * m, rv, m, rv);
      g2.term(F.Finv[v], rv, pl->u[v], rv, rv);
    }
    rec.gemm(a, s, g1);
    rec.gemm(a, s, g2);
  }
  // leaves: z2 += V (w - t) ; x = S^{-T} z2
  {
    GemmBatch g1(0, 0), g2(1, 0);
    for (int v = lf; v < lf + lc; ++v) {
      const int nv = F.rho[v];
      if (F.r[v] > 0) {
        g1.add(z2 + T.start[v], nv, m, Ni, 1.0);
        g1.term(F.V[v], nv, F.blk(pl->ws, v, m), F.blk_ld(v), F.r[v], 1.0);
        g1.term(F.V[v], nv, F.blk(pl->ts, v, m), F.blk_ld(v), F.r[v], -1.0);
      }
      g2.add(pl->z + T.start[v], nv, m, Ni);
      g2.term(F.Sinv[v], nv, z2 + T.start[v], Ni, nv);
    }
    rec.gemm(a, s, g1);
    rec.gemm(a, s, g2);
  }
  SPD_HIP(hipStreamSynchronize(s));
  U.plan = std::move(pl);
}

double* ulv_plan_z(ULVModel& U, int m) {
  if (!U.plan || U.plan->ncols != m) {
    U.plan.reset();
    build_apply_plan(U, m);
  }
  return U.plan->z;
}

void ulv_apply_tree(ULVModel& U, const double* b, double* x, int m) {
  double* z = ulv_plan_z(U, m);
  const int64_t N = U.f->T.N;
  if (b != z)
    SPD_HIP(hipMemcpyAsync(z, b, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, U.s));
  U.plan->rec.replay(U.s);
  if (x != z)
    SPD_HIP(hipMemcpyAsync(x, z, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, U.s));
}

// ------------------------------------------------------------------ PCG --
// One iteration (product, preconditioner sweeps, dot products, updates) is
// captured into a HIP graph on a private stream and replayed; the host reads
// the convergence flags every few iterations.  Columns that have converged are
// frozen by the kernels themselves (they test the device-side active flags),
// so iterations run past convergence change nothing and the per-column
// iteration counters, kept on the device, stay exact.
static constexpr int kCheckEvery = 8;

PcgResult pcg_tree(H2Model& H, ULVModel* U, const double* bt, double* xt, int m, double rtol,
                   int maxit) {
  hipStream_t caller = H.s;
  hipStream_t s = nullptr;
  SPD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t ev = nullptr;
  struct Restore {
    H2Model& H;
    ULVModel* U;
    hipStream_t caller, s;
    hipEvent_t ev;
    ~Restore() {
      H.s = caller;
      if (U) U->s = caller;
      if (ev) (void)hipEventDestroy(ev);
      if (s) (void)hipStreamDestroy(s);
    }
  } restore{H, U, caller, s, nullptr};
  SPD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  restore.ev = ev;
  SPD_HIP(hipEventRecord(ev, caller));
  SPD_HIP(hipStreamWaitEvent(s, ev, 0));
  H.s = s;
  if (U) U->s = s;

  const int64_t N = H.T.N;
  const size_t bytes = (size_t)N * m * sizeof(double);
  Arena a;
  double* r = a.get_n<double>((size_t)N * m);
  double* z = a.get_n<double>((size_t)N * m);
  double* p = h2_plan_x(H, m);   // the product reads p in place
  double* q = h2_plan_y(H, m);   // and writes q in place
  if (U) ulv_plan_z(*U, m);
  const int nblk = ceil_div(N, 8192);
  double* partial = a.get_n<double>((size_t)nblk * m);
  double* sc = a.get_n<double>((size_t)8 * m);
  double* rz = sc, *rzn = sc + m, *pq = sc + 2 * m, *rr = sc + 3 * m, *bb = sc + 4 * m;
  int* active = a.get_n<int>(2 * m + 1);
  int* any = active + m;
  int* iters = active + m + 1;
  auto precond = [&](const double* in, double* out) {
    if (U) ulv_apply_tree(*U, in, out, m);
    else SPD_HIP(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s));
  };
  launch_fill(s, xt, 0.0, (int64_t)N * m);
  SPD_HIP(hipMemcpyAsync(r, bt, bytes, hipMemcpyDeviceToDevice, s));
  precond(r, z);
  SPD_HIP(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, s));
  launch_coldot(s, r, z, N, m, N, partial, rz);
  launch_coldot(s, bt, bt, N, m, N, partial, bb);
  launch_coldot(s, r, r, N, m, N, partial, rr);
  {
    std::vector<int> init(2 * m + 1, 0);
    for (int c = 0; c < m; ++c) init[c] = 1;
    SPD_HIP(hipMemcpyAsync(active, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SPD_HIP(hipStreamSynchronize(s));
  }
  launch_pcg_active(s, rr, bb, rtol, active, m, any);
  auto body = [&]() {
    h2_plan_run(H);  // q = A p
    launch_coldot(s, p, q, N, m, N, partial, pq);
    launch_pcg_update_xr(s, xt, r, p, q, rz, pq, active, N, m, N, iters);
    launch_coldot(s, r, r, N, m, N, partial, rr);
    launch_pcg_active(s, rr, bb, rtol, active, m, any);
    precond(r, z);
    launch_coldot(s, r, z, N, m, N, partial, rzn);
    launch_pcg_update_p(s, p, z, rzn, rz, active, N, m, N);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = getenv("SPDHSS_NO_GRAPH") == nullptr;
  if (use_graph) {
    SPD_HIP(hipStreamSynchronize(s));
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      body();
      if (hipStreamEndCapture(s, &graph) != hipSuccess ||
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        use_graph = false;
      }
    } else {
      (void)hipGetLastError();
      use_graph = false;
    }
  }
  int h_any = 1;
  int done = 0;
  while (done < maxit) {
    SPD_HIP(hipMemcpyAsync(&h_any, any, sizeof(int), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    if (!h_any) break;
    const int chunk = std::min(kCheckEvery, maxit - done);
    for (int c = 0; c < chunk; ++c) {
      if (use_graph) SPD_HIP(hipGraphLaunch(exec, s));
      else body();
    }
    done += chunk;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  PcgResult res;
  std::vector<int> act(2 * m + 1);
  SPD_HIP(hipMemcpyAsync(act.data(), active, act.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  // true residual
  SPD_HIP(hipMemcpyAsync(p, xt, bytes, hipMemcpyDeviceToDevice, s));
  h2_plan_run(H);
  SPD_HIP(hipMemcpyAsync(r, bt, bytes, hipMemcpyDeviceToDevice, s));
  launch_axpby(s, r, q, -1.0, 1.0, N, m, N);
  launch_coldot(s, r, r, N, m, N, partial, rr);
  std::vector<double> hrr(m), hbb(m);
  SPD_HIP(hipMemcpyAsync(hrr.data(), rr, m * sizeof(double), hipMemcpyDeviceToHost, s));
  SPD_HIP(hipMemcpyAsync(hbb.data(), bb, m * sizeof(double), hipMemcpyDeviceToHost, s));
  SPD_HIP(hipStreamSynchronize(s));
  res.iters.assign(act.begin() + m + 1, act.end());
  res.relres.resize(m);
  for (int c = 0; c < m; ++c) {
    res.relres[c] = hbb[c] > 0 ? std::sqrt(hrr[c] / hbb[c]) : std::sqrt(hrr[c]);
    if (act[c]) res.converged = false;
  }
  return res;
}

// Time the dominant kernel of the product (the leaf-level near-field pass)
// with HIP events on the stream it runs on.
void h2_time_near(H2Model& H, int m, int reps, double* ms, double* bytes) {
  double* x = h2_plan_x(H, m);
  (void)x;
  H2Model::NearStats st = h2_near_stats(H, m);
  hipEvent_t e0, e1;
  SPD_HIP(hipEventCreate(&e0));
  SPD_HIP(hipEventCreate(&e1));
  h2_plan_run_last(H);  // warm
  SPD_HIP(hipEventRecord(e0, H.s));
  for (int i = 0; i < reps; ++i) h2_plan_run_last(H);
  SPD_HIP(hipEventRecord(e1, H.s));
  SPD_HIP(hipEventSynchronize(e1));
  float t = 0;
  SPD_HIP(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  *bytes = st.bytes;
}

}  // namespace spd
