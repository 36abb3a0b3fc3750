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
// The sweeps are run in an equivalent form with one product per level.  With
// Z = S^{-T} V (leaf) or F^{-T} V-bar (nonleaf) and d = w - t:
//   up:    t_v = Z_v^T b_v (leaf),  t_v = Z_v^T [t_c] (nonleaf)
//   root:  [d_c] = ((I + bold B_root)^{-1} - I) [t_c]
//   down:  [d_c] = ((I + bold B_v)^{-1} - I) [t_c] + Z_v d_v
//   leaf:  x_v = A_vv^{-1} b_v + Z_v d_v
// since F^{-T}(F^{-1} t + V-bar d) - t = (F^{-T} F^{-1} - I) t + Z d and
// S^{-T}(S^{-1} b + V d) = (S S^T)^{-1} b + Z d.  The matrices are formed once
// by ulv_factor from explicit inverses of the triangular factors.
//
// PCG (Section 6): x0 = 0, one recurrence per right-hand side, a column stops
// once its recursively updated residual satisfies ||r|| <= rtol ||b||.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>

namespace spd {

struct ULVModel::ApplyPlan {
  int ncols = 0;
  Arena arena;
  Recorder rec;
  double* in = nullptr;   // tree-order right-hand sides (read)
  double* out = nullptr;  // tree-order solution (written)
  double* ts = nullptr;   // stacked t blocks
  double* ds = nullptr;   // stacked d = w - t blocks
};

ULVModel::ULVModel() = default;
ULVModel::~ULVModel() = default;

// The solve's matrices (see the top of this file): explicit inverses X of the
// triangular factors (S_v at the leaves, F_v above) by triangular solves
// against the identity, in scratch memory; then Dm_v = X^T X (leaf) or
// X^T X - I, and Z_v and Z_v^T copied from the construction, so that every
// product of the solve reads its matrix down columns.
static void form_solve_ops(Factors& F, const HSSModel& M, Stage& st, hipStream_t s) {
  if (F.ops_ready) return;
  const TreeHost& T = F.T;
  F.Dm.assign(T.nnodes, nullptr);
  F.Zs.assign(T.nnodes, nullptr);
  F.ZsT.assign(T.nnodes, nullptr);
  Arena tmp;
  BlockBatch eye, dm_init, cp;
  TrsmBatch tb;
  GemmBatch g(1, 0);
  for (int v = 0; v < T.nnodes; ++v) {
    const bool leaf = T.is_leaf(v);
    const double* L = leaf ? F.S[v] : F.F[v];
    const int n = F.rho[v];
    if (!L || n <= 0) continue;
    double* X = tmp.get_n<double>((size_t)n * n);
    eye.add(X, n, n, n, 0.0, 1);
    tb.add(L, n, X, n, n, n);
    F.Dm[v] = F.arena.get_n<double>((size_t)n * n);
    if (!leaf) dm_init.add(F.Dm[v], n, n, n, 0.0, 1);
    g.add(F.Dm[v], n, n, n, leaf ? 0.0 : -1.0);
    g.term(X, n, X, n, n);
    const int r = F.r[v];
    if (v > 0 && r > 0 && (size_t)v < M.Z.size() && M.Z[v]) {
      F.Zs[v] = F.arena.get_n<double>((size_t)n * r);
      F.ZsT[v] = F.arena.get_n<double>((size_t)n * r);
      cp.add(F.Zs[v], n, r, n);
      cp.term(M.Z[v], n);
      cp.add(F.ZsT[v], r, n, r);
      cp.term(M.Z[v], n, 1.0, 1);
    }
  }
  eye.run(s, st);
  tb.run(s, st, 0);
  dm_init.run(s, st);
  g.run(s, st);
  cp.run(s, st);
  SPD_HIP(hipStreamSynchronize(s));
  st.reset();
  F.ops_ready = true;
}

// FP32 copies of the solve operators for the mixed-precision apply.
static void form_solve_ops_f32(Factors& F, Stage& st, hipStream_t s) {
  if (F.ops32_ready) return;
  const int nn = F.T.nnodes;
  F.Dm32.assign(nn, nullptr);
  F.Zs32.assign(nn, nullptr);
  F.ZsT32.assign(nn, nullptr);
  std::vector<CvtProblem> cv;
  auto copy = [&](const double* src, float*& dst, int64_t n) {
    if (!src || n <= 0) return;
    dst = F.arena.get_n<float>((size_t)n);
    cv.push_back({src, dst, n});
  };
  for (int v = 0; v < nn; ++v) {
    const int64_t n = F.rho[v], r = F.r[v];
    copy(F.Dm[v], F.Dm32[v], n * n);
    if (F.Zs[v]) {
      copy(F.Zs[v], F.Zs32[v], n * r);
      copy(F.ZsT[v], F.ZsT32[v], n * r);
    }
  }
  if (!cv.empty()) {
    auto* d = (const CvtProblem*)st.push(s, cv.data(), cv.size() * sizeof(CvtProblem));
    launch_to_f32(s, d, (int)cv.size());
  }
  SPD_HIP(hipStreamSynchronize(s));
  st.reset();
  F.ops32_ready = true;
}

void ulv_factor_impl(HSSModel& M, ULVModel& U, hipStream_t s) {
  U.f = M.f;
  U.s = s;
  Factors& F = *U.f;
  const TreeHost& T = F.T;
  if (T.L == 1 || F.root_factored) {
    F.root_factored = true;
    form_solve_ops(F, M, U.stage, s);
    if (U.precision == 1) form_solve_ops_f32(F, U.stage, s);
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
  form_solve_ops(F, M, U.stage, s);
  if (U.precision == 1) form_solve_ops_f32(F, U.stage, s);
}

// The sweeps as batched products, one launch per level.  With at most 4
// columns every product is a dot-form product (transposed storage: Z_v for
// Z_v^T, Z_v^T for Z_v, and the symmetric Dm_v for itself), whose lanes run
// down stored columns; with more columns the same products run on MFMA.
// region: the plan's buffers, descriptors and partial results come from
// [region, region + region_bytes) only (no device allocation), else from the
// plan's own arena.
static std::unique_ptr<ULVModel::ApplyPlan> make_apply_plan(ULVModel& U, int m, void* region = nullptr,
                                                            size_t region_bytes = 0) {
  auto pl = std::make_unique<ULVModel::ApplyPlan>();
  if (region) pl->arena.use_region(region, region_bytes);
  pl->ncols = m;
  Factors& F = *U.f;
  const TreeHost& T = F.T;
  const int L = T.L;
  const int64_t N = T.N;
  hipStream_t s = U.s;
  Arena& a = pl->arena;
  Recorder& rec = pl->rec;
  pl->in = a.get_n<double>((size_t)N * m);
  pl->out = a.get_n<double>((size_t)N * m);
  const int lf = T.first_at(1), lc = T.count_at(1);
  const int Ni = (int)N;
  const int tA = m <= 4 ? 1 : 0;
  // mixed precision: FP32 operators, read by the dot-form products (<= 4
  // columns) or by the symmetric-pair kernel's row sums (5-16 columns)
  const bool f32 = U.precision == 1 && m <= 16;
  auto op = [&](const std::vector<double*>& d, const std::vector<float*>& f, int v) -> const double* {
    return f32 ? (const double*)f[v] : d[v];
  };
  auto batch = [&]() {
    GemmBatch g(tA, 0);
    g.a_f32 = f32 ? 1 : 0;
    return g;
  };
  if (L == 1) {
    GemmBatch g = batch();
    g.add(pl->out, Ni, m, Ni);
    g.term(op(F.Dm, F.Dm32, 0), Ni, pl->in, Ni, Ni);
    rec.gemm(a, s, g);
    SPD_HIP(hipStreamSynchronize(s));
    return pl;
  }
  const int64_t rows = std::max<int64_t>(F.stack_rows, 1);
  pl->ts = a.get_n<double>((size_t)rows * m);
  pl->ds = a.get_n<double>((size_t)rows * m);
  // leaves: t_v = Z_v^T b_v
  {
    GemmBatch g = batch();
    for (int v = lf; v < lf + lc; ++v) {
      if (F.r[v] == 0) continue;
      g.add(F.blk(pl->ts, v, m), F.r[v], m, F.blk_ld(v));
      if (tA) g.term(op(F.Zs, F.Zs32, v), F.rho[v], pl->in + T.start[v], Ni, F.rho[v]);
      else g.term(op(F.ZsT, F.ZsT32, v), F.r[v], pl->in + T.start[v], Ni, F.rho[v]);
    }
    rec.gemm(a, s, g);
  }
  // upward: t_v = Z_v^T [t_c]
  for (int lev = 2; lev <= L - 1; ++lev) {
    GemmBatch g = batch();
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      if (F.r[v] == 0 || F.rho[v] == 0) continue;
      g.add(F.blk(pl->ts, v, m), F.r[v], m, F.blk_ld(v));
      if (tA) g.term(op(F.Zs, F.Zs32, v), F.rho[v], pl->ts + F.par_off[v] * m, F.rho[v], F.rho[v]);
      else g.term(op(F.ZsT, F.ZsT32, v), F.r[v], pl->ts + F.par_off[v] * m, F.rho[v], F.rho[v]);
    }
    rec.gemm(a, s, g);
  }
  // root: [d_c] = ((I + bold B_root)^{-1} - I) [t_c]
  if (F.rho[0] > 0) {
    const int rv = F.rho[0];
    GemmBatch g = batch();
    g.add(pl->ds + F.par_off[0] * m, rv, m, rv);
    g.term(op(F.Dm, F.Dm32, 0), rv, pl->ts + F.par_off[0] * m, rv, rv);
    rec.gemm(a, s, g);
  }
  // downward: [d_c] = ((I + bold B_v)^{-1} - I) [t_c] + Z_v d_v
  for (int lev = L - 1; lev >= 2; --lev) {
    GemmBatch g = batch();
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      const int rv = F.rho[v];
      if (rv == 0) continue;
      g.add(pl->ds + F.par_off[v] * m, rv, m, rv);
      g.term(op(F.Dm, F.Dm32, v), rv, pl->ts + F.par_off[v] * m, rv, rv);
      if (F.r[v] > 0) {
        if (tA) g.term(op(F.ZsT, F.ZsT32, v), F.r[v], F.blk(pl->ds, v, m), F.blk_ld(v), F.r[v]);
        else g.term(op(F.Zs, F.Zs32, v), rv, F.blk(pl->ds, v, m), F.blk_ld(v), F.r[v]);
      }
    }
    rec.gemm(a, s, g);
  }
  // leaves: x_v = A_vv^{-1} b_v + Z_v d_v
  {
    GemmBatch g = batch();
    for (int v = lf; v < lf + lc; ++v) {
      const int nv = F.rho[v];
      g.add(pl->out + T.start[v], nv, m, Ni);
      g.term(op(F.Dm, F.Dm32, v), nv, pl->in + T.start[v], Ni, nv);
      if (F.r[v] > 0) {
        if (tA) g.term(op(F.ZsT, F.ZsT32, v), F.r[v], F.blk(pl->ds, v, m), F.blk_ld(v), F.r[v]);
        else g.term(op(F.Zs, F.Zs32, v), nv, F.blk(pl->ds, v, m), F.blk_ld(v), F.r[v]);
      }
    }
    rec.gemm(a, s, g);
  }
  SPD_HIP(hipStreamSynchronize(s));
  return pl;
}

static void build_apply_plan(ULVModel& U, int m) { U.plan = make_apply_plan(U, m); }

double* ulv_plan_in(ULVModel& U, int m) {
  if (!U.plan || U.plan->ncols != m) {
    U.plan.reset();
    build_apply_plan(U, m);
  }
  return U.plan->in;
}

double* ulv_plan_out(ULVModel& U, int m) {
  ulv_plan_in(U, m);
  return U.plan->out;
}

// ------------------------------------------------------ allocation-free apply --
// A fixed device array per GPU for the variant of the apply that allocates
// nothing: its tree-order right-hand sides and solution, the stacked rank-space
// blocks, the launch descriptors and any partial results all live here.  Every
// call on a device shares that device's copy, so calls that overlap on one
// GPU race; nothing in it has to start at zero (every block is written before
// it is read).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// The array's device address, taken once per device with that device current
// (the host-side name is only a stand-in for the symbol, not an address).
static char* scratch_address() {
  static std::mutex mu;
  static char* addr[64] = {};
  int dev = 0;
  SPD_HIP(hipGetDevice(&dev));
  SPD_REQUIRE(dev >= 0 && dev < 64, SPD_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(SPD_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = static_cast<char*>(p);
  }
  return addr[dev];
}

int64_t ulv_noalloc_bytes(const ULVModel& U, int m) {
  const Factors& F = *U.f;
  const int64_t rows = std::max<int64_t>(F.stack_rows, 1);
  return 8 * ((int64_t)2 * F.T.N * m + (F.T.L > 1 ? 2 * rows * m : 0));
}

void ulv_apply_noalloc_impl(ULVModel& U, const double* b, double* x, int m, int64_t ld) {
  const int64_t need = ulv_noalloc_bytes(U, m);
  SPD_REQUIRE(need <= (int64_t)kNoAllocScratchBytes, SPD_E_INVALID,
              "allocation-free apply: " + std::to_string(need) + " bytes of vectors exceed the " +
                  std::to_string(kNoAllocScratchBytes) + "-byte scratch array (use fewer right-hand sides)");
  char* base = scratch_address();
  auto pl = make_apply_plan(U, m, base, kNoAllocScratchBytes);
  const Factors& F = *U.f;
  const int64_t N = F.T.N;
  hipStream_t s = U.s;
  launch_gather_rows(s, b, ld, pl->in, N, F.perm_d, N, m);
  pl->rec.replay(s);
  launch_scatter_rows(s, pl->out, N, x, ld, F.perm_d, N, m);
  SPD_HIP(hipStreamSynchronize(s));
}

void ulv_apply_tree(ULVModel& U, const double* b, double* x, int m) {
  double* in = ulv_plan_in(U, m);
  double* out = U.plan->out;
  const int64_t N = U.f->T.N;
  if (b != in)
    SPD_HIP(hipMemcpyAsync(in, b, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, U.s));
  U.plan->rec.replay(U.s);
  if (x != out)
    SPD_HIP(hipMemcpyAsync(x, out, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, U.s));
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
                   int maxit, bool op_f32) {
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
  // the product reads p and writes q in place; the preconditioner reads r and
  // writes z in place
  double* r = U ? ulv_plan_in(*U, m) : a.get_n<double>((size_t)N * m);
  double* z = U ? ulv_plan_out(*U, m) : a.get_n<double>((size_t)N * m);
  double* p = h2_plan_x(H, m);
  double* q = h2_plan_y(H, m);
  if (op_f32) h2_plan_prepare32(H, m);
  const int nblk = coldot_chunks(N);
  double* partial = a.get_n<double>((size_t)nblk * m);
  // per-chunk partial dot products of the iteration (see k_pcg_xr_dot)
  double* pqp = a.get_n<double>((size_t)nblk * m);
  double* rrp = a.get_n<double>((size_t)nblk * m);
  double* rzp = a.get_n<double>((size_t)nblk * m);
  // flexible (Polak-Ribiere) beta when the preconditioner is applied in FP32:
  // partials of r_new . z_old, taken before z is overwritten
  const bool flexible = U && U->precision == 1;
  double* rzop = flexible ? a.get_n<double>((size_t)nblk * m) : nullptr;
  double* sc = a.get_n<double>((size_t)8 * m);
  double* rz = sc, *rzv = sc + m, *rr = sc + 3 * m, *bb = sc + 4 * m;
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
  launch_coldot_partial(s, r, z, N, m, N, rzp);
  launch_coldot(s, bt, bt, N, m, N, partial, bb);
  launch_coldot(s, r, r, N, m, N, partial, rr);
  {
    std::vector<int> init(2 * m + 1, 0);
    for (int c = 0; c < m; ++c) init[c] = 1;
    SPD_HIP(hipMemcpyAsync(active, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice, s));
    SPD_HIP(hipStreamSynchronize(s));
  }
  launch_pcg_active(s, rr, bb, rtol, active, m, any);
  // one iteration: q = A p; alpha = (r.z)/(p.q); x, r update; stop test;
  // z = M r; beta = (r.z)_new/(r.z)_old; p update.  The dot products stay as
  // per-chunk partials read by the next kernel.
  auto body = [&]() {
    if (op_f32) h2_plan_run32(H, m);
    else h2_plan_run(H);
    launch_coldot_partial(s, p, q, N, m, N, pqp);
    launch_pcg_xr_dot(s, xt, r, p, q, rzp, pqp, active, N, m, N, iters, rzv, rrp,
                      flexible ? z : nullptr, rzop);
    launch_pcg_active_partial(s, rrp, N, bb, rtol, active, m, any);
    precond(r, z);
    launch_coldot_partial(s, r, z, N, m, N, rzp);
    launch_pcg_update_p_partial(s, p, z, rzp, rzv, active, N, m, N, rzop);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the iteration runs as a captured graph; if capture is not available on
  // the stream (or instantiation fails) the same launches run eagerly
  bool use_graph = true;
  {
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
  PcgResult res;
  // Reliable updates (op_f32).  The recursively updated residual follows the
  // FP32 product, and drifts from b - A x by the rounding of the blocks times
  // the steps taken.  Whenever some active column's recursive residual has
  // dropped below kReliableDelta times its norm at the last replacement (checked
  // every kCheckEvery steps), every column's r is replaced by b - A x from the
  // FP64 product; p, z and the scalars carry on, so the Krylov recurrence is
  // not restarted.  Measured on the Matern N = 100k workload: 0.01 -> 3,736,
  // 0.1 -> 3,428, 0.5 -> 3,038 iterations (1,934 with the FP64 product).
  constexpr double kReliableDelta = 0.5;
  std::vector<double> ref(m, 0.0), hrrp((size_t)nblk * m);
  std::vector<int> hact(m);
  double* psave = op_f32 ? a.get_n<double>((size_t)N * m) : nullptr;
  auto replace_residual = [&]() {
    SPD_HIP(hipMemcpyAsync(psave, p, bytes, hipMemcpyDeviceToDevice, s));
    SPD_HIP(hipMemcpyAsync(p, xt, bytes, hipMemcpyDeviceToDevice, s));
    h2_plan_run(H);
    SPD_HIP(hipMemcpyAsync(r, bt, bytes, hipMemcpyDeviceToDevice, s));
    launch_axpby(s, r, q, -1.0, 1.0, N, m, N);
    SPD_HIP(hipMemcpyAsync(p, psave, bytes, hipMemcpyDeviceToDevice, s));
    launch_coldot(s, r, r, N, m, N, partial, rr);
    std::vector<double> h(m);
    SPD_HIP(hipMemcpyAsync(h.data(), rr, m * sizeof(double), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < m; ++c) ref[c] = std::sqrt(h[c]);
    ++res.replacements;
  };
  if (op_f32) {
    std::vector<double> h(m);
    SPD_HIP(hipMemcpyAsync(h.data(), rr, m * sizeof(double), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < m; ++c) ref[c] = std::sqrt(h[c]);
  }
  auto iterate = [&]() {
    while (done < maxit) {
      SPD_HIP(hipMemcpyAsync(&h_any, any, sizeof(int), hipMemcpyDeviceToHost, s));
      if (op_f32 && done > 0) {
        SPD_HIP(hipMemcpyAsync(hrrp.data(), rrp, hrrp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        SPD_HIP(hipMemcpyAsync(hact.data(), active, m * sizeof(int), hipMemcpyDeviceToHost, s));
      }
      SPD_HIP(hipStreamSynchronize(s));
      if (!h_any) break;
      if (op_f32 && done > 0) {
        bool due = false;
        for (int c = 0; c < m && !due; ++c) {
          if (!hact[c]) continue;
          double t = 0.0;
          for (int b = 0; b < nblk; ++b) t += hrrp[b + (size_t)c * nblk];
          due = std::sqrt(t) < kReliableDelta * ref[c];
        }
        if (due) replace_residual();
      }
      const int chunk = std::min(kCheckEvery, maxit - done);
      for (int c = 0; c < chunk; ++c) {
        if (use_graph) SPD_HIP(hipGraphLaunch(exec, s));
        else body();
      }
      done += chunk;
    }
  };
  // r = b - A x (true residual) and its relative norms per column
  std::vector<double> hrr(m), hbb(m), rel(m);
  auto true_residual = [&]() {
    SPD_HIP(hipMemcpyAsync(p, xt, bytes, hipMemcpyDeviceToDevice, s));
    h2_plan_run(H);
    SPD_HIP(hipMemcpyAsync(r, bt, bytes, hipMemcpyDeviceToDevice, s));
    launch_axpby(s, r, q, -1.0, 1.0, N, m, N);
    launch_coldot(s, r, r, N, m, N, partial, rr);
    SPD_HIP(hipMemcpyAsync(hrr.data(), rr, m * sizeof(double), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipMemcpyAsync(hbb.data(), bb, m * sizeof(double), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < m; ++c) rel[c] = hbb[c] > 0 ? std::sqrt(hrr[c] / hbb[c]) : std::sqrt(hrr[c]);
  };
  iterate();
  true_residual();
  // Residual replacement (beyond the paper, whose PCG stops on the recursively
  // updated residual): a column whose recursive residual met rtol while its
  // true residual is still above rtol (the two drift apart on ill-conditioned
  // systems) continues from the true residual, within maxit and at most
  // kMaxRestarts times, so that a converged result meets rtol on the true
  // residual.
  constexpr double kRestartFactor = 1.0;
  constexpr int kMaxRestarts = 4;
  for (int restart = 0; restart < kMaxRestarts && done < maxit; ++restart) {
    std::vector<int> act(m + 1, 0);
    SPD_HIP(hipMemcpyAsync(act.data(), active, (m + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    SPD_HIP(hipStreamSynchronize(s));
    bool again = false;
    for (int c = 0; c < m; ++c) {
      act[c] = (!act[c] && rel[c] > kRestartFactor * rtol) ? 1 : act[c];
      again |= act[c] != 0;
    }
    if (!again) break;
    act[m] = 1;  // any
    SPD_HIP(hipMemcpyAsync(active, act.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    // r holds the true residual: z = M r, p = z, then the iteration continues
    for (int c = 0; c < m; ++c) ref[c] = std::sqrt(hrr[c]);
    precond(r, z);
    SPD_HIP(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, s));
    launch_coldot_partial(s, r, z, N, m, N, rzp);
    SPD_HIP(hipStreamSynchronize(s));
    iterate();
    true_residual();
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  std::vector<int> act(2 * m + 1);
  SPD_HIP(hipMemcpyAsync(act.data(), active, act.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  SPD_HIP(hipStreamSynchronize(s));
  res.iters.assign(act.begin() + m + 1, act.end());
  res.relres = rel;
  for (int c = 0; c < m; ++c)
    if (act[c] || rel[c] > kRestartFactor * rtol) res.converged = false;
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
