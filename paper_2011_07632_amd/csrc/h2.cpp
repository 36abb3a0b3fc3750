// H^2 representation of shift*I + K(X, X): construction and product.
//
// Section 5.1 (eq. uniformbasis_h2): far blocks A_ij = U_i B_ij U_j^T with
// nested bases U_i = diag(U_children) R_i (eq. nested); dense near blocks at
// the leaf level; only Type-3 couplings are stored (Section 5.2.2).
//
// Bases come from an interpolative decomposition against proxy points (the
// paper uses H2Pack's proxy-point method without describing it; this is the
// library's own construction): for each node, candidates are its points (leaf)
// or its children's skeletons (nonleaf); G = K(proxies, candidates) with
// proxies on spheres between the nearest far box and the farthest root-box
// corner; a column-pivoted QR of G with relative truncation picks the skeleton
// and W = [I; (R11^{-1} R12)^T] (rows in candidate order) is U_i or R_i.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace spd {

// The recorded product.  With at most 4 columns the near-field pass reads only
// x, so its product launch (`side`) runs on the side stream beside the
// far-field chain (`rec`: upward, coupling, downward down to the leaves, which
// writes the far-field part of y); `tail` then adds the near-field parts into
// y once both are done.  Otherwise everything is in `rec`.
struct H2Model::MatvecPlan {
  int ncols = 0;
  Arena arena;
  Recorder rec, side, tail;
  double* xh = nullptr;
  double* yh = nullptr;
  double* xt = nullptr;  // tree-order input
  double* yt = nullptr;  // tree-order output
};

H2Model::H2Model() = default;
H2Model::~H2Model() {
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (side_s) (void)hipStreamDestroy(side_s);
}

// Run the recorded product on H.s (the side part forked onto H.side_s and
// joined before the tail); stream-ordered and capturable into a graph.
static void replay_plan(H2Model& H, const H2Model::MatvecPlan& pl) {
  if (pl.side.recs.empty()) {
    pl.rec.replay(H.s);
    pl.tail.replay(H.s);
    return;
  }
  SPD_HIP(hipEventRecord(H.ev_fork, H.s));
  SPD_HIP(hipStreamWaitEvent(H.side_s, H.ev_fork, 0));
  pl.side.replay(H.side_s);
  SPD_HIP(hipEventRecord(H.ev_join, H.side_s));
  pl.rec.replay(H.s);
  SPD_HIP(hipStreamWaitEvent(H.s, H.ev_join, 0));
  pl.tail.replay(H.s);
}

// X = R^{-1} B in place for every problem (R upper triangular k x k, ld ldr;
// B k x n, ld ldb), for orders above what the batched triangular kernel holds
// in LDS: back substitution by row blocks of 256, each block row first updated
// with the rows already solved (an MFMA product), then its diagonal block
// solved by the batched triangular kernel.
struct UpperSolve {
  const double* R;
  int ldr;
  double* B;
  int ldb, k, n;
};
static void upper_solve_blocked(hipStream_t s, Stage& st, const std::vector<UpperSolve>& ps) {
  constexpr int NB = 256;
  int steps = 0;
  for (const UpperSolve& p : ps) steps = std::max(steps, ceil_div(p.k, NB));
  for (int step = 0; step < steps; ++step) {
    GemmBatch g(0, 0);
    TrsmBatch tb;
    for (const UpperSolve& p : ps) {
      const int b = ceil_div(p.k, NB) - 1 - step;
      if (b < 0 || p.n <= 0) continue;
      const int r0 = b * NB, rb = std::min(NB, p.k - r0), below = p.k - r0 - rb;
      if (below > 0) {
        g.add(p.B + r0, rb, p.n, p.ldb, 1.0, -1.0);
        g.term(p.R + r0 + (size_t)(r0 + rb) * p.ldr, p.ldr, p.B + r0 + rb, p.ldb, below);
      }
      tb.add(p.R + r0 + (size_t)r0 * p.ldr, p.ldr, p.B + r0, p.ldb, rb, p.n);
    }
    if (!g.empty()) g.run(s, st);
    tb.run(s, st, 1, 1);
  }
}

void h2_build_impl(H2Model& H, const double* points, int64_t npts) {
  hipStream_t s = H.s;
  const double t0 = now_seconds();
  std::vector<double> hp((size_t)3 * npts);
  SPD_HIP(hipMemcpyAsync(hp.data(), points, (size_t)3 * npts * sizeof(double), hipMemcpyDeviceToHost, s));
  SPD_HIP(hipStreamSynchronize(s));
  for (double x : hp) SPD_REQUIRE(std::isfinite(x), SPD_E_INVALID, "non-finite point coordinate");
  // The RPY tensor acts on 3 rows per particle (row 3p + c is component c of
  // particle p): the tree, lists and IDs work on these rows, each placed at
  // its particle, and the kernel blocks read a row's component from its
  // original index.
  const bool tensor = H.kern.kind == SPD_K_RPY;
  const int64_t n = tensor ? 3 * npts : npts;
  if (tensor) {
    std::vector<double> h3((size_t)3 * n);
    for (int64_t p = 0; p < npts; ++p)
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 3; ++k) h3[(size_t)3 * (3 * p + c) + k] = hp[(size_t)3 * p + k];
    hp.swap(h3);
  }
  TreeHost& T = H.T;
  T.build(hp.data(), n, H.opts.leaf_size, H.opts.eta, H.opts.tree);
  const int nn = T.nnodes, L = T.L;
  H.perm_d = upload(H.arena, s, T.perm);
  H.pts = H.arena.get_n<double>((size_t)3 * n);
  if (tensor) {
    double* rows = H.arena.get_n<double>((size_t)3 * n);
    SPD_HIP(hipMemcpyAsync(rows, hp.data(), (size_t)3 * n * sizeof(double), hipMemcpyHostToDevice, s));
    launch_soa_points(s, rows, H.perm_d, n, H.pts);
    SPD_HIP(hipStreamSynchronize(s));
  } else {
    launch_soa_points(s, points, H.perm_d, n, H.pts);
  }
  const double t1 = now_seconds();

  H.k.assign(nn, 0);
  H.cand.assign(nn, 0);
  H.cand_d.assign(nn, nullptr);
  H.cand_h.assign(nn, {});
  H.skel_h.assign(nn, {});
  H.W.assign(nn, nullptr);
  H.piv_d.assign(nn, nullptr);
  H.E.assign(nn, nullptr);
  H.ET.assign(nn, nullptr);
  {
    std::vector<int> pos(n);
    std::iota(pos.begin(), pos.end(), 0);
    int* leafpos = upload(H.arena, s, pos);
    for (int v = T.first_at(1); v < T.first_at(1) + T.count_at(1); ++v) {
      H.cand[v] = (int)T.size(v);
      H.cand_d[v] = leafpos + T.start[v];
      H.cand_h[v].resize(T.size(v));
      std::iota(H.cand_h[v].begin(), H.cand_h[v].end(), (int)T.start[v]);
    }
  }
  const int Q = H.opts.proxy_shells;
  H.proxy_n.assign(nn, 0);
  H.sketched.assign(nn, 0);
  Stage& st = H.stage;
  for (int lev = 1; lev < L; ++lev) {
    // per node: proxies per sphere, proxy rows M, candidates c, and the rows
    // m of the matrix whose pivoted QR picks the skeleton (the sketch of
    // l = max(2c, c + 16) rows when M exceeds l, else the proxy matrix)
    struct Job {
      int v, per, M, c, m;
      bool sk;
      double rin, rout;
    };
    std::vector<Job> jobs;
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      double rin, rout;
      if (H.cand[v] == 0 || !T.proxy_radii(v, rin, rout)) continue;
      Job jb;
      jb.v = v;
      jb.rin = rin;
      jb.rout = rout;
      // the RPY tensor: its ell is the particle radius, not a length scale of
      // a far field that decays like 1/r, so the count per sphere is fixed at
      // twice proxy_per_shell, and every proxy point gives 3 columns
      jb.per = tensor ? std::min(2 * H.opts.proxy_per_shell, H.opts.proxy_per_shell_max)
                      : proxy_count(rin, H.kern.ell, H.opts.proxy_per_shell, H.opts.proxy_per_shell_max,
                                    H.opts.proxy_density);
      jb.M = Q * jb.per * (tensor ? 3 : 1);
      jb.c = H.cand[v];
      const int l = std::max(2 * jb.c, jb.c + 16);
      jb.sk = jb.M > l;
      jb.m = jb.sk ? l : jb.M;
      SPD_REQUIRE(jb.m <= kCpqrWideRows, SPD_E_INVALID,
                  "H^2 proxy ID: more than 8000 candidates at node " + std::to_string(v) +
                      " (level " + std::to_string(lev) + ")");
      H.proxy_n[v] = jb.per;
      H.sketched[v] = jb.sk;
      jobs.push_back(jb);
    }
    size_t i = 0;
    while (i < jobs.size()) {
      // a batch of nodes whose proxy matrices, sketches, R factors and shared
      // Omega stay within about 16 GB (a level's nodes then run side by side,
      // one pivoted QR per workgroup)
      size_t j = i, bytes = 0;
      int64_t om_rows = 0, om_cols = 0;
      while (j < jobs.size()) {
        const Job& jb = jobs[j];
        size_t b = (size_t)jb.M * jb.c + (size_t)std::min(jb.m, jb.c) * jb.c + jb.c;
        if (jb.sk) b += (size_t)jb.m * jb.c;
        b *= 8;
        const int64_t r2 = jb.sk ? std::max<int64_t>(om_rows, jb.M) : om_rows;
        const int64_t c2 = jb.sk ? std::max<int64_t>(om_cols, jb.m) : om_cols;
        if (j > i && bytes + b + (size_t)(r2 * c2 * 8) > (size_t(16) << 30)) break;
        bytes += b;
        om_rows = r2;
        om_cols = c2;
        ++j;
      }
      const int nj = (int)(j - i);
      Arena tmp;
      std::vector<KBlockProblem> kb(nj);
      std::vector<CpqrProblem> cq(nj);
      std::vector<double*> Rp(nj);
      std::vector<int*> pivp(nj);
      int* d_rank = tmp.get_n<int>(nj);
      int maxc = 0, maxM = 0, maxm = 0;
      double* Om = om_rows > 0 ? tmp.get_n<double>((size_t)om_rows * om_cols) : nullptr;
      GemmBatch sketch(1, 0);
      for (int q = 0; q < nj; ++q) {
        const Job& jb = jobs[i + q];
        const int v = jb.v, c = jb.c, mr = std::min(jb.m, c);
        maxc = std::max(maxc, c);
        maxM = std::max(maxM, jb.M);
        maxm = std::max(maxm, jb.m);
        double* G = tmp.get_n<double>((size_t)jb.M * c);
        double* A = G;
        if (jb.sk) {
          A = tmp.get_n<double>((size_t)jb.m * c);
          sketch.add(A, jb.m, c, jb.m);
          sketch.term(Om, (int)om_rows, G, jb.M, jb.M);
        }
        Rp[q] = tmp.get_n<double>((size_t)mr * c);
        pivp[q] = tmp.get_n<int>(c);
        KBlockProblem& kp = kb[q];
        kp = KBlockProblem{};
        kp.out = G;
        kp.ia = nullptr;
        kp.ib = T.is_leaf(v) ? nullptr : H.cand_d[v];
        kp.offa = 0;
        kp.offb = T.is_leaf(v) ? T.start[v] : 0;
        kp.na = jb.M;
        kp.nb = c;
        kp.ld = jb.M;
        kp.proxy = 1;
        kp.shells = Q;
        kp.per_shell = jb.per;
        kp.cx = T.center[3 * v];
        kp.cy = T.center[3 * v + 1];
        kp.cz = T.center[3 * v + 2];
        kp.rin = jb.rin;
        kp.rout = jb.rout;
        CpqrProblem& cp = cq[q];
        cp = CpqrProblem{};
        cp.A = A;
        cp.R = Rp[q];
        cp.piv = pivp[q];
        cp.rank = d_rank + q;
        cp.m = jb.m;
        cp.n = c;
        cp.lda = jb.m;
        cp.maxrank = mr;
        cp.tol = H.opts.tol;
        cp.nrm = tmp.get_n<double>(2 * (size_t)c + mr + 2);  // the wide form's workspace
      }
      auto* dkb = (const KBlockProblem*)st.push(s, kb.data(), kb.size() * sizeof(KBlockProblem));
      launch_kblock(s, dkb, nj, maxM, maxc, H.pts, n, H.kern.kind, H.kern.ell, H.kern.shift, H.perm_d);
      if (!sketch.empty()) {
        launch_sketch_fill(s, Om, om_rows, (int)om_cols, om_rows, H.opts.sketch_seed);
        sketch.run(s, st);
      }
      auto* dcq = (const CpqrProblem*)st.push(s, cq.data(), cq.size() * sizeof(CpqrProblem));
      cpqr_global(s, st, cq, dcq, maxm, maxc);
      std::vector<int> ranks(nj);
      SPD_HIP(hipMemcpyAsync(ranks.data(), d_rank, nj * sizeof(int), hipMemcpyDeviceToHost, s));
      SPD_HIP(hipStreamSynchronize(s));
      st.reset();
      // E = R11^{-1} R12 in place of R12
      TrsmBatch tb;
      std::vector<UpperSolve> big;
      for (int q = 0; q < nj; ++q) {
        const Job& jb = jobs[i + q];
        const int c = jb.c, mr = std::min(jb.m, c), k = ranks[q];
        if (k > 0 && c > k) {
          if (k <= 2048) tb.add(Rp[q], mr, Rp[q] + (size_t)k * mr, mr, k, c - k);
          else big.push_back({Rp[q], mr, Rp[q] + (size_t)k * mr, mr, k, c - k});
        }
      }
      tb.run(s, st, 1, 1);
      if (!big.empty()) upper_solve_blocked(s, st, big);
      std::vector<std::vector<int>> pivh(nj);
      BlockBatch ecp;  // E_v and E_v^T, kept for the streaming product
      for (int q = 0; q < nj; ++q) {
        const Job& jb = jobs[i + q];
        const int v = jb.v, c = jb.c, mr = std::min(jb.m, c), k = ranks[q];
        H.k[v] = k;
        if (k > 0) {
          H.W[v] = H.arena.get_n<double>((size_t)c * k);
          launch_scatter_interp(s, H.W[v], c, Rp[q] + (size_t)k * mr, mr, pivp[q], c, k);
          H.piv_d[v] = H.arena.get_n<int>(c);
          SPD_HIP(hipMemcpyAsync(H.piv_d[v], pivp[q], c * sizeof(int), hipMemcpyDeviceToDevice, s));
          if (c > k) {
            H.E[v] = H.arena.get_n<double>((size_t)k * (c - k));
            H.ET[v] = H.arena.get_n<double>((size_t)k * (c - k));
            ecp.add(H.E[v], k, c - k, k);
            ecp.term(Rp[q] + (size_t)k * mr, mr);
            ecp.add(H.ET[v], c - k, k, c - k);
            ecp.term(Rp[q] + (size_t)k * mr, mr, 1.0, 1);
          }
        }
        pivh[q].resize(k);
        if (k > 0)
          SPD_HIP(hipMemcpyAsync(pivh[q].data(), pivp[q], k * sizeof(int), hipMemcpyDeviceToHost, s));
      }
      ecp.run(s, st);
      SPD_HIP(hipStreamSynchronize(s));
      st.reset();
      for (int q = 0; q < nj; ++q) {
        const int v = jobs[i + q].v;
        std::vector<int> sk(pivh[q].size());
        for (size_t t = 0; t < sk.size(); ++t) sk[t] = H.cand_h[v][pivh[q][t]];
        H.skel_h[v] = std::move(sk);
      }
      i = j;
    }
    // nodes without a far field keep no skeleton
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v)
      if (H.k[v] == 0) H.skel_h[v].clear();
    // parents' candidates: children's skeletons in child order
    for (int p = T.first_at(lev + 1); p < T.first_at(lev + 1) + T.count_at(lev + 1); ++p) {
      const int c1 = 2 * p + 1, c2 = 2 * p + 2;
      std::vector<int> cc(H.skel_h[c1]);
      cc.insert(cc.end(), H.skel_h[c2].begin(), H.skel_h[c2].end());
      H.cand[p] = (int)cc.size();
      H.cand_d[p] = cc.empty() ? H.arena.get_n<int>(1) : upload(H.arena, s, cc);
      H.cand_h[p] = std::move(cc);
    }
  }
  // W_v^T for the upward pass
  H.WT.assign(nn, nullptr);
  {
    BlockBatch tr;
    for (int v = 1; v < nn; ++v) {
      if (H.k[v] == 0 || H.cand[v] == 0) continue;
      H.WT[v] = H.arena.get_n<double>((size_t)H.k[v] * H.cand[v]);
      tr.add(H.WT[v], H.k[v], H.cand[v], H.k[v]);
      tr.term(H.W[v], H.cand[v], 1.0, 1);
    }
    tr.run(s, st);
    SPD_HIP(hipStreamSynchronize(s));
    st.reset();
  }
  const double t2 = now_seconds();

  // coupling blocks B_ij = K(skel_i, skel_j) and dense near blocks
  H.Bh.assign(T.coup_idx.size(), nullptr);
  H.nearA.assign(T.near_idx.size(), nullptr);
  {
    std::vector<KBlockProblem> kb;
    int mm = 0, mn = 0;
    // the blocks of one block row are adjacent in memory (one allocation), so
    // the product streams a row's couplings with adjacent columns as one
    for (int v = 1; v < nn; ++v) {
      size_t row = 0;
      for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) row += (size_t)H.k[T.coup_idx[e]];
      const int ld = H.coup_ld(v);
      double* base = (H.k[v] > 0 && row > 0) ? H.arena.get_n<double>((size_t)ld * row) : nullptr;
      if (base) launch_fill(s, base, 0.0, (int64_t)ld * row);
      for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
        const int j = T.coup_idx[e];
        if (H.k[v] == 0 || H.k[j] == 0) continue;
        H.Bh[e] = base;
        base += (size_t)ld * H.k[j];
        KBlockProblem kp{};
        kp.out = H.Bh[e];
        kp.ia = H.skel_d(v);
        kp.ib = H.skel_d(j);
        kp.na = H.k[v];
        kp.nb = H.k[j];
        kp.ld = ld;
        kb.push_back(kp);
        mm = std::max(mm, kp.na);
        mn = std::max(mn, kp.nb);
      }
    }
    for (int v = T.first_at(1); v < T.first_at(1) + T.count_at(1); ++v) {
      size_t row = 0;
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) row += (size_t)T.size(T.near_idx[e]);
      const int ld = std::max(H.near_ld(v), 16);
      double* base = H.arena.get_n<double>(std::max<size_t>((size_t)ld * row, 1));
      launch_fill(s, base, 0.0, std::max<int64_t>((int64_t)ld * row, 1));
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        const int ni = (int)T.size(v), nj = (int)T.size(j);
        H.nearA[e] = base;
        base += (size_t)ld * nj;
        KBlockProblem kp{};
        kp.out = H.nearA[e];
        kp.offa = T.start[v];
        kp.offb = T.start[j];
        kp.na = ni;
        kp.nb = nj;
        kp.ld = ld;
        kp.diag_shift = (v == j);
        kb.push_back(kp);
        mm = std::max(mm, ni);
        mn = std::max(mn, nj);
      }
    }
    // launch in bounded chunks of descriptors
    const size_t chunk = 1 << 16;
    for (size_t a = 0; a < kb.size(); a += chunk) {
      const size_t b = std::min(kb.size(), a + chunk);
      auto* d = (const KBlockProblem*)st.push(s, kb.data() + a, (b - a) * sizeof(KBlockProblem));
      launch_kblock(s, d, (int)(b - a), mm, mn, H.pts, n, H.kern.kind, H.kern.ell, H.kern.shift, H.perm_d);
    }
    SPD_HIP(hipStreamSynchronize(s));
    st.reset();
  }
  H.par_off.assign(nn, 0);
  H.stack_rows = 0;
  for (int p = 0; p < nn; ++p)
    if (!T.is_leaf(p)) {
      H.par_off[p] = H.stack_rows;
      H.stack_rows += H.cand[p];
    }
  const double t3 = now_seconds();
  H.times[0] = t1 - t0;
  H.times[1] = t2 - t1;
  H.times[2] = t3 - t2;
  H.times[3] = t3 - t0;
}

// ------------------------------------------------------------- product --
// Workgroups of the near-field product when it runs beside the far-field
// chain: few enough to leave the latency-bound level passes room.  With
// 512 leaves each workgroup takes one or two leaf rows.  Measured on the
// N = 100k Matern workload (ms per PCG iteration, 1,934 iterations in every
// case, since the cap only changes which workgroup takes which row):
// 128 -> 1.976, 256 -> 1.941, 320 -> 1.935, 352 -> 1.931, 384 -> 1.927,
// 416 -> 1.924, 448 -> 1.929, 512 (one row per workgroup) -> 1.939.
static constexpr int kNearCap = 416;

// Bytes of near blocks per part of a leaf row in the 5-16 column product.
// Each part writes its own m x n partial result, which the block sum reads
// back; leaf rows at N = 1M hold about 6.7 MB of blocks.  Measured there with
// 16 columns (near-field launch + its block sum, ms): 1 MiB 5.09 + 0.45,
// 2 MiB 5.02 + 0.40, 4 MiB 5.09 + 0.36.  The coupling rows keep 1 MiB
// (2 MiB: 3.86 + 0.43 against 3.72 + 0.46).
static double near_split(int ncols) { return ncols > 4 ? 2.0 * (1 << 20) : 0.0; }

// FP32 copies of the blocks that the symmetric-pair product reads.
static void make_f32_blocks(H2Model& H) {
  if (!H.Bh32.empty() || !H.nearA32.empty()) return;
  const TreeHost& T = H.T;
  hipStream_t s = H.s;
  H.Bh32.assign(H.Bh.size(), nullptr);
  H.nearA32.assign(H.nearA.size(), nullptr);
  std::vector<CvtProblem> cv;
  auto flush = [&]() {
    if (cv.empty()) return;
    auto* d = (const CvtProblem*)H.stage.push(s, cv.data(), cv.size() * sizeof(CvtProblem));
    launch_to_f32(s, d, (int)cv.size());
    SPD_HIP(hipStreamSynchronize(s));
    H.stage.reset();
    cv.clear();
  };
  // one allocation per block row, blocks in list order (as the FP64 rows)
  auto row = [&](int64_t e0, int64_t e1, auto keep, auto rows, auto cols, std::vector<double*>& src,
                 std::vector<float*>& dst) {
    size_t total = 0;
    for (int64_t e = e0; e < e1; ++e)
      if (keep(e) && src[e]) total += (size_t)rows(e) * cols(e);
    if (total == 0) return;
    float* base = H.arena32.get_n<float>(total);
    for (int64_t e = e0; e < e1; ++e) {
      if (!keep(e) || !src[e]) continue;
      const int64_t n = (int64_t)rows(e) * cols(e);
      dst[e] = base;
      cv.push_back({src[e], base, n});
      base += n;
      if (cv.size() >= 4096) flush();
    }
  };
  for (int v = 1; v < T.nnodes; ++v)
    row(T.coup_ptr[v], T.coup_ptr[v + 1], [&](int64_t e) { return T.coup_idx[e] > v; },
        [&](int64_t) { return H.coup_ld(v); }, [&](int64_t e) { return H.k[T.coup_idx[e]]; }, H.Bh, H.Bh32);
  for (int v = T.first_at(1); v < T.first_at(1) + T.count_at(1); ++v)
    row(T.near_ptr[v], T.near_ptr[v + 1], [&](int64_t e) { return T.near_idx[e] >= v; },
        [&](int64_t) { return std::max(H.near_ld(v), 16); },
        [&](int64_t e) { return (int)T.size(T.near_idx[e]); }, H.nearA, H.nearA32);
  flush();
}

// f32: the near and coupling launches read the FP32 block copies; the plan
// then shares the input, output and skeleton-space buffers of the FP64 plan
// for the same column count (which must exist).
static void build_plan(H2Model& H, int m, bool f32 = false) {
  auto pl = std::make_unique<H2Model::MatvecPlan>();
  pl->ncols = m;
  const TreeHost& T = H.T;
  const int L = T.L;
  const int64_t N = T.N;
  hipStream_t s = H.s;
  Arena& a = pl->arena;
  if (f32) {
    SPD_REQUIRE(m <= 16 && H.plan && H.plan->ncols == m, SPD_E_INVALID,
                "the FP32 product needs at most 16 columns");
    make_f32_blocks(H);
    pl->xt = H.plan->xt;
    pl->yt = H.plan->yt;
    pl->xh = H.plan->xh;
    pl->yh = H.plan->yh;
  } else {
    pl->xt = a.get_n<double>((size_t)N * m);
    pl->yt = a.get_n<double>((size_t)N * m);
    pl->xh = a.get_n<double>((size_t)std::max<int64_t>(H.stack_rows, 1) * m);
    pl->yh = a.get_n<double>((size_t)std::max<int64_t>(H.stack_rows, 1) * m);
  }
  // A operand of a symmetric-pair term: the FP64 block or its FP32 copy
  auto blk = [&](const std::vector<double*>& d, const std::vector<float*>& f, int64_t e) {
    return f32 ? (const double*)f[e] : (const double*)d[e];
  };
  Recorder& rec = pl->rec;
  const int lf = T.first_at(1), lc = T.count_at(1);
  // With at most 4 columns the interpolation W_v = Pi_v [I; E_v^T] is applied
  // in that form: the identity rows are a gather (upward) or scatter
  // (downward) of the vector, and only E_v is streamed, as dot products down
  // the columns of E_v^T (upward) or E_v (downward).
  const bool eform = m <= 4;
  // with up to 16 columns the coupling and near-field blocks are read once
  // for both products of a symmetric pair (k_symv up to 4 columns, the MFMA
  // form k_symm16 above)
  const bool sym = m <= 16;
  if (L > 1) {
    // upward: x-hat_v = W_v^T x_v (leaf) or W_v^T [x-hat_c1; x-hat_c2]
    //         = x[Pi_v(0:k)] + E_v x[Pi_v(k:cand)]
    for (int lev = 1; lev < L; ++lev) {
      GemmBatch g(eform ? 1 : 0, 0);  // E form: dot products down the columns of E^T
      for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
        if (H.k[v] == 0) continue;
        const double* xin = lev == 1 ? pl->xt + T.start[v] : pl->xh + H.par_off[v] * m;
        const int ldin = lev == 1 ? (int)N : H.cand[v];
        if (eform) {
          const int k = H.k[v], c = H.cand[v];
          g.add_indexed(H.hat(pl->xh, v, m), k, m, H.hat_ld(v), 0.0, nullptr, xin, H.piv_d[v], ldin);
          if (c > k) g.term_gathered(H.ET[v], c - k, xin, ldin, H.piv_d[v] + k, c - k);
        } else {
          g.add(H.hat(pl->xh, v, m), H.k[v], m, H.hat_ld(v));
          g.term(H.WT[v], H.k[v], xin, ldin, H.cand[v]);
        }
      }
      const size_t first = rec.recs.size();
      rec.gemm(a, s, g);
      rec.tag_from(first, 100 + lev);
    }
    // coupling: y-hat_v = sum_j B_vj x-hat_j.  With at most 16 columns the
    // blocks B_vj with j > v are read once for both B_vj x-hat_j and
    // B_jv x-hat_v = B_vj^T x-hat_v (B^{H2} is symmetric: B_jv = B_vj^T).
    if (sym) {
      std::vector<SymRow> rows;
      std::vector<int> row_of(T.nnodes, -1);
      for (int v = 1; v < T.nnodes; ++v) {
        if (H.k[v] == 0) continue;
        row_of[v] = (int)rows.size();
        rows.push_back(SymRow{H.hat(pl->yh, v, m), H.hat_ld(v), H.hat(pl->xh, v, m), H.hat_ld(v), H.k[v], {}});
      }
      for (int v = 1; v < T.nnodes; ++v) {
        if (H.k[v] == 0) continue;
        SymRow& R = rows[row_of[v]];
        for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
          const int j = T.coup_idx[e];
          if (H.k[j] == 0 || j < v) continue;
          R.terms.push_back({blk(H.Bh, H.Bh32, e), H.coup_ld(v), H.hat(pl->xh, j, m), H.hat_ld(j), H.k[j],
                             row_of[j]});
        }
      }
      const size_t first = rec.recs.size();
      rec.symv(a, s, rows, m, 0.0, f32);
      rec.tag_from(first, 200);
    } else {
      GemmBatch g(0, 0);
      for (int v = 1; v < T.nnodes; ++v) {
        if (H.k[v] == 0) continue;
        g.add(H.hat(pl->yh, v, m), H.k[v], m, H.hat_ld(v));
        for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
          const int j = T.coup_idx[e];
          if (H.k[j] == 0) continue;
          g.term(H.Bh[e], H.coup_ld(v), H.hat(pl->xh, j, m), H.hat_ld(j), H.k[j]);
        }
      }
      const size_t first = rec.recs.size();
      rec.gemm(a, s, g);
      rec.tag_from(first, 200);
    }
    // downward: [y-hat_c1; y-hat_c2] += W_v y-hat_v; with the E form the
    // skeleton rows Pi_v(0:k) receive y-hat_v and the others E_v^T y-hat_v.
    // The E form continues to the leaves (level 1), where W_v y-hat_v is the
    // far-field part of y_v; the leaf pass then adds the near field.
    for (int lev = L - 1; lev >= (eform ? 1 : 2); --lev) {
      GemmBatch g(eform ? 1 : 0, 0);  // E form: dot products down the columns of E
      for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
        const bool leaf = lev == 1;
        double* yout = leaf ? pl->yt + T.start[v] : pl->yh + H.par_off[v] * m;
        const int ldout = leaf ? (int)N : H.cand[v];
        const double beta = leaf ? 0.0 : 1.0;
        const int k = H.k[v], c = H.cand[v];
        if (eform) {
          if (k == 0) {
            if (leaf) g.add((double*)yout, (int)T.size(v), m, ldout);  // no far field: zero rows
            continue;
          }
          g.add_indexed(yout, k, m, ldout, beta, H.piv_d[v], H.hat(pl->yh, v, m), nullptr, H.hat_ld(v));
          if (c > k) {
            g.add_indexed(yout, c - k, m, ldout, beta, H.piv_d[v] + k, nullptr, nullptr, 0);
            g.term(H.E[v], k, H.hat(pl->yh, v, m), H.hat_ld(v), k);
          }
        } else {
          if (k == 0 || c == 0) continue;
          g.add(yout, c, m, ldout, 1.0);
          g.term(H.W[v], c, H.hat(pl->yh, v, m), H.hat_ld(v), k);
        }
      }
      const size_t first = rec.recs.size();
      rec.gemm(a, s, g);
      rec.tag_from(first, 300 + lev);
    }
  }
  if (eform && L == 1) {  // a single leaf: no far field
    GemmBatch g(0, 0);
    g.add(pl->yt, (int)N, m, (int)N);
    rec.gemm(a, s, g);
  }
  // leaves: y_v = W_v y-hat_v + sum_{j near v} A_vj x_j.  With at most 4
  // columns the near blocks A_vj with j > v also give A_jv x_v = A_vj^T x_v.
  if (eform) {
    // the far-field part of y is already in place (downward pass at level 1)
    std::vector<SymRow> rows;
    for (int v = lf; v < lf + lc; ++v)
      rows.push_back(SymRow{pl->yt + T.start[v], (int)N, pl->xt + T.start[v], (int)N, (int)T.size(v), {}});
    for (int v = lf; v < lf + lc; ++v) {
      SymRow& R = rows[v - lf];
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        if (j < v) continue;
        R.terms.push_back({blk(H.nearA, H.nearA32, e), std::max(H.near_ld(v), 16), pl->xt + T.start[j],
                           (int)N, (int)T.size(j), j == v ? -1 : j - lf});
      }
    }
    Recorder near;
    near.symv(a, s, rows, m, 1.0, f32, near_split(m));
    near.tag_from(0, 400);
    // the product launch goes to the side stream, the block sum into y after the join
    pl->side.recs.push_back(near.recs[0]);
    pl->side.recs[0].cap = kNearCap;
    pl->tail.recs.assign(near.recs.begin() + 1, near.recs.end());
    if (!H.side_s) {
      SPD_HIP(hipStreamCreateWithFlags(&H.side_s, hipStreamNonBlocking));
      SPD_HIP(hipEventCreateWithFlags(&H.ev_fork, hipEventDisableTiming));
      SPD_HIP(hipEventCreateWithFlags(&H.ev_join, hipEventDisableTiming));
    }
  } else if (sym) {
    // far-field part of y at the leaves, y_v = W_v y-hat_v, then the near
    // field by symmetric pairs added onto it
    GemmBatch g(0, 0);
    for (int v = lf; v < lf + lc; ++v) {
      g.add(pl->yt + T.start[v], (int)T.size(v), m, (int)N);
      if (L > 1 && H.k[v] > 0) g.term(H.W[v], H.cand[v], H.hat(pl->yh, v, m), H.hat_ld(v), H.k[v]);
    }
    size_t first = rec.recs.size();
    rec.gemm(a, s, g);
    std::vector<SymRow> rows;
    for (int v = lf; v < lf + lc; ++v)
      rows.push_back(SymRow{pl->yt + T.start[v], (int)N, pl->xt + T.start[v], (int)N, (int)T.size(v), {}});
    for (int v = lf; v < lf + lc; ++v) {
      SymRow& R = rows[v - lf];
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        if (j < v) continue;
        R.terms.push_back({blk(H.nearA, H.nearA32, e), std::max(H.near_ld(v), 16), pl->xt + T.start[j], (int)N,
                           (int)T.size(j), j == v ? -1 : j - lf});
      }
    }
    rec.symv(a, s, rows, m, 1.0, f32, near_split(m));
    rec.tag_from(first, 400);
  } else {
    GemmBatch g(0, 0);
    for (int v = lf; v < lf + lc; ++v) {
      g.add(pl->yt + T.start[v], (int)T.size(v), m, (int)N);
      if (L > 1 && H.k[v] > 0) g.term(H.W[v], H.cand[v], H.hat(pl->yh, v, m), H.hat_ld(v), H.k[v]);
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        g.term(H.nearA[e], std::max(H.near_ld(v), 16), pl->xt + T.start[j], (int)N, (int)T.size(j));
      }
    }
    const size_t first = rec.recs.size();
    rec.gemm(a, s, g);
    rec.tag_from(first, 400);
  }
  SPD_HIP(hipStreamSynchronize(s));
  if (f32) H.plan32 = std::move(pl);
  else H.plan = std::move(pl);
}

void h2_matvec_tree(H2Model& H, const double* x, double* y, int m, bool f32) {
  if (!H.plan || H.plan->ncols != m) {
    H.plan32.reset();
    H.plan.reset();
    build_plan(H, m);
  }
  if (f32 && (!H.plan32 || H.plan32->ncols != m)) build_plan(H, m, true);
  const int64_t N = H.T.N;
  auto& pl = *H.plan;
  if (x != pl.xt)
    SPD_HIP(hipMemcpyAsync(pl.xt, x, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, H.s));
  replay_plan(H, f32 ? *H.plan32 : pl);
  if (y != pl.yt)
    SPD_HIP(hipMemcpyAsync(y, pl.yt, (size_t)N * m * sizeof(double), hipMemcpyDeviceToDevice, H.s));
}

double* h2_plan_x(H2Model& H, int m) {
  if (!H.plan || H.plan->ncols != m) {
    H.plan32.reset();
    H.plan.reset();
    build_plan(H, m);
  }
  return H.plan->xt;
}
double* h2_plan_y(H2Model& H, int m) {
  h2_plan_x(H, m);
  return H.plan->yt;
}
void h2_plan_run(H2Model& H) { replay_plan(H, *H.plan); }
void h2_plan_prepare32(H2Model& H, int m) {
  h2_plan_x(H, m);
  if (!H.plan32 || H.plan32->ncols != m) build_plan(H, m, true);
}
void h2_plan_run32(H2Model& H, int m) {
  h2_plan_prepare32(H, m);
  replay_plan(H, *H.plan32);
}

// every recorded launch of the product, in stream order
static std::vector<LaunchRec> all_launches(const H2Model::MatvecPlan& pl) {
  std::vector<LaunchRec> v(pl.rec.recs);
  v.insert(v.end(), pl.side.recs.begin(), pl.side.recs.end());
  v.insert(v.end(), pl.tail.recs.begin(), pl.tail.recs.end());
  return v;
}

// the launches of the near-field (leaf) pass, on H.s
void h2_plan_run_last(H2Model& H) {
  Recorder one;
  for (const LaunchRec& r : all_launches(*H.plan))
    if (r.tag == 400) one.recs.push_back(r);
  one.replay(H.s);
}

// Algorithmic bytes of the leaf pass: the sum over its recorded launches
// (every near block read, the leaf bases and skeleton-space inputs, x and y).
H2Model::NearStats h2_near_stats(H2Model& H, int m) {
  h2_plan_x(H, m);
  double b = 0;
  for (const LaunchRec& r : all_launches(*H.plan))
    if (r.tag == 400) b += r.bytes;
  H2Model::NearStats st;
  st.bytes = b;
  return st;
}

// Time every launch of the product separately (HIP events on the product's
// stream); returns the number of launches written.
int h2_time_launches(H2Model& H, int m, int reps, double* ms, double* bytes, int* tags, int cap) {
  h2_plan_x(H, m);
  const std::vector<LaunchRec> recs = all_launches(*H.plan);
  hipEvent_t e0, e1;
  SPD_HIP(hipEventCreate(&e0));
  SPD_HIP(hipEventCreate(&e1));
  const int n = std::min<int>((int)recs.size(), cap);
  for (int i = 0; i < n; ++i) {
    Recorder one;
    one.recs.push_back(recs[i]);
    one.replay(H.s);
    SPD_HIP(hipEventRecord(e0, H.s));
    for (int r = 0; r < reps; ++r) one.replay(H.s);
    SPD_HIP(hipEventRecord(e1, H.s));
    SPD_HIP(hipEventSynchronize(e1));
    float t = 0;
    SPD_HIP(hipEventElapsedTime(&t, e0, e1));
    ms[i] = t / reps;
    bytes[i] = recs[i].bytes;
    if (tags) tags[i] = recs[i].tag;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return n;
}

}  // namespace spd
