// Accelerated SPD HSS construction (Algorithm 5.3) on the device.
//
// Level by level from the leaves, every node is scaled by its symmetric
// factor (leaf: Cholesky S_i of A_ii; nonleaf: Cholesky F_i of I + bold B_ii,
// eqs. Aii0/Si0/Si with a Cholesky factor in place of the square root), its
// sample Lambda_{ii^c} Omega_{i^c} is compressed by a column-pivoted QR
// (Algorithm 5.1) and the Type-1/Type-3 couplings of the level are formed
// (eqs. Mijk, type3_Mij), with Phi_i U_i^H2 by its nested recursion and
// R_i = F_i V-bar_i (eq. Rik).
//
// Sampling.  Algorithm 5.3 computes Y^(k) = (A - diag_k(A)) Omega for every
// nonroot level (eq. Yk) and pushes each through Algorithm 5.2.  Here the same
// quantities Phi-projected are formed without materialising the far-field part
// of any Y^(k): a far block U_p B_pq U_q^T contributes Phi_a U_p ... which, by
// the nested recursion of Phi_i U_i^H2 (Section 5.2.2, Case 1), equals
// (Phi U)_p B_pq x-hat_q added at the level of p, or (Phi U)_c times the
// downward-accumulated skeleton-space vector for blocks above the target
// level.  Near blocks are summed once per lowest-common-ancestor level
// ("class"), since a block enters Y^(k) exactly when its class exceeds k.
// The result equals Algorithm 5.2's output up to rounding order.
#include "model.h"

#include <algorithm>
#include <map>

namespace spd {

namespace {

struct Ctx {
  H2Model& H;
  HSSModel& M;
  Factors& F;
  const TreeHost& T;
  hipStream_t s;
  Stage st;
  int S;  // sample columns
  Ctx(H2Model& h, HSSModel& m, Factors& f, hipStream_t str)
      : H(h), M(m), F(f), T(h.T), s(str), S(0) {}
  void sync() {
    SPD_HIP(hipStreamSynchronize(s));
    st.reset();
  }
};

// HSS coupling block of a pair at one level (near or coupling entry).
const double* pair_block(const Ctx& c, int a, int b) {
  const int64_t e = c.T.near_pos(a, b);
  if (e >= 0) return c.M.Bn[e];
  const int64_t f = c.T.coup_pos(a, b);
  SPD_REQUIRE(f >= 0, SPD_E_INVALID, "internal: missing child pair");
  return c.M.Bc[f];
}

void check_fail(Ctx& c, int* d_fail, const std::vector<int>& nodes, const char* what) {
  std::vector<int> fl(nodes.size());
  if (nodes.empty()) return;
  SPD_HIP(hipMemcpyAsync(fl.data(), d_fail, fl.size() * sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  for (size_t i = 0; i < fl.size(); ++i)
    if (fl[i])
      throw Error(SPD_E_NOT_SPD, std::string(what) + " not positive definite at node " +
                                     std::to_string(nodes[i]) + " (level " +
                                     std::to_string(c.T.level(nodes[i])) + ")");
}

// Type-1 and Type-3 HSS couplings of one level (for pairs i < j; B_ji = B_ij^T).
void couplings(Ctx& c, int lev, Arena& out) {
  const TreeHost& T = c.T;
  const auto& r = c.F.r;
  const auto& hk = c.H.k;
  const int f0 = T.first_at(lev), cnt = T.count_at(lev);
  struct PairJob { int i, j; int64_t e; bool near; };
  std::vector<PairJob> jobs;
  for (int i = f0; i < f0 + cnt; ++i) {
    for (int64_t e = T.near_ptr[i]; e < T.near_ptr[i + 1]; ++e) {
      const int j = T.near_idx[e];
      if (j == i) continue;
      c.M.Bn[e] = out.get_n<double>((size_t)std::max(r[i] * r[j], 1));
      if (i < j) jobs.push_back({i, j, e, true});
    }
    for (int64_t e = T.coup_ptr[i]; e < T.coup_ptr[i + 1]; ++e) {
      const int j = T.coup_idx[e];
      c.M.Bc[e] = out.get_n<double>((size_t)std::max(r[i] * r[j], 1));
      if (i < j) jobs.push_back({i, j, e, false});
    }
  }
  // process in chunks bounding the temporaries
  size_t a = 0;
  while (a < jobs.size()) {
    size_t b = a, bytes = 0;
    while (b < jobs.size()) {
      const PairJob& p = jobs[b];
      const size_t sz = p.near ? (size_t)c.F.rho[p.i] * (c.F.rho[p.j] + r[p.j]) * 8
                               : (size_t)hk[p.i] * r[p.j] * 8;
      if (b > a && bytes + sz > (size_t(1) << 30)) break;
      bytes += sz;
      ++b;
    }
    Arena tmp;
    BlockBatch asmb;     // bold B_ij assembly (nonleaf near pairs)
    GemmBatch g1(0, 0);  // M = A_ij Z_j  |  M = bold B_ij Z_j  |  M = B^H2 (PhiU_j)^T
    GemmBatch g1t(0, 1);
    GemmBatch g2(1, 0);  // B_ij = Z_i^T M
    GemmBatch g2n(0, 0); // B_ij = PhiU_i M
    BlockBatch zero;
    for (size_t q = a; q < b; ++q) {
      const PairJob& p = jobs[q];
      const int i = p.i, j = p.j;
      double* Bij = p.near ? c.M.Bn[p.e] : c.M.Bc[p.e];
      if (r[i] == 0 || r[j] == 0) continue;
      if (p.near) {
        const int ri = c.F.rho[i], rj = c.F.rho[j];
        double* Mt = tmp.get_n<double>((size_t)ri * r[j]);
        const double* Aij;
        int ldA = ri;
        if (lev == 1) {
          Aij = c.H.nearA[p.e];
          ldA = std::max(c.H.near_ld(i), 16);
        } else {
          double* Bb = tmp.get_n<double>((size_t)ri * rj);
          const int ci[2] = {2 * i + 1, 2 * i + 2}, cj[2] = {2 * j + 1, 2 * j + 2};
          int ro = 0;
          for (int x = 0; x < 2; ++x) {
            int co = 0;
            for (int y = 0; y < 2; ++y) {
              const int ra = r[ci[x]], rb = r[cj[y]];
              if (ra > 0 && rb > 0) {
                asmb.add(Bb + ro + (size_t)co * ri, ra, rb, ri);
                asmb.term(pair_block(c, ci[x], cj[y]), ra);
              }
              co += rb;
            }
            ro += r[ci[x]];
          }
          Aij = Bb;
        }
        g1.add(Mt, ri, r[j], ri);
        g1.term(Aij, ldA, c.M.Z[j], rj, rj);
        g2.add(Bij, r[i], r[j], r[i]);
        g2.term(c.M.Z[i], ri, Mt, ri, ri);
      } else {
        const int ki = hk[i], kj = hk[j];
        if (ki == 0 || kj == 0) {
          zero.add(Bij, r[i], r[j], r[i]);
          continue;
        }
        double* Mt = tmp.get_n<double>((size_t)ki * r[j]);
        g1t.add(Mt, ki, r[j], ki);
        g1t.term(c.H.Bh[p.e], c.H.coup_ld(i), c.M.PhiU[j], r[j], kj);
        g2n.add(Bij, r[i], r[j], r[i]);
        g2n.term(c.M.PhiU[i], r[i], Mt, ki, ki);
      }
    }
    asmb.run(c.s, c.st);
    zero.run(c.s, c.st);
    g1.run(c.s, c.st);
    g1t.run(c.s, c.st);
    g2.run(c.s, c.st);
    g2n.run(c.s, c.st);
    c.sync();
    a = b;
  }
  // B_ji = B_ij^T
  BlockBatch tr;
  for (const PairJob& p : jobs) {
    const int i = p.i, j = p.j;
    if (r[i] == 0 || r[j] == 0) continue;
    const double* Bij = p.near ? c.M.Bn[p.e] : c.M.Bc[p.e];
    double* Bji = p.near ? c.M.Bn[T.near_pos(j, i)] : c.M.Bc[T.coup_pos(j, i)];
    tr.add(Bji, r[j], r[i], r[j]);
    tr.term(Bij, r[i], 1.0, 1);
  }
  tr.run(c.s, c.st);
  c.sync();
}

}  // namespace

void spdhss_build_impl(H2Model& H, const spd_hss_opts& o, HSSModel& M, hipStream_t s) {
  const TreeHost& T = H.T;
  const int L = T.L, nn = T.nnodes;
  const int64_t N = T.N;
  const int S = o.max_rank + o.oversample;
  SPD_REQUIRE(o.max_rank >= 0 && o.oversample >= 0 && S >= 1, SPD_E_INVALID, "bad rank options");
  SPD_REQUIRE(S <= 256, SPD_E_INVALID, "max_rank + oversample must not exceed 256");
  SPD_REQUIRE(o.tol >= 0.0, SPD_E_INVALID, "negative tolerance");
  M.opts = o;
  M.opts.omega = nullptr;
  M.s = S;
  M.f = std::make_shared<Factors>();
  Factors& F = *M.f;
  F.T = T;
  Ctx c(H, M, F, s);
  c.S = S;
  Arena& out = M.arena;
  const double t_begin = now_seconds();
  F.perm_d = F.arena.get_n<int64_t>(N);
  SPD_HIP(hipMemcpyAsync(F.perm_d, H.perm_d, N * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  F.r.assign(nn, 0);
  F.rho.assign(nn, 0);
  F.S.assign(nn, nullptr);
  F.V.assign(nn, nullptr);
  F.F.assign(nn, nullptr);
  M.Z.assign(nn, nullptr);
  M.R.assign(nn, nullptr);
  M.PhiU.assign(nn, nullptr);
  M.piv.assign(nn, nullptr);
  M.Bn.assign(T.near_idx.size(), nullptr);
  M.Bc.assign(T.coup_idx.size(), nullptr);
  M.hk = H.k;
  M.lists = T;
  const auto& hk = H.k;
  const int lf = T.first_at(1), lc = T.count_at(1);
  Arena tmp;
  int* d_fail = tmp.get_n<int>(nn + 2);
  int* d_rank = tmp.get_n<int>(nn);

  // ---- Omega in tree order
  double* Om = tmp.get_n<double>((size_t)N * S);
  if (o.omega)
    launch_gather_rows(s, o.omega, N, Om, N, H.perm_d, N, S);
  else
    launch_gaussian_fill(s, Om, N, S, N, H.perm_d, o.seed);

  if (L == 1) {
    // a single leaf: the HSS matrix is the dense block itself
    F.rho[0] = (int)N;
    F.S[0] = F.arena.get_n<double>((size_t)N * N);
    BlockBatch cp;
    cp.add(F.S[0], (int)N, (int)N, (int)N);
    cp.term(H.nearA[T.near_ptr[0]], std::max(H.near_ld(0), 16));
    cp.run(s, c.st);
    std::vector<CholProblem> ch{{F.S[0], (int)N, (int)N}};
    launch_fill(s, (double*)d_fail, 0.0, (nn + 1) / 2);
    auto* dch = (const CholProblem*)c.st.push(s, ch.data(), sizeof(CholProblem));
    launch_chol(s, dch, 1, (int)N, d_fail);
    check_fail(c, d_fail, {0}, "diagonal block");
    F.root_factored = true;
    M.times[7] = now_seconds() - t_begin;
    return;
  }

  // ---- far field in skeleton space: x-hat = U^T Omega (upward)
  double* xh = tmp.get_n<double>((size_t)std::max<int64_t>(H.stack_rows, 1) * S);
  for (int lev = 1; lev < L; ++lev) {
    GemmBatch g(1, 0);
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      if (hk[v] == 0) continue;
      g.add(H.hat(xh, v, S), hk[v], S, H.hat_ld(v));
      if (lev == 1)
        g.term(H.W[v], H.cand[v], Om + T.start[v], (int)N, H.cand[v]);
      else
        g.term(H.W[v], H.cand[v], xh + H.par_off[v] * S, H.cand[v], H.cand[v]);
    }
    g.run(s, c.st);
  }
  // coupling sums per (node, class): c-hat_v^(lam) = sum_{j in coup(v), lca = lam} B_vj x-hat_j
  std::vector<std::vector<std::pair<int, double*>>> chat(nn);
  {
    GemmBatch g(0, 0);
    for (int v = 1; v < nn; ++v) {
      if (hk[v] == 0) continue;
      std::map<int, std::vector<int64_t>> cls;
      for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
        const int j = T.coup_idx[e];
        if (hk[j] == 0) continue;
        cls[T.lca_level(v, j)].push_back(e);
      }
      for (auto& kv : cls) {
        double* slot = tmp.get_n<double>((size_t)hk[v] * S);
        chat[v].push_back({kv.first, slot});
        g.add(slot, hk[v], S, hk[v]);
        for (int64_t e : kv.second) {
          const int j = T.coup_idx[e];
          g.term(H.Bh[e], H.coup_ld(v), H.hat(xh, j, S), H.hat_ld(j), hk[j]);
        }
      }
    }
    g.run(s, c.st);
  }
  // downward accumulation y-down (skeleton space), top to bottom
  double* yd = tmp.get_n<double>((size_t)std::max<int64_t>(H.stack_rows, 1) * S);
  launch_fill(s, yd, 0.0, std::max<int64_t>(H.stack_rows, 1) * S);
  for (int lev = L - 1; lev >= 1; --lev) {
    if (lev < L - 1) {
      GemmBatch g(0, 0);
      for (int p = T.first_at(lev + 1); p < T.first_at(lev + 1) + T.count_at(lev + 1); ++p) {
        if (hk[p] == 0 || H.cand[p] == 0) continue;
        g.add(yd + H.par_off[p] * S, H.cand[p], S, H.cand[p], 1.0);
        g.term(H.W[p], H.cand[p], H.hat(yd, p, S), H.hat_ld(p), hk[p]);
      }
      g.run(s, c.st);
    }
    BlockBatch bb;
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) {
      if (hk[v] == 0 || chat[v].empty()) continue;
      bb.add(H.hat(yd, v, S), hk[v], S, H.hat_ld(v), 1.0);
      for (auto& cs : chat[v]) bb.term(cs.second, hk[v]);
    }
    bb.run(s, c.st);
  }
  // near-field class sums at the leaves: N_v^(lam) = sum_{j near v, lca = lam} A_vj Omega_j
  std::vector<std::vector<std::pair<int, double*>>> nsum(nn);
  {
    GemmBatch g(0, 0);
    for (int v = lf; v < lf + lc; ++v) {
      std::map<int, std::vector<int64_t>> cls;
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        if (j == v) continue;
        cls[T.lca_level(v, j)].push_back(e);
      }
      const int nv = (int)T.size(v);
      for (auto& kv : cls) {
        double* slot = tmp.get_n<double>((size_t)std::max(nv, 1) * S);
        nsum[v].push_back({kv.first, slot});
        g.add(slot, nv, S, std::max(nv, 1));
        for (int64_t e : kv.second) {
          const int j = T.near_idx[e];
          g.term(H.nearA[e], std::max(H.near_ld(v), 16), Om + T.start[j], (int)N, (int)T.size(j));
        }
      }
    }
    g.run(s, c.st);
  }
  c.sync();
  const double t_sample = now_seconds();

  // ---- leaf level
  std::vector<int> leaves(lc);
  for (int q = 0; q < lc; ++q) leaves[q] = lf + q;
  Arena lvl_tmp;
  std::vector<double*> Psi(nn, nullptr);
  {
    BlockBatch cp, y1;
    std::vector<CholProblem> ch;
    int maxn = 0;
    for (int v : leaves) {
      const int nv = (int)T.size(v);
      maxn = std::max(maxn, nv);
      F.rho[v] = nv;
      F.S[v] = F.arena.get_n<double>((size_t)std::max(nv * nv, 1));
      cp.add(F.S[v], nv, nv, std::max(nv, 1));
      cp.term(H.nearA[T.near_pos(v, v)], std::max(H.near_ld(v), 16));
      ch.push_back({F.S[v], nv, std::max(nv, 1)});
      Psi[v] = lvl_tmp.get_n<double>((size_t)std::max(nv, 1) * S);
      y1.add(Psi[v], nv, S, std::max(nv, 1));
      for (auto& cs : nsum[v]) y1.term(cs.second, std::max(nv, 1));
    }
    cp.run(s, c.st);
    y1.run(s, c.st);
    GemmBatch far(0, 0);
    for (int v : leaves)
      if (hk[v] > 0) {
        const int nv = (int)T.size(v);
        far.add(Psi[v], nv, S, std::max(nv, 1), 1.0);
        far.term(H.W[v], H.cand[v], H.hat(yd, v, S), H.hat_ld(v), hk[v]);
      }
    far.run(s, c.st);
    launch_fill(s, (double*)d_fail, 0.0, (nn + 1) / 2);
    auto* dch = (const CholProblem*)c.st.push(s, ch.data(), ch.size() * sizeof(CholProblem));
    launch_chol(s, dch, (int)ch.size(), maxn, d_fail);
    check_fail(c, d_fail, leaves, "leaf diagonal block");
    // Psi = S^{-1} Y^(1)
    TrsmBatch tb;
    for (int v : leaves) tb.add(F.S[v], F.rho[v], Psi[v], F.rho[v], F.rho[v], S);
    tb.run(s, c.st, 0);
  }
  const double t_leaf_scale = now_seconds();

  // compress the samples of one level; returns ranks on the host
  // More than 128 samples (r_max + p > 128) exceed the register-resident
  // kernel; the global-memory kernel then factors the samples in place
  // (they are not needed afterwards) and a second launch forms Q.
  const bool glob = S > 128;
  auto compress = [&](const std::vector<int>& nodes) {
    std::vector<CpqrProblem> cq;
    Arena wk;
    int mm = 1;
    for (size_t q = 0; q < nodes.size(); ++q) {
      const int v = nodes[q];
      const int m = F.rho[v];
      const int mr = std::min(std::min(m, S), o.max_rank);
      F.V[v] = F.arena.get_n<double>((size_t)std::max(m * mr, 1));
      // the global kernel writes the whole column order (S entries)
      M.piv[v] = out.get_n<int>(std::max(glob ? S : mr, 1));
      CpqrProblem p{};
      p.A = Psi[v];
      p.Q = F.V[v];
      p.V = wk.get_n<double>((size_t)std::max(m * mr, 1));
      p.piv = M.piv[v];
      p.rank = d_rank + q;
      p.m = m;
      p.n = S;
      p.lda = std::max(m, 1);
      p.ldq = std::max(m, 1);
      p.maxrank = mr;
      p.tol = o.tol;
      if (glob) p.hbeta = wk.get_n<double>((size_t)std::max(mr, 1));
      cq.push_back(p);
      mm = std::max(mm, m);
      if (glob) SPD_REQUIRE(m <= 2048, SPD_E_INVALID, "basis rows exceed 2048");
      else SPD_REQUIRE(cpqr_reg_fits(m, S), SPD_E_INVALID, "basis rows exceed 512");
    }
    auto* d = (const CpqrProblem*)c.st.push(s, cq.data(), cq.size() * sizeof(CpqrProblem));
    if (glob) {
      launch_cpqr_glob(s, d, (int)cq.size(), mm, S);
      launch_cpqr_formq(s, d, (int)cq.size());
    } else {
      launch_cpqr_reg(s, d, (int)cq.size(), mm, S);
    }
    std::vector<int> rk(nodes.size());
    SPD_HIP(hipMemcpyAsync(rk.data(), d_rank, rk.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    c.sync();
    for (size_t q = 0; q < nodes.size(); ++q) F.r[nodes[q]] = rk[q];
  };
  // Z = op(factor)^{-T} V
  auto make_Z = [&](const std::vector<int>& nodes, bool leaf) {
    BlockBatch cp;
    TrsmBatch tb;
    for (int v : nodes) {
      const int m = F.rho[v], rv = F.r[v];
      M.Z[v] = out.get_n<double>((size_t)std::max(m * rv, 1));
      if (rv == 0) continue;
      cp.add(M.Z[v], m, rv, m);
      cp.term(F.V[v], m);
      tb.add(leaf ? F.S[v] : F.F[v], m, M.Z[v], m, m, rv);
    }
    cp.run(s, c.st);
    tb.run(s, c.st, 1);
  };

  compress(leaves);
  make_Z(leaves, true);
  {
    GemmBatch g(1, 0);
    for (int v : leaves) {
      M.PhiU[v] = out.get_n<double>((size_t)std::max(F.r[v] * hk[v], 1));
      if (F.r[v] == 0 || hk[v] == 0) continue;
      g.add(M.PhiU[v], F.r[v], hk[v], F.r[v]);
      g.term(M.Z[v], F.rho[v], H.W[v], H.cand[v], F.rho[v]);
    }
    g.run(s, c.st);
  }
  c.sync();
  const double t_leaf_comp = now_seconds();
  couplings(c, 1, out);

  // stacked parents' buffers of T-blocks for the targets above this level
  F.par_off.assign(nn, 0);
  auto stack_for = [&](int lev, Arena& ar, int nt) {
    // parents at lev+1; returns per-parent pointers (rho_p x S*nt)
    std::vector<double*> G(nn, nullptr);
    for (int p = T.first_at(lev + 1); p < T.first_at(lev + 1) + T.count_at(lev + 1); ++p) {
      const int rp = F.r[2 * p + 1] + F.r[2 * p + 2];
      G[p] = ar.get_n<double>((size_t)std::max(rp, 1) * S * std::max(nt, 1));
    }
    return G;
  };
  auto rowoff = [&](int v) { return (v % 2 == 0) ? F.r[v - 1] : 0; };
  auto rho_par = [&](int v) { const int p = (v - 1) / 2; return F.r[2 * p + 1] + F.r[2 * p + 2]; };

  // T-blocks of the leaves for targets 2..L-1
  std::unique_ptr<Arena> g_ar(new Arena());
  std::vector<double*> Gst;
  int nt = L - 2;
  if (nt > 0) {
    Gst = stack_for(1, *g_ar, nt);
    Arena pt;
    GemmBatch gz(1, 0), gp(0, 0);
    BlockBatch acc;
    for (int v : leaves) {
      const int rv = F.r[v], nv = F.rho[v];
      std::map<int, double*> P;
      if (rv == 0) continue;
      for (auto& cs : nsum[v]) {
        if (cs.first < 3) continue;
        double*& slot = P[cs.first];
        if (!slot) slot = pt.get_n<double>((size_t)rv * S);
        gz.add(slot, rv, S, rv);
        gz.term(M.Z[v], nv, cs.second, nv, nv);
      }
      for (auto& cs : chat[v]) {
        if (cs.first < 3 || hk[v] == 0) continue;
        double*& slot = P[cs.first];
        const bool fresh = !slot;
        if (!slot) slot = pt.get_n<double>((size_t)rv * S);
        gp.add(slot, rv, S, rv, fresh ? 0.0 : 1.0);
        gp.term(M.PhiU[v], rv, cs.second, hk[v], hk[v]);
      }
      const int p = (v - 1) / 2, rp = rho_par(v);
      for (int k = 2; k <= L - 1; ++k) {
        acc.add(Gst[p] + rowoff(v) + (size_t)(k - 2) * S * rp, rv, S, rp);
        for (auto& kv : P)
          if (kv.first > k) acc.term(kv.second, rv);
      }
    }
    gz.run(s, c.st);
    gp.run(s, c.st);
    acc.run(s, c.st);
    c.sync();
  }
  const double t_leaf = now_seconds();

  // ---- levels 2 .. L-1
  for (int lev = 2; lev <= L - 1; ++lev) {
    lvl_tmp.release();
    std::vector<int> nodes;
    for (int v = T.first_at(lev); v < T.first_at(lev) + T.count_at(lev); ++v) nodes.push_back(v);
    // I + bold B_ii and its Cholesky factor
    BlockBatch as;
    std::vector<CholProblem> ch;
    int maxr = 1;
    for (int v : nodes) {
      const int c1 = 2 * v + 1, c2 = 2 * v + 2, r1 = F.r[c1], r2 = F.r[c2], rv = r1 + r2;
      F.rho[v] = rv;
      maxr = std::max(maxr, rv);
      F.F[v] = F.arena.get_n<double>((size_t)std::max(rv * rv, 1));
      if (rv == 0) continue;
      if (r1 > 0) as.add(F.F[v], r1, r1, rv, 0.0, 1);
      if (r2 > 0) as.add(F.F[v] + r1 + (size_t)r1 * rv, r2, r2, rv, 0.0, 1);
      if (r1 > 0 && r2 > 0) {
        as.add(F.F[v] + (size_t)r1 * rv, r1, r2, rv);
        as.term(pair_block(c, c1, c2), r1);
        as.add(F.F[v] + r1, r2, r1, rv);
        as.term(pair_block(c, c2, c1), r2);
      }
      ch.push_back({F.F[v], rv, rv});
    }
    as.run(s, c.st);
    launch_fill(s, (double*)d_fail, 0.0, (nn + 1) / 2);
    std::vector<int> chn;
    for (int v : nodes) if (F.rho[v] > 0) chn.push_back(v);
    if (!ch.empty()) {
      auto* dch = (const CholProblem*)c.st.push(s, ch.data(), ch.size() * sizeof(CholProblem));
      launch_chol(s, dch, (int)ch.size(), maxr, d_fail);
    }
    check_fail(c, d_fail, chn, "I + B_ii");
    // DW_v = diag(PhiU_c1, PhiU_c2) W_v ; Psi_v = F^{-1} (G_v[:, 0:S] + DW_v y-down_v)
    std::vector<double*> DW(nn, nullptr);
    {
      GemmBatch g(0, 0);
      BlockBatch cp;
      for (int v : nodes) {
        const int c1 = 2 * v + 1, c2 = 2 * v + 2, r1 = F.r[c1], r2 = F.r[c2], rv = F.rho[v];
        DW[v] = lvl_tmp.get_n<double>((size_t)std::max(rv * hk[v], 1));
        Psi[v] = lvl_tmp.get_n<double>((size_t)std::max(rv, 1) * S);
        if (rv == 0) continue;
        if (hk[v] > 0) {
          if (r1 > 0 && hk[c1] > 0) {
            g.add(DW[v], r1, hk[v], rv);
            g.term(M.PhiU[c1], r1, H.W[v], H.cand[v], hk[c1]);
          } else if (r1 > 0) {
            cp.add(DW[v], r1, hk[v], rv);
          }
          if (r2 > 0 && hk[c2] > 0) {
            g.add(DW[v] + r1, r2, hk[v], rv);
            g.term(M.PhiU[c2], r2, H.W[v] + hk[c1], H.cand[v], hk[c2]);
          } else if (r2 > 0) {
            cp.add(DW[v] + r1, r2, hk[v], rv);
          }
        }
        cp.add(Psi[v], rv, S, rv);
        cp.term(Gst[v], rv);
      }
      cp.run(s, c.st);
      g.run(s, c.st);
      GemmBatch g2(0, 0);
      for (int v : nodes) {
        const int rv = F.rho[v];
        if (rv == 0 || hk[v] == 0) continue;
        g2.add(Psi[v], rv, S, rv, 1.0);
        g2.term(DW[v], rv, H.hat(yd, v, S), H.hat_ld(v), hk[v]);
      }
      g2.run(s, c.st);
      TrsmBatch tb;
      for (int v : nodes) tb.add(F.F[v], F.rho[v], Psi[v], F.rho[v], F.rho[v], S);
      tb.run(s, c.st, 0);
    }
    std::vector<int> live;
    for (int v : nodes) if (F.rho[v] > 0) live.push_back(v);
    for (int v : nodes)
      if (F.rho[v] == 0) {
        F.r[v] = 0;
        F.V[v] = F.arena.get_n<double>(1);
        M.piv[v] = out.get_n<int>(1);
      }
    if (!live.empty()) compress(live);
    make_Z(nodes, false);
    {
      GemmBatch gphi(1, 0), gr(0, 0);
      for (int v : nodes) {
        const int rv = F.r[v], m = F.rho[v];
        M.PhiU[v] = out.get_n<double>((size_t)std::max(rv * hk[v], 1));
        M.R[v] = out.get_n<double>((size_t)std::max(m * rv, 1));
        if (rv == 0) continue;
        if (hk[v] > 0) {
          gphi.add(M.PhiU[v], rv, hk[v], rv);
          gphi.term(M.Z[v], m, DW[v], m, m);
        }
        gr.add(M.R[v], m, rv, m);
        gr.term(F.F[v], m, F.V[v], m, m);
      }
      gphi.run(s, c.st);
      gr.run(s, c.st);
    }
    c.sync();
    couplings(c, lev, out);
    // T-blocks for the targets above this level
    const int ntn = L - 1 - lev;
    if (ntn > 0) {
      std::unique_ptr<Arena> nar(new Arena());
      std::vector<double*> Gn = stack_for(lev, *nar, ntn);
      Arena pt;
      GemmBatch gz(1, 0), gp(0, 0);
      BlockBatch acc;
      for (int v : nodes) {
        const int rv = F.r[v], m = F.rho[v];
        if (rv == 0) continue;
        const int p = (v - 1) / 2, rp = rho_par(v);
        // propagated part: Z-bar^T G_v[:, S:]
        gz.add(Gn[p] + rowoff(v), rv, S * ntn, rp);
        gz.term(M.Z[v], m, Gst[v] + (size_t)S * m, m, m);
        std::map<int, double*> P;
        for (auto& cs : chat[v]) {
          if (cs.first < lev + 2 || hk[v] == 0) continue;
          double* slot = pt.get_n<double>((size_t)rv * S);
          P[cs.first] = slot;
          gp.add(slot, rv, S, rv);
          gp.term(M.PhiU[v], rv, cs.second, hk[v], hk[v]);
        }
        for (int k = lev + 1; k <= L - 1; ++k) {
          bool any = false;
          for (auto& kv : P) any |= kv.first > k;
          if (!any) continue;
          acc.add(Gn[p] + rowoff(v) + (size_t)(k - lev - 1) * S * rp, rv, S, rp, 1.0);
          for (auto& kv : P)
            if (kv.first > k) acc.term(kv.second, rv);
        }
      }
      gz.run(s, c.st);
      gp.run(s, c.st);
      acc.run(s, c.st);
      c.sync();
      g_ar = std::move(nar);
      Gst = std::move(Gn);
    }
  }
  c.sync();
  // stacked rank-space layout for the solves
  F.stack_rows = 0;
  for (int p = 0; p < nn; ++p)
    if (!T.is_leaf(p)) {
      F.par_off[p] = F.stack_rows;
      F.stack_rows += F.r[2 * p + 1] + F.r[2 * p + 2];
      if (p == 0 || T.level(p) >= 2) F.rho[p] = F.r[2 * p + 1] + F.r[2 * p + 2];
    }
  const double t_end = now_seconds();
  M.times[0] = t_sample - t_begin;
  M.times[1] = t_leaf_scale - t_sample;
  M.times[2] = t_leaf_comp - t_leaf_scale;
  M.times[3] = t_leaf - t_leaf_comp;
  M.times[4] = t_end - t_leaf;
  M.times[7] = t_end - t_begin;
}

}  // namespace spd
