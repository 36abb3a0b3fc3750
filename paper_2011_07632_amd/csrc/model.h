// Host-side model of the library's handles: the tree, the H^2 matrix, the SPD
// HSS matrix and its nested factors, plus the descriptor staging used to
// launch the batched kernels.
#pragma once
#include "common.h"

#include <memory>

namespace spd {

// ------------------------------------------------------------------ tree --
struct TreeHost {
  int64_t N = 0;
  int leaf = 0, D = 0, L = 0, nnodes = 0, kind = SPD_TREE_KD;
  double eta = 1.0;
  std::vector<int64_t> perm, start, end;
  std::vector<double> lo, hi, center, radius;
  std::vector<int64_t> near_ptr, coup_ptr;
  std::vector<int> near_idx, coup_idx;

  void build(const double* pts_rowmajor, int64_t n, int leaf_size, double eta, int kind);
  void split(const double* pts, int v, int axis);
  bool admissible(int i, int j) const;
  void build_lists();
  int depth(int v) const { int d = 0; while ((1 << (d + 1)) - 1 <= v) ++d; return d; }
  int level(int v) const { return L - depth(v); }
  bool is_leaf(int v) const { return depth(v) == D; }
  int first_at(int k) const { return (1 << (L - k)) - 1; }
  int count_at(int k) const { return 1 << (L - k); }
  int64_t size(int v) const { return end[v] - start[v]; }
  int lca_level(int i, int j) const;
  int64_t near_pos(int i, int j) const;
  int64_t coup_pos(int i, int j) const;
  bool proxy_radii(int v, double& rin, double& rout) const;
};
int proxy_count(double rin, double ell, int lo, int hi, double density);

// --------------------------------------------------- descriptor staging --
// Collects descriptor arrays on the host and copies them to device memory.
// A device copy stays valid until reset(), which the owner calls only after
// synchronizing the stream; filling a chunk opens a new one and never frees
// an earlier chunk, whose descriptors may still be waiting for their launch.
class Stage {
 public:
  ~Stage();
  void* push(hipStream_t s, const void* data, size_t bytes);
  void reset();

 private:
  struct Chunk {
    char* dev = nullptr;
    char* host = nullptr;
    size_t cap = 0;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, off_ = 0;
};

// Pivoted QR of problems in global memory (launch_cpqr_glob), in the wide
// form (one launch per step over many workgroups) above 2048 rows or for fewer
// than 128 problems; h are the host copies of the device descriptors d.
void cpqr_global(hipStream_t s, Stage& st, const std::vector<CpqrProblem>& h, const CpqrProblem* d,
                 int max_m, int max_n);

struct GemmBatch {
  std::vector<GemmProblem> probs;
  std::vector<GemmTerm> terms;
  int max_m = 0, max_n = 0, transA = 0, transB = 0, max_k = 0;
  int a_f32 = 0;  // A operands are FP32 (set before adding terms)
  explicit GemmBatch(int ta = 0, int tb = 0) : transA(ta), transB(tb) {}
  void add(double* C, int m, int n, int ldc, double beta = 0.0, double alpha = 1.0);
  void term(const double* A, int lda, const double* B, int ldb, int k, double scale = 1.0);
  // indexed forms (at most 4 columns): scattered C rows and an addend D with
  // optional row gather; a term whose B rows are gathered through bidx
  void add_indexed(double* C, int m, int n, int ldc, double beta, const int* cidx, const double* D,
                   const int* didx, int ldd);
  void term_gathered(const double* A, int lda, const double* B, int ldb, const int* bidx, int k);
  bool indexed = false;
  void run(hipStream_t s, Stage& st);
  bool empty() const { return probs.empty(); }
};

struct BlockBatch {
  std::vector<BlockProblem> probs;
  std::vector<BlockTerm> terms;
  int max_m = 0, max_n = 0;
  void add(double* dst, int m, int n, int ldd, double beta = 0.0, int add_eye = 0);
  void term(const double* src, int lds, double alpha = 1.0, int trans = 0);
  void run(hipStream_t s, Stage& st);
};

struct TrsmBatch {
  std::vector<TrsmProblem> probs;
  int max_n = 0, max_nrhs = 0;
  void add(const double* L, int ldl, double* B, int ldb, int n, int nrhs);
  void run(hipStream_t s, Stage& st, int trans, int upper = 0);
};

// A recorded launch with descriptors resident in device memory, replayed by
// the solve loops (matvec and preconditioner apply) without host work.
struct LaunchRec {
  int type;  // 0 gemm, 1 block, 2 trsm, 3 symmetric-pair product
  const void* probs;
  const void* terms;
  int nprob, max_m, max_n, transA, transB;
  double bytes;  // algorithmic bytes: every A operand once, distinct B operands once, C once
  int tag = -1;  // caller-defined label (which pass of a product)
  int max_k = 1 << 30;  // bound on the terms' inner dimension (gemm records)
  int cap = 0;          // workgroup cap (symmetric-pair records), 0 = none
  int a_f32 = 0;        // FP32 A operands (gemm records)
  int mir = 1;          // symmetric-pair records: some term has a mirrored output
  const int* tiles = nullptr;  // tile list (block records)
  int ntiles = 0;
};
// One block row of a symmetric product with at most 4 right-hand columns:
// y = sum_t A_t B_t, and every mirrored term (an off-diagonal block A_ij of a
// symmetric matrix, stored once) also adds A_ij^T x to the output of row
// `mirror`, where x are this row's own input rows.
struct SymRow {
  double* y;
  int ldy;
  const double* x;
  int ldx;
  int m;
  struct Term {
    const double* A;
    int lda;
    const double* B;
    int ldb;
    int k;
    int mirror;  // index of the receiving row, or -1
  };
  std::vector<Term> terms;
};

struct Recorder {
  std::vector<LaunchRec> recs;
  void gemm(Arena& a, hipStream_t s, const GemmBatch& b);
  // the same product on the symmetric-pair kernel (row sums only)
  void gemm_symm(Arena& a, hipStream_t s, const GemmBatch& b, double bytes);
  // symmetric product of n <= 4 columns over rows (one product launch and one
  // launch that sums each row's partial results in a fixed order into
  // y = beta * y + sum)
  // (a_f32: the terms' A pointers address FP32 copies with the same layout)
  // (split_bytes: bytes of A per part of a row, 0 = the default of 1 MiB)
  void symv(Arena& a, hipStream_t s, const std::vector<SymRow>& rows, int n, double beta = 0.0,
            bool a_f32 = false, double split_bytes = 0.0);
  void block(Arena& a, hipStream_t s, const BlockBatch& b);
  void trsm(Arena& a, hipStream_t s, const TrsmBatch& b, int trans);
  void replay(hipStream_t s) const;
  void tag_from(size_t first, int tag) {
    for (size_t i = first; i < recs.size(); ++i) recs[i].tag = tag;
  }
};

// ---------------------------------------------------------------- H^2 --
struct H2Model {
  spd_kernel kern{};
  spd_h2_opts opts{};
  TreeHost T;
  Arena arena;
  Stage stage;
  hipStream_t s = nullptr;
  // side stream of the product (the near-field pass runs beside the far-field
  // chain) and its fork/join events; created with the first product plan
  hipStream_t side_s = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* pts = nullptr;        // SoA, tree order: x[N] y[N] z[N]
  int64_t* perm_d = nullptr;    // tree position -> original index
  // per node (heap order)
  std::vector<int> k;             // skeleton size k_v
  std::vector<int> proxy_n;       // points per proxy sphere (0: no ID at this node)
  std::vector<int> sketched;      // the proxy matrix was sketched before the pivoted QR
  std::vector<int> cand;          // candidates: n_v (leaf) or k_c1 + k_c2
  std::vector<int*> cand_d;       // device candidate tree positions (nonleaf: [skel_c1; skel_c2])
  std::vector<std::vector<int>> cand_h;  // host copy (tree positions)
  std::vector<std::vector<int>> skel_h;  // skeleton of every node (tree positions)
  std::vector<double*> W;         // U_v (leaf) or R_v (nonleaf): cand_v x k_v, ld cand_v
  std::vector<double*> WT;        // W_v^T (k_v x cand_v, ld k_v): coalesced upward pass
  // W_v = Pi_v [I; E_v^T]: the ID's column order Pi_v (cand_v positions, the
  // skeleton first) and E_v = R11^{-1} R12 (k_v x (cand_v - k_v)) and its transpose
  std::vector<int*> piv_d;
  std::vector<double*> E, ET;
  std::vector<double*> Bh;        // per coupling entry: K(skel_i, skel_j), k_i x k_j, ld coup_ld(i)
  std::vector<double*> nearA;     // per leaf near entry: n_i x n_j, ld near_ld(i)
  // Leading dimensions of the stored blocks: the rows rounded up to 16
  // doubles, so that every column starts on a 128-byte line and a streamed
  // column touches no partial line at its start (the pad rows hold zeros and
  // are never read as data).
  int coup_ld(int v) const { return (k[v] + 15) / 16 * 16; }
  int near_ld(int v) const { return ((int)T.size(v) + 15) / 16 * 16; }
  // FP32 copies of the blocks the symmetric-pair product reads (coupling
  // entries j > i, near entries j >= i; null elsewhere), made on first use by
  // the mixed-precision product; each block row's copies are one allocation
  std::vector<float*> Bh32, nearA32;
  Arena arena32;
  double times[4] = {0, 0, 0, 0};
  // stacked layout of skeleton-space blocks: the two children of a node share
  // one (cand_p x ncols, ld cand_p) buffer; par_off[p] is its row offset.
  std::vector<int64_t> par_off;
  int64_t stack_rows = 0;
  struct MatvecPlan;
  std::unique_ptr<MatvecPlan> plan;
  // the same product with the FP32 block copies; shares plan's input and
  // output buffers (so h2_plan_x / h2_plan_y serve both)
  std::unique_ptr<MatvecPlan> plan32;
  struct NearStats {
    double bytes = 0;  // algorithmic bytes of one near-field launch
  };

  H2Model();
  ~H2Model();
  const int* skel_d(int v) const {
    const int p = (v - 1) / 2;
    return cand_d[p] + ((v % 2 == 0) ? k[v - 1] : 0);
  }
  // block of node v (k_v x ncols, ld cand_parent) inside a stacked buffer
  double* hat(double* base, int v, int ncols) const {
    const int p = (v - 1) / 2;
    return base + par_off[p] * ncols + ((v % 2 == 0) ? k[v - 1] : 0);
  }
  int hat_ld(int v) const { return cand[(v - 1) / 2]; }
  int64_t n(int v) const { return T.size(v); }
};

void h2_build_impl(H2Model& H, const double* points, int64_t n);
void h2_matvec_tree(H2Model& H, const double* x, double* y, int ncols, bool f32 = false);

// --------------------------------------------------- SPD HSS + factors --
// Nested factors shared by an HSS handle and the ULV handle made from it.
struct Factors {
  Arena arena;
  TreeHost T;             // tree shape and ranges
  int64_t* perm_d = nullptr;
  std::vector<int> r;     // HSS rank per node
  std::vector<int> rho;   // rows of the node's basis: n_v at leaves, r_c1 + r_c2 above
  std::vector<double*> S; // leaf Cholesky factors S_v (n_v x n_v)
  std::vector<double*> V; // V_v (leaf, n_v x r_v) or V-bar_v (rho_v x r_v)
  std::vector<double*> F; // factor of I + bold B_v (rho_v x rho_v), nonleaf incl. root
  // operators of the solve, formed by ulv_factor:
  //   Dm: leaf A_vv^{-1} = S_v^{-T} S_v^{-1}; nonleaf and root (I + bold B_vv)^{-1} - I
  //   Zs: Z_v = S_v^{-T} V_v (leaf) or F_v^{-T} V-bar_v (nonleaf); ZsT: Z_v^T
  std::vector<double*> Dm, Zs, ZsT;
  // FP32 copies of Dm, Zs, ZsT for the mixed-precision apply
  std::vector<float*> Dm32, Zs32, ZsT32;
  bool ops32_ready = false;
  bool root_factored = false;
  bool ops_ready = false;  // Dm, Zs, ZsT formed
  // stacked rank-space layout: the children of p share a rho_p-row buffer
  std::vector<int64_t> par_off;
  int64_t stack_rows = 0;
  double* blk(double* base, int v, int ncols) const {
    const int p = (v - 1) / 2;
    return base + par_off[p] * ncols + ((v % 2 == 0) ? r[v - 1] : 0);
  }
  int blk_ld(int v) const { return rho[(v - 1) / 2]; }
};

struct HSSModel {
  std::shared_ptr<Factors> f;
  spd_hss_opts opts{};
  int s = 0;
  Arena arena;
  std::vector<double*> Z;     // S^{-T} V (leaf) or F^{-T} V-bar (nonleaf)
  std::vector<double*> R;     // transfer matrices F V-bar (nonleaf)
  std::vector<double*> PhiU;  // Phi_v U_v^H2: r_v x k_v
  std::vector<int*> piv;      // pivots of the node's CPQR
  std::vector<double*> Bn;    // HSS couplings per near entry (self entries null)
  std::vector<double*> Bc;    // per coupling entry
  std::vector<int> hk;        // H^2 ranks (copy)
  TreeHost lists;             // tree with lists (for coupling queries)
  double times[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double flops[4] = {0, 0, 0, 0};
};

void spdhss_build_impl(H2Model& H, const spd_hss_opts& o, HSSModel& M, hipStream_t s);

struct ULVModel {
  std::shared_ptr<Factors> f;
  int precision = 0;  // 0: FP64 apply; 1: FP32 operators, FP64 vectors and sums
  Stage stage;
  hipStream_t s = nullptr;
  struct ApplyPlan;
  std::unique_ptr<ApplyPlan> plan;
  ULVModel();
  ~ULVModel();
};

void ulv_factor_impl(HSSModel& M, ULVModel& U, hipStream_t s);
void ulv_apply_tree(ULVModel& U, const double* b, double* x, int ncols);
// The apply with every device buffer in a fixed per-GPU array of
// kNoAllocScratchBytes (see solve.cpp); b and x as for ulv_apply.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
int64_t ulv_noalloc_bytes(const ULVModel& U, int ncols);
void ulv_apply_noalloc_impl(ULVModel& U, const double* b, double* x, int ncols, int64_t ld);
// apply plan buffers: ulv_plan_in is read and ulv_plan_out written in place
double* ulv_plan_in(ULVModel& U, int m);
double* ulv_plan_out(ULVModel& U, int m);

// product plan buffers: h2_plan_x is read and h2_plan_y written in place
double* h2_plan_x(H2Model& H, int m);
double* h2_plan_y(H2Model& H, int m);
void h2_plan_run(H2Model& H);
// the product with FP32 near and coupling blocks (FP64 accumulation, vectors
// and interpolation), at most 4 columns; same buffers as h2_plan_x / h2_plan_y
void h2_plan_run32(H2Model& H, int m);
void h2_plan_prepare32(H2Model& H, int m);  // build the FP32 plan (outside graph capture)
void h2_plan_run_last(H2Model& H);
H2Model::NearStats h2_near_stats(H2Model& H, int m);
void h2_time_near(H2Model& H, int m, int reps, double* ms, double* bytes);
int h2_time_launches(H2Model& H, int m, int reps, double* ms, double* bytes, int* tags, int cap);

struct PcgResult {
  std::vector<int> iters;
  std::vector<double> relres;
  bool converged = true;
  int replacements = 0;  // residual replacements with the FP64 product (op_f32)
};
// op_f32: the iterations use the product with FP32 blocks (h2_plan_run32) and
// the residual is replaced by b - A x with the FP64 product whenever it has
// halved since the last replacement (reliable updates)
PcgResult pcg_tree(H2Model& H, ULVModel* U, const double* bt, double* xt, int m, double rtol,
                   int maxit, bool op_f32 = false);

double now_seconds();
const char* last_error_cstr();

}  // namespace spd
