// Shared declarations of the spdhss library: descriptor structs for the batched
// kernels, launch wrappers, error handling and a bump-allocating device arena.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>
#include <stdexcept>

#include "spdhss.h"

namespace spd {

// ---------------------------------------------------------------- errors --
struct Error : std::runtime_error {
  spd_status code;
  Error(spd_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);
// frees the cached arena chunks of every device (none of them is in use)
void release_cached_chunks();

#define SPD_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::spd::Error(SPD_E_DEVICE, std::string(#call) + ": " +             \
                                           hipGetErrorString(e_));             \
  } while (0)

#define SPD_REQUIRE(cond, code, msg)                                           \
  do {                                                                         \
    if (!(cond)) throw ::spd::Error((code), (msg));                            \
  } while (0)

// ------------------------------------------------------------ descriptors --
// C = beta * C + alpha * sum_t op(A_t) op(B_t); all terms of a problem share
// (m, n); each term has its own inner size k.  Column-major storage.
// C = alpha * sum_t scale_t op(A_t) op(B_t) + beta * C (+ D).  The index and
// addend fields are for products with at most 4 columns (the streaming kernel)
// and are null otherwise:
//   cidx: row r of C is row cidx[r] of the C array (scatter);
//   D, didx, ldd: D row (didx ? didx[r] : r) is added to C row r;
//   bidx: row c of B is row bidx[c] of the B array (gather; B not transposed).
struct GemmProblem {
  double* C;
  int m, n, ldc;
  int term_begin, term_end;
  double alpha, beta;
  const int* cidx;
  const double* D;
  const int* didx;
  int ldd, pad;
};
struct GemmTerm {
  const double* A;
  const double* B;
  double scale;  // multiplies this term's product
  int k, lda, ldb, pad;
  const int* bidx;
};

// Symmetric-pair product for at most 4 right-hand columns.  For every term t
// of a problem, with A_t an m x k_t block of a symmetric matrix whose mirror
// block is A_t^T:
//   C = alpha * sum_t scale_t A_t B_t + beta * C         (row results, m x n)
//   P_t = scale_t A_t^T X   for every term with P_t set  (k_t x n, ldp)
// X (m x n) holds the problem's own input rows.  When the problem's rows are
// cut into row tiles, tile r writes its part of A_t^T X at P_t + r * ptile.
struct SymProblem {
  double* C;
  const double* X;
  int64_t ptile;
  int m, n, ldc, ldx, ldp;
  int term_begin, term_end;
  int pad;
  double alpha, beta;
};
struct SymTerm {
  const double* A;  // FP64, or FP32 elements for an a_f32 launch
  const double* B;
  double* P;      // null: row result only (diagonal blocks, bases)
  double scale;
  int k, lda, ldb, pad;
};

// dst (m x n) = beta * dst + sum_t alpha_t * src_t  (+ identity if add_eye)
struct BlockProblem {
  double* dst;
  int m, n, ldd;
  int term_begin, term_end;
  int add_eye;
  double beta;
  int tile0;  // first workgroup of this problem in its launch's tile list
};
struct BlockTerm {
  const double* src;
  int lds, trans;
  double alpha;
};

// Dense kernel block out(i, j) = K(x_a[ia(i)], x_b[ib(j)]) (+ shift if i == j
// and diag_shift).  Points are gathered from SoA arrays through index lists
// (idx == nullptr means the contiguous range starting at off); when proxy is
// set, the a-side (row) points are generated as `shells` Fibonacci spheres of
// `per_shell` points around the given centre (see proxy_point).
struct KBlockProblem {
  double* out;
  const int* ia;
  const int* ib;
  int64_t offa, offb;
  int na, nb, ld, diag_shift;
  int proxy;          // a side is a proxy set
  int shells, per_shell;
  int pad;
  double cx, cy, cz;  // proxy centre
  double rin, rout;   // proxy radii
};

// Cholesky / triangular solves on column-major matrices.
struct CholProblem {
  double* A;
  int n, lda;
};
struct TrsmProblem {
  const double* L;  // triangular factor
  double* B;        // right-hand sides, overwritten
  int n, nrhs, ldl, ldb;
};

// Column-pivoted QR of a column-major m x n matrix.
struct CpqrProblem {
  double* A;        // input (destroyed for the global-memory variant)
  double* Q;        // out: first rank columns of Q (ldq), may be null
  double* V;        // workspace: Householder vectors (m x maxrank, ld m)
  double* R;        // out (global variant): R rows in pivot order, rank x n, ld maxrank
  int* piv;         // out: pivot column indices (maxrank)
  int* rank;        // out
  double* diag;     // out: |R_tt|
  int m, n, lda, ldq;
  int maxrank;
  double tol;
  double* hbeta;    // global variant with Q: out, Householder factors (maxrank); else null
  double* nrm;      // global variant, more than 2048 rows: workspace of n doubles
};

// ----------------------------------------------------------- launchers --
// All launchers enqueue on `s` and copy their descriptor arrays from device
// memory (`d_*` pointers) that the caller keeps alive until completion.
// dot-form product (op(A) = A^T stored K x m, at most 4 columns); max_k bounds
// the terms' K
void launch_gemv_t(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob, int max_m,
                   int max_n, int max_k, int transB, int a_f32 = 0);
// FP32 copy of an FP64 array
struct CvtProblem {
  const double* src;
  float* dst;
  int64_t n;
};
void launch_to_f32(hipStream_t s, const CvtProblem* d_p, int nprob);
// cap > 0 bounds the number of workgroups (they then walk the problems with a
// stride), so that the launch can run beside latency-bound work.  a_f32: the
// terms' A operands are FP32 (same element layout), widened to FP64 on load.
// mir = 0 declares that no term has a mirrored output (T.P null throughout):
// 5-16 columns then take the plain-product form of the kernel.
void launch_symv(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob, int max_m,
                 int max_n, int cap = 0, int a_f32 = 0, int mir = 1);
// rows per workgroup of launch_symv for a launch whose largest problem has max_m rows
int symv_row_tile(int max_m, int ncols);
// max_k bounds the terms' inner dimension (used to pick the dot-form variant
// when transA is set and there are at most 4 columns)
// a_f32: the A operands are FP32 (dot-form product only)
void launch_gemm(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                 int max_m, int max_n, int transA, int transB, int max_k = 1 << 30, int a_f32 = 0);
// Block sums over a tile list: tile t belongs to problem tiles[t] (made by
// block_tiles, which also sets BlockProblem::tile0); tiles of 64 rows x 16
// columns when every problem has at most 16 columns (max_n <= 16), else 64 x 64.
int block_tile_cols(int max_n);
std::vector<int> block_tiles(std::vector<BlockProblem>& probs, int max_n);
void launch_block(hipStream_t s, const BlockProblem* d_p, const BlockTerm* d_t,
                  const int* d_tiles, int ntiles, int max_n);
// perm: tree position -> original index (for the RPY tensor, whose rows are
// point components: component = original index mod 3); may be null otherwise
void launch_kblock(hipStream_t s, const KBlockProblem* d_p, int nprob, int max_m,
                   int max_n, const double* px, int64_t stride, int kind,
                   double ell, double shift, const int64_t* perm);
void launch_chol(hipStream_t s, const CholProblem* d_p, int nprob, int max_n,
                 int* d_fail);
void launch_trsm(hipStream_t s, const TrsmProblem* d_p, int nprob, int max_n,
                 int max_nrhs, int trans, int upper);
void launch_cpqr_reg(hipStream_t s, const CpqrProblem* d_p, int nprob, int max_m,
                     int max_n);
// After launch_cpqr_glob on problems with V (m x maxrank, ld m) and hbeta set:
// Q's first rank columns from the stored Householder vectors, the signs
// making R's diagonal non-negative (as the register kernel's Q).
void launch_cpqr_formq(hipStream_t s, const CpqrProblem* d_p, int nprob);
// Above 2048 rows (at most kCpqrBigRows) every problem must carry its nrm
// workspace.
constexpr int kCpqrBigRows = 8000;
// rows of the wide form (cpqr_global above 2048 rows): the Householder vector
// is staged in LDS up to kCpqrBigRows rows and read from the pivot column above
constexpr int kCpqrWideRows = 16000;
void launch_cpqr_glob(hipStream_t s, const CpqrProblem* d_p, int nprob, int max_m,
                      int max_n);
// The wide form of the global-memory variant (one launch per step, columns
// over many workgroups; same results as launch_cpqr_glob above 2048 rows).
// Every problem's nrm workspace holds 2n + maxrank + 2 doubles and P.R is
// set.  d_wg: workgroup table (problem, first column, end column, 0); d_done:
// one flag per problem, set once the problem has stopped; d_fix: (problem,
// step) for every step below the problem's min(m, n, maxrank); d_rc:
// (problem, column) for every column.
void launch_cpqr_wide_norms(hipStream_t s, const CpqrProblem* d_p, const int4* d_wg, int nwg,
                            int* d_done);
void launch_cpqr_wide_step(hipStream_t s, const CpqrProblem* d_p, const int4* d_wg, int nwg,
                           int max_m, int t, int* d_done);
void launch_cpqr_wide_finish(hipStream_t s, const CpqrProblem* d_p, int nprob, const int2* d_fix,
                             int nfix, const int2* d_rc, int nrc);
bool cpqr_reg_fits(int m, int n);

// vector kernels
void launch_gather_rows(hipStream_t s, const double* src, int64_t lds, double* dst,
                        int64_t ldd, const int64_t* perm, int64_t n, int ncols);
void launch_scatter_rows(hipStream_t s, const double* src, int64_t lds, double* dst,
                         int64_t ldd, const int64_t* perm, int64_t n, int ncols);
void launch_gaussian_fill(hipStream_t s, double* dst, int64_t n, int ncols,
                          int64_t ldd, const int64_t* perm, uint64_t seed);
// dst(t, j) = standard normal of the counter (t << 24) | j under seed, for
// t < rows, j < cols (column-major, ld): the sketch of the proxy ID
void launch_sketch_fill(hipStream_t s, double* dst, int64_t rows, int cols, int64_t ld,
                        uint64_t seed);
void launch_soa_points(hipStream_t s, const double* pts_rowmajor,
                       const int64_t* perm, int64_t n, double* soa);
// Fused PCG step kernels over per-chunk partial dot products (coldot_chunks(n)
// chunks per column): partials of x.y; x, r update with the partials of the
// new r.r; the active test; the p update.
int coldot_chunks(int64_t n);
void launch_coldot_partial(hipStream_t s, const double* x, const double* y, int64_t n, int ncols,
                           int64_t ld, double* partial);
void launch_pcg_xr_dot(hipStream_t s, double* x, double* r, const double* p, const double* q,
                       const double* rzp, const double* pqp, const int* active, int64_t n, int ncols,
                       int64_t ld, int* iters, double* rzv, double* rrp, const double* zold = nullptr,
                       double* rzop = nullptr);
void launch_pcg_active_partial(hipStream_t s, const double* rrp, int64_t n, const double* bb,
                               double rtol, int* active, int ncols, int* any_active);
void launch_pcg_update_p_partial(hipStream_t s, double* p, const double* z, const double* rzp,
                                 const double* rzv, const int* active, int64_t n, int ncols,
                                 int64_t ld, const double* rzop = nullptr);
// column dot products: out[c] = sum_i x[i,c] * y[i,c] (deterministic, two-stage)
void launch_coldot(hipStream_t s, const double* x, const double* y, int64_t n,
                   int ncols, int64_t ld, double* partial, double* out);
void launch_pcg_active(hipStream_t s, const double* rr, const double* bb,
                       double rtol, int* active, int ncols, int* any_active);
void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b,
                  int64_t n, int ncols, int64_t ld);
void launch_fill(hipStream_t s, double* p, double v, int64_t count);
void launch_scatter_interp(hipStream_t s, double* W, int ldw, const double* E,
                           int lde, const int* perm_full, int cand, int k);
void launch_gather_skel(hipStream_t s, const int* cand, const int* piv, int k, int* out);

// --------------------------------------------------------------- arena --
// Device memory handed out by bumping through large hipMalloc'd chunks; all of
// it is released together when the owning handle is destroyed.
// Device memory in 256 MiB chunks (larger requests get a dedicated
// allocation).  Released chunks go to a process-wide cache per device and are
// handed to the next arena instead of being freed: hipFree waits for the whole
// device, which would stall every other stream (concurrent instances).  An
// arena is released only after the work that used it has completed (every
// entry point synchronizes its stream before returning); dedicated allocations
// are freed.  release_cached_chunks() frees the cache.
class Arena {
 public:
  ~Arena();
  // Hand out memory from [base, base + bytes) only (caller-owned, never freed
  // here); a request beyond it throws SPD_E_NOMEM.  No device allocation is
  // made in this mode.
  void use_region(void* base, size_t bytes);
  void* get(size_t bytes);
  template <class T>
  T* get_n(size_t n) { return static_cast<T*>(get(n * sizeof(T))); }
  void release();
  size_t bytes_used() const { return used_; }

 private:
  std::vector<std::pair<void*, size_t>> chunks_;
  char* cur_ = nullptr;
  size_t left_ = 0;
  size_t used_ = 0;
  bool region_ = false;
};

// Upload a host vector into arena memory (synchronous w.r.t. the host data).
template <class T>
T* upload(Arena& a, hipStream_t s, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  T* d = a.get_n<T>(v.size());
  SPD_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SPD_HIP(hipStreamSynchronize(s));
  return d;
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace spd
