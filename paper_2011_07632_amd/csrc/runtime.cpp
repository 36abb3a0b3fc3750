// Runtime pieces of the library: device arena, descriptor staging, batch
// builders and error bookkeeping.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <chrono>
#include <cstring>

namespace spd {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- arena --
static constexpr size_t kChunk = size_t(256) << 20;

namespace {
std::mutex g_chunk_mu;
std::vector<std::pair<int, void*>> g_chunk_cache;  // (device, chunk)

void* take_chunk() {
  int dev = 0;
  SPD_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_chunk_mu);
    for (size_t i = g_chunk_cache.size(); i-- > 0;)
      if (g_chunk_cache[i].first == dev) {
        void* p = g_chunk_cache[i].second;
        g_chunk_cache.erase(g_chunk_cache.begin() + i);
        return p;
      }
  }
  void* p = nullptr;
  if (hipMalloc(&p, kChunk) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void give_chunk(void* p) {
  int dev = 0;
  if (hipPointerAttribute_t a{}; hipPointerGetAttributes(&a, p) == hipSuccess) dev = a.device;
  else (void)hipGetLastError();
  std::lock_guard<std::mutex> lk(g_chunk_mu);
  g_chunk_cache.push_back({dev, p});
}
}  // namespace

void release_cached_chunks() {
  std::vector<std::pair<int, void*>> all;
  {
    std::lock_guard<std::mutex> lk(g_chunk_mu);
    all.swap(g_chunk_cache);
  }
  for (auto& c : all) (void)hipFree(c.second);
}

Arena::~Arena() { release(); }

void Arena::use_region(void* base, size_t bytes) {
  release();
  region_ = true;
  cur_ = static_cast<char*>(base);
  left_ = bytes;
}

void Arena::release() {
  if (region_) {
    region_ = false;
    cur_ = nullptr;
    left_ = 0;
    used_ = 0;
    return;
  }
  for (auto& c : chunks_) {
    if (c.second == kChunk) give_chunk(c.first);
    else (void)hipFree(c.first);
  }
  chunks_.clear();
  cur_ = nullptr;
  left_ = 0;
  used_ = 0;
}

void* Arena::get(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  if (region_) {
    if (bytes > left_)
      throw Error(SPD_E_NOMEM, "scratch region exhausted (" + std::to_string(used_ + bytes) +
                                   " bytes needed, " + std::to_string(used_ + left_) + " available)");
    void* r = cur_;
    cur_ += bytes;
    left_ -= bytes;
    used_ += bytes;
    return r;
  }
  if (bytes > left_) {
    const size_t sz = bytes > kChunk / 4 ? bytes : kChunk;
    void* p = nullptr;
    if (sz == kChunk) {
      p = take_chunk();
    } else if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) throw Error(SPD_E_NOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
    chunks_.push_back({p, sz});
    used_ += sz;
    if (sz != kChunk) return p;  // dedicated allocation; keep the current chunk
    cur_ = static_cast<char*>(p);
    left_ = sz;
  }
  void* r = cur_;
  cur_ += bytes;
  left_ -= bytes;
  return r;
}

// ---------------------------------------------------------------- stage --
Stage::~Stage() {
  for (Chunk& c : chunks_) {
    if (c.dev) (void)hipFree(c.dev);
    if (c.host) (void)hipHostFree(c.host);
  }
}

void Stage::reset() {
  // keep only the largest chunk for reuse; the caller has synchronized
  if (chunks_.size() > 1) {
    size_t best = 0;
    for (size_t i = 1; i < chunks_.size(); ++i)
      if (chunks_[i].cap > chunks_[best].cap) best = i;
    for (size_t i = 0; i < chunks_.size(); ++i)
      if (i != best) {
        (void)hipFree(chunks_[i].dev);
        (void)hipHostFree(chunks_[i].host);
      }
    Chunk keep = chunks_[best];
    chunks_.assign(1, keep);
  }
  cur_ = 0;
  off_ = 0;
}

void* Stage::push(hipStream_t s, const void* data, size_t bytes) {
  const size_t aligned = (bytes + 255) & ~size_t(255);
  if (chunks_.empty() || off_ + aligned > chunks_[cur_].cap) {
    if (!chunks_.empty() && cur_ + 1 < chunks_.size() && chunks_[cur_ + 1].cap >= aligned) {
      ++cur_;
    } else {
      size_t cap = size_t(4) << 20;
      while (cap < aligned) cap *= 2;
      Chunk c;
      SPD_HIP(hipMalloc(&c.dev, cap));
      SPD_HIP(hipHostMalloc((void**)&c.host, cap, hipHostMallocDefault));
      c.cap = cap;
      chunks_.push_back(c);
      cur_ = chunks_.size() - 1;
    }
    off_ = 0;
  }
  Chunk& c = chunks_[cur_];
  std::memcpy(c.host + off_, data, bytes);
  void* d = c.dev + off_;
  SPD_HIP(hipMemcpyAsync(d, c.host + off_, bytes, hipMemcpyHostToDevice, s));
  off_ += aligned;
  return d;
}

// -------------------------------------------------------------- batches --
void GemmBatch::add(double* C, int m, int n, int ldc, double beta, double alpha) {
  GemmProblem p{};
  p.C = C;
  p.m = m;
  p.n = n;
  p.ldc = ldc;
  p.term_begin = p.term_end = (int)terms.size();
  p.alpha = alpha;
  p.beta = beta;
  probs.push_back(p);
  max_m = std::max(max_m, m);
  max_n = std::max(max_n, n);
}

// A term that continues the previous term of the same problem in memory (its
// first column of op(A) follows that term's last, and likewise its rows of
// op(B)) is merged into it: a longer unbroken stream for the kernels.
void GemmBatch::term(const double* A, int lda, const double* B, int ldb, int k, double scale) {
  if (k <= 0) return;
  GemmProblem& p = probs.back();
  if (p.term_end > p.term_begin && !terms.back().bidx && !a_f32) {
    GemmTerm& q = terms.back();
    const int64_t acs = transA ? 1 : q.lda, bcs = transB ? q.ldb : 1;
    if (q.lda == lda && (q.ldb == ldb || (p.n == 1 && !transB)) && q.scale == scale &&
        A == q.A + acs * q.k && B == q.B + bcs * q.k) {
      q.k += k;
      max_k = std::max(max_k, q.k);
      return;
    }
  }
  GemmTerm t{};
  t.A = A;
  t.B = B;
  t.scale = scale;
  t.k = k;
  t.lda = lda;
  t.ldb = ldb;
  terms.push_back(t);
  p.term_end = (int)terms.size();
  max_k = std::max(max_k, k);
}

void GemmBatch::add_indexed(double* C, int m, int n, int ldc, double beta, const int* cidx,
                            const double* D, const int* didx, int ldd) {
  add(C, m, n, ldc, beta);
  GemmProblem& p = probs.back();
  p.cidx = cidx;
  p.D = D;
  p.didx = didx;
  p.ldd = ldd;
  indexed = true;
}

void GemmBatch::term_gathered(const double* A, int lda, const double* B, int ldb, const int* bidx,
                              int k) {
  if (k <= 0) return;
  GemmTerm t{};
  t.A = A;
  t.B = B;
  t.scale = 1.0;
  t.k = k;
  t.lda = lda;
  t.ldb = ldb;
  t.bidx = bidx;
  terms.push_back(t);
  probs.back().term_end = (int)terms.size();
  indexed = true;
  max_k = std::max(max_k, k);
}

void GemmBatch::run(hipStream_t s, Stage& st) {
  if (probs.empty() || max_m == 0 || max_n == 0) return;
  if (indexed && max_n > 4) throw Error(SPD_E_INVALID, "indexed products support at most 4 columns");
  const GemmTerm dummy{};
  auto* dp = (const GemmProblem*)st.push(s, probs.data(), probs.size() * sizeof(GemmProblem));
  auto* dt = (const GemmTerm*)st.push(s, terms.empty() ? &dummy : terms.data(),
                                      std::max<size_t>(1, terms.size()) * sizeof(GemmTerm));
  launch_gemm(s, dp, dt, (int)probs.size(), max_m, max_n, transA, transB, std::max(max_k, 1), a_f32);
}

void BlockBatch::add(double* dst, int m, int n, int ldd, double beta, int add_eye) {
  BlockProblem p{};
  p.dst = dst;
  p.m = m;
  p.n = n;
  p.ldd = ldd;
  p.term_begin = p.term_end = (int)terms.size();
  p.add_eye = add_eye;
  p.beta = beta;
  probs.push_back(p);
  max_m = std::max(max_m, m);
  max_n = std::max(max_n, n);
}

void BlockBatch::term(const double* src, int lds, double alpha, int trans) {
  BlockTerm t{};
  t.src = src;
  t.lds = lds;
  t.trans = trans;
  t.alpha = alpha;
  terms.push_back(t);
  probs.back().term_end = (int)terms.size();
}

void BlockBatch::run(hipStream_t s, Stage& st) {
  if (probs.empty() || max_m == 0 || max_n == 0) return;
  const BlockTerm dummy{};
  const std::vector<int> tl = block_tiles(probs, max_n);
  if (tl.empty()) return;
  auto* dp = (const BlockProblem*)st.push(s, probs.data(), probs.size() * sizeof(BlockProblem));
  auto* dt = (const BlockTerm*)st.push(s, terms.empty() ? &dummy : terms.data(),
                                       std::max<size_t>(1, terms.size()) * sizeof(BlockTerm));
  auto* dl = (const int*)st.push(s, tl.data(), tl.size() * sizeof(int));
  launch_block(s, dp, dt, dl, (int)tl.size(), max_n);
}

void cpqr_global(hipStream_t s, Stage& st, const std::vector<CpqrProblem>& h, const CpqrProblem* d,
                 int max_m, int max_n) {
  const int nprob = (int)h.size();
  if (nprob == 0) return;
  // one workgroup per problem fills the chip only with many problems
  if (max_m <= 2048 && nprob >= 128) {
    launch_cpqr_glob(s, d, nprob, max_m, max_n);
    return;
  }
  // about 768 workgroups over all columns, 16 columns (a column per wave) or more each
  int64_t cols = 0;
  int kmax = 0;
  for (const CpqrProblem& p : h) {
    cols += p.n;
    kmax = std::max(kmax, std::min(std::min(p.m, p.n), p.maxrank));
  }
  const int cb = 16 * (int)std::max<int64_t>(1, (cols + 16 * 768 - 1) / (16 * 768));
  std::vector<int4> wg;
  std::vector<int2> fix, rc;
  for (int q = 0; q < nprob; ++q) {
    for (int c = 0; c < h[q].n; c += cb) wg.push_back(make_int4(q, c, std::min(h[q].n, c + cb), 0));
    // a problem without columns still needs the workgroup that sets up its state
    if (h[q].n <= 0) wg.push_back(make_int4(q, 0, 0, 0));
    const int km = std::min(std::min(h[q].m, h[q].n), h[q].maxrank);
    for (int t = 0; t < km; ++t) fix.push_back(make_int2(q, t));
    for (int j = 0; j < h[q].n; ++j) rc.push_back(make_int2(q, j));
  }
  const std::vector<int> zero(nprob, 0);
  auto* dwg = (const int4*)st.push(s, wg.data(), wg.size() * sizeof(int4));
  auto* dfix = fix.empty() ? nullptr : (const int2*)st.push(s, fix.data(), fix.size() * sizeof(int2));
  auto* drc = (const int2*)st.push(s, rc.data(), rc.size() * sizeof(int2));
  auto* ddone = (int*)st.push(s, zero.data(), zero.size() * sizeof(int));
  launch_cpqr_wide_norms(s, d, dwg, (int)wg.size(), ddone);
  std::vector<int> done(nprob);
  for (int t = 0; t <= kmax; ++t) {
    launch_cpqr_wide_step(s, d, dwg, (int)wg.size(), max_m, t, ddone);
    // every 32 steps: stop once every problem has stopped
    if ((t & 31) == 31 && t < kmax) {
      SPD_HIP(hipMemcpyAsync(done.data(), ddone, nprob * sizeof(int), hipMemcpyDeviceToHost, s));
      SPD_HIP(hipStreamSynchronize(s));
      if (std::all_of(done.begin(), done.end(), [](int x) { return x != 0; })) break;
    }
  }
  launch_cpqr_wide_finish(s, d, nprob, dfix, (int)fix.size(), drc, (int)rc.size());
}

void TrsmBatch::add(const double* L, int ldl, double* B, int ldb, int n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return;
  TrsmProblem p{};
  p.L = L;
  p.B = B;
  p.n = n;
  p.nrhs = nrhs;
  p.ldl = ldl;
  p.ldb = ldb;
  probs.push_back(p);
  max_n = std::max(max_n, n);
  max_nrhs = std::max(max_nrhs, nrhs);
}

void TrsmBatch::run(hipStream_t s, Stage& st, int trans, int upper) {
  if (probs.empty()) return;
  auto* dp = (const TrsmProblem*)st.push(s, probs.data(), probs.size() * sizeof(TrsmProblem));
  launch_trsm(s, dp, (int)probs.size(), max_n, max_nrhs, trans, upper);
}

// ------------------------------------------------------------- recorder --
template <class T>
static const void* keep(Arena& a, hipStream_t s, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  return upload(a, s, v);
}

// Products with at most 16 columns are bandwidth-bound; a problem that streams
// more than kSplitBytes of A is cut into parts of about equal width (terms are
// cut at column boundaries where needed), each written to its own partial
// result, and a second launch sums the partials in part order into C
// (deterministic).  This balances the work over workgroups when per-problem
// work is uneven (the coupling pass).
static constexpr double kSplitBytes = 1.0 * (1 << 20);
static constexpr int64_t kFillTiles = 1024;

// Algorithmic bytes of a batch: every A operand once, C once (twice with
// beta), and the union of the B ranges read (B operands of different terms
// may overlap, e.g. skeleton vectors shared by many coupling rows).
static double batch_bytes(const GemmBatch& b) {
  double bytes = 0;
  std::vector<std::pair<const double*, const double*>> rs;
  for (const GemmProblem& p : b.probs) {
    bytes += 8.0 * p.m * p.n * (p.beta != 0.0 ? 2.0 : 1.0);
    if (p.D) bytes += 8.0 * p.m * p.n + (p.didx ? 4.0 * p.m : 0.0);
    if (p.cidx) bytes += 4.0 * p.m;
    for (int q = p.term_begin; q < p.term_end; ++q) {
      const GemmTerm& g = b.terms[q];
      bytes += (b.a_f32 ? 4.0 : 8.0) * p.m * g.k;
      if (g.bidx) {
        bytes += 8.0 * g.k * p.n + 4.0 * g.k;  // gathered rows and their indices
        continue;
      }
      if (!b.transB)
        for (int j = 0; j < p.n; ++j) rs.push_back({g.B + (int64_t)j * g.ldb, g.B + (int64_t)j * g.ldb + g.k});
      else
        for (int c = 0; c < g.k; ++c) rs.push_back({g.B + (int64_t)c * g.ldb, g.B + (int64_t)c * g.ldb + p.n});
    }
  }
  std::sort(rs.begin(), rs.end());
  const double* end = nullptr;
  for (const auto& r : rs) {
    const double* lo = (end && r.first < end) ? end : r.first;
    if (r.second > lo) bytes += 8.0 * (double)(r.second - lo);
    if (!end || r.second > end) end = r.second;
  }
  return bytes;
}

// A product of 5-16 right-hand columns that streams its A operands (not
// transposed, no gathered rows) runs on the symmetric-pair kernel with no
// mirrored terms: the row sums alone are C = alpha sum_t scale_t A_t B_t +
// beta C, with every A read once per 256-row tile.  Launches of fewer than
// kSymmMinWork tiles stay on the tiled GEMM, which splits them finer, unless
// their A operands are FP32 copies, which only this kernel reads.
static constexpr int64_t kSymmMinWork = 1024;

static bool symm_form(const GemmBatch& b) {
  if (b.transA || b.transB || b.indexed || b.max_n < 5 || b.max_n > 16) return false;
  const int64_t esz = b.a_f32 ? 4 : 8;
  int64_t work = 0;
  for (const GemmProblem& p : b.probs) {
    if (p.cidx || p.D || p.didx) return false;
    work += (p.m + 255) / 256;
    for (int q = p.term_begin; q < p.term_end; ++q) {
      const GemmTerm& t = b.terms[q];
      if (t.bidx || esz * (int64_t)t.lda * t.k >= (1ll << 31) ||
          8 * ((int64_t)(p.n - 1) * t.ldb + t.k) >= (1ll << 31))
        return false;
    }
  }
  return b.a_f32 || work >= kSymmMinWork;
}

void Recorder::gemm_symm(Arena& a, hipStream_t s, const GemmBatch& b, double bytes) {
  std::vector<SymProblem> probs;
  std::vector<SymTerm> terms;
  probs.reserve(b.probs.size());
  for (const GemmProblem& g : b.probs) {
    SymProblem P{};
    P.C = g.C;
    P.X = g.C;  // never multiplied (no mirrored terms); any rows of the right size
    P.ptile = 0;
    P.m = g.m;
    P.n = g.n;
    P.ldc = g.ldc;
    P.ldx = g.ldc;
    P.ldp = 1;
    P.alpha = g.alpha;
    P.beta = g.beta;
    P.term_begin = (int)terms.size();
    for (int q = g.term_begin; q < g.term_end; ++q) {
      const GemmTerm& t = b.terms[q];
      if (t.k <= 0) continue;
      SymTerm u{};
      u.A = t.A;
      u.B = t.B;
      u.P = nullptr;
      u.scale = t.scale;
      u.k = t.k;
      u.lda = t.lda;
      u.ldb = t.ldb;
      terms.push_back(u);
    }
    P.term_end = (int)terms.size();
    probs.push_back(P);
  }
  if (terms.empty()) terms.push_back(SymTerm{});
  LaunchRec r{3, keep(a, s, probs), keep(a, s, terms), (int)probs.size(), b.max_m, b.max_n, 0, 0, bytes,
              -1};
  r.a_f32 = b.a_f32;
  r.mir = 0;  // plain products: no mirrored outputs
  recs.push_back(r);
}

void Recorder::gemm(Arena& a, hipStream_t s, const GemmBatch& b) {
  if (b.probs.empty() || b.max_m == 0 || b.max_n == 0) return;
  const double bytes = batch_bytes(b);
  auto width = [&](const GemmProblem& p) {
    int64_t k = 0;
    for (int q = p.term_begin; q < p.term_end; ++q) k += b.terms[q].k;
    return k;
  };
  if (b.indexed && b.max_n > 4) throw Error(SPD_E_INVALID, "indexed products support at most 4 columns");
  // Parts per problem: by bytes (about kSplitBytes of A each), and, for a
  // 5-16 column launch of fewer than kFillTiles row tiles (the upper levels of
  // the sweeps: a few large nodes, one workgroup each), by the inner dimension
  // too, so that the launch fills the GPU (parts of at least 128 columns).
  int64_t tiles = 0;
  for (const GemmProblem& p : b.probs) tiles += (p.m + 63) / 64;
  const int64_t fill =
      (!b.transA && b.max_n > 4 && b.max_n <= 16 && tiles > 0 && tiles < kFillTiles) ? (kFillTiles + tiles - 1) / tiles : 1;
  auto nparts_of = [&](const GemmProblem& p) -> int64_t {
    const int64_t K = width(p);
    if (K <= 1) return 1;
    int64_t np = 8.0 * p.m * K > kSplitBytes ? (int64_t)std::ceil(8.0 * p.m * K / kSplitBytes) : 1;
    np = std::max<int64_t>(np, std::min<int64_t>(fill, K / 128));
    return std::max<int64_t>(1, std::min<int64_t>(np, K));
  };
  bool split = false;
  if (b.max_n <= 16 && !b.indexed && !b.a_f32)
    for (const GemmProblem& p : b.probs)
      if (nparts_of(p) > 1) { split = true; break; }
  if (!split && symm_form(b)) {
    gemm_symm(a, s, b, bytes);
    return;
  }
  if (!split) {
    std::vector<GemmTerm> t = b.terms;
    if (t.empty()) t.push_back(GemmTerm{});
    recs.push_back({0, keep(a, s, b.probs), keep(a, s, t), (int)b.probs.size(), b.max_m, b.max_n,
                    b.transA, b.transB, bytes, -1});
    recs.back().max_k = std::max(b.max_k, 1);
    recs.back().a_f32 = b.a_f32;
    return;
  }
  GemmBatch parts(b.transA, b.transB);
  BlockBatch red;
  // partial results live in this recorder's arena for its lifetime
  for (const GemmProblem& p : b.probs) {
    const int64_t K = width(p);
    const int64_t nparts = nparts_of(p);
    if (nparts <= 1) {
      parts.probs.push_back(p);
      parts.probs.back().term_begin = (int)parts.terms.size();
      for (int q = p.term_begin; q < p.term_end; ++q) parts.terms.push_back(b.terms[q]);
      parts.probs.back().term_end = (int)parts.terms.size();
      parts.max_m = std::max(parts.max_m, p.m);
      parts.max_n = std::max(parts.max_n, p.n);
      continue;
    }
    red.add(p.C, p.m, p.n, p.ldc, p.beta);
    int q = p.term_begin;
    int64_t off = 0;  // columns of term q already assigned
    for (int64_t part = 0; part < nparts; ++part) {
      int64_t want = K * (part + 1) / nparts - K * part / nparts;
      double* dst = a.get_n<double>((size_t)p.m * p.n);
      parts.add(dst, p.m, p.n, p.m, 0.0, 1.0);
      while (want > 0) {
        const GemmTerm& g = b.terms[q];
        const int64_t take = std::min<int64_t>(want, g.k - off);
        GemmTerm t = g;
        const int64_t acs = b.transA ? 1 : g.lda, bcs = b.transB ? g.ldb : 1;
        t.A = g.A + acs * off;
        t.B = g.B + bcs * off;
        t.k = (int)take;
        parts.terms.push_back(t);
        want -= take;
        off += take;
        if (off == g.k) {
          ++q;
          off = 0;
        }
      }
      parts.probs.back().term_end = (int)parts.terms.size();
      red.term(dst, p.m, p.alpha);
    }
  }
  if (symm_form(parts)) {
    gemm_symm(a, s, parts, bytes);
  } else {
    recs.push_back({0, keep(a, s, parts.probs), keep(a, s, parts.terms), (int)parts.probs.size(),
                    parts.max_m, parts.max_n, parts.transA, parts.transB, bytes, -1});
    recs.back().max_k = std::max(b.max_k, 1);
  }
  block(a, s, red);
}

// Symmetric-pair product: the rows' terms are cut into parts of about
// kSplitBytes of A (at column granularity) and written as SymProblems whose
// row results go to per-part buffers; the mirrored products A^T x go to
// per-row regions [row tile][mirrored columns x n].  A block launch then forms
// every output row as the sum, in a fixed order, of its own parts and of the
// mirrored products addressed to it.
void Recorder::symv(Arena& a, hipStream_t s, const std::vector<SymRow>& rows, int n, double beta,
                    bool a_f32, double split_bytes) {
  if (split_bytes <= 0) split_bytes = kSplitBytes;
  // the terms' A pointers address FP64 or (a_f32) FP32 elements
  const int64_t esz = a_f32 ? 4 : 8;
  auto a_at = [esz](const double* A, int64_t elems) {
    return (const double*)((const char*)A + esz * elems);
  };
  if (rows.empty() || n <= 0) return;
  int max_m = 0;
  for (const SymRow& R : rows) max_m = std::max(max_m, R.m);
  if (max_m == 0) return;
  const int tile = symv_row_tile(max_m, n);
  std::vector<SymProblem> probs;
  std::vector<SymTerm> terms;
  // contributions to each row's output, in order: (source, leading dimension)
  std::vector<std::vector<std::pair<const double*, int>>> contrib(rows.size());
  double bytes = 0;
  std::vector<std::pair<const double*, const double*>> bset;
  for (size_t i = 0; i < rows.size(); ++i) {
    const SymRow& R = rows[i];
    if (R.m <= 0) continue;
    // merge adjacent terms that continue each other in A and B (and are both
    // mirrored or both not); mirrored terms take consecutive columns of P
    struct MT { const double* A; const double* B; int lda, ldb, k; bool mir; std::vector<std::pair<int, int>> tgt; };
    std::vector<MT> mt;
    int64_t kmir = 0;
    for (const SymRow::Term& t : R.terms) {
      if (t.k <= 0) continue;
      const bool mir = t.mirror >= 0;
      if (!mt.empty()) {
        MT& q = mt.back();
        if (q.mir == mir && q.lda == t.lda && (q.ldb == t.ldb || n == 1) && t.A == a_at(q.A, (int64_t)q.lda * q.k) &&
            t.B == q.B + q.k) {
          if (mir) q.tgt.push_back({t.mirror, t.k});
          q.k += t.k;
          if (mir) kmir += t.k;
          continue;
        }
      }
      MT m{t.A, t.B, t.lda, t.ldb, t.k, mir, {}};
      if (mir) {
        m.tgt.push_back({t.mirror, t.k});
        kmir += t.k;
      }
      mt.push_back(m);
    }
    const int tiles = ceil_div(R.m, tile);
    double* pb = kmir > 0 ? a.get_n<double>((size_t)tiles * kmir * n) : nullptr;
    // P column of every merged term; mirrored products addressed to their rows
    std::vector<int64_t> pcol(mt.size(), -1);
    {
      int64_t c = 0;
      for (size_t q = 0; q < mt.size(); ++q) {
        if (!mt[q].mir) continue;
        pcol[q] = c;
        for (const auto& tg : mt[q].tgt) {
          for (int r = 0; r < tiles; ++r)
            contrib[tg.first].push_back({pb + (int64_t)r * kmir * n + c, (int)kmir});
          c += tg.second;
        }
      }
    }
    int64_t K = 0;
    for (const MT& q : mt) K += q.k;
    const int64_t nparts =
        K == 0 ? 1 : std::max<int64_t>(1, std::min<int64_t>(K, (int64_t)std::ceil(8.0 * R.m * K / split_bytes)));
    size_t q = 0;
    int64_t off = 0;
    for (int64_t part = 0; part < nparts; ++part) {
      int64_t want = K * (part + 1) / nparts - K * part / nparts;
      double* dst = a.get_n<double>((size_t)R.m * n);
      SymProblem P{};
      P.C = dst;
      P.X = R.x;
      P.ptile = kmir * n;
      P.m = R.m;
      P.n = n;
      P.ldc = R.m;
      P.ldx = R.ldx;
      P.ldp = (int)std::max<int64_t>(kmir, 1);
      P.term_begin = (int)terms.size();
      P.alpha = 1.0;
      P.beta = 0.0;
      while (want > 0) {
        const MT& g = mt[q];
        const int64_t take = std::min<int64_t>(want, g.k - off);
        // the 5-16 column kernel addresses a term through 32-bit buffer ranges
        SPD_REQUIRE(n <= 4 || (esz * (int64_t)g.lda * take < (1ll << 31) &&
                               8 * ((int64_t)(n - 1) * g.ldb + take) < (1ll << 31)),
                    SPD_E_INVALID, "symmetric-pair term above 2 GiB of addressed bytes");
        SymTerm t{};
        t.A = a_at(g.A, (int64_t)g.lda * off);
        t.B = g.B + off;
        t.P = g.mir ? pb + pcol[q] + off : nullptr;
        t.scale = 1.0;
        t.k = (int)take;
        t.lda = g.lda;
        t.ldb = g.ldb;
        terms.push_back(t);
        want -= take;
        off += take;
        if (off == g.k) {
          ++q;
          off = 0;
        }
      }
      P.term_end = (int)terms.size();
      probs.push_back(P);
      contrib[i].insert(contrib[i].begin() + part, {dst, R.m});
    }
    // algorithmic bytes: every block once, own rows, B ranges once, row and mirrored results
    for (const MT& g : mt) {
      bytes += (double)esz * R.m * g.k;
      for (int j = 0; j < n; ++j) bset.push_back({g.B + (int64_t)j * g.ldb, g.B + (int64_t)j * g.ldb + g.k});
    }
    bytes += 8.0 * R.m * n * 2.0 + 8.0 * tiles * kmir * n;
  }
  std::sort(bset.begin(), bset.end());
  const double* end = nullptr;
  for (const auto& r : bset) {
    const double* lo = (end && r.first < end) ? end : r.first;
    if (r.second > lo) bytes += 8.0 * (double)(r.second - lo);
    if (!end || r.second > end) end = r.second;
  }
  if (terms.empty()) terms.push_back(SymTerm{});
  recs.push_back({3, keep(a, s, probs), keep(a, s, terms), (int)probs.size(), max_m, n, 0, 0, bytes, -1});
  recs.back().a_f32 = a_f32 ? 1 : 0;
  BlockBatch red;
  for (size_t i = 0; i < rows.size(); ++i) {
    const SymRow& R = rows[i];
    if (R.m <= 0) continue;
    red.add(R.y, R.m, n, R.ldy, beta);
    for (const auto& c : contrib[i]) red.term(c.first, c.second, 1.0);
  }
  block(a, s, red);
}

void Recorder::block(Arena& a, hipStream_t s, const BlockBatch& b) {
  if (b.probs.empty() || b.max_m == 0 || b.max_n == 0) return;
  std::vector<BlockProblem> p = b.probs;
  const std::vector<int> tl = block_tiles(p, b.max_n);
  if (tl.empty()) return;
  std::vector<BlockTerm> t = b.terms;
  if (t.empty()) t.push_back(BlockTerm{});
  recs.push_back({1, keep(a, s, p), keep(a, s, t), (int)p.size(), b.max_m, b.max_n, 0, 0, 0.0, -1});
  recs.back().tiles = (const int*)keep(a, s, tl);
  recs.back().ntiles = (int)tl.size();
}

void Recorder::trsm(Arena& a, hipStream_t s, const TrsmBatch& b, int trans) {
  if (b.probs.empty()) return;
  recs.push_back({2, keep(a, s, b.probs), nullptr, (int)b.probs.size(), b.max_n, b.max_nrhs, trans,
                  0, 0.0, -1});
}

void Recorder::replay(hipStream_t s) const {
  for (const LaunchRec& r : recs) {
    if (r.type == 0)
      launch_gemm(s, (const GemmProblem*)r.probs, (const GemmTerm*)r.terms, r.nprob, r.max_m,
                  r.max_n, r.transA, r.transB, r.max_k, r.a_f32);
    else if (r.type == 1)
      launch_block(s, (const BlockProblem*)r.probs, (const BlockTerm*)r.terms, r.tiles, r.ntiles,
                   r.max_n);
    else if (r.type == 3)
      launch_symv(s, (const SymProblem*)r.probs, (const SymTerm*)r.terms, r.nprob, r.max_m, r.max_n,
                  r.cap, r.a_f32, r.mir);
    else
      launch_trsm(s, (const TrsmProblem*)r.probs, r.nprob, r.max_m, r.max_n, r.transA, 0);
  }
}

}  // namespace spd
