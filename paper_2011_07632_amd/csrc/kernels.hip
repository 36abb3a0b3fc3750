// Device kernels of the spdhss library (gfx950, FP64).
//
// Every kernel takes an array of per-problem descriptors so that one launch
// covers all nodes (or node pairs) of a tree level: the level-parallel axis of
// the construction (all blocks of one level can be scaled and compressed
// independently, Section 1).
#include "common.h"

#include <algorithm>

#include <cmath>
#include <type_traits>

namespace spd {

// Global-memory pointer (global_load instead of flat_load), and a pointer to
// memory that no workgroup writes while the kernel runs (the compiler may then
// read wave-uniform addresses through the scalar cache).
typedef const double __attribute__((address_space(1))) gdouble;
typedef const double __attribute__((address_space(4))) rdouble;

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ reductions --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off, 64);
  }
}

// argmax with ties to the lowest index; every lane gets the result
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// ------------------------------------------------------------------- GEMM --
// Grouped GEMM on FP64 MFMA (v_mfma_f64_16x16x4f64).  One workgroup computes a
// BM x BN tile of one problem, summing over all of the problem's terms in
// order (deterministic).  Four waves tile the block as (BM/WM) x (BN/WN).
// Operand layout of the 16x16x4 f64 MFMA: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result element v of lane l is D[l/16 + 4*v][l%16].
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm(const GemmProblem* __restrict__ probs,
                                              const GemmTerm* __restrict__ terms,
                                              int tiles_max, int transA, int transB) {
  constexpr int BK = 16;
  constexpr int NWM = BM / WM;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BK * BN / 256;  // elements each thread stages
  static_assert((BM / WM) * (BN / WN) == 4, "four waves");
  static_assert(LA * 256 == BM * BK && LB * 256 == BK * BN, "whole tiles per thread");
  // Two LDS buffers: the (term, k) step after the current one is fetched into
  // registers while the current one is multiplied, then stored into the other
  // buffer, so one barrier per step separates the two.  Steps run in the same
  // order as a single-buffered loop, so the sums are the same bit for bit.
  __shared__ double As[2][BK][BM + 1];
  __shared__ double Bs[2][BK][BN + 1];
  const int p = blockIdx.x / tiles_max, tile = blockIdx.x % tiles_max;
  const GemmProblem P = probs[p];
  const int tm = (P.m + BM - 1) / BM, tn = (P.n + BN - 1) / BN;
  if (tile >= tm * tn) return;
  const int i0 = (tile % tm) * BM, j0 = (tile / tm) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % NWM, wn = wave / NWM;
  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // the (term, k0) steps in order; t == term_end marks the end
  int t = P.term_begin, k0 = 0;
  while (t < P.term_end && terms[t].k <= 0) ++t;
  if (t >= P.term_end) goto store;
  {
    double ra[LA], rb[LB];
    auto fetch = [&](int tt, int kk0) {
      const GemmTerm T = terms[tt];
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + 256 * q;
        int i, kk;
        if (!transA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
        const int gi = i0 + i, gk = kk0 + kk;
        double v = 0.0;
        if (gi < P.m && gk < T.k)
          v = T.scale * (transA ? T.A[gk + (int64_t)gi * T.lda] : T.A[gi + (int64_t)gk * T.lda]);
        ra[q] = v;
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + 256 * q;
        int j, kk;
        if (!transB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
        const int gj = j0 + j, gk = kk0 + kk;
        double v = 0.0;
        if (gj < P.n && gk < T.k)
          v = transB ? T.B[gj + (int64_t)gk * T.ldb] : T.B[gk + (int64_t)gj * T.ldb];
        rb[q] = v;
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int e = tid + 256 * q;
        int i, kk;
        if (!transA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
        As[buf][kk][i] = ra[q];
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int e = tid + 256 * q;
        int j, kk;
        if (!transB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
        Bs[buf][kk][j] = rb[q];
      }
    };
    auto advance = [&](int& tt, int& kk0) {
      kk0 += BK;
      if (kk0 >= terms[tt].k) {
        kk0 = 0;
        ++tt;
        while (tt < P.term_end && terms[tt].k <= 0) ++tt;
      }
    };
    fetch(t, k0);
    stash(0);
    __syncthreads();
    int cur = 0;
    for (;;) {
      int tn_ = t, kn = k0;
      advance(tn_, kn);
      const bool more = tn_ < P.term_end;
      if (more) fetch(tn_, kn);
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        double af[FM], bf[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) af[a] = As[cur][ks + (lane >> 4)][wm * WM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b) bf[b] = Bs[cur][ks + (lane >> 4)][wn * WN + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      if (!more) break;
      stash(cur ^ 1);
      __syncthreads();
      cur ^= 1;
      t = tn_;
      k0 = kn;
    }
  }
store:
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wm * WM + a * 16 + (lane >> 4) + 4 * v;
        const int j = j0 + wn * WN + b * 16 + (lane & 15);
        if (i < P.m && j < P.n) {
          double* c = P.C + i + (int64_t)j * P.ldc;
          double val = P.alpha * acc[a][b][v];
          if (P.beta != 0.0) val += P.beta * (*c);
          *c = val;
        }
      }
}

// Sum over the 64 lanes of V values at once (V a power of two, at most 64):
// at each of the first log2(V) exchange steps a lane keeps half of its values
// and trades the other half with its partner, then the last steps are a plain
// butterfly.  Lane l returns the total of value index
// sum_s bit(l, 5 - s) * V / 2^(s+1); every lane whose low 6 - log2(V) bits are
// zero holds a distinct index.  The order of additions is fixed.
template <int V>
__device__ __forceinline__ double wave_sum_many(double (&v)[V], int lane) {
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int d = 32 >> s;
    constexpr int kV = V;
    const int nv = kV >> s;
    if (nv >= 2) {
      const int h = nv / 2;
      const bool up = (lane & d) != 0;
#pragma unroll
      for (int q = 0; q < kV / 2; ++q) {
        if (q < h) {
          const double give = up ? v[q] : v[q + h];
          const double keep = up ? v[q + h] : v[q];
          v[q] = keep + __shfl_xor(give, d);
        }
      }
    } else {
      v[0] += __shfl_xor(v[0], d);
    }
  }
  return v[0];
}

template <int V>
__device__ __forceinline__ int wave_sum_index(int lane) {
  int idx = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s)
    if ((V >> s) >= 2 && (lane & (32 >> s))) idx += V >> (s + 1);
  return idx;
}

template <int V>
__device__ __forceinline__ bool wave_sum_holder(int lane) {
  int hs = 0;
#pragma unroll
  for (int s = 0; s < 6; ++s)
    if ((V >> s) >= 2) ++hs;
  return (lane & ((64 >> hs) - 1)) == 0;
}

// Skinny grouped GEMM for at most 4 right-hand columns: bandwidth-bound
// streaming of A.  A workgroup of NW waves owns up to 64*RG rows of one
// problem (lane l of row group g owns row i0 + 64 g + l), so every column of a
// block is read by one workgroup only: no cache line is fetched by two
// workgroups, which may sit on different XCDs with separate L2s.  The waves
// take the columns of each term in runs of U adjacent columns (a step of the
// workgroup covers NW*U adjacent columns, wave w reading run w), so a cache
// line shared by adjacent columns is read within one wave's step; all loads
// of a step are issued back to back; in the
// last step of a term, out-of-range columns load from an in-range address and
// are zeroed afterwards.  Small launches use 16 waves per workgroup so that
// each wave's chain of dependent memory round trips stays short.  The NW
// partial sums are added pairwise in a fixed tree through LDS, so results are
// deterministic.  The wave index is made wave-uniform so that the B entries,
// the same for every lane, come from scalar loads.  A is read with
// non-temporal loads: it is streamed once per launch.  Long term lists are
// split into several problems by the host (see Recorder::gemm).
template <int NC, int RG, int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_skinny(const GemmProblem* __restrict__ probs,
                                                          const GemmTerm* __restrict__ terms,
                                                          int tiles_max, int transA, int transB) {
  constexpr int U = (RG == 1) ? 8 : (RG == 2 ? 6 : 4);
  constexpr int TR = 64 * RG;
  __shared__ double red[NW / 2][TR][NC];
  const int p = blockIdx.x / tiles_max, tile = blockIdx.x % tiles_max;
  const GemmProblem P = probs[p];
  const int i0 = tile * TR;
  if (i0 >= P.m || P.n <= 0) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = P.n;
  int jc[NC];  // right-hand columns past n read column 0 and are never stored
#pragma unroll
  for (int j = 0; j < NC; ++j) jc[j] = j < n ? j : 0;
  int rowc[RG];  // rows past the problem read row i0 and are never stored
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int r = i0 + 64 * g + lane;
    rowc[g] = r < P.m ? r : i0;
  }
  double acc[RG][NC];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[g][c] = 0.0;
  for (int t = P.term_begin; t < P.term_end; ++t) {
    const GemmTerm T = terms[t];
    const int K = T.k;
    if (w * U >= K) continue;
    const int64_t lda = T.lda, ldb = T.ldb;
    const double sc = T.scale;
    // op(A)(r, c) = transA ? A[c + r lda] : A[r + c lda];  op(B)(c, j) likewise
    const int64_t acs = transA ? 1 : lda, ars = transA ? lda : 1;
    const int64_t bcs = transB ? ldb : 1, bjs = transB ? 1 : ldb;
    const int64_t astep = acs, bstep = bcs;
    gdouble* ap[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) ap[g] = (gdouble*)T.A + (int64_t)rowc[g] * ars + (int64_t)w * U * acs;
    rdouble* bp = (rdouble*)T.B + (int64_t)w * U * bcs;
    // gathered B: row c of B is row bidx[c] of T.B
    const int __attribute__((address_space(4)))* bix =
        T.bidx ? (const int __attribute__((address_space(4)))*)T.bidx + w * U : nullptr;
    rdouble* B0 = (rdouble*)T.B;
    int c = w * U;  // this wave's next column; a step reads columns c, ..., c + U - 1
    for (; c + U - 1 < K; c += NW * U) {
      double a[U][RG], b[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int g = 0; g < RG; ++g) a[u][g] = __builtin_nontemporal_load(&ap[g][u * astep]);
        if (bix) {
          const int64_t row = bix[u];
#pragma unroll
          for (int j = 0; j < NC; ++j) b[u][j] = B0[row + jc[j] * bjs];
        } else {
#pragma unroll
          for (int j = 0; j < NC; ++j) b[u][j] = bp[u * bstep + jc[j] * bjs];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const double av = sc * a[u][g];
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[g][j] += av * b[u][j];
        }
#pragma unroll
      for (int g = 0; g < RG; ++g) ap[g] += NW * U * astep;
      bp += NW * U * bstep;
      if (bix) bix += U * NW;
    }
    if (c < K) {  // fewer than U columns left: clamp to column c, zero afterwards
      double a[U][RG], b[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t uu = (c + u < K) ? u : 0;
#pragma unroll
        for (int g = 0; g < RG; ++g) a[u][g] = (double)__builtin_nontemporal_load(&ap[g][uu * astep]);
        if (bix) {
          const int64_t row = bix[uu];
#pragma unroll
          for (int j = 0; j < NC; ++j) b[u][j] = B0[row + jc[j] * bjs];
        } else {
#pragma unroll
          for (int j = 0; j < NC; ++j) b[u][j] = bp[uu * bstep + jc[j] * bjs];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool cok = c + u < K;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const double av = cok ? sc * a[u][g] : 0.0;
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[g][j] += av * (cok ? b[u][j] : 0.0);
        }
      }
    }
  }
  // pairwise tree over the waves: at width h, wave w < h adds wave w + h
#pragma unroll
  for (int h = NW / 2; h >= 1; h /= 2) {
    if (w >= h && w < 2 * h) {
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int j = 0; j < NC; ++j) red[w - h][64 * g + lane][j] = acc[g][j];
    }
    __syncthreads();
    if (w < h) {
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[g][j] += red[w][64 * g + lane][j];
    }
    __syncthreads();
  }
  if (w == 0) {
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int r = i0 + 64 * g + lane;
      if (r >= P.m) continue;
      const int64_t rc = P.cidx ? P.cidx[r] : r;
      const int64_t rd = P.didx ? P.didx[r] : r;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (j >= n) continue;
        double* cp = P.C + rc + (int64_t)j * P.ldc;
        double val = P.alpha * acc[g][j];
        if (P.beta != 0.0) val += P.beta * (*cp);
        if (P.D) val += P.D[rd + (int64_t)j * P.ldd];
        *cp = val;
      }
    }
  }
}

template <int NC, int NW>
static void launch_skinny_nw(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                             int max_m, int transA, int transB) {
  if (max_m <= 64) {
    hipLaunchKernelGGL((k_gemm_skinny<NC, 1, NW>), dim3((unsigned)nprob), dim3(64 * NW), 0, s, d_p,
                       d_t, 1, transA, transB);
  } else if (max_m <= 128) {
    hipLaunchKernelGGL((k_gemm_skinny<NC, 2, NW>), dim3((unsigned)nprob), dim3(64 * NW), 0, s, d_p,
                       d_t, 1, transA, transB);
  } else {
    const int tiles = ceil_div(max_m, 256);
    hipLaunchKernelGGL((k_gemm_skinny<NC, 4, NW>), dim3((unsigned)nprob * tiles), dim3(64 * NW), 0,
                       s, d_p, d_t, tiles, transA, transB);
  }
}

// Dot-form product for at most 4 right-hand columns with A stored transposed
// (op(A) = A^T, A stored K x m): output row r is column r of A dotted with B,
// so lanes run along the contiguous K dimension.  Each wave owns U output rows
// and keeps U x KU loads in flight (KU chunks of 64 along K), which covers
// K <= 64 KU in one round trip; the U x NC lane sums are added across the wave
// with wave_sum_many and stored by the holding lanes.  Waves are independent
// (no LDS, no barrier).  This is the kernel for the small per-level products
// of the solve sweeps and of the H^2 interpolation, whose cost is the chain of
// dependent memory round trips rather than bandwidth.
template <int NC, int U, int KU, typename TA>
__global__ __launch_bounds__(256) void k_gemv_t(const GemmProblem* __restrict__ probs,
                                               const GemmTerm* __restrict__ terms, int tiles_max,
                                               int transB) {
  constexpr int V = U * NC;
  const int p = blockIdx.x / tiles_max, tile = blockIdx.x % tiles_max;
  const GemmProblem P = probs[p];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r0 = (tile * 4 + w) * U;  // this wave's first output row
  if (r0 >= P.m || P.n <= 0) return;
  const int n = P.n;
  int jc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) jc[j] = j < n ? j : 0;
  int rc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) rc[u] = min(r0 + u, P.m - 1);
  double acc[U][NC];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[u][j] = 0.0;
  for (int t = P.term_begin; t < P.term_end; ++t) {
    const GemmTerm T = terms[t];
    const int K = T.k;
    const int64_t lda = T.lda, ldb = T.ldb;
    const double sc = T.scale;
    const TA __attribute__((address_space(1)))* A = (const TA __attribute__((address_space(1)))*)T.A;
    gdouble* B = (gdouble*)T.B;
    const int* __restrict__ bidx = T.bidx;
    // op(B)(k, j) = transB ? B[j + k ldb] : B[k + j ldb]
    const int64_t bks = transB ? ldb : 1, bjs = transB ? 1 : ldb;
    for (int k0 = 0; k0 < K; k0 += 64 * KU) {
      double a[U][KU], b[KU][NC];
#pragma unroll
      for (int q = 0; q < KU; ++q) {
        const int k = k0 + 64 * q + lane;
        const int kc = k < K ? k : K - 1;
        const int64_t brow = bidx ? bidx[kc] : kc;
#pragma unroll
        for (int j = 0; j < NC; ++j) b[q][j] = k < K ? B[brow * bks + jc[j] * bjs] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
          a[u][q] = (double)__builtin_nontemporal_load(&A[kc + (int64_t)rc[u] * lda]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < KU; ++q)
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[u][j] += sc * a[u][q] * b[q][j];
    }
  }
  double v[V];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int j = 0; j < NC; ++j) v[u * NC + j] = acc[u][j];
  const double tot = wave_sum_many<V>(v, lane);
  const int idx = wave_sum_index<V>(lane);
  const int r = r0 + idx / NC, j = idx % NC;
  if (wave_sum_holder<V>(lane) && r < P.m && j < n) {
    const int64_t row = P.cidx ? P.cidx[r] : r;
    double* cp = P.C + row + (int64_t)j * P.ldc;
    double val = P.alpha * tot;
    if (P.beta != 0.0) val += P.beta * (*cp);
    if (P.D) val += P.D[(P.didx ? P.didx[r] : r) + (int64_t)j * P.ldd];
    *cp = val;
  }
}

// rows per workgroup of the dot-form kernel: 4 waves of U rows
template <int NC, int U, typename TA>
static void launch_gemv_t_u(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                            int max_m, int max_k, int transB) {
  const int tiles = ceil_div(max_m, 4 * U);
  const dim3 grid((unsigned)nprob * tiles);
  if (max_k <= 256)
    hipLaunchKernelGGL((k_gemv_t<NC, U, 4, TA>), grid, dim3(256), 0, s, d_p, d_t, tiles, transB);
  else
    hipLaunchKernelGGL((k_gemv_t<NC, U, 8, TA>), grid, dim3(256), 0, s, d_p, d_t, tiles, transB);
}

template <typename TA>
static void launch_gemv_t_ta(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                             int max_m, int max_n, int max_k, int transB) {
  if (max_n == 1) launch_gemv_t_u<1, 4, TA>(s, d_p, d_t, nprob, max_m, max_k, transB);
  else if (max_n == 2) launch_gemv_t_u<2, 2, TA>(s, d_p, d_t, nprob, max_m, max_k, transB);
  else launch_gemv_t_u<4, 1, TA>(s, d_p, d_t, nprob, max_m, max_k, transB);
}

void launch_gemv_t(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob, int max_m,
                   int max_n, int max_k, int transB, int a_f32) {
  if (nprob <= 0 || max_m <= 0 || max_n <= 0) return;
  if (max_n > 4) throw Error(SPD_E_INVALID, "dot-form product supports at most 4 columns");
  if (a_f32) launch_gemv_t_ta<float>(s, d_p, d_t, nprob, max_m, max_n, max_k, transB);
  else launch_gemv_t_ta<double>(s, d_p, d_t, nprob, max_m, max_n, max_k, transB);
  SPD_HIP(hipGetLastError());
}

// FP32 copies of FP64 arrays: one descriptor per array, grid over (array, chunk)
__global__ __launch_bounds__(256) void k_to_f32(const CvtProblem* __restrict__ probs, int chunks) {
  const CvtProblem P = probs[blockIdx.x / chunks];
  const int64_t chunk = (P.n + chunks - 1) / chunks;
  const int64_t lo = (blockIdx.x % chunks) * chunk, hi = min(P.n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) P.dst[i] = (float)P.src[i];
}
void launch_to_f32(hipStream_t s, const CvtProblem* d_p, int nprob) {
  if (nprob <= 0) return;
  constexpr int chunks = 16;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)nprob * chunks), dim3(256), 0, s, d_p, chunks);
  SPD_HIP(hipGetLastError());
}

// Workgroups below which a launch uses 16 waves per workgroup (two per SIMD
// of every CU at 4 waves).
static constexpr int kSkinnyWide = 2048;

template <int NC>
static void launch_skinny(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                          int max_m, int transA, int transB) {
  const int64_t blocks = (int64_t)nprob * ceil_div(max_m, 256);
  if (blocks < kSkinnyWide)
    launch_skinny_nw<NC, 16>(s, d_p, d_t, nprob, max_m, transA, transB);
  else
    launch_skinny_nw<NC, 4>(s, d_p, d_t, nprob, max_m, transA, transB);
}

// Symmetric-pair product (see SymProblem).  The row results follow the
// streaming GEMV above (a workgroup owns the problem's rows of a row tile, the
// waves take runs of U adjacent columns).  For a term with P set, each
// loaded column a is also dotted with the problem's own rows X: the lane
// partial sums of the U columns of a step are added across the wave by
// wave_sum_many and stored by the holding lanes, so every off-diagonal block
// is read once for both of its products.
template <int NC, int RG, int NW, typename TA>
__global__ __launch_bounds__(64 * NW) void k_symv(const SymProblem* __restrict__ probs,
                                                   const SymTerm* __restrict__ terms, int tiles_max,
                                                   int nwork, int nprob) {
  constexpr int U = (RG == 1) ? 8 : 4;
  constexpr int V = U * NC;
  constexpr int TR = 64 * RG;
  __shared__ double red[NW / 2][TR][NC];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // a capped grid walks the (problem, row tile) items with a stride.  XCD-aware
  // decode: items are dealt to the 8 XCDs round-robin (item & 7), and the row
  // tiles of one problem take consecutive slots of the same XCD, so the cache
  // line they share at their boundary is fetched once into that XCD's L2.
  for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
  const int x8 = item & 7, rest = item >> 3;
  const int tile = rest % tiles_max, p = (rest / tiles_max) * 8 + x8;
  if (p >= nprob) continue;
  const SymProblem P = probs[p];
  const int i0 = tile * TR;
  if (i0 >= P.m || P.n <= 0) continue;
  const int n = P.n;
  int jc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) jc[j] = j < n ? j : 0;
  int rowc[RG];
  double xi[RG][NC];  // the problem's own input rows; zero past the last row
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int r = i0 + 64 * g + lane;
    const bool ok = r < P.m;
    rowc[g] = ok ? r : i0;
#pragma unroll
    for (int j = 0; j < NC; ++j) xi[g][j] = ok ? P.X[rowc[g] + (int64_t)jc[j] * P.ldx] : 0.0;
  }
  double acc[RG][NC];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[g][j] = 0.0;
  const int vidx = wave_sum_index<V>(lane);
  const bool holder = wave_sum_holder<V>(lane);
  const int hu = vidx / NC, hj = vidx % NC;  // the (column step, right-hand column) a holder stores
  for (int t = P.term_begin; t < P.term_end; ++t) {
    const SymTerm T = terms[t];
    const int K = T.k;
    if (w * U >= K) continue;
    const int64_t lda = T.lda, ldb = T.ldb;
    const double sc = T.scale;
    const int64_t astep = lda;
    // A in FP64 or (mixed-precision product) FP32, widened to FP64 on load
    typedef const TA __attribute__((address_space(1))) gta;
    gta* ap[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) ap[g] = (gta*)T.A + rowc[g] + (int64_t)w * U * lda;
    rdouble* bp = (rdouble*)T.B + w * U;
    double* pt = T.P ? T.P + (int64_t)tile * P.ptile : nullptr;
    for (int c = w * U; c < K; c += NW * U) {
      double a[U][RG], b[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t uu = (c + u < K) ? u : 0;
#pragma unroll
        for (int g = 0; g < RG; ++g) a[u][g] = (double)__builtin_nontemporal_load(&ap[g][uu * astep]);
#pragma unroll
        for (int j = 0; j < NC; ++j) b[u][j] = bp[uu + jc[j] * ldb];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool cok = c + u < K;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const double av = cok ? sc * a[u][g] : 0.0;
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[g][j] += av * (cok ? b[u][j] : 0.0);
        }
      }
      if (pt) {
        double v[V];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            double sum = 0.0;
#pragma unroll
            for (int g = 0; g < RG; ++g) sum += a[u][g] * xi[g][j];
            v[u * NC + j] = sum;
          }
        const double tot = wave_sum_many<V>(v, lane);
        const int col = c + hu;
        if (holder && col < K && hj < n) pt[col + (int64_t)hj * P.ldp] = sc * tot;
      }
#pragma unroll
      for (int g = 0; g < RG; ++g) ap[g] += NW * U * lda;
      bp += U * NW;
    }
  }
#pragma unroll
  for (int h = NW / 2; h >= 1; h /= 2) {
    if (w >= h && w < 2 * h) {
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int j = 0; j < NC; ++j) red[w - h][64 * g + lane][j] = acc[g][j];
    }
    __syncthreads();
    if (w < h) {
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[g][j] += red[w][64 * g + lane][j];
    }
    __syncthreads();
  }
  if (w == 0) {
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int r = i0 + 64 * g + lane;
      if (r >= P.m) continue;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (j >= n) continue;
        double* cp = P.C + r + (int64_t)j * P.ldc;
        double val = P.alpha * acc[g][j];
        if (P.beta != 0.0) val += P.beta * (*cp);
        *cp = val;
      }
    }
  }
  }
}

int symv_row_tile(int max_m, int ncols) {
  if (ncols > 4) return 256;
  return max_m <= 64 ? 64 : (max_m <= 128 ? 128 : 256);
}

template <int NC, int NW, typename TA>
static void launch_symv_nw(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob,
                           int max_m, int cap) {
  const int tiles = max_m <= 128 ? 1 : ceil_div(max_m, 256);
  const int nwork = ceil_div(nprob, 8) * 8 * tiles;  // problems padded to a multiple of 8 (XCDs)
  const int capped = cap > 0 ? std::max(8, cap / 8 * 8) : nwork;  // keep item & 7 == block & 7
  const dim3 grid((unsigned)std::min(capped, nwork));
  if (max_m <= 64)
    hipLaunchKernelGGL((k_symv<NC, 1, NW, TA>), grid, dim3(64 * NW), 0, s, d_p, d_t, 1, nwork, nprob);
  else if (max_m <= 128)
    hipLaunchKernelGGL((k_symv<NC, 2, NW, TA>), grid, dim3(64 * NW), 0, s, d_p, d_t, 1, nwork, nprob);
  else
    hipLaunchKernelGGL((k_symv<NC, 4, NW, TA>), grid, dim3(64 * NW), 0, s, d_p, d_t, tiles, nwork,
                       nprob);
}

// 16-wave workgroups for small launches with one right-hand column only (more
// columns would not fit the register budget of a 1024-thread workgroup).
template <int NC, typename TA>
static void launch_symv_nc(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob,
                           int max_m, int cap) {
  const int64_t blocks = (int64_t)nprob * ceil_div(max_m, 256);
  if (NC == 1 && blocks < kSkinnyWide && cap <= 0)
    launch_symv_nw<NC, 16, TA>(s, d_p, d_t, nprob, max_m, cap);
  else
    launch_symv_nw<NC, 4, TA>(s, d_p, d_t, nprob, max_m, cap);
}

template <typename TA>
static void launch_symv_ta(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob,
                           int max_m, int max_n, int cap) {
  if (max_n == 1) launch_symv_nc<1, TA>(s, d_p, d_t, nprob, max_m, cap);
  else if (max_n == 2) launch_symv_nc<2, TA>(s, d_p, d_t, nprob, max_m, cap);
  else launch_symv_nc<4, TA>(s, d_p, d_t, nprob, max_m, cap);
}

// Symmetric-pair product for 5 to 16 right-hand columns on FP64 MFMA
// (v_mfma_f64_16x16x4f64; lane l holds A[l%16][l/16] and B[l/16][l%16], and
// element v of the result D[l/16 + 4v][l%16]).  Same descriptors and outputs
// as k_symv: a work item is (problem, tile of up to 256 rows).  The tile's
// rows are cut into R strips of 64 (R = 1, 2 or 4, the fewest that cover
// them) and the four waves into R x G with G = 4 / R: wave (s, g) takes strip
// s and every G-th chunk of 16 columns starting at chunk g, so that short
// tiles keep all four waves on rows that exist.  Per chunk:
//   row sums:  C[rows] += A[rows, chunk] B[chunk, :]        (16 MFMAs)
//   mirrored:  P[chunk, :] = A[rows, chunk]^T X[rows, :]     (16 MFMAs per wave,
//              the R strips' parts summed in strip order through LDS)
// The mirrored product contracts over rows, so each wave transposes its
// 64 x 16 chunk through its own LDS slot before the second set of MFMAs.  The
// G groups' row sums are added in group order at the end of the item.  A
// operands are FP64, or FP32 copies (TA = float) widened to FP64 as they are
// loaded; B, X and all arithmetic stay FP64.
// Every block element is read from HBM once.  Columns past n are zero in the
// inputs and not written.
//
// A wave walks its chunks of all the item's terms as one sequence and loads
// the next chunk (of the same or the next term) while it multiplies the
// current one.  It waits for the current chunk's loads before it issues the
// next ones: the mirrored results are stored inside the loop, and with stores
// and loads both outstanding the wait for the older loads is a wait for
// everything, which would otherwise include the loads just issued.
// Descriptors read through the constant address space: uniform scalar loads
// (a generic pointer to memory that stores may reach gives vector loads).
// Buffer resource word 3 for raw (unswizzled, unformatted) buffer loads on
// gfx9-family parts, the nontemporal cache policy bit of a buffer load, and
// the s_waitcnt operand that waits for vmcnt = 0 only (expcnt 7, lgkmcnt 15).
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufNT = 2;
constexpr int kWaitVm0 = 0x0F70;
typedef const __attribute__((address_space(4))) SymProblem cSymProblem;
typedef const __attribute__((address_space(4))) SymTerm cSymTerm;
static __device__ inline SymProblem sym_problem(const SymProblem* p, int i) {
  const cSymProblem* c = (const cSymProblem*)p + i;
  SymProblem P;
  P.C = c->C;
  P.X = c->X;
  P.ptile = c->ptile;
  P.m = c->m;
  P.n = c->n;
  P.ldc = c->ldc;
  P.ldx = c->ldx;
  P.ldp = c->ldp;
  P.term_begin = c->term_begin;
  P.term_end = c->term_end;
  P.pad = 0;
  P.alpha = c->alpha;
  P.beta = c->beta;
  return P;
}
static __device__ inline SymTerm sym_term(const SymTerm* t, int i) {
  const cSymTerm* c = (const cSymTerm*)t + i;
  SymTerm T;
  T.A = c->A;
  T.B = c->B;
  T.P = c->P;
  T.scale = c->scale;
  T.k = c->k;
  T.lda = c->lda;
  T.ldb = c->ldb;
  T.pad = 0;
  return T;
}

// MIR = false: plain products (no term has a mirrored output), whose waves
// keep no mirrored state and make no transposes.
template <typename TA, bool MIR>
__device__ __forceinline__ void symm16_body(const SymProblem* __restrict__ probs,
                                            const SymTerm* __restrict__ terms, int tiles_max,
                                            int nwork, int nprob) {
  constexpr int ES = (int)sizeof(TA);  // bytes of an A element (FP64, or FP32 copies widened on load)
  __shared__ double tr[4][64][17];      // per-wave transpose slot; row-sum exchange between groups
  __shared__ double red[2][4][16][17];  // per-wave mirrored partials, two chunks in flight
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  int buf = 0;
  for (int item = blockIdx.x; item < nwork; item += gridDim.x) {
    const int x8 = item & 7, rest = item >> 3;
    const int tile = rest % tiles_max, p = (rest / tiles_max) * 8 + x8;
    if (p >= nprob) continue;
    const SymProblem P = sym_problem(probs, p);
    const int i0 = tile * 256;
    if (i0 >= P.m || P.n <= 0) continue;
    const int n = P.n, m = P.m;
    const int mt = min(256, m - i0);
    const int lgR = mt <= 64 ? 0 : (mt <= 128 ? 1 : 2);  // R = 1 << lgR strips
    const int R = 1 << lgR, G = 4 >> lgR;
    const int st = w & (R - 1), g = w >> lgR;
    const int r0 = i0 + 64 * st;  // this wave's first row
    // 16-row quads of this wave's strip that hold rows of the block (0 to 4;
    // uniform per wave): quads past the last row take no loads, MFMAs or
    // transposes
    const int nq = min(4, max(0, (m - r0 + 15) >> 4));
    const bool colok = lr < n;
    // the mirrored product's right operand: this wave's own input rows,
    // X[r0 + 4r + l/16][l%16] for row quads r = 0..15
    double xop[16];
    if constexpr (MIR) {
      gdouble* Xg = (gdouble*)P.X;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = r0 + 4 * r + lk;
        const double mk = (row < m && colok) ? 1.0 : 0.0;
        xop[r] = Xg[(row < m ? row : m - 1) + (int64_t)(colok ? lr : 0) * P.ldx] * mk;
      }
    }
    const int lrc = colok ? lr : 0;
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    // pending mirrored result of the last chunk: ov (per lane), its block,
    // first column and column count (uniform)
    double ov[4];
    bool pend = false;
    double* ppt = nullptr;
    int pc0 = 0, pK = 0;
    // the chunk sequence: term t, chunk c0 = 16 (it G + g), it < niter(t)
    struct Cur {
      const TA* A;
      const double* B;
      double* pt;
      int ldab, bext;  // A's column stride and B's extent from its first row, in bytes
      double sc;
      int K, niter, t, it;
      uint32_t va[4], vb;  // this lane's byte offsets in a chunk's first column
    };
    auto open = [&](int t, Cur& c) {  // first nonempty term at or after t; false at the end
      for (; t < P.term_end; ++t) {
        const SymTerm T = sym_term(terms, t);
        if (T.k <= 0) continue;
        c.A = (const TA*)T.A;
        c.B = T.B;
        c.pt = T.P ? T.P + (int64_t)tile * P.ptile : nullptr;
        c.ldab = ES * T.lda;
        c.bext = 8 * ((n - 1) * T.ldb + T.k);
        c.sc = T.scale;
        c.K = T.k;
        c.niter = (((T.k + 15) >> 4) + G - 1) >> (2 - lgR);
        c.t = t;
        c.it = 0;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) c.va[s4] = (uint32_t)ES * (uint32_t)(lk * T.lda + r0 + 16 * s4 + lr);
        c.vb = 8u * (uint32_t)(lk + lrc * T.ldb);
        return true;
      }
      return false;
    };
    // A chunk's operands: A[r0 + 16s + l%16][c0 + 4q + l/16] and
    // B[c0 + 4q + l/16][l%16], as buffer loads from the chunk's column c0 + 4q
    // whose range ends at the term's last column: the columns past K read
    // zeros (so do rows past the block's last element).  B's columns past K
    // are still zeroed when the chunk is multiplied, since the rows of B past
    // K belong to other data.  Nothing else needs a mask: rows past m meet
    // zero rows of X in the mirrored product and give row sums that are never
    // stored, and columns past K give mirrored entries that are never stored;
    // values of columns past n reach only outputs that are never stored.
    auto issue = [&](auto nqc, const Cur& c, int q, double (&ra)[4][4], double (&rb)[4]) {
      constexpr int NQ = decltype(nqc)::value;
      if constexpr (NQ == 0) return;
      const int col0 = 16 * (c.it * G + g) + 4 * q, rem = c.K - col0;
      const __amdgpu_buffer_rsrc_t sa = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(c.A + (int64_t)col0 * (c.ldab / ES)), (short)0, rem > 0 ? rem * c.ldab : 0, kBufWord3);
      const __amdgpu_buffer_rsrc_t sb = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(c.B + col0), (short)0, rem > 0 ? c.bext - 8 * col0 : 0, kBufWord3);
#pragma unroll
      for (int s4 = 0; s4 < NQ; ++s4) {
        if constexpr (ES == 8)
          ra[s4][q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(sa, c.va[s4], 0, kBufNT));
        else
          ra[s4][q] = (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sa, c.va[s4], 0, kBufNT));
      }
      rb[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(sb, c.vb, 0, 0));
    };
    auto load = [&](auto nqc, const Cur& c, double (&ra)[4][4], double (&rb)[4]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) issue(nqc, c, q, ra, rb);
    };
    // wait for every load issued so far (the current chunk's), before the
    // next chunk's loads are issued
    auto ready = [&]() {
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      __builtin_amdgcn_sched_barrier(0);
    };
    // one step: the loads of chunk c have arrived in (ca, cb); the loads of
    // the next chunk nx go out between the row-sum MFMAs of c, and so do the
    // LDS transposes of c
    auto process = [&](auto nqc, const Cur& c, const double (&ca)[4][4], const double (&cb)[4],
                       const Cur& nx, double (&na)[4][4], double (&nb)[4], bool more) {
      constexpr int NQ = decltype(nqc)::value;
      const int c0 = 16 * (c.it * G + g);
      double bs[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) bs[q] = (NQ > 0 && c0 + 4 * q + lk < c.K) ? c.sc * cb[q] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int s4 = 0; s4 < NQ; ++s4)
          acc[s4] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[s4][q], bs[q], acc[s4], 0, 0, 0);
        if (more) issue(nqc, nx, q, na, nb);
        if constexpr (MIR) {
#pragma unroll
          for (int s4 = 0; s4 < NQ; ++s4) tr[w][16 * s4 + lr][4 * q + lk] = ca[s4][q];
        }
      }
      // issue order per column quad: MFMAs alternating with the buffer loads
      // and LDS writes (scheduling-group masks: 0x008 MFMA, 0x020 vector
      // memory read, 0x200 LDS write)
      if constexpr (MIR && NQ == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
      } else if constexpr (NQ > 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int j = 0; j < NQ; ++j) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          }
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
          if constexpr (MIR) __builtin_amdgcn_sched_group_barrier(0x200, NQ, 0);
        }
      }
      if (!MIR || !c.pt) return;  // uniform across the workgroup (per term)
      // LDS-only ordering: the prefetched global loads of the next chunk
      // stay in flight (a full fence would wait for them)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      // four independent accumulation chains over the row quads
      d4 pa[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pa[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4 * NQ; ++r)
        pa[r & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[w][4 * r + lk][lr], xop[r], pa[r & 3], 0, 0, 0);
      // the chunk's mirrored result is stored after the next chunk's wait
      // (so that waiting for a chunk's loads never waits for a store just issued)
      pend = true;
      ppt = c.pt;
      pc0 = c0;
      pK = c.K;
      if (R == 1) {
        // one strip: the wave's own sums are the chunk's mirrored result
#pragma unroll
        for (int v = 0; v < 4; ++v) ov[v] = c.sc * ((pa[0][v] + pa[1][v]) + (pa[2][v] + pa[3][v]));
        return;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        red[buf][w][lk + 4 * v][lr] = (pa[0][v] + pa[1][v]) + (pa[2][v] + pa[3][v]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      // the group's 256 outputs, G = 256 / (64 R) per lane: output i is entry
      // e = 64 (st + R i) + lane, the R strips summed in order
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i >= G) break;
        const int e = 64 * (st + R * i) + lane;
        const int kk = e >> 4, cc = e & 15;
        double v = red[buf][g << lgR][kk][cc];
        for (int s = 1; s < R; ++s) v += red[buf][(g << lgR) + s][kk][cc];
        ov[i] = c.sc * v;
      }
      buf ^= 1;
    };
    // store the pending mirrored result (lanes and entries past K or n skip)
    auto flush = [&]() {
      if (!pend) return;  // uniform
      pend = false;
      if (R == 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int kk = lk + 4 * v;
          if (pc0 + kk < pK && colok) ppt[pc0 + kk + (int64_t)lr * P.ldp] = ov[v];
        }
        return;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i >= G) break;
        const int e = 64 * (st + R * i) + lane;
        const int kk = e >> 4, cc = e & 15;
        if (pc0 + kk < pK && cc < n) ppt[pc0 + kk + (int64_t)cc * P.ldp] = ov[i];
      }
    };
    // advance to the next chunk in the sequence; false at the end
    auto next = [&](const Cur& c, Cur& nx) {
      if (c.it + 1 < c.niter) {
        nx = c;
        nx.it = c.it + 1;
        return true;
      }
      return open(c.t + 1, nx);
    };
    // the chunk loop for this wave's quad count (a constant inside)
    auto run = [&](auto nqc) {
      // two operand buffers in turn
      double a0[4][4], b0[4], a1[4][4], b1[4];
      Cur c0s, c1s;
      if (open(P.term_begin, c0s)) {
        load(nqc, c0s, a0, b0);
        while (true) {
          ready();
          flush();
          const bool more0 = next(c0s, c1s);
          process(nqc, c0s, a0, b0, c1s, a1, b1, more0);
          if (!more0) break;
          ready();
          flush();
          const bool more1 = next(c1s, c0s);
          process(nqc, c1s, a1, b1, c0s, a0, b0, more1);
          if (!more1) break;
        }
        flush();
      }
    };
    switch (nq) {
      case 0: run(std::integral_constant<int, 0>{}); break;
      case 1: run(std::integral_constant<int, 1>{}); break;
      case 2: run(std::integral_constant<int, 2>{}); break;
      case 3: run(std::integral_constant<int, 3>{}); break;
      default: run(std::integral_constant<int, 4>{}); break;
    }
    // row sums: D[l/16 + 4v][l%16] of strip s is row r0 + 16s + l/16 + 4v,
    // column l%16; with G > 1 the groups' sums are added in group order
    if (G > 1) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int v = 0; v < 4; ++v) tr[w][16 * s4 + lk + 4 * v][lr] = acc[s4][v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      if (g == 0) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double sum = acc[s4][v];
            for (int h = 1; h < G; ++h) sum += tr[st + (h << lgR)][16 * s4 + lk + 4 * v][lr];
            acc[s4][v] = sum;
          }
      }
      // the slots are written again by the next item's transposes
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
    if (g == 0) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 16 * s4 + lk + 4 * v;
          if (row < m && colok) {
            double* cp = P.C + row + (int64_t)lr * P.ldc;
            double val = P.alpha * acc[s4][v];
            if (P.beta != 0.0) val += P.beta * (*cp);
            *cp = val;
          }
        }
    }
  }
}

template <typename TA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_symm16(
    const SymProblem* __restrict__ probs, const SymTerm* __restrict__ terms, int tiles_max, int nwork, int nprob) {
  symm16_body<TA, true>(probs, terms, tiles_max, nwork, nprob);
}

// The same for plain products: without the mirrored state three waves fit a SIMD.
template <typename TA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_rows16(
    const SymProblem* __restrict__ probs, const SymTerm* __restrict__ terms, int tiles_max, int nwork, int nprob) {
  symm16_body<TA, false>(probs, terms, tiles_max, nwork, nprob);
}

static void launch_symm16(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob,
                          int max_m, int cap, int a_f32, int mir) {
  const int tiles = ceil_div(max_m, 256);
  const int nwork = ceil_div(nprob, 8) * 8 * tiles;
  const int capped = cap > 0 ? std::max(8, cap / 8 * 8) : nwork;
  const dim3 grid((unsigned)std::min(capped, nwork));
  if (mir) {
    if (a_f32)
      hipLaunchKernelGGL(k_symm16<float>, grid, dim3(256), 0, s, d_p, d_t, tiles, nwork, nprob);
    else
      hipLaunchKernelGGL(k_symm16<double>, grid, dim3(256), 0, s, d_p, d_t, tiles, nwork, nprob);
  } else {
    if (a_f32)
      hipLaunchKernelGGL(k_rows16<float>, grid, dim3(256), 0, s, d_p, d_t, tiles, nwork, nprob);
    else
      hipLaunchKernelGGL(k_rows16<double>, grid, dim3(256), 0, s, d_p, d_t, tiles, nwork, nprob);
  }
}

void launch_symv(hipStream_t s, const SymProblem* d_p, const SymTerm* d_t, int nprob, int max_m,
                 int max_n, int cap, int a_f32, int mir) {
  if (nprob <= 0 || max_m <= 0 || max_n <= 0) return;
  if (max_n > 16) throw Error(SPD_E_INVALID, "symmetric-pair product supports at most 16 columns");
  if (max_n > 4) {
    launch_symm16(s, d_p, d_t, nprob, max_m, cap, a_f32, mir);
    SPD_HIP(hipGetLastError());
    return;
  }
  if (a_f32) launch_symv_ta<float>(s, d_p, d_t, nprob, max_m, max_n, cap);
  else launch_symv_ta<double>(s, d_p, d_t, nprob, max_m, max_n, cap);
  SPD_HIP(hipGetLastError());
}

// Problems per launch of a kernel with `tiles` workgroups of `threads` per
// problem, so that one launch stays below 2^31 work-items (the dispatch
// packet's grid size is a 32-bit count of work-items).
static int probs_per_launch(int64_t tiles, int threads) {
  const int64_t lim = ((int64_t)1 << 31) / (tiles * threads);
  return (int)std::max<int64_t>(1, std::min<int64_t>(lim, 1 << 30));
}

template <int BM, int BN, int WM, int WN>
static void launch_gemm_tiles(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                              int max_m, int max_n, int transA, int transB) {
  const int tiles = ceil_div(max_m, BM) * ceil_div(max_n, BN);
  const int per = probs_per_launch(tiles, 256);
  for (int p0 = 0; p0 < nprob; p0 += per) {
    const int np = std::min(per, nprob - p0);
    hipLaunchKernelGGL((k_gemm<BM, BN, WM, WN>), dim3((unsigned)np * tiles), dim3(256), 0, s,
                       d_p + p0, d_t, tiles, transA, transB);
  }
}

void launch_gemm(hipStream_t s, const GemmProblem* d_p, const GemmTerm* d_t, int nprob,
                 int max_m, int max_n, int transA, int transB, int max_k, int a_f32) {
  if (nprob <= 0 || max_m <= 0 || max_n <= 0) return;
  if (transA && max_n <= 4) {
    launch_gemv_t(s, d_p, d_t, nprob, max_m, max_n, max_k, transB, a_f32);
    return;
  }
  if (a_f32) throw Error(SPD_E_INVALID, "FP32 A only in the dot-form product (transposed, <= 4 columns)");
  if (max_n <= 4) {
    if (max_n == 1) launch_skinny<1>(s, d_p, d_t, nprob, max_m, transA, transB);
    else if (max_n <= 2) launch_skinny<2>(s, d_p, d_t, nprob, max_m, transA, transB);
    else launch_skinny<4>(s, d_p, d_t, nprob, max_m, transA, transB);
  } else if (max_n <= 16) {
    launch_gemm_tiles<64, 16, 16, 16>(s, d_p, d_t, nprob, max_m, max_n, transA, transB);
  } else if (max_n <= 32) {
    launch_gemm_tiles<64, 32, 32, 16>(s, d_p, d_t, nprob, max_m, max_n, transA, transB);
  } else {
    launch_gemm_tiles<64, 64, 32, 32>(s, d_p, d_t, nprob, max_m, max_n, transA, transB);
  }
  SPD_HIP(hipGetLastError());
}

// ---------------------------------------------------------- block updates --
// dst = beta dst + sum_t alpha_t op(src_t) (+ I), per element in term order:
// beta dst first, then the terms one by one.  Workgroups come from a tile
// list, so problems of very different sizes launch no empty workgroups.
int block_tile_cols(int max_n) { return max_n <= 16 ? 16 : 64; }

std::vector<int> block_tiles(std::vector<BlockProblem>& probs, int max_n) {
  const int bn = block_tile_cols(max_n);
  std::vector<int> t;
  for (size_t p = 0; p < probs.size(); ++p) {
    probs[p].tile0 = (int)t.size();
    const int64_t n = (int64_t)ceil_div(probs[p].m, 64) * ceil_div(probs[p].n, bn);
    t.insert(t.end(), (size_t)n, (int)p);
  }
  return t;
}

__device__ __forceinline__ double block_src(const BlockTerm& T, int i, int j) {
  return T.alpha * (T.trans ? T.src[j + (int64_t)i * T.lds] : T.src[i + (int64_t)j * T.lds]);
}

// 64 x BN tiles: element e of the tile is row e mod 64, column e / 64
template <int BN>
__global__ __launch_bounds__(256) void k_block(const BlockProblem* __restrict__ probs,
                                               const BlockTerm* __restrict__ terms,
                                               const int* __restrict__ tiles, int tile_base) {
  const int g = tile_base + blockIdx.x;
  const BlockProblem P = probs[tiles[g]];
  const int tile = g - P.tile0;
  const int tm = (P.m + 63) / 64;
  const int i0 = (tile % tm) * 64, j0 = (tile / tm) * BN;
  for (int e = threadIdx.x; e < 64 * BN; e += 256) {
    const int i = i0 + (e & 63), j = j0 + (e >> 6);
    if (i >= P.m || j >= P.n) continue;
    double* d = P.dst + i + (int64_t)j * P.ldd;
    double v = (P.beta != 0.0) ? P.beta * (*d) : 0.0;
    // terms in groups of 8: the loads of a group are issued together, the sum
    // keeps term order
    int t = P.term_begin;
    for (; t + 8 <= P.term_end; t += 8) {
      double x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = block_src(terms[t + q], i, j);
#pragma unroll
      for (int q = 0; q < 8; ++q) v += x[q];
    }
    for (; t < P.term_end; ++t) v += block_src(terms[t], i, j);
    if (P.add_eye && i == j) v += 1.0;
    *d = v;
  }
}

void launch_block(hipStream_t s, const BlockProblem* d_p, const BlockTerm* d_t, const int* d_tiles,
                  int ntiles, int max_n) {
  if (ntiles <= 0 || max_n <= 0) return;
  const int per = probs_per_launch(1, 256);  // workgroups per launch below 2^31 work-items
  for (int t0 = 0; t0 < ntiles; t0 += per) {
    const dim3 grid((unsigned)std::min(per, ntiles - t0));
    if (block_tile_cols(max_n) == 16)
      hipLaunchKernelGGL(k_block<16>, grid, dim3(256), 0, s, d_p, d_t, d_tiles, t0);
    else
      hipLaunchKernelGGL(k_block<64>, grid, dim3(256), 0, s, d_p, d_t, d_tiles, t0);
  }
  SPD_HIP(hipGetLastError());
}

// ------------------------------------------------------- kernel entries --
__device__ __forceinline__ double kfun(int kind, double ell, double r2) {
  if (kind == SPD_K_GAUSSIAN) return exp(-r2 / (ell * ell));
  if (kind == SPD_K_MATERN32) {
    const double t = 1.7320508075688772 * sqrt(r2) / ell;
    return (1.0 + t) * exp(-t);
  }
  if (kind == SPD_K_EXPONENTIAL) return exp(-sqrt(r2) / ell);
  return 1.0 / sqrt(r2 + ell * ell);
}

// Proxy point t of a node: sphere q = t / per_shell at radius
// rin (rout/rin)^(q/(shells-1)), Fibonacci lattice point u = t % per_shell.
__device__ __forceinline__ void proxy_point(const KBlockProblem& P, int t, double& x, double& y,
                                            double& z) {
  const int shells = P.shells, per_shell = P.per_shell;
  const int q = t / per_shell, u = t % per_shell;
  const double zz = 1.0 - (2.0 * u + 1.0) / per_shell;
  const double rho = sqrt(fmax(0.0, 1.0 - zz * zz));
  const double phi = u * (3.141592653589793 * (3.0 - 2.23606797749979));
  const double rad =
      shells == 1 ? P.rin : P.rin * pow(P.rout / P.rin, (double)q / (double)(shells - 1));
  x = P.cx + rad * (rho * cos(phi));
  y = P.cy + rad * (rho * sin(phi));
  z = P.cz + rad * zz;
}

// Entry [ca][cb] of the RPY tensor with particle radius a at r = (dx, dy, dz)
// (Section 6, normalized so that the self term is I / a):
//   |r| >= 2a:  3/(4|r|) (I + rr) + 3a^2/(2|r|^3) (I/3 - rr)
//   |r| <  2a:  (1/a)(1 - 9|r|/(32a)) I + 3|r|/(32a^2) rr,   rr = r r^T / |r|^2
// (the two branches agree at |r| = 2a).
__device__ __forceinline__ double rpy_entry(double a, double dx, double dy, double dz, int ca, int cb) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double eye = ca == cb ? 1.0 : 0.0;
  if (r2 == 0.0) return eye / a;
  const double d[3] = {dx, dy, dz};
  const double r = sqrt(r2);
  const double rr = d[ca] * d[cb] / r2;
  if (r >= 2.0 * a) return 0.75 / r * (eye + rr) + 1.5 * a * a / (r2 * r) * (eye / 3.0 - rr);
  return (1.0 - 9.0 * r / (32.0 * a)) / a * eye + 3.0 * r / (32.0 * a * a) * rr;
}

// Dense kernel blocks.  For the RPY tensor every row and column is a point's
// component: a point's component is its original index mod 3 (row 3p + c is
// component c of particle p), and proxy index t is component t mod 3 of proxy
// point t / 3.
__global__ __launch_bounds__(256) void k_kblock(const KBlockProblem* __restrict__ probs,
                                                int tiles_max, const double* __restrict__ px,
                                                int64_t stride, int kind, double ell,
                                                double shift, const int64_t* __restrict__ perm) {
  __shared__ double ax[64], ay[64], az[64], bx[64], by[64], bz[64];
  __shared__ int ac[64], bc[64];
  const bool tensor = kind == SPD_K_RPY;
  const int p = blockIdx.x / tiles_max, tile = blockIdx.x % tiles_max;
  const KBlockProblem P = probs[p];
  const int tm = (P.na + 63) / 64, tn = (P.nb + 63) / 64;
  if (tile >= tm * tn) return;
  const int i0 = (tile % tm) * 64, j0 = (tile / tm) * 64;
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int i = i0 + tid;
    if (i < P.na) {
      double x, y, z;
      int c = 0;
      if (P.proxy) {
        proxy_point(P, tensor ? i / 3 : i, x, y, z);
        c = tensor ? i % 3 : 0;
      } else {
        const int64_t g = P.ia ? (int64_t)P.ia[i] : P.offa + i;
        x = px[g];
        y = px[g + stride];
        z = px[g + 2 * stride];
        c = tensor ? (int)(perm[g] % 3) : 0;
      }
      ax[tid] = x;
      ay[tid] = y;
      az[tid] = z;
      ac[tid] = c;
    }
  } else if (tid < 128) {
    const int j = j0 + tid - 64;
    if (j < P.nb) {
      const int64_t g = P.ib ? (int64_t)P.ib[j] : P.offb + j;
      bx[tid - 64] = px[g];
      by[tid - 64] = px[g + stride];
      bz[tid - 64] = px[g + 2 * stride];
      bc[tid - 64] = tensor ? (int)(perm[g] % 3) : 0;
    }
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int il = e & 63, jl = e >> 6;
    const int i = i0 + il, j = j0 + jl;
    if (i >= P.na || j >= P.nb) continue;
    const double dx = ax[il] - bx[jl], dy = ay[il] - by[jl], dz = az[il] - bz[jl];
    double v;
    if (tensor) {
      v = rpy_entry(ell, dx, dy, dz, ac[il], bc[jl]);
    } else {
      const double r2 = dx * dx + dy * dy + dz * dz;
      v = kfun(kind, ell, r2);
    }
    if (P.diag_shift && i == j) v += shift;
    P.out[i + (int64_t)j * P.ld] = v;
  }
}

void launch_kblock(hipStream_t s, const KBlockProblem* d_p, int nprob, int max_m, int max_n,
                   const double* px, int64_t stride, int kind, double ell, double shift,
                   const int64_t* perm) {
  if (nprob <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tiles = ceil_div(max_m, 64) * ceil_div(max_n, 64);
  const int per = probs_per_launch(tiles, 256);
  for (int p0 = 0; p0 < nprob; p0 += per)
    hipLaunchKernelGGL(k_kblock, dim3((unsigned)std::min(per, nprob - p0) * tiles), dim3(256), 0, s,
                       d_p + p0, tiles, px, stride, kind, ell, shift, perm);
  SPD_HIP(hipGetLastError());
}

// --------------------------------------------------------------- Cholesky --
// In-place lower Cholesky, one workgroup per matrix, left-looking by panels of
// 32 columns.  The strictly upper triangle is set to zero on exit.
__global__ __launch_bounds__(256) void k_chol(const CholProblem* __restrict__ probs, int* fail) {
  __shared__ double W[32][33];
  __shared__ double D[32][33];
  __shared__ int bad;
  const CholProblem P = probs[blockIdx.x];
  const int n = P.n, lda = P.lda, tid = threadIdx.x;
  double* A = P.A;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += 32) {
    const int jb = min(32, n - j0);
    const int nrows = n - j0;
    // panel update A[j0:n, j0:j0+jb] -= A[j0:n, 0:j0] A[j0:j0+jb, 0:j0]^T
    for (int rbase = 0; rbase < nrows; rbase += 256) {
      const int r = rbase + tid;
      const bool act = r < nrows;
      double acc[32];
#pragma unroll
      for (int c = 0; c < 32; ++c)
        acc[c] = (act && c < jb) ? A[(j0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
      for (int k0 = 0; k0 < j0; k0 += 32) {
        __syncthreads();
        for (int e = tid; e < 32 * 32; e += 256) {
          const int c = e & 31, kk = e >> 5;
          W[c][kk] = (c < jb) ? A[(j0 + c) + (int64_t)(k0 + kk) * lda] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < 32; ++kk) {
          const double a = act ? A[(j0 + r) + (int64_t)(k0 + kk) * lda] : 0.0;
#pragma unroll
          for (int c = 0; c < 32; ++c) acc[c] -= a * W[c][kk];
        }
      }
      if (act) {
#pragma unroll
        for (int c = 0; c < 32; ++c)
          if (c < jb) A[(j0 + r) + (int64_t)(j0 + c) * lda] = acc[c];
      }
    }
    __syncthreads();
    // factor the diagonal block in LDS
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e & 31, c = e >> 5;
      D[r][c] = (r < jb && c < jb && c <= r) ? A[(j0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < jb; ++c) {
      if (tid == 0) {
        const double d = D[c][c];
        if (!(d > 0.0)) bad = 1;
        D[c][c] = sqrt(fmax(d, 0.0));
      }
      __syncthreads();
      const double dc = D[c][c];
      if (tid > c && tid < jb) D[tid][c] = (dc > 0.0) ? D[tid][c] / dc : 0.0;
      __syncthreads();
      for (int e = tid; e < 32 * 32; e += 256) {
        const int r = e & 31, q = e >> 5;
        if (q > c && r >= q && r < jb) D[r][q] -= D[r][c] * D[q][c];
      }
      __syncthreads();
    }
    if (bad) break;
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e & 31, c = e >> 5;
      if (r < jb && c < jb && c <= r) A[(j0 + r) + (int64_t)(j0 + c) * lda] = D[r][c];
    }
    // rows below the diagonal block: X D^T = P
    for (int rbase = jb; rbase < nrows; rbase += 256) {
      const int r = rbase + tid;
      if (r < nrows) {
        double x[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) x[c] = (c < jb) ? A[(j0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
#pragma unroll
        for (int c = 0; c < 32; ++c) {
          if (c < jb) {
            double sacc = x[c];
#pragma unroll
            for (int q = 0; q < c; ++q) sacc -= x[q] * D[c][q];
            x[c] = sacc / D[c][c];
          }
        }
#pragma unroll
        for (int c = 0; c < 32; ++c)
          if (c < jb) A[(j0 + r) + (int64_t)(j0 + c) * lda] = x[c];
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) fail[blockIdx.x] = 1;
    return;
  }
  for (int64_t e = tid; e < (int64_t)n * n; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    if (r < c) A[r + (int64_t)c * lda] = 0.0;
  }
}

void launch_chol(hipStream_t s, const CholProblem* d_p, int nprob, int max_n, int* d_fail) {
  if (nprob <= 0 || max_n <= 0) return;
  hipLaunchKernelGGL(k_chol, dim3(nprob), dim3(256), 0, s, d_p, d_fail);
  SPD_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- TRSM --
// B <- op(L)^{-1} B for lower-triangular L (trans: L^T).  With upper = 1 the
// factor is read as L(i, j) = M[j + i*ld], i.e. the transpose of an upper
// triangular M, so (trans=1, upper=1) computes M^{-1} B.  One workgroup per
// (problem, block of CB right-hand sides); the block stays in LDS.
template <int CB>
__global__ __launch_bounds__(256) void k_trsm(const TrsmProblem* __restrict__ probs, int nprob,
                                              int ncb, int trans, int upper) {
  extern __shared__ double X[];  // n x CB, row-major
  __shared__ double Dg[32][33];
  // XCD-aware decode: all column blocks of one problem share blockIdx % 8.
  const int b = blockIdx.x;
  const int x8 = b & 7, rest = b >> 3;
  const int cb = rest % ncb, p = (rest / ncb) * 8 + x8;
  if (p >= nprob) return;
  const TrsmProblem P = probs[p];
  const int n = P.n, ldl = P.ldl, tid = threadIdx.x;
  const int c0 = cb * CB;
  const int ncol = min(CB, P.nrhs - c0);
  if (ncol <= 0 || n <= 0) return;
  auto Lg = [&](int i, int j) -> double {
    return upper ? P.L[j + (int64_t)i * ldl] : P.L[i + (int64_t)j * ldl];
  };
  for (int e = tid; e < n * CB; e += 256) {
    const int r = e % n, c = e / n;
    X[r * CB + c] = (c < ncol) ? P.B[r + (int64_t)(c0 + c) * P.ldb] : 0.0;
  }
  __syncthreads();
  constexpr int CPT = CB / 8;  // columns per thread in the update
  const int nblk = (n + 31) / 32;
  for (int bi = 0; bi < nblk; ++bi) {
    const int blk = trans ? (nblk - 1 - bi) : bi;
    const int r0 = blk * 32, rb = min(32, n - r0);
    const int r = tid & 31, cg = tid >> 5;
    double acc[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) acc[q] = 0.0;
    if (r < rb) {
      if (!trans) {
        for (int k = 0; k < r0; ++k) {
          const double l = Lg(r0 + r, k);
#pragma unroll
          for (int q = 0; q < CPT; ++q) acc[q] += l * X[k * CB + cg * CPT + q];
        }
      } else {
        for (int k = r0 + rb; k < n; ++k) {
          const double l = Lg(k, r0 + r);
#pragma unroll
          for (int q = 0; q < CPT; ++q) acc[q] += l * X[k * CB + cg * CPT + q];
        }
      }
#pragma unroll
      for (int q = 0; q < CPT; ++q) X[(r0 + r) * CB + cg * CPT + q] -= acc[q];
    }
    for (int e = tid; e < 32 * 32; e += 256) {
      const int rr = e & 31, qq = e >> 5;
      Dg[rr][qq] = (rr < rb && qq < rb && qq <= rr) ? Lg(r0 + rr, r0 + qq) : 0.0;
    }
    __syncthreads();
    if (tid < CB) {
      double x[32];
#pragma unroll
      for (int rr = 0; rr < 32; ++rr) x[rr] = (rr < rb) ? X[(r0 + rr) * CB + tid] : 0.0;
      if (!trans) {
#pragma unroll
        for (int rr = 0; rr < 32; ++rr) {
          if (rr < rb) {
            double sacc = x[rr];
#pragma unroll
            for (int qq = 0; qq < rr; ++qq) sacc -= Dg[rr][qq] * x[qq];
            x[rr] = sacc / Dg[rr][rr];
          }
        }
      } else {
#pragma unroll
        for (int rr = 31; rr >= 0; --rr) {
          if (rr < rb) {
            double sacc = x[rr];
#pragma unroll
            for (int qq = rr + 1; qq < 32; ++qq)
              if (qq < rb) sacc -= Dg[qq][rr] * x[qq];
            x[rr] = sacc / Dg[rr][rr];
          }
        }
      }
#pragma unroll
      for (int rr = 0; rr < 32; ++rr)
        if (rr < rb) X[(r0 + rr) * CB + tid] = x[rr];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * ncol; e += 256) {
    const int r = e % n, c = e / n;
    P.B[r + (int64_t)(c0 + c) * P.ldb] = X[r * CB + c];
  }
}

void launch_trsm(hipStream_t s, const TrsmProblem* d_p, int nprob, int max_n, int max_nrhs,
                 int trans, int upper) {
  if (nprob <= 0 || max_n <= 0 || max_nrhs <= 0) return;
  const int np8 = (nprob + 7) / 8 * 8;
  if (max_n <= 256) {
    constexpr int CB = 32;
    const int ncb = ceil_div(max_nrhs, CB);
    hipLaunchKernelGGL((k_trsm<CB>), dim3((unsigned)np8 * ncb), dim3(256),
                       (size_t)max_n * CB * sizeof(double), s, d_p, nprob, ncb, trans, upper);
  } else {
    SPD_REQUIRE(max_n <= 2048, SPD_E_INVALID, "triangular solve: order above 2048");
    constexpr int CB = 8;
    const int ncb = ceil_div(max_nrhs, CB);
    hipLaunchKernelGGL((k_trsm<CB>), dim3((unsigned)np8 * ncb), dim3(256),
                       (size_t)max_n * CB * sizeof(double), s, d_p, nprob, ncb, trans, upper);
  }
  SPD_HIP(hipGetLastError());
}

// --------------------------------------------------------------- CPQR --
// Register-resident Householder QR with column pivoting (Algorithm 5.1,
// step 3).  Wave w owns columns w + NW*c, lane l owns rows l + 64*q.  At step t
// the pivot is the unused column with the largest exactly recomputed trailing
// norm (rows >= t), ties to the lowest column index; the factorization stops
// when t reaches maxrank or min(m, n), or when that norm is not larger than
// tol times the first pivot norm.  Q's first rank columns are then formed by
// applying the reflectors to the identity, with signs making R_tt >= 0.
template <int NW, int RPL, int CPW>
__global__ __launch_bounds__(NW * 64) void k_cpqr_reg(const CpqrProblem* __restrict__ probs) {
  constexpr int NC = NW * CPW;
  __shared__ double nrm2[NC];
  __shared__ double vbuf[64 * RPL];
  __shared__ double betas[NC];
  __shared__ double alphas[NC];
  __shared__ double sh_beta;
  const CpqrProblem P = probs[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = P.m, n = P.n;
  double a[CPW][RPL];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int col = w + NW * c;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int row = lane + 64 * q;
      a[c][q] = (col < n && row < m) ? P.A[row + (int64_t)col * P.lda] : 0.0;
    }
  }
  {
    double s2[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      s2[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) s2[c] += a[c][q] * a[c][q];
    }
    wave_sum_n<CPW>(s2);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int col = w + NW * c;
        nrm2[col] = (col < n) ? s2[c] : -1.0;
      }
    }
  }
  __syncthreads();
  const int kmax = min(min(m, n), P.maxrank);
  uint32_t used = 0;
  double ref = 0.0;
  int rank = 0;
  for (int t = 0; t < kmax; ++t) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int j = lane; j < NC; j += 64) {
      const double v = nrm2[j];
      if (v > best) { best = v; bi = j; }
    }
    wave_argmax(best, bi);
    const double nrm = sqrt(fmax(best, 0.0));
    if (t == 0) ref = nrm;
    if (!(nrm > P.tol * ref) || nrm == 0.0) break;
    __syncthreads();  // everyone has read nrm2 of this step
    const int owner = bi % NW, slot = bi / NW;
    if (w == owner) {
      double col[RPL];
#pragma unroll
      for (int q = 0; q < RPL; ++q) col[q] = 0.0;
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        if (c == slot)
#pragma unroll
          for (int q = 0; q < RPL; ++q) col[q] = a[c][q];
      double xt = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (q == t / 64) xt = col[q];
      xt = __shfl(xt, t % 64, 64);
      const double alpha = (xt >= 0.0) ? -nrm : nrm;
      const double beta = 1.0 / (nrm * (nrm + fabs(xt)));
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int row = lane + 64 * q;
        double v = (row >= t) ? col[q] : 0.0;
        if (row == t) v = xt - alpha;
        vbuf[row] = v;
        if (row < m && P.V) P.V[row + (int64_t)t * m] = v;
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        if (c == slot)
#pragma unroll
          for (int q = 0; q < RPL; ++q) {
            const int row = lane + 64 * q;
            if (row == t) a[c][q] = alpha;
            else if (row > t) a[c][q] = 0.0;
          }
      if (lane == 0) {
        sh_beta = beta;
        betas[t] = beta;
        alphas[t] = alpha;
        P.piv[t] = bi;
        if (P.diag) P.diag[t] = nrm;
      }
      used |= (1u << slot);
    }
    __syncthreads();
    const double beta = sh_beta;
    double v[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) v[q] = vbuf[lane + 64 * q];
    double d[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      d[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) d[c] += v[q] * a[c][q];
    }
    wave_sum_n<CPW>(d);
    double s2[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const bool live = !((used >> c) & 1u);
      s2[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        if (live) a[c][q] -= beta * d[c] * v[q];
        const int row = lane + 64 * q;
        if (row > t) s2[c] += a[c][q] * a[c][q];
      }
    }
    wave_sum_n<CPW>(s2);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int col = w + NW * c;
        if (col < NC) nrm2[col] = (col < n && !((used >> c) & 1u)) ? s2[c] : -1.0;
      }
    }
    rank = t + 1;
    __syncthreads();
  }
  if (threadIdx.x == 0) *P.rank = rank;
  if (!P.Q) return;
  // form Q = H_0 ... H_{rank-1} [I; 0]
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int col = w + NW * c;
#pragma unroll
    for (int q = 0; q < RPL; ++q) a[c][q] = (col < rank && lane + 64 * q == col) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int t = rank - 1; t >= 0; --t) {
    double v[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int row = lane + 64 * q;
      v[q] = (row < m && row >= t) ? P.V[row + (int64_t)t * m] : 0.0;
    }
    const double beta = betas[t];
    double d[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      d[c] = 0.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) d[c] += v[q] * a[c][q];
    }
    wave_sum_n<CPW>(d);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int col = w + NW * c;
      if (col >= t && col < rank)
#pragma unroll
        for (int q = 0; q < RPL; ++q) a[c][q] -= beta * d[c] * v[q];
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int col = w + NW * c;
    if (col < rank) {
      const double sg = (alphas[col] < 0.0) ? -1.0 : 1.0;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int row = lane + 64 * q;
        if (row < m) P.Q[row + (int64_t)col * P.ldq] = sg * a[c][q];
      }
    }
  }
}

bool cpqr_reg_fits(int m, int n) { return m <= 512 && n <= 128; }

void launch_cpqr_reg(hipStream_t s, const CpqrProblem* d_p, int nprob, int max_m, int max_n) {
  if (nprob <= 0) return;
  SPD_REQUIRE(cpqr_reg_fits(max_m, max_n), SPD_E_INVALID, "cpqr: shape exceeds register kernel");
  if (max_m <= 256)
    hipLaunchKernelGGL((k_cpqr_reg<8, 4, 16>), dim3(nprob), dim3(512), 0, s, d_p);
  else
    hipLaunchKernelGGL((k_cpqr_reg<16, 8, 8>), dim3(nprob), dim3(1024), 0, s, d_p);
  SPD_HIP(hipGetLastError());
}

// Global-memory variant for tall or wide matrices (the proxy interpolative
// decomposition).  The matrix is updated in place; each column is streamed
// through registers once per step (RCH chunks of 64 rows per lane).  On exit
// P.piv holds the full column order (pivots first, then the unused columns in
// ascending order) and P.R the first rank rows of R in that order.
template <int RCH>
__global__ __launch_bounds__(1024) void k_cpqr_glob(const CpqrProblem* __restrict__ probs,
                                                    double* nrm_ws) {
  constexpr int NW = 16;
  extern __shared__ double sm[];  // vbuf[64*RCH] | nrm2[n]
  __shared__ double sh_beta;
  const CpqrProblem P = probs[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = P.m, n = P.n;
  double* vbuf = sm;
  double* nrm2 = sm + 64 * RCH;
  double* A = P.A;
  const int64_t lda = P.lda;
  for (int col = w; col < n; col += NW) {
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
      const int row = lane + 64 * q;
      if (row < m) { const double x = A[row + col * lda]; s2 += x * x; }
    }
    s2 = wave_sum(s2);
    if (lane == 0) nrm2[col] = s2;
  }
  __syncthreads();
  const int kmax = min(min(m, n), P.maxrank);
  double ref = 0.0;
  int rank = 0;
  for (int t = 0; t < kmax; ++t) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int j = lane; j < n; j += 64) {
      const double v = nrm2[j];
      if (v > best) { best = v; bi = j; }
    }
    wave_argmax(best, bi);
    const double nrm = sqrt(fmax(best, 0.0));
    if (t == 0) ref = nrm;
    if (!(nrm > P.tol * ref) || nrm == 0.0) break;
    __syncthreads();
    if (w == bi % NW) {
      const double xt = A[t + bi * lda];
      const double alpha = (xt >= 0.0) ? -nrm : nrm;
      const double beta = 1.0 / (nrm * (nrm + fabs(xt)));
#pragma unroll
      for (int q = 0; q < RCH; ++q) {
        const int row = lane + 64 * q;
        double v = 0.0;
        if (row < m && row >= t) v = (row == t) ? xt - alpha : A[row + bi * lda];
        vbuf[row] = v;
        if (row < m && row >= t) A[row + bi * lda] = (row == t) ? alpha : 0.0;
        // keep the reflector for Q (rows above t are zero)
        if (P.hbeta && row < m) P.V[row + (int64_t)t * m] = v;
      }
      if (lane == 0) {
        if (P.hbeta) P.hbeta[t] = beta;
        sh_beta = beta;
        P.piv[t] = bi;
        if (P.diag) P.diag[t] = nrm;
        nrm2[bi] = -1.0;
      }
    }
    __syncthreads();
    const double beta = sh_beta;
    for (int col = w; col < n; col += NW) {
      if (nrm2[col] < 0.0) continue;  // used (the pivot's owner wrote -1 before the barrier)
      double x[RCH];
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < RCH; ++q) {
        const int row = lane + 64 * q;
        x[q] = (row < m && row >= t) ? A[row + col * lda] : 0.0;
        d += vbuf[row] * x[q];
      }
      d = wave_sum(d);
      double s2 = 0.0;
#pragma unroll
      for (int q = 0; q < RCH; ++q) {
        const int row = lane + 64 * q;
        if (row < m && row >= t) {
          x[q] -= beta * d * vbuf[row];
          A[row + col * lda] = x[q];
          if (row > t) s2 += x[q] * x[q];
        }
      }
      s2 = wave_sum(s2);
      if (lane == 0) nrm2[col] = s2;
    }
    rank = t + 1;
    __syncthreads();
  }
  if (threadIdx.x == 0) *P.rank = rank;
  __syncthreads();
  // complete the permutation with the unused columns in ascending order
  if (threadIdx.x == 0) {
    int pos = rank;
    for (int j = 0; j < n; ++j)
      if (nrm2[j] >= 0.0) P.piv[pos++] = j;
  }
  __syncthreads();
  if (P.R) {
    const int64_t ldr = P.maxrank;
    for (int64_t e = threadIdx.x; e < (int64_t)rank * n; e += blockDim.x) {
      const int i = (int)(e % rank), j = (int)(e / rank);
      P.R[i + j * ldr] = A[i + (int64_t)P.piv[j] * lda];
    }
  }
  (void)nrm_ws;
}

// Variant for more rows than the register chunks hold (2048 < m <= 8000):
// the Householder vector is staged in LDS (m doubles), the squared trailing
// norms live in the problem's global workspace P.nrm, and each remaining
// column is read twice per step (its dot product with the vector, then the
// update).  Pivot choice, norms (rows > t after step t) and outputs are those
// of k_cpqr_glob; each lane owns the rows lane + 64 q as there.
__global__ __launch_bounds__(1024) void k_cpqr_big(const CpqrProblem* __restrict__ probs) {
  constexpr int NW = 16;
  extern __shared__ double vbuf[];  // m
  __shared__ double sh_beta;
  const CpqrProblem P = probs[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = P.m, n = P.n;
  double* A = P.A;
  double* nrm2 = P.nrm;
  const int64_t lda = P.lda;
  for (int col = w; col < n; col += NW) {
    double s2 = 0.0;
    for (int row = lane; row < m; row += 64) {
      const double x = A[row + col * lda];
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (lane == 0) nrm2[col] = s2;
  }
  __threadfence_block();
  __syncthreads();
  const int kmax = min(min(m, n), P.maxrank);
  double ref = 0.0;
  int rank = 0;
  for (int t = 0; t < kmax; ++t) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int j = lane; j < n; j += 64) {
      const double v = nrm2[j];
      if (v > best) { best = v; bi = j; }
    }
    wave_argmax(best, bi);
    const double nrm = sqrt(fmax(best, 0.0));
    if (t == 0) ref = nrm;
    if (!(nrm > P.tol * ref) || nrm == 0.0) break;
    __syncthreads();
    if (w == bi % NW) {
      const double xt = A[t + bi * lda];
      const double alpha = (xt >= 0.0) ? -nrm : nrm;
      const double beta = 1.0 / (nrm * (nrm + fabs(xt)));
      for (int row = lane; row < m; row += 64) {
        if (row < t) continue;
        const double v = (row == t) ? xt - alpha : A[row + bi * lda];
        vbuf[row] = v;
        A[row + bi * lda] = (row == t) ? alpha : 0.0;
        if (P.hbeta) P.V[row + (int64_t)t * m] = v;
      }
      if (P.hbeta)
        for (int row = lane; row < t; row += 64) P.V[row + (int64_t)t * m] = 0.0;
      if (lane == 0) {
        if (P.hbeta) P.hbeta[t] = beta;
        sh_beta = beta;
        P.piv[t] = bi;
        if (P.diag) P.diag[t] = nrm;
        nrm2[bi] = -1.0;
      }
    }
    __threadfence_block();
    __syncthreads();
    const double beta = sh_beta;
    for (int col = w; col < n; col += NW) {
      if (nrm2[col] < 0.0) continue;
      double d = 0.0;
      for (int row = lane; row < m; row += 64)
        if (row >= t) d += vbuf[row] * A[row + col * lda];
      d = wave_sum(d);
      double s2 = 0.0;
      for (int row = lane; row < m; row += 64) {
        if (row < t) continue;
        const double x = A[row + col * lda] - beta * d * vbuf[row];
        A[row + col * lda] = x;
        if (row > t) s2 += x * x;
      }
      s2 = wave_sum(s2);
      if (lane == 0) nrm2[col] = s2;
    }
    rank = t + 1;
    __threadfence_block();
    __syncthreads();
  }
  if (threadIdx.x == 0) *P.rank = rank;
  __syncthreads();
  if (threadIdx.x == 0) {
    int pos = rank;
    for (int j = 0; j < n; ++j)
      if (nrm2[j] >= 0.0) P.piv[pos++] = j;
  }
  __threadfence_block();
  __syncthreads();
  if (P.R) {
    const int64_t ldr = P.maxrank;
    for (int64_t e = threadIdx.x; e < (int64_t)rank * n; e += blockDim.x) {
      const int i = (int)(e % rank), j = (int)(e / rank);
      P.R[i + j * ldr] = A[i + (int64_t)P.piv[j] * lda];
    }
  }
}

// Wide form of the global-memory variant, for a few large problems (the upper
// levels of the H^2 construction, where one workgroup per problem leaves the
// chip nearly idle): one launch per step t, the columns of every problem split
// over many workgroups.  Each column is still updated by one wave with the
// loops of k_cpqr_big, and every workgroup finds the pivot with the same
// reduction, so pivots, norms and outputs are those of k_cpqr_big.  Workspace
// (P.nrm, 2n + maxrank + 2 doubles): the squared trailing norms in two
// buffers (step t reads buffer t mod 2 and writes the other, so no workgroup
// reads a norm written in its own launch), alpha_t per step, the first
// pivot's norm, and the problem's state (negative while running, else its
// rank).  The pivot column itself is only read during its step; its R
// diagonal and zeros below are written by k_cpqr_wide_fix at the end.
// Workgroup table entry: (problem, first column, end column, 0).
struct CpqrWs {
  double *n0, *n1, *alpha, *ref, *state;
};
__device__ __forceinline__ CpqrWs cpqr_ws(const CpqrProblem& P) {
  CpqrWs w;
  w.n0 = P.nrm;
  w.n1 = P.nrm + P.n;
  w.alpha = P.nrm + 2 * (int64_t)P.n;
  w.ref = w.alpha + P.maxrank;
  w.state = w.ref + 1;
  return w;
}

__global__ __launch_bounds__(1024) void k_cpqr_wide_norms(const CpqrProblem* __restrict__ probs,
                                                          const int4* __restrict__ wg, int* done) {
  constexpr int NW = 16;
  const int4 g = wg[blockIdx.x];
  const CpqrProblem P = probs[g.x];
  const CpqrWs ws = cpqr_ws(P);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t lda = P.lda;
  for (int col = g.y + w; col < g.z; col += NW) {
    double s2 = 0.0;
    for (int row = lane; row < P.m; row += 64) {
      const double x = P.A[row + col * lda];
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (lane == 0) ws.n0[col] = s2;
  }
  if (g.y == 0 && threadIdx.x == 0) {
    *ws.state = -1.0;
    done[g.x] = 0;
  }
}

// vlds: the Householder vector is staged in LDS (at most kCpqrBigRows rows);
// otherwise every use reads it from the pivot column, which nobody writes
// during the step.
__global__ __launch_bounds__(1024) void k_cpqr_wide_step(const CpqrProblem* __restrict__ probs,
                                                         const int4* __restrict__ wg, int t,
                                                         int* done, int vlds) {
  constexpr int NW = 16;
  extern __shared__ double vbuf[];  // m, when vlds
  const int4 g = wg[blockIdx.x];
  const CpqrProblem P = probs[g.x];
  const CpqrWs ws = cpqr_ws(P);
  if (*ws.state >= 0.0) return;  // finished (uniform)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = P.m, n = P.n;
  const int64_t lda = P.lda;
  const double* nin = (t & 1) ? ws.n1 : ws.n0;
  double* nout = (t & 1) ? ws.n0 : ws.n1;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int j = lane; j < n; j += 64) {
    const double v = nin[j];
    if (v > best) { best = v; bi = j; }
  }
  wave_argmax(best, bi);
  const double nrm = sqrt(fmax(best, 0.0));
  const double ref = (t == 0) ? nrm : *ws.ref;
  const int kmax = min(min(m, n), P.maxrank);
  if (t >= kmax || !(nrm > P.tol * ref) || nrm == 0.0) {
    if (g.y == 0 && threadIdx.x == 0) {
      *ws.state = (double)t;
      done[g.x] = 1;
    }
    return;
  }
  const double xt = P.A[t + (int64_t)bi * lda];
  const double alpha = (xt >= 0.0) ? -nrm : nrm;
  const double beta = 1.0 / (nrm * (nrm + fabs(xt)));
  const bool first = g.y == 0;  // the problem's first workgroup records the step
  const double* pcol = P.A + (int64_t)bi * lda;
  if (vlds || (first && P.hbeta)) {
    for (int row = threadIdx.x; row < m; row += 1024) {
      const double v = row < t ? 0.0 : (row == t ? xt - alpha : pcol[row]);
      if (vlds) vbuf[row] = v;
      if (first && P.hbeta) P.V[row + (int64_t)t * m] = v;
    }
  }
  auto vat = [&](int row) {  // the vector's entry in row >= t
    return vlds ? vbuf[row] : (row == t ? xt - alpha : pcol[row]);
  };
  if (first && threadIdx.x == 0) {
    if (P.hbeta) P.hbeta[t] = beta;
    P.piv[t] = bi;
    if (P.diag) P.diag[t] = nrm;
    ws.alpha[t] = alpha;
    if (t == 0) *ws.ref = nrm;
  }
  __syncthreads();
  for (int col = g.y + w; col < g.z; col += NW) {
    if (col == bi || nin[col] < 0.0) {
      if (lane == 0) nout[col] = -1.0;
      continue;
    }
    double d = 0.0;
    for (int row = lane; row < m; row += 64)
      if (row >= t) d += vat(row) * P.A[row + col * lda];
    d = wave_sum(d);
    double s2 = 0.0;
    for (int row = lane; row < m; row += 64) {
      if (row < t) continue;
      const double x = P.A[row + col * lda] - beta * d * vat(row);
      P.A[row + col * lda] = x;
      if (row > t) s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (lane == 0) nout[col] = s2;
  }
}

// The pivot column of step s (one workgroup per (problem, s) entry of the
// table, x: problem, y: s): R diagonal alpha_s in row s, zeros below.
__global__ __launch_bounds__(256) void k_cpqr_wide_fix(const CpqrProblem* __restrict__ probs,
                                                       const int2* __restrict__ fx) {
  const int2 f = fx[blockIdx.x];
  const CpqrProblem P = probs[f.x];
  const CpqrWs ws = cpqr_ws(P);
  const int rank = (int)*ws.state, s = f.y;
  if (s >= rank) return;
  double* col = P.A + (int64_t)P.piv[s] * P.lda;
  for (int row = s + threadIdx.x; row < P.m; row += 256) col[row] = row == s ? ws.alpha[s] : 0.0;
}

// Rank, the unused columns after the pivots in ascending order (one
// workgroup per problem).
__global__ void k_cpqr_wide_perm(const CpqrProblem* __restrict__ probs) {
  const CpqrProblem P = probs[blockIdx.x];
  const CpqrWs ws = cpqr_ws(P);
  if (threadIdx.x != 0) return;
  const int rank = (int)*ws.state;
  const double* fin = (rank & 1) ? ws.n1 : ws.n0;  // written by the last step (step rank - 1)
  *P.rank = rank;
  int pos = rank;
  for (int j = 0; j < P.n; ++j)
    if (fin[j] >= 0.0) P.piv[pos++] = j;
}

// R rows in pivot order (one workgroup per (problem, column) entry).
__global__ __launch_bounds__(256) void k_cpqr_wide_r(const CpqrProblem* __restrict__ probs,
                                                     const int2* __restrict__ rc) {
  const int2 f = rc[blockIdx.x];
  const CpqrProblem P = probs[f.x];
  if (!P.R) return;
  const int rank = *P.rank, j = f.y;
  const double* col = P.A + (int64_t)P.piv[j] * P.lda;
  for (int i = threadIdx.x; i < rank; i += 256) P.R[i + (int64_t)j * P.maxrank] = col[i];
}

void launch_cpqr_wide_norms(hipStream_t s, const CpqrProblem* d_p, const int4* d_wg, int nwg,
                            int* d_done) {
  if (nwg <= 0) return;
  hipLaunchKernelGGL(k_cpqr_wide_norms, dim3(nwg), dim3(1024), 0, s, d_p, d_wg, d_done);
  SPD_HIP(hipGetLastError());
}
void launch_cpqr_wide_step(hipStream_t s, const CpqrProblem* d_p, const int4* d_wg, int nwg,
                           int max_m, int t, int* d_done) {
  if (nwg <= 0) return;
  SPD_REQUIRE(max_m <= kCpqrWideRows, SPD_E_INVALID, "cpqr: more than 16000 rows");
  const int vlds = max_m <= kCpqrBigRows ? 1 : 0;
  hipLaunchKernelGGL(k_cpqr_wide_step, dim3(nwg), dim3(1024), vlds ? (size_t)max_m * sizeof(double) : 0, s,
                     d_p, d_wg, t, d_done, vlds);
  SPD_HIP(hipGetLastError());
}
void launch_cpqr_wide_finish(hipStream_t s, const CpqrProblem* d_p, int nprob, const int2* d_fix,
                             int nfix, const int2* d_rc, int nrc) {
  if (nfix > 0) hipLaunchKernelGGL(k_cpqr_wide_fix, dim3(nfix), dim3(256), 0, s, d_p, d_fix);
  if (nprob > 0) hipLaunchKernelGGL(k_cpqr_wide_perm, dim3(nprob), dim3(64), 0, s, d_p);
  if (nrc > 0) hipLaunchKernelGGL(k_cpqr_wide_r, dim3(nrc), dim3(256), 0, s, d_p, d_rc);
  SPD_HIP(hipGetLastError());
}

// Q = H_0 H_1 ... H_{rank-1} [I; 0] by backward accumulation: start from the
// first rank columns of the identity and apply H_t = I - beta_t v_t v_t^T for
// t = rank-1 down to 0 (it touches rows >= t of columns >= t only); then flip
// column c where R_cc (the in-place alpha of the global kernel) is negative.
// One 1024-thread workgroup per problem, a wave per column.
__global__ __launch_bounds__(1024) void k_cpqr_formq(const CpqrProblem* __restrict__ probs) {
  constexpr int NW = 16;
  const CpqrProblem P = probs[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = P.m, rank = *P.rank;
  const int64_t ldq = P.ldq;
  double* Q = P.Q;
  for (int64_t e = threadIdx.x; e < (int64_t)m * rank; e += blockDim.x) {
    const int i = (int)(e % m), c = (int)(e / m);
    Q[i + c * ldq] = (i == c) ? 1.0 : 0.0;
  }
  __threadfence_block();
  __syncthreads();
  for (int t = rank - 1; t >= 0; --t) {
    const double beta = P.hbeta[t];
    const double* v = P.V + (int64_t)t * m;
    for (int c = t + w; c < rank; c += NW) {
      double d = 0.0;
      for (int i = t + lane; i < m; i += 64) d += v[i] * Q[i + c * ldq];
      d = wave_sum(d);
      for (int i = t + lane; i < m; i += 64) Q[i + c * ldq] -= beta * d * v[i];
    }
    __threadfence_block();
    __syncthreads();
  }
  for (int c = w; c < rank; c += NW) {
    const double rcc = P.A[c + (int64_t)P.piv[c] * P.lda];
    if (rcc < 0.0)
      for (int i = lane; i < m; i += 64) Q[i + c * ldq] = -Q[i + c * ldq];
  }
}

void launch_cpqr_formq(hipStream_t s, const CpqrProblem* d_p, int nprob) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(k_cpqr_formq, dim3(nprob), dim3(1024), 0, s, d_p);
  SPD_HIP(hipGetLastError());
}

void launch_cpqr_glob(hipStream_t s, const CpqrProblem* d_p, int nprob, int max_m, int max_n) {
  if (nprob <= 0) return;
  const size_t sh = 0;
  (void)sh;
  if (max_m <= 1024) {
    const size_t bytes = (64 * 16 + (size_t)max_n) * sizeof(double);
    hipLaunchKernelGGL((k_cpqr_glob<16>), dim3(nprob), dim3(1024), bytes, s, d_p, nullptr);
  } else if (max_m <= 2048) {
    const size_t bytes = (64 * 32 + (size_t)max_n) * sizeof(double);
    hipLaunchKernelGGL((k_cpqr_glob<32>), dim3(nprob), dim3(1024), bytes, s, d_p, nullptr);
  } else {
    SPD_REQUIRE(max_m <= kCpqrBigRows, SPD_E_INVALID, "cpqr: more than 8000 rows");
    const size_t bytes = (size_t)max_m * sizeof(double);
    hipLaunchKernelGGL(k_cpqr_big, dim3(nprob), dim3(1024), bytes, s, d_p);
  }
  SPD_HIP(hipGetLastError());
}

// ---------------------------------------------------------- vectors --
__global__ void k_gather_rows(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                              int64_t ldd, const int64_t* __restrict__ perm, int64_t n, int ncols) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n && c < ncols) dst[i + c * ldd] = src[perm[i] + c * lds];
}
void launch_gather_rows(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd,
                        const int64_t* perm, int64_t n, int ncols) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(ceil_div(n, 256), ncols), dim3(256), 0, s, src, lds, dst,
                     ldd, perm, n, ncols);
  SPD_HIP(hipGetLastError());
}

__global__ void k_scatter_rows(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                               int64_t ldd, const int64_t* __restrict__ perm, int64_t n, int ncols) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n && c < ncols) dst[perm[i] + c * ldd] = src[i + c * lds];
}
void launch_scatter_rows(hipStream_t s, const double* src, int64_t lds, double* dst, int64_t ldd,
                         const int64_t* perm, int64_t n, int ncols) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_scatter_rows, dim3(ceil_div(n, 256), ncols), dim3(256), 0, s, src, lds, dst,
                     ldd, perm, n, ncols);
  SPD_HIP(hipGetLastError());
}

// SplitMix64 (Steele, Lea, Flood 2014) on the counter (seed, original row,
// column), two draws turned into a standard normal by the Box-Muller formula.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_gaussian_fill(double* __restrict__ dst, int64_t n, int ncols, int64_t ldd,
                                const int64_t* __restrict__ perm, uint64_t seed) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n) return;
  const uint64_t ctr = (uint64_t)perm[i] * (uint64_t)ncols + (uint64_t)c;
  const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * ctr));
  const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * ctr + 1));
  const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  dst[i + c * ldd] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
__global__ void k_sketch_fill(double* __restrict__ dst, int64_t rows, int cols, int64_t ld,
                              uint64_t seed) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (t >= rows || j >= cols) return;
  const uint64_t ctr = ((uint64_t)t << 24) | (uint64_t)j;
  const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * ctr));
  const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * ctr + 1));
  const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  dst[t + j * ld] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
void launch_sketch_fill(hipStream_t s, double* dst, int64_t rows, int cols, int64_t ld,
                        uint64_t seed) {
  if (rows <= 0 || cols <= 0) return;
  SPD_REQUIRE(cols < (1 << 24), SPD_E_INVALID, "sketch: too many columns");
  hipLaunchKernelGGL(k_sketch_fill, dim3(ceil_div(rows, 256), cols), dim3(256), 0, s, dst, rows,
                     cols, ld, seed);
  SPD_HIP(hipGetLastError());
}

void launch_gaussian_fill(hipStream_t s, double* dst, int64_t n, int ncols, int64_t ldd,
                          const int64_t* perm, uint64_t seed) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_gaussian_fill, dim3(ceil_div(n, 256), ncols), dim3(256), 0, s, dst, n, ncols,
                     ldd, perm, seed);
  SPD_HIP(hipGetLastError());
}

__global__ void k_soa_points(const double* __restrict__ pts, const int64_t* __restrict__ perm,
                             int64_t n, double* __restrict__ soa) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = perm[i];
  soa[i] = pts[3 * o];
  soa[n + i] = pts[3 * o + 1];
  soa[2 * n + i] = pts[3 * o + 2];
}
void launch_soa_points(hipStream_t s, const double* pts, const int64_t* perm, int64_t n,
                       double* soa) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_soa_points, dim3(ceil_div(n, 256)), dim3(256), 0, s, pts, perm, n, soa);
  SPD_HIP(hipGetLastError());
}

// Deterministic column dot products: fixed-size chunks reduced per block, the
// partials then summed in order by one block per column.
constexpr int DOT_CHUNK = 8192;
__global__ __launch_bounds__(256) void k_coldot_partial(const double* __restrict__ x,
                                                        const double* __restrict__ y, int64_t n,
                                                        int64_t ld, double* __restrict__ partial,
                                                        int nblk) {
  __shared__ double red[4];
  const int b = blockIdx.x, c = blockIdx.y;
  const int64_t lo = (int64_t)b * DOT_CHUNK, hi = min(n, lo + DOT_CHUNK);
  double sacc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) sacc += x[i + c * ld] * y[i + c * ld];
  sacc = wave_sum(sacc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sacc;
  __syncthreads();
  if (threadIdx.x == 0) partial[b + (int64_t)c * nblk] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(64) void k_coldot_final(const double* __restrict__ partial, int nblk,
                                                     double* __restrict__ out) {
  const int c = blockIdx.x;
  double sacc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) sacc += partial[b + (int64_t)c * nblk];
  sacc = wave_sum(sacc);
  if (threadIdx.x == 0) out[c] = sacc;
}
void launch_coldot(hipStream_t s, const double* x, const double* y, int64_t n, int ncols, int64_t ld,
                   double* partial, double* out) {
  if (ncols <= 0) return;
  const int nblk = ceil_div(n, DOT_CHUNK);
  hipLaunchKernelGGL(k_coldot_partial, dim3(nblk, ncols), dim3(256), 0, s, x, y, n, ld, partial, nblk);
  hipLaunchKernelGGL(k_coldot_final, dim3(ncols), dim3(64), 0, s, partial, nblk, out);
  SPD_HIP(hipGetLastError());
}

// Fused PCG updates.  Column dot products are kept as per-chunk partial sums
// (DOT_CHUNK entries per workgroup of k_coldot_partial); every consumer adds
// the partials of its column in chunk order, so all blocks agree bit for bit
// and no separate finishing launch is needed.
__device__ __forceinline__ double chunk_sum(const double* __restrict__ partial, int nblk, int c) {
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[b + (int64_t)c * nblk];
  return s;
}

// x += alpha p, r -= alpha q with alpha = (r.z) / (p.q), then the partial sums
// of the updated r.r; block (0, c) counts the iteration and records r.z for
// the next beta.
// With zold set (flexible form), the partial sums of r_new . z_old go to rzop.
__global__ __launch_bounds__(256) void k_pcg_xr_dot(double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ rzp,
                                                    const double* __restrict__ pqp, int nblk,
                                                    const int* __restrict__ active, int64_t n,
                                                    int64_t ld, int* __restrict__ iters,
                                                    double* __restrict__ rzv,
                                                    double* __restrict__ rrp,
                                                    const double* __restrict__ zold,
                                                    double* __restrict__ rzop) {
  __shared__ double red[4], red2[4];
  __shared__ double salpha;
  const int b = blockIdx.x, c = blockIdx.y;
  if (!active[c]) return;  // uniform across the block
  // the scalars once per block (the same sums in the same order as every
  // other block), handed to its threads through LDS
  if (threadIdx.x == 0) {
    const double rz = chunk_sum(rzp, nblk, c);
    salpha = rz / chunk_sum(pqp, nblk, c);
    if (b == 0) {
      if (iters) iters[c] += 1;
      rzv[c] = rz;
    }
  }
  __syncthreads();
  const double alpha = salpha;
  const int64_t lo = (int64_t)b * DOT_CHUNK, hi = min(n, lo + DOT_CHUNK);
  double sacc = 0.0, sz = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    x[i + c * ld] += alpha * p[i + c * ld];
    const double rn = r[i + c * ld] - alpha * q[i + c * ld];
    r[i + c * ld] = rn;
    sacc += rn * rn;
    if (zold) sz += rn * zold[i + c * ld];
  }
  sacc = wave_sum(sacc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sacc;
  if (zold) {
    sz = wave_sum(sz);
    if ((threadIdx.x & 63) == 0) red2[threadIdx.x >> 6] = sz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rrp[b + (int64_t)c * nblk] = (red[0] + red[1]) + (red[2] + red[3]);
    if (zold) rzop[b + (int64_t)c * nblk] = (red2[0] + red2[1]) + (red2[2] + red2[3]);
  }
}

// active[c] stays set while ||r_c|| > rtol ||b_c||, with r.r from its partials
__global__ void k_pcg_active_partial(const double* __restrict__ rrp, int nblk,
                                     const double* __restrict__ bb, double rtol,
                                     int* __restrict__ active, int ncols, int* any_active) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    if (active[c]) {
      const bool a = sqrt(chunk_sum(rrp, nblk, c)) > rtol * sqrt(bb[c]);
      active[c] = a ? 1 : 0;
      if (a) atomicOr(&any, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *any_active = any;
}

// p = z + beta p with beta = (r.z)_new / (r.z)_old, (r.z)_new from its
// partials; with rzop set (flexible form, for an inexact preconditioner)
// beta = (r_new . (z_new - z_old)) / (r.z)_old.
__global__ void k_pcg_update_p_partial(double* __restrict__ p, const double* __restrict__ z,
                                       const double* __restrict__ rzp, int nblk,
                                       const double* __restrict__ rzv,
                                       const int* __restrict__ active, int64_t n, int64_t ld,
                                       const double* __restrict__ rzop) {
  __shared__ double sbeta;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (!active[c]) return;  // uniform across the block
  if (threadIdx.x == 0) {  // beta once per block, handed over through LDS
    double num = chunk_sum(rzp, nblk, c);
    if (rzop) num -= chunk_sum(rzop, nblk, c);
    sbeta = num / rzv[c];
  }
  __syncthreads();
  if (i >= n) return;
  p[i + c * ld] = z[i + c * ld] + sbeta * p[i + c * ld];
}

void launch_coldot_partial(hipStream_t s, const double* x, const double* y, int64_t n, int ncols,
                           int64_t ld, double* partial) {
  if (ncols <= 0) return;
  const int nblk = ceil_div(n, DOT_CHUNK);
  hipLaunchKernelGGL(k_coldot_partial, dim3(nblk, ncols), dim3(256), 0, s, x, y, n, ld, partial, nblk);
  SPD_HIP(hipGetLastError());
}

int coldot_chunks(int64_t n) { return ceil_div(n, DOT_CHUNK); }

void launch_pcg_xr_dot(hipStream_t s, double* x, double* r, const double* p, const double* q,
                       const double* rzp, const double* pqp, const int* active, int64_t n, int ncols,
                       int64_t ld, int* iters, double* rzv, double* rrp, const double* zold,
                       double* rzop) {
  const int nblk = ceil_div(n, DOT_CHUNK);
  hipLaunchKernelGGL(k_pcg_xr_dot, dim3(nblk, ncols), dim3(256), 0, s, x, r, p, q, rzp, pqp, nblk,
                     active, n, ld, iters, rzv, rrp, zold, rzop);
  SPD_HIP(hipGetLastError());
}

void launch_pcg_active_partial(hipStream_t s, const double* rrp, int64_t n, const double* bb,
                               double rtol, int* active, int ncols, int* any_active) {
  hipLaunchKernelGGL(k_pcg_active_partial, dim3(1), dim3(64), 0, s, rrp, ceil_div(n, DOT_CHUNK), bb,
                     rtol, active, ncols, any_active);
  SPD_HIP(hipGetLastError());
}

void launch_pcg_update_p_partial(hipStream_t s, double* p, const double* z, const double* rzp,
                                 const double* rzv, const int* active, int64_t n, int ncols,
                                 int64_t ld, const double* rzop) {
  hipLaunchKernelGGL(k_pcg_update_p_partial, dim3(ceil_div(n, 256), ncols), dim3(256), 0, s, p, z, rzp,
                     ceil_div(n, DOT_CHUNK), rzv, active, n, ld, rzop);
  SPD_HIP(hipGetLastError());
}

__global__ void k_pcg_active(const double* __restrict__ rr, const double* __restrict__ bb,
                             double rtol, int* __restrict__ active, int ncols, int* any_active) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    if (active[c]) {
      const bool a = sqrt(rr[c]) > rtol * sqrt(bb[c]);
      active[c] = a ? 1 : 0;
      if (a) atomicOr(&any, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *any_active = any;
}
void launch_pcg_active(hipStream_t s, const double* rr, const double* bb, double rtol, int* active,
                       int ncols, int* any_active) {
  hipLaunchKernelGGL(k_pcg_active, dim3(1), dim3(64), 0, s, rr, bb, rtol, active, ncols, any_active);
  SPD_HIP(hipGetLastError());
}

__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b,
                        int64_t n, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n) y[i + c * ld] = a * x[i + c * ld] + (b != 0.0 ? b * y[i + c * ld] : 0.0);
}
void launch_axpby(hipStream_t s, double* y, const double* x, double a, double b, int64_t n,
                  int ncols, int64_t ld) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(ceil_div(n, 256), ncols), dim3(256), 0, s, y, x, a, b, n, ld);
  SPD_HIP(hipGetLastError());
}

__global__ void k_fill(double* __restrict__ p, double v, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
void launch_fill(hipStream_t s, double* p, double v, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(ceil_div(count, 256)), dim3(256), 0, s, p, v, count);
  SPD_HIP(hipGetLastError());
}

// W (cand x k) of an interpolative decomposition from E = R11^{-1} R12 and
// the full column order: identity rows at the skeleton, E^T rows elsewhere.
__global__ void k_scatter_interp(double* __restrict__ W, int ldw, const double* __restrict__ E,
                                 int lde, const int* __restrict__ perm, int cand, int k) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)cand * k) return;
  const int j = (int)(e / k), i = (int)(e % k);  // row position j in pivot order, column i
  const int row = perm[j];
  double v;
  if (j < k) v = (i == j) ? 1.0 : 0.0;
  else v = E[i + (int64_t)(j - k) * lde];
  W[row + (int64_t)i * ldw] = v;
}
void launch_scatter_interp(hipStream_t s, double* W, int ldw, const double* E, int lde,
                           const int* perm, int cand, int k) {
  if ((int64_t)cand * k <= 0) return;
  hipLaunchKernelGGL(k_scatter_interp, dim3(ceil_div((int64_t)cand * k, 256)), dim3(256), 0, s, W, ldw,
                     E, lde, perm, cand, k);
  SPD_HIP(hipGetLastError());
}

__global__ void k_gather_skel(const int* __restrict__ cand, const int* __restrict__ piv, int k,
                              int* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) out[j] = cand[piv[j]];
}
void launch_gather_skel(hipStream_t s, const int* cand, const int* piv, int k, int* out) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_gather_skel, dim3(ceil_div(k, 256)), dim3(256), 0, s, cand, piv, k, out);
  SPD_HIP(hipGetLastError());
}

}  // namespace spd
