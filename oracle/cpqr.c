/* Householder QR with column pivoting (oracle; test infrastructure only).
 *
 * The plain loop of oracle/linalg.py's CPQR written in C, for the large proxy
 * and sketch matrices of the H^2 construction, where the interpreted loop
 * takes minutes per node.  Same definition (Algorithm 5.1, step 3, with the
 * readings of the oracle): at step t the pivot is the unused column whose
 * trailing part (rows t..m-1) has the largest exactly recomputed 2-norm,
 * lowest column index on ties; the factorization stops before step t at
 * max_rank, at min(m, n), or when that norm is not above tol times the first
 * pivot's norm.  Columns stay in place; the pivot order is recorded.
 *
 * A is column-major m x n (lda = m) and is overwritten: on return rows
 * 0..rank-1 of the pivot columns hold R (diagonal alpha_t, before any sign
 * normalisation) and the other columns hold Q^T applied to them.  V (m x
 * max_rank, column-major) receives the Householder vectors (zero above row
 * t), betas the factors of H_t = I - beta_t v_t v_t^T, alpha the diagonal.
 * Returns the rank.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle_cpqr(int m, int n, double *A, double tol, int max_rank, int *piv, double *alpha,
                double *betas, double *V) {
  int kmax = m < n ? m : n;
  if (max_rank < kmax) kmax = max_rank < 0 ? 0 : max_rank;
  char *used = (char *)calloc((size_t)n, 1);
  double *nrm2 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double ref = -1.0;
  int rank = 0;
  for (int c = 0; c < n; ++c) {
    const double *col = A + (size_t)c * m;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += col[i] * col[i];
    nrm2[c] = s;
  }
  for (int t = 0; t < kmax; ++t) {
    int j = -1;
    double best = -1.0;
    for (int c = 0; c < n; ++c)
      if (!used[c] && nrm2[c] > best) { best = nrm2[c]; j = c; }
    if (j < 0) break;
    const double nrm = sqrt(best);
    if (ref < 0.0) ref = nrm;
    if (!(nrm > tol * ref) || nrm == 0.0) break;
    double *x = A + (size_t)j * m;
    double *v = V + (size_t)t * m;
    memset(v, 0, sizeof(double) * (size_t)m);
    const double a = x[t] >= 0.0 ? -nrm : nrm; /* H x = a e_t */
    for (int i = t; i < m; ++i) v[i] = x[i];
    v[t] -= a;
    double vv = 0.0;
    for (int i = t; i < m; ++i) vv += v[i] * v[i];
    const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
    used[j] = 1;
    for (int c = 0; c < n; ++c) {
      if (used[c]) continue;
      double *col = A + (size_t)c * m;
      double d = 0.0;
      for (int i = t; i < m; ++i) d += v[i] * col[i];
      double s = 0.0;
      for (int i = t; i < m; ++i) {
        col[i] -= beta * (v[i] * d);
        if (i > t) s += col[i] * col[i];
      }
      nrm2[c] = s;
    }
    for (int i = t; i < m; ++i) x[i] = 0.0;
    x[t] = a;
    piv[t] = j;
    alpha[t] = a;
    betas[t] = beta;
    rank = t + 1;
  }
  free(used);
  free(nrm2);
  return rank;
}
