/*
 * Oracle (test infrastructure only): classical modified interpolation of
 * Section 3.1, written as a plain loop over the rows of A.
 *
 * Coarse numbering: C points in ascending fine index (cidx).  A C row of P is
 * the identity.  For an F row i let
 *   C_i  = strong dependencies of i that are C points,
 *   F_i  = strong dependencies of i that are F points,
 *   W_i  = every other off-diagonal entry of row i (weak).
 * For k in F_i the distribution coefficients of row k keep only entries of
 * the opposite sign to its diagonal:
 *   ahat_kj = a_kj   if sign(a_kj) != sign(a_kk),   else 0,
 *   sigma_ik = sum over j in C_i (ascending j) of ahat_kj, starting from 0.
 * A strong F neighbour with sigma_ik == 0 shares no usable C point with i and
 * is lumped into the diagonal together with the weak entries:
 *   at_ii = a_ii + sum of a_in over n in W_i or lumped   (ascending column),
 *   w_ij  = -(a_ij + sum over non-lumped k in F_i of (a_ik * ahat_kj) / sigma_ik)
 *           / at_ii                                       (ascending k),
 * for j in C_i.  No truncation.  An F row with C_i empty is empty.
 *
 * Every sum is evaluated left to right, one IEEE operation per term; build
 * with -ffp-contract=off so that no product is fused into a sum.
 */
#include <stdint.h>

static int sign_of(double v) { return (v > 0.0) - (v < 0.0); }

/* Value of A(k, j), or 0 when row k stores no column j (binary search over
 * the sorted columns of row k). */
static double entry(const int64_t* indptr, const int32_t* indices, const double* data,
                    int64_t k, int64_t j) {
  int64_t lo = indptr[k], hi = indptr[k + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (indices[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return (lo < indptr[k + 1] && indices[lo] == j) ? data[lo] : 0.0;
}

static double diag_of(const int64_t* indptr, const int32_t* indices, const double* data,
                      int64_t k) {
  return entry(indptr, indices, data, k, k);
}

/*
 * n        rows of A (square); indptr[n+1], indices, data: CSR, sorted columns.
 * strong   one flag per stored entry (1: the column is a strong dependency).
 * cf       1 = C point, -1 = F point.
 * cidx     coarse index of every C point (ascending fine order).
 * sigma    scratch of at least max row length doubles.
 * p_*      output CSR of P with room for nnz(A) + n entries.
 * Returns the number of entries of P.
 */
int64_t oracle_interpolation(int64_t n, const int64_t* indptr, const int32_t* indices,
                             const double* data, const uint8_t* strong, const int8_t* cf,
                             const int64_t* cidx, double* sigma, int64_t* p_indptr,
                             int32_t* p_indices, double* p_data) {
  int64_t nnz_p = 0;
  p_indptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t a0 = indptr[i], a1 = indptr[i + 1];
    if (cf[i] == 1) {
      p_indices[nnz_p] = (int32_t)cidx[i];
      p_data[nnz_p] = 1.0;
      ++nnz_p;
      p_indptr[i + 1] = nnz_p;
      continue;
    }
    /* sigma_ik for every strong F neighbour k (stored at the entry's offset) */
    for (int64_t e = a0; e < a1; ++e) {
      const int64_t k = indices[e];
      sigma[e - a0] = 0.0;
      if (!strong[e] || cf[k] == 1) continue;
      const int sk = sign_of(diag_of(indptr, indices, data, k));
      double s = 0.0;
      for (int64_t f = a0; f < a1; ++f) {
        const int64_t j = indices[f];
        if (!strong[f] || cf[j] != 1) continue;
        const double akj = entry(indptr, indices, data, k, j);
        const double ahat = sign_of(akj) != sk ? akj : 0.0;
        s = s + ahat;
      }
      sigma[e - a0] = s;
    }
    /* modified diagonal: weak entries and lumped strong F entries */
    double at = diag_of(indptr, indices, data, i);
    for (int64_t e = a0; e < a1; ++e) {
      const int64_t k = indices[e];
      if (k == i) continue;
      const int weak = !strong[e];
      const int lumped = strong[e] && cf[k] != 1 && sigma[e - a0] == 0.0;
      if (weak || lumped) at = at + data[e];
    }
    /* one weight per strong C point j, ascending j */
    for (int64_t f = a0; f < a1; ++f) {
      const int64_t j = indices[f];
      if (!strong[f] || cf[j] != 1) continue;
      double num = data[f];
      for (int64_t e = a0; e < a1; ++e) {
        const int64_t k = indices[e];
        if (!strong[e] || cf[k] == 1 || sigma[e - a0] == 0.0) continue;
        const int sk = sign_of(diag_of(indptr, indices, data, k));
        const double akj = entry(indptr, indices, data, k, j);
        const double ahat = sign_of(akj) != sk ? akj : 0.0;
        num = num + (data[e] * ahat) / sigma[e - a0];
      }
      p_indices[nnz_p] = (int32_t)cidx[j];
      p_data[nnz_p] = -num / at;
      ++nnz_p;
    }
    p_indptr[i + 1] = nnz_p;
  }
  return nnz_p;
}
