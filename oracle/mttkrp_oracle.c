/*
 * ORACLE — test infrastructure only.  Plain, slow, fp64 CPU reference for the
 * sparse MTTKRP and the sparse CP fit loss.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the library never does.
 * It shares no code, header or table with the GPU library.
 *
 * Notation follows the paper: an N-mode sparse tensor X with non-zeros
 * x_k at coordinates (i_1^k, ..., i_N^k), 0-based here, and factor matrices
 * A^(m) of shape I_m x R stored row-major (row i = R contiguous doubles).
 *
 * Build: gcc -O2 -fPIC -shared oracle/mttkrp_oracle.c -o oracle/liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Mode-n MTTKRP, Eq. (1) of Section 2.3, in the per-non-zero form of Figure 3:
 * for each non-zero, fetch row i_m of every A^(m), m != n (step 1), take their
 * Hadamard product (step 2), scale by x_k (step 3) and add it to row i_n of M
 * (step 4).  Non-zeros are visited in input order; m ascends inside a term.
 *
 * M and S are I_n x R, overwritten.  S accumulates |term|, the scale used to
 * normalise the difference between two summation orders.
 */
void oracle_mttkrp(int N, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                   const double* vals, const double* const* factors, int R, int mode,
                   double* M, double* S) {
  size_t out_elems = (size_t)dims[mode] * (size_t)R;
  memset(M, 0, out_elems * sizeof(double));
  if (S) memset(S, 0, out_elems * sizeof(double));
  for (int64_t k = 0; k < nnz; ++k) {
    size_t row = (size_t)coords[mode][k] * (size_t)R;
    for (int r = 0; r < R; ++r) {
      double p = vals[k];
      for (int m = 0; m < N; ++m) {
        if (m == mode) continue;
        p *= factors[m][(size_t)coords[m][k] * (size_t)R + (size_t)r];
      }
      M[row + (size_t)r] += p;
      if (S) S[row + (size_t)r] += fabs(p);
    }
  }
}

/*
 * The same definition restricted to the output rows listed in `rows`
 * (distinct indices of mode n): out row j of M_rows/S_rows holds M[rows[j], :].
 * Every non-zero is still visited in input order; those whose i_n is not
 * listed contribute to no listed row and are skipped.
 */
void oracle_mttkrp_rows(int N, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                        const double* vals, const double* const* factors, int R, int mode,
                        int64_t nrows, const uint32_t* rows, double* M_rows, double* S_rows) {
  int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)dims[mode]);
  for (uint64_t i = 0; i < dims[mode]; ++i) slot[i] = -1;
  for (int64_t j = 0; j < nrows; ++j) slot[rows[j]] = j;
  memset(M_rows, 0, sizeof(double) * (size_t)nrows * (size_t)R);
  if (S_rows) memset(S_rows, 0, sizeof(double) * (size_t)nrows * (size_t)R);
  for (int64_t k = 0; k < nnz; ++k) {
    int64_t j = slot[coords[mode][k]];
    if (j < 0) continue;
    for (int r = 0; r < R; ++r) {
      double p = vals[k];
      for (int m = 0; m < N; ++m) {
        if (m == mode) continue;
        p *= factors[m][(size_t)coords[m][k] * (size_t)R + (size_t)r];
      }
      M_rows[(size_t)j * (size_t)R + (size_t)r] += p;
      if (S_rows) S_rows[(size_t)j * (size_t)R + (size_t)r] += fabs(p);
    }
  }
  free(slot);
}

/*
 * CP model at the non-zeros (Section 2.2: X is approximated by the sum over r
 * of the outer products of the r-th columns of the factors):
 *   xhat_k = sum_r prod_{m=1..N} A^(m)[i_m^k, r].
 */
void oracle_cp_model(int N, int64_t nnz, const uint32_t* const* coords,
                     const double* const* factors, int R, double* xhat) {
  for (int64_t k = 0; k < nnz; ++k) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) {
      double p = 1.0;
      for (int m = 0; m < N; ++m) p *= factors[m][(size_t)coords[m][k] * (size_t)R + (size_t)r];
      s += p;
    }
    xhat[k] = s;
  }
}

/*
 * Sparse CP fit loss over the non-zeros, f = 1/2 sum_k (x_k - xhat_k)^2.
 * Writes the residuals e_k = x_k - xhat_k and returns f.
 */
double oracle_cp_loss(int N, int64_t nnz, const uint32_t* const* coords, const double* vals,
                      const double* const* factors, int R, double* resid) {
  oracle_cp_model(N, nnz, coords, factors, R, resid);
  double f = 0.0;
  for (int64_t k = 0; k < nnz; ++k) {
    double e = vals[k] - resid[k];
    resid[k] = e;
    f += 0.5 * e * e;
  }
  return f;
}

/*
 * oracle_mttkrp_rows with fp32 values and factors, each converted exactly to
 * fp64 as it is read (same definition, same visiting order; no fp64 copies of
 * large factor matrices are needed).
 */
void oracle_mttkrp_rows_f32(int N, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                            const float* vals, const float* const* factors, int R, int mode,
                            int64_t nrows, const uint32_t* rows, double* M_rows, double* S_rows) {
  int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)dims[mode]);
  for (uint64_t i = 0; i < dims[mode]; ++i) slot[i] = -1;
  for (int64_t j = 0; j < nrows; ++j) slot[rows[j]] = j;
  memset(M_rows, 0, sizeof(double) * (size_t)nrows * (size_t)R);
  if (S_rows) memset(S_rows, 0, sizeof(double) * (size_t)nrows * (size_t)R);
  for (int64_t k = 0; k < nnz; ++k) {
    int64_t j = slot[coords[mode][k]];
    if (j < 0) continue;
    for (int r = 0; r < R; ++r) {
      double p = (double)vals[k];
      for (int m = 0; m < N; ++m) {
        if (m == mode) continue;
        p *= (double)factors[m][(size_t)coords[m][k] * (size_t)R + (size_t)r];
      }
      M_rows[(size_t)j * (size_t)R + (size_t)r] += p;
      if (S_rows) S_rows[(size_t)j * (size_t)R + (size_t)r] += fabs(p);
    }
  }
  free(slot);
}
