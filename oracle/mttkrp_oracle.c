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
 * Build: gcc -O2 -fPIC -shared -fopenmp oracle/mttkrp_oracle.c -o oracle/liboracle.so -lm
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

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

/*
 * oracle_mttkrp on several host threads (OpenMP), for timing the oracle on
 * all cores of a machine; the definition and the per-term arithmetic are
 * those of oracle_mttkrp.  The non-zeros are cut into one contiguous chunk
 * per thread, each visited in input order.  When nthreads private copies of
 * M (and S) fit in a quarter of physical memory (and in 64 GiB), each thread sums its chunk
 * into its own copy and the copies are added in thread order afterwards
 * (deterministic for a given thread count); otherwise, or when force_atomic
 * is set, the threads add into M and S with atomic updates.  Only the order
 * of the additions differs from oracle_mttkrp.  nthreads <= 0 takes
 * omp_get_max_threads().  Returns the number of threads used, negated when
 * the atomic form was taken.
 */
int oracle_mttkrp_omp(int N, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                      const double* vals, const double* const* factors, int R, int mode,
                      double* M, double* S, int nthreads, int force_atomic) {
  const size_t out_elems = (size_t)dims[mode] * (size_t)R;
  int T = nthreads > 0 ? nthreads : omp_get_max_threads();
  if (T < 1) T = 1;
  const double phys = (double)sysconf(_SC_PHYS_PAGES) * (double)sysconf(_SC_PAGESIZE);
  const double priv = (double)T * (double)out_elems * sizeof(double) * (S ? 2.0 : 1.0);
  const int atomic = force_atomic || priv > 0.25 * phys || priv > 64.0 * (1 << 30);
  memset(M, 0, out_elems * sizeof(double));
  if (S) memset(S, 0, out_elems * sizeof(double));
  double** pm = NULL;
  double** ps = NULL;
  if (!atomic) {
    pm = (double**)calloc((size_t)T, sizeof(double*));
    ps = (double**)calloc((size_t)T, sizeof(double*));
  }
#pragma omp parallel num_threads(T)
  {
    const int tid = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    const int64_t lo = nnz * tid / nt, hi = nnz * (tid + 1) / nt;
    double* m = M;
    double* s = S;
    if (!atomic) {
      m = tid == 0 ? M : (double*)calloc(out_elems, sizeof(double));
      s = (S == NULL) ? NULL : (tid == 0 ? S : (double*)calloc(out_elems, sizeof(double)));
      if (!m || (S && !s)) {
        fprintf(stderr, "oracle_mttkrp_omp: out of memory for a private output\n");
        abort();
      }
      pm[tid] = m;
      ps[tid] = s;
    }
    for (int64_t k = lo; k < hi; ++k) {
      const size_t row = (size_t)coords[mode][k] * (size_t)R;
      for (int r = 0; r < R; ++r) {
        double p = vals[k];
        for (int q = 0; q < N; ++q) {
          if (q == mode) continue;
          p *= factors[q][(size_t)coords[q][k] * (size_t)R + (size_t)r];
        }
        if (atomic) {
#pragma omp atomic
          M[row + (size_t)r] += p;
          if (S) {
            const double a = fabs(p);
#pragma omp atomic
            S[row + (size_t)r] += a;
          }
        } else {
          m[row + (size_t)r] += p;
          if (s) s[row + (size_t)r] += fabs(p);
        }
      }
    }
#pragma omp barrier
    if (!atomic) {
      /* thread-order sum of the private copies, each thread over its slice of entries */
      const size_t e0 = out_elems * (size_t)tid / (size_t)nt;
      const size_t e1 = out_elems * (size_t)(tid + 1) / (size_t)nt;
      for (int u = 1; u < nt; ++u)
        for (size_t e = e0; e < e1; ++e) {
          M[e] += pm[u][e];
          if (S) S[e] += ps[u][e];
        }
#pragma omp barrier
      if (tid > 0) {
        free(m);
        if (s) free(s);
      }
    }
    if (tid == 0) T = nt;
  }
  free(pm);
  free(ps);
  return atomic ? -T : T;
}

/*
 * oracle_mttkrp_rows on several host threads (OpenMP), for the full-size
 * parity checks: fp64 values, fp32 factors widened exactly as they are read
 * (as in oracle_mttkrp_rows_f32).  The non-zeros are cut into one contiguous
 * chunk per thread, each visited in input order into a private copy of the
 * listed rows; the copies are added in thread order.  Only the order of the
 * additions differs from the serial definition.  nthreads <= 0 takes
 * omp_get_max_threads(); returns the number of threads used.
 */
int oracle_mttkrp_rows_omp(int N, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                           const double* vals, const float* const* factors, int R, int mode,
                           int64_t nrows, const uint32_t* rows, double* M_rows, double* S_rows,
                           int nthreads) {
  int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)dims[mode]);
  for (uint64_t i = 0; i < dims[mode]; ++i) slot[i] = -1;
  for (int64_t j = 0; j < nrows; ++j) slot[rows[j]] = j;
  const size_t elems = (size_t)nrows * (size_t)R;
  int T = nthreads > 0 ? nthreads : omp_get_max_threads();
  if (T < 1) T = 1;
  double* pm = (double*)calloc((size_t)T * elems + 1, sizeof(double));
  double* ps = (double*)calloc((size_t)T * elems + 1, sizeof(double));
  if (!slot || !pm || !ps) {
    fprintf(stderr, "oracle_mttkrp_rows_omp: out of memory\n");
    abort();
  }
  int used = 1;
#pragma omp parallel num_threads(T)
  {
    const int tid = omp_get_thread_num();
    const int nt = omp_get_num_threads();
    const int64_t lo = nnz * tid / nt, hi = nnz * (tid + 1) / nt;
    double* m = pm + (size_t)tid * elems;
    double* s = ps + (size_t)tid * elems;
    for (int64_t k = lo; k < hi; ++k) {
      const int64_t j = slot[coords[mode][k]];
      if (j < 0) continue;
      for (int r = 0; r < R; ++r) {
        double p = vals[k];
        for (int q = 0; q < N; ++q) {
          if (q == mode) continue;
          p *= (double)factors[q][(size_t)coords[q][k] * (size_t)R + (size_t)r];
        }
        m[(size_t)j * (size_t)R + (size_t)r] += p;
        s[(size_t)j * (size_t)R + (size_t)r] += fabs(p);
      }
    }
    if (tid == 0) used = nt;
  }
  memset(M_rows, 0, sizeof(double) * elems);
  if (S_rows) memset(S_rows, 0, sizeof(double) * elems);
  for (int u = 0; u < used; ++u)
    for (size_t e = 0; e < elems; ++e) {
      M_rows[e] += pm[(size_t)u * elems + e];
      if (S_rows) S_rows[e] += ps[(size_t)u * elems + e];
    }
  free(pm);
  free(ps);
  free(slot);
  return used;
}

/*
 * oracle_cp_model with the non-zeros shared among host threads (OpenMP): each
 * xhat_k is computed exactly as in oracle_cp_model, so the result is the same
 * bit for bit.
 */
void oracle_cp_model_omp(int N, int64_t nnz, const uint32_t* const* coords,
                         const double* const* factors, int R, double* xhat, int nthreads) {
  const int T = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for num_threads(T) schedule(static)
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
