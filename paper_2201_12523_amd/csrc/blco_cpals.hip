// CP-ALS (Algorithm 1) around the BLCO MTTKRP, for AMD Instinct MI355X (gfx950).
//
// Per iteration and mode n: V = Hadamard product of the Gram matrices of the
// other factors, M = mode-n MTTKRP, A^(n) = M V^+.  The small dense steps run
// in their own kernels: Gram matrices (fp32 products, fp64 sums; on the
// matrix cores for R <= 32), the R x R
// pseudo-inverse of V in one workgroup (fp64), the row-wise product M V^+
// (fp64 sums), and the fit.  The MTTKRP is the library's (blco_mttkrp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "blco_internal.h"

using blco::set_error;
using blco::clear_error;

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(BLCO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

namespace {

constexpr int kMaxRank = 64;       // largest rank of the dense steps
constexpr int kGramRows = 64;      // rows staged in LDS per Gram step
constexpr int kGramThreads = 256;
constexpr int kSolveThreads = 1024;
// V is positive definite to working precision when every elimination pivot
// exceeds this fraction of V's largest diagonal entry
constexpr double kPivotTol = 1e-13;

template <typename FT>
__device__ __forceinline__ float ld_elem(const FT* p, int64_t i);
template <>
__device__ __forceinline__ float ld_elem<float>(const float* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ float ld_elem<uint16_t>(const uint16_t* p, int64_t i) {
  return __uint_as_float((uint32_t)p[i] << 16);
}

__global__ void k_zero_f64(double* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_zero_i32(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// G += A^T A over this workgroup's rows: products in fp32 over kGramRows rows
// at a time, sums in fp64; one fp64 atomic per entry per workgroup.
template <typename FT>
__global__ __launch_bounds__(kGramThreads) void k_gram(const FT* __restrict__ A, int64_t rows,
                                                       int R, int64_t per, double* __restrict__ G) {
  __shared__ float s_a[kGramRows * kMaxRank];
  constexpr int E = kMaxRank * kMaxRank / kGramThreads;   // entries per thread (max)
  const int tid = threadIdx.x;
  const int RR = R * R;
  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(rows, lo + per);
  for (int64_t r0 = lo; r0 < hi; r0 += kGramRows) {
    const int nr = (int)min<int64_t>(kGramRows, hi - r0);
    __syncthreads();
    for (int i = tid; i < nr * R; i += kGramThreads) s_a[i] = ld_elem<FT>(A, r0 * R + i);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ent = tid + e * kGramThreads;
      if (ent < RR) {
        const int a = ent / R, b = ent - (ent / R) * R;
        float s = 0.f;
        for (int i = 0; i < nr; ++i) s = fmaf(s_a[i * R + a], s_a[i * R + b], s);
        acc[e] += (double)s;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int ent = tid + e * kGramThreads;
    if (ent < RR && lo < hi) atomicAdd(&G[ent], acc[e]);
  }
}

// G += A^T A for R <= 32 on the matrix cores: each wave takes a contiguous
// range of rows and, two rows per step, feeds the 2 x 32 tile X of those rows
// to v_mfma_f32_32x32x2f32 as both operands (A-operand X^T, B-operand X: lane l
// holds X[l / 32][l % 32] for both), accumulating the 32 x 32 product in fp32;
// every kGramFlush rows the accumulators are added into fp64 registers, and
// at the end each wave adds its fp64 sums into G with fp64 atomics.  Output
// layout of the instruction: register v of lane l holds row
// 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
constexpr int kGramFlush = 64;   // rows summed in fp32 before moving to fp64
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <typename FT>
__global__ __launch_bounds__(256) void k_gram_mfma(const FT* __restrict__ A, int64_t rows, int R,
                                                   int64_t per_wave, double* __restrict__ G) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t lo = wave * per_wave;
  const int64_t hi = min(rows, lo + per_wave);
  if (lo >= hi) return;
  const int col = lane & 31;
  const int kk = lane >> 5;
  const bool cact = col < R;
  double acc64[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc64[v] = 0.0;
  for (int64_t r0 = lo; r0 < hi; r0 += kGramFlush) {
    const int64_t r1 = min(hi, r0 + kGramFlush);
    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    constexpr int S = 8;   // row pairs loaded before the first use
    for (int64_t r = r0; r < r1; r += 2 * S) {
      float x[S];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const int64_t row = r + 2 * q + kk;
        x[q] = (cact && row < r1) ? ld_elem<FT>(A, row * R + col) : 0.f;
      }
#pragma unroll
      for (int q = 0; q < S; ++q) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(x[q], x[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) acc64[v] += (double)acc[v];
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * kk + (v & 3);
    if (i < R && cact) atomicAdd(&G[i * R + col], acc64[v]);
  }
}

// *out += sum_i x[i] * y[i] (fp32 inputs, fp64 sums; one atomic per workgroup)
__global__ __launch_bounds__(256) void k_dot(const float* __restrict__ x, const float* __restrict__ y,
                                             int64_t n, double* __restrict__ out) {
  __shared__ double s_w[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += (double)x[i] * (double)y[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, s_w[0] + s_w[1] + s_w[2] + s_w[3]);
}

// V = Hadamard product of the Gram matrices of every mode but `skip` (all ones
// when there is none), into a (R x R, row-major), by all threads of the block.
__device__ void hadamard(const double* __restrict__ grams, int N, int skip, int R, double* a) {
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != skip) v *= grams[(size_t)m * R * R + e];
    a[e] = v;
  }
}

// In-place Gauss-Jordan inverse of the R x R matrix in `a` (LDS or global),
// diagonal pivots; returns false (uniformly) when a pivot is <= tol.
__device__ bool gauss_jordan(double* a, int R, double tol, double* row, double* col) {
  for (int k = 0; k < R; ++k) {
    __syncthreads();
    const double piv = a[k * R + k];
    if (!(piv > tol)) return false;
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
      row[i] = a[k * R + i];
      col[i] = a[i * R + k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
      const int i = e / R, j = e - (e / R) * R;
      const double nr = (j == k ? 1.0 : row[j]) / piv;   // new pivot-row entry
      if (i == k)
        a[e] = nr;
      else
        a[e] = (j == k ? 0.0 : a[e]) - col[i] * nr;
    }
  }
  __syncthreads();
  return true;
}

// V^+ of V = Hadamard of the other modes' Grams (one workgroup, fp64).
// Positive definite to working precision: Gauss-Jordan inverse in LDS.
// Otherwise: rank-revealing pivoted Cholesky P^T V P = L L^T (L: R x k, full
// column rank), and V^+ = P L (L^T L)^-2 L^T P^T, with the matrices in `scratch`
// (3 R x R).  `fallbacks` counts the calls that took the second route.
__global__ __launch_bounds__(kSolveThreads) void k_pinv_v(const double* __restrict__ grams, int N,
                                                          int n, int R, double* __restrict__ vinv,
                                                          double* __restrict__ scratch,
                                                          int* __restrict__ fallbacks) {
  __shared__ double s_a[kMaxRank * kMaxRank];
  __shared__ double s_row[kMaxRank], s_col[kMaxRank];
  __shared__ int s_perm[kMaxRank];
  __shared__ double s_tol;
  __shared__ int s_piv, s_rank;
  const int tid = threadIdx.x;
  hadamard(grams, N, n, R, s_a);
  __syncthreads();
  if (tid == 0) {
    double d = 0.0;
    for (int i = 0; i < R; ++i) d = fmax(d, s_a[i * R + i]);
    s_tol = kPivotTol * d;
  }
  __syncthreads();
  const double tol = s_tol;
  if (gauss_jordan(s_a, R, tol, s_row, s_col)) {
    for (int e = tid; e < R * R; e += blockDim.x) vinv[e] = s_a[e];
    return;
  }
  // ---- rank-revealing pivoted Cholesky of V (reloaded)
  __syncthreads();
  if (tid == 0) atomicAdd(fallbacks, 1);
  hadamard(grams, N, n, R, s_a);
  for (int i = tid; i < R; i += blockDim.x) s_perm[i] = i;
  if (tid == 0) s_rank = 0;
  for (int k = 0; k < R; ++k) {
    __syncthreads();
    if (tid == 0) {
      int j = k;
      for (int i = k + 1; i < R; ++i)
        if (s_a[i * R + i] > s_a[j * R + j]) j = i;
      s_piv = (s_a[j * R + j] > tol) ? j : -1;
      if (s_piv >= 0) s_rank = k + 1;
    }
    __syncthreads();
    const int j = s_piv;
    if (j < 0) break;
    if (j != k) {   // symmetric swap of rows and columns k and j
      for (int e = tid; e < R; e += blockDim.x) {
        const double t = s_a[k * R + e];
        s_a[k * R + e] = s_a[j * R + e];
        s_a[j * R + e] = t;
      }
      __syncthreads();
      for (int e = tid; e < R; e += blockDim.x) {
        const double t = s_a[e * R + k];
        s_a[e * R + k] = s_a[e * R + j];
        s_a[e * R + j] = t;
      }
      if (tid == 0) {
        const int t = s_perm[k];
        s_perm[k] = s_perm[j];
        s_perm[j] = t;
      }
      __syncthreads();
    }
    const double d = sqrt(s_a[k * R + k]);
    __syncthreads();
    for (int i = tid; i < R; i += blockDim.x) {
      if (i > k) s_a[i * R + k] /= d;
    }
    if (tid == 0) s_a[k * R + k] = d;
    __syncthreads();
    for (int e = tid; e < R * R; e += blockDim.x) {
      const int i = e / R, c = e - (e / R) * R;
      if (i > k && c > k) s_a[e] -= s_a[i * R + k] * s_a[c * R + k];
    }
  }
  __syncthreads();
  const int rk = s_rank;
  double* L = scratch;                 // R x rk (stride R)
  double* C = scratch + R * R;         // rk x rk (stride R): L^T L, then its inverse
  double* T = scratch + 2 * R * R;     // R x rk (stride R): L (L^T L)^-1
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int i = e / R, c = e - (e / R) * R;
    L[e] = (c < rk && c <= i) ? s_a[e] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < rk * rk; e += blockDim.x) {
    const int a = e / rk, b = e - (e / rk) * rk;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += L[i * R + a] * L[i * R + b];
    s_a[a * rk + b] = s;
  }
  __syncthreads();
  if (rk > 0) gauss_jordan(s_a, rk, 0.0, s_row, s_col);   // L^T L is positive definite
  for (int e = tid; e < rk * rk; e += blockDim.x) C[(e / rk) * R + e % rk] = s_a[e];
  __syncthreads();
  for (int e = tid; e < R * rk; e += blockDim.x) {
    const int i = e / rk, c = e - (e / rk) * rk;
    double s = 0.0;
    for (int q = 0; q < rk; ++q) s += L[i * R + q] * C[q * R + c];
    T[i * R + c] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += blockDim.x) {
    const int a = e / R, b = e - (e / R) * R;
    double s = 0.0;
    for (int q = 0; q < rk; ++q) s += T[a * R + q] * T[b * R + q];
    vinv[s_perm[a] * R + s_perm[b]] = s;
  }
}

// A = M V^+ row by row (fp64 sums of fp32 M and fp64 V^+).
__global__ __launch_bounds__(256) void k_apply_vinv(const float* __restrict__ M, int64_t rows,
                                                    int R, const double* __restrict__ vinv,
                                                    float* __restrict__ A) {
  __shared__ double s_v[kMaxRank * kMaxRank];
  for (int e = threadIdx.x; e < R * R; e += 256) s_v[e] = vinv[e];
  __syncthreads();
  const int per = 256 / R;            // rows per pass of the block
  const int lr = threadIdx.x / R, c = threadIdx.x - (threadIdx.x / R) * R;
  if (lr >= per) return;
  for (int64_t i = (int64_t)blockIdx.x * per + lr; i < rows; i += (int64_t)gridDim.x * per) {
    const float* m = M + i * R;
    double s = 0.0;
    for (int q = 0; q < R; ++q) s += (double)m[q] * s_v[q * R + c];
    A[i * R + c] = (float)s;
  }
}

// scal[0] = ||X||^2, scal[1] = <X, Xhat>; writes scal[2] = fit
__global__ void k_fit(const double* __restrict__ grams, int N, int R, double* __restrict__ scal) {
  __shared__ double s_w[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < N; ++m) v *= grams[(size_t)m * R * R + e];
    s += v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double model2 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) model2 += s_w[w];
    const double x2 = scal[0];
    const double r2 = fmax(x2 - 2.0 * scal[1] + model2, 0.0);
    scal[2] = 1.0 - sqrt(r2) / sqrt(x2);
  }
}

int launch_gram(const void* A, int dtype, int64_t rows, int R, double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, G, R * R);
  HIPCHK(hipGetLastError());
  if (rows <= 0) return BLCO_OK;
  if (R <= 32) {
    // matrix cores: about 2048 waves, each over at least one flush block of rows
    int64_t per = std::max<int64_t>((rows + 2047) / 2048, kGramFlush);
    per = (per + kGramFlush - 1) / kGramFlush * kGramFlush;
    const int64_t waves = (rows + per - 1) / per;
    const int64_t nwg = (waves + 3) / 4;
    if (dtype == BLCO_BF16)
      hipLaunchKernelGGL(k_gram_mfma<uint16_t>, dim3((unsigned)nwg), dim3(256), 0, s,
                         static_cast<const uint16_t*>(A), rows, R, per, G);
    else
      hipLaunchKernelGGL(k_gram_mfma<float>, dim3((unsigned)nwg), dim3(256), 0, s,
                         static_cast<const float*>(A), rows, R, per, G);
    HIPCHK(hipGetLastError());
    return BLCO_OK;
  }
  const int64_t want = 512;
  int64_t per = std::max<int64_t>((rows + want - 1) / want, kGramRows);
  const int64_t nwg = (rows + per - 1) / per;
  if (dtype == BLCO_BF16)
    hipLaunchKernelGGL(k_gram<uint16_t>, dim3((unsigned)nwg), dim3(kGramThreads), 0, s,
                       static_cast<const uint16_t*>(A), rows, R, per, G);
  else
    hipLaunchKernelGGL(k_gram<float>, dim3((unsigned)nwg), dim3(kGramThreads), 0, s,
                       static_cast<const float*>(A), rows, R, per, G);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

int launch_dot(const float* x, const float* y, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return BLCO_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_dot, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n, out);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int blco_gram(const void* A, int dtype, int64_t rows, int rank, double* G,
                         void* stream) {
  clear_error();
  if (!A && rows > 0) return set_error(BLCO_EINVAL, "A is NULL");
  if (!G) return set_error(BLCO_EINVAL, "G is NULL");
  if (rows < 0) return set_error(BLCO_EINVAL, "rows %lld < 0", (long long)rows);
  if (rank < 1 || rank > kMaxRank)
    return set_error(BLCO_EINVAL, "rank %d outside 1..%d", rank, kMaxRank);
  if (dtype != BLCO_F32 && dtype != BLCO_BF16) return set_error(BLCO_EINVAL, "dtype %d", dtype);
  return launch_gram(A, dtype, rows, rank, G, static_cast<hipStream_t>(stream));
}

extern "C" int blco_cp_als(blco_tensor* t, float* const* factors, int rank,
                           const blco_cpals_opts* opts, double* fits, blco_cpals_report* report,
                           void* stream) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "CP-ALS needs a tensor placed in device memory");
  const int N = t->lay.N;
  if (rank < 1 || rank > kMaxRank)
    return set_error(BLCO_EINVAL, "rank %d outside 1..%d", rank, kMaxRank);
  if (!factors) return set_error(BLCO_EINVAL, "factors is NULL");
  for (int m = 0; m < N; ++m)
    if (!factors[m]) return set_error(BLCO_EINVAL, "factors[%d] is NULL", m);
  blco_cpals_opts o = {25, 1e-5, BLCO_F32};
  if (opts) o = *opts;
  if (o.max_iters < 1) return set_error(BLCO_EINVAL, "max_iters %d < 1", o.max_iters);
  if (o.tol != o.tol) return set_error(BLCO_EINVAL, "tol is NaN");
  if (o.factor_dtype != BLCO_F32 && o.factor_dtype != BLCO_BF16)
    return set_error(BLCO_EINVAL, "factor dtype %d", o.factor_dtype);
  if (t->nnz == 0) return set_error(BLCO_EINVAL, "the tensor has no non-zeros");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int R = rank;
  uint64_t maxI = 0, sumI = 0;
  for (int m = 0; m < N; ++m) {
    maxI = std::max<uint64_t>(maxI, t->lay.dims[m]);
    sumI += t->lay.dims[m];
  }
  // workspace: M, Grams, V^+, pseudo-inverse scratch, scalars, counter, bf16 copies
  const size_t bytes_M = (size_t)maxI * R * sizeof(float);
  const size_t bytes_G = (size_t)N * R * R * sizeof(double);
  const size_t bytes_V = (size_t)R * R * sizeof(double);
  const size_t bytes_S = 3 * bytes_V;
  const size_t bytes_sc = 4 * sizeof(double) + sizeof(int) * 2;
  const size_t bytes_h = o.factor_dtype == BLCO_BF16 ? (size_t)sumI * R * sizeof(uint16_t) : 0;
  auto align = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t total = align(bytes_M) + align(bytes_G) + align(bytes_V) + align(bytes_S) +
                       align(bytes_sc) + align(bytes_h);
  DevBuf ws;
  HIPCHK(hipMalloc(&ws.p, total));
  char* base = static_cast<char*>(ws.p);
  float* dM = reinterpret_cast<float*>(base);
  base += align(bytes_M);
  double* dG = reinterpret_cast<double*>(base);
  base += align(bytes_G);
  double* dV = reinterpret_cast<double*>(base);
  base += align(bytes_V);
  double* dS = reinterpret_cast<double*>(base);
  base += align(bytes_S);
  double* dsc = reinterpret_cast<double*>(base);
  int* dfb = reinterpret_cast<int*>(dsc + 4);
  base += align(bytes_sc);
  uint16_t* dh = bytes_h ? reinterpret_cast<uint16_t*>(base) : nullptr;
  std::vector<const void*> mt(N);
  std::vector<uint16_t*> half(N, nullptr);
  {
    size_t off = 0;
    for (int m = 0; m < N; ++m) {
      if (dh) {
        half[m] = dh + off;
        off += (size_t)t->lay.dims[m] * R;
      }
      mt[m] = dh ? static_cast<const void*>(half[m]) : static_cast<const void*>(factors[m]);
    }
  }
  const int mdt = o.factor_dtype;
  int rc;
  // ||X||^2, the Grams, the bf16 copies
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, dsc, 4);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, dfb, 2);
  HIPCHK(hipGetLastError());
  if ((rc = launch_dot(t->d_vals, t->d_vals, t->nnz, dsc, s)) != BLCO_OK) return rc;
  for (int m = 0; m < N; ++m) {
    if ((rc = launch_gram(factors[m], BLCO_F32, (int64_t)t->lay.dims[m], R,
                          dG + (size_t)m * R * R, s)) != BLCO_OK)
      return rc;
    if (dh && (rc = blco_cast_bf16(factors[m], half[m], (int64_t)t->lay.dims[m] * R, s)) != BLCO_OK)
      return rc;
  }
  int it = 0;
  double prev = 0.0;
  for (; it < o.max_iters; ++it) {
    for (int n = 0; n < N; ++n) {
      const int64_t In = (int64_t)t->lay.dims[n];
      hipLaunchKernelGGL(k_pinv_v, dim3(1), dim3(kSolveThreads), 0, s, dG, N, n, R, dV, dS, dfb);
      HIPCHK(hipGetLastError());
      if ((rc = blco_mttkrp(t, n, mt.data(), mdt, R, dM, s)) != BLCO_OK) return rc;
      const int per = 256 / R;
      const int64_t blocks = std::min<int64_t>((In + per - 1) / per, 4096);
      hipLaunchKernelGGL(k_apply_vinv, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0,
                         s, dM, In, R, dV, factors[n]);
      HIPCHK(hipGetLastError());
      if ((rc = launch_gram(factors[n], BLCO_F32, In, R, dG + (size_t)n * R * R, s)) != BLCO_OK)
        return rc;
      if (dh && (rc = blco_cast_bf16(factors[n], half[n], In * R, s)) != BLCO_OK) return rc;
    }
    // <X, Xhat> from the last mode's MTTKRP (still in dM) and its new factor
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, dsc + 1, 1);
    HIPCHK(hipGetLastError());
    const int64_t Il = (int64_t)t->lay.dims[N - 1];
    if ((rc = launch_dot(dM, factors[N - 1], Il * R, dsc + 1, s)) != BLCO_OK) return rc;
    hipLaunchKernelGGL(k_fit, dim3(1), dim3(1024), 0, s, dG, N, R, dsc);
    HIPCHK(hipGetLastError());
    double fit = 0.0;
    HIPCHK(hipMemcpyAsync(&fit, dsc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (fits) fits[it] = fit;
    const bool stop = it > 0 && fit - prev < o.tol;
    prev = fit;
    if (stop) {
      ++it;
      break;
    }
  }
  int fb = 0;
  HIPCHK(hipMemcpyAsync(&fb, dfb, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (report) {
    report->iters = std::min(it, o.max_iters);
    report->pinv_fallbacks = fb;
  }
  return BLCO_OK;
}
