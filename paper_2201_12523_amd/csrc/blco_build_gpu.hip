// BLCO construction on the GPU (Sections 4.1-4.2), from coordinates and values
// already in device memory.
//
// Steps, each a kernel or a device-wide primitive on the caller's stream:
//   1. ALTO linearization of every coordinate (Section 4.1): bit j of mode n
//      goes to position pos[n][j] of a 64- or 128-bit index (per-byte deposit
//      tables); out-of-range coordinates are flagged;
//   2. a stable radix sort along the encoding line (blco_sort.hip), least
//      significant digits first, the values moved along: one sort over the low
//      64 bits, then, for indices over 64 bits, one over the high bits.  The first
//      also moves the high bits (32-bit words for indices of at most 96 bits), the
//      second the low bits, so no array follows a permutation by gathers;
//   3. re-encoding in sorted order (Figure 6b) from the sorted index: every
//      index bit below K moves to its mode's field (a byte table), the block
//      key is the index above bit K;
//   4. runs of equal block key (flags and a stream compaction), copied to the host, where
//      the block list, per-run high bits and tile table are finished by the
//      same code as the host builder;
//   5. the frequent rows of each mode (sampled rows sorted and run-length
//      counted, then a stable descending radix sort of the counts).
// The result equals blco_build's bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "blco_internal.h"

using namespace blco;

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(BLCO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

namespace {

struct LinParams {
  const uint32_t* coords[BLCO_MAX_MODES];
  uint64_t dims[BLCO_MAX_MODES];
  uint8_t pos[BLCO_MAX_MODES][32];
  int b[BLCO_MAX_MODES];
  int w[BLCO_MAX_MODES];
  int s[BLCO_MAX_MODES];
  int N;
  int K;
  int T;
};

// ALTO index of every non-zero (lo: bits 0..63; hi: bits 64..127, or hi32: bits
// 64..95 of an index of at most 96 bits; or neither); *bad = smallest non-zero
// number with a coordinate out of range.
// dep[((m * 4 + k) * 256 + v) * 2 + {0, 1}]: the (lo, hi) index bits of byte k of a
// mode-m coordinate holding v.  Without a high part the lo halves of the table are
// staged in LDS (N * 8 KiB of dynamic LDS), once per workgroup of a grid that
// strides over the non-zeros.
__global__ __launch_bounds__(256) void k_linearize(LinParams p, int64_t n,
                                                   const uint64_t* __restrict__ dep,
                                                   uint64_t* __restrict__ lo,
                                                   uint64_t* __restrict__ hi,
                                                   uint32_t* __restrict__ hi32,
                                                   unsigned long long* __restrict__ bad) {
  extern __shared__ uint64_t s_dep[];   // [(m * 4 + k) * 256 + v], lo halves (no high part)
  const bool wide = hi || hi32;
  if (!wide) {
    for (int j = threadIdx.x; j < p.N * 4 * 256; j += 256) s_dep[j] = dep[2 * j];
    __syncthreads();
  }
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
  uint64_t l = 0, h = 0;
  for (int m = 0; m < p.N; ++m) {
    uint32_t c = p.coords[m][i];
    if ((uint64_t)c >= p.dims[m]) {
      atomicMin(bad, (unsigned long long)i);
      c = 0;
    }
    if (!wide) {
      const uint64_t* d = s_dep + (size_t)m * 4 * 256;
#pragma unroll
      for (int k = 0; k < 4; ++k) l |= d[k * 256 + ((c >> (8 * k)) & 255u)];
    } else {
      const uint64_t* d = dep + (size_t)m * 4 * 256 * 2;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t v = (c >> (8 * k)) & 255u;
        l |= d[(k * 256 + v) * 2];
        h |= d[(k * 256 + v) * 2 + 1];
      }
    }
  }
  lo[i] = l;
  if (hi) hi[i] = h;
  if (hi32) hi32[i] = (uint32_t)h;
  }
}

// Keys and block keys in sorted order, from the sorted index (slo: bits 0..63;
// shi: bits 64..127, or shi32: bits 64..95; or neither): the key gathers every index
// bit below K into its mode's field through a byte table (enc[k][v]: key bits of
// byte k holding v); the block key is the index above bit K.  The values are
// already in place: the sorts moved them.
constexpr int kEncBytes = 8;   // K <= 64
__global__ __launch_bounds__(256) void k_encode(int64_t n, int K, const uint64_t* __restrict__ enc,
                                                const uint64_t* __restrict__ slo,
                                                const uint64_t* __restrict__ shi,
                                                const uint32_t* __restrict__ shi32,
                                                uint64_t* __restrict__ keys,
                                                uint64_t* __restrict__ bkey) {
  __shared__ uint64_t s_enc[kEncBytes * 256];
  for (int i = threadIdx.x; i < kEncBytes * 256; i += 256) s_enc[i] = enc[i];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t l = slo[i], h = shi ? shi[i] : shi32 ? (uint64_t)shi32[i] : 0;
  const uint64_t low = K >= 64 ? l : (l & ((1ULL << K) - 1));
  uint64_t key = 0;
#pragma unroll
  for (int k = 0; k < kEncBytes; ++k) key |= s_enc[k * 256 + ((low >> (8 * k)) & 255)];
  keys[i] = key;
  if (!bkey) return;
  uint64_t B;
  if (K >= 64)
    B = h >> (K - 64);
  else if (K == 0)
    B = l;
  else
    B = (l >> K) | (h << (64 - K));
  bkey[i] = B;
}

__global__ __launch_bounds__(256) void k_run_flags(const uint64_t* __restrict__ bkey, int64_t n,
                                                   uint8_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || bkey[i] != bkey[i - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_gather_keys(const uint64_t* __restrict__ bkey,
                                                     const int64_t* __restrict__ starts,
                                                     int64_t nruns, uint64_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < nruns) out[r] = bkey[starts[r]];
}

__global__ __launch_bounds__(256) void k_sample(const uint32_t* __restrict__ c, int64_t samples,
                                                int64_t step, uint32_t* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s < samples) out[s] = c[s * step];
}

__global__ __launch_bounds__(256) void k_row_flags(const uint32_t* __restrict__ sorted, int64_t n,
                                                   uint8_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1 : 0;
}

// Run-length encoding from the run starts of a sorted array: the value and the
// length of every run.
__global__ __launch_bounds__(256) void k_runs(const uint32_t* __restrict__ sorted,
                                              const int64_t* __restrict__ starts, int64_t nruns,
                                              int64_t n, uint32_t* __restrict__ uniq,
                                              uint32_t* __restrict__ cnt) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nruns) return;
  const int64_t a = starts[r], e = r + 1 < nruns ? starts[r + 1] : n;
  uniq[r] = sorted[a];
  cnt[r] = (uint32_t)(e - a);
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) { *p = v; }

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>((n + 255) / 256, 1); }

constexpr unsigned kStrideGrid = 2048;   // workgroups of grid-stride kernels (8 per CU)

// Events at the stage boundaries of one build on its stream (released on return).
struct StageEvents {
  static constexpr int kN = 6;
  hipEvent_t ev[kN] = {};
  bool ok = true;
  StageEvents() {
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) ok = false;
  }
  ~StageEvents() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int k, hipStream_t s) {
    if (ok) (void)hipEventRecord(ev[k], s);
  }
  // elapsed ms between consecutive marks, once the last has completed
  void read(double* ms) {
    if (!ok || hipEventSynchronize(ev[kN - 1]) != hipSuccess) return;
    for (int k = 0; k + 1 < kN; ++k) {
      float x = 0.f;
      if (hipEventElapsedTime(&x, ev[k], ev[k + 1]) == hipSuccess) ms[k] = x;
    }
  }
};

// device allocations released on every return path
struct Pool {
  std::vector<void*> ptrs;
  ~Pool() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int get(T** out, size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
      return set_error(BLCO_ENOMEM, "device allocation of %zu bytes failed",
                       std::max<size_t>(count, 1) * sizeof(T));
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return BLCO_OK;
  }
};

template <typename T>
int upload_to(T** dst, const T* src, size_t count, hipStream_t s, size_t* acc) {
  const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
  HIPCHK(hipMalloc((void**)dst, bytes));
  if (count) HIPCHK(hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s));
  *acc += bytes;
  return BLCO_OK;
}

void release_tensor_arrays(blco_tensor* t) {
  for (void* p : {(void*)t->d_keys, (void*)t->d_vals, (void*)t->d_run_start,
                  (void*)t->d_run_base, (void*)t->d_tile_run, (void*)t->d_hot})
    if (p) (void)hipFree(p);
  t->d_keys = nullptr;
  t->d_vals = nullptr;
  t->d_run_start = nullptr;
  t->d_run_base = nullptr;
  t->d_tile_run = nullptr;
  t->d_hot = nullptr;
  free_host_arrays(t);
}

void pinned_release(void* p) { (void)hipHostFree(p); }

// Frequent rows of every mode, as find_hot_rows: the rows of every step-th
// non-zero are sorted and run-length counted (no atomics: hot rows would
// serialise), then the kHotMax + 1 most frequent (ties by row, as the stable
// sort keeps ascending rows) are kept and those reaching the threshold marked.
int gpu_hot_rows(const LinParams& lp, int64_t nnz, int64_t min_count, Pool& pool, hipStream_t s,
                 blco_tensor* t) {
  const int N = lp.N;
  t->hot.assign((size_t)N * kHotMax, 0xFFFFFFFFu);
  t->hot_cnt.assign((size_t)N * (kHotMax + 1), 0);
  for (int n = 0; n < N; ++n) t->nhot[n] = 0;
  if (nnz <= 0 || min_count < 0) return BLCO_OK;
  const int64_t step = std::max<int64_t>(1, nnz / ((int64_t)1 << 22));
  const int64_t samples = (nnz + step - 1) / step;
  const uint64_t need = (uint64_t)std::max<int64_t>(1, (min_count + step - 1) / step);
  int rc;
  uint32_t *smp, *sorted, *uniq, *cnt, *cnt2, *row2, *tk, *tv;
  uint8_t* flag;
  int64_t* starts;
  unsigned int* ws;
  if ((rc = pool.get(&smp, samples)) || (rc = pool.get(&sorted, samples)) ||
      (rc = pool.get(&uniq, samples)) || (rc = pool.get(&cnt, samples)) ||
      (rc = pool.get(&cnt2, samples)) || (rc = pool.get(&row2, samples)) ||
      (rc = pool.get(&tk, samples)) || (rc = pool.get(&tv, samples)) ||
      (rc = pool.get(&flag, samples)) || (rc = pool.get(&starts, samples)) ||
      (rc = pool.get(&ws, std::max(sort_workspace_words(samples), select_workspace_words(samples)))))
    return rc;
  for (int n = 0; n < N; ++n) {
    const uint64_t I = lp.dims[n];
    if (I > ((uint64_t)1 << 26)) continue;
    const int bits = std::max(1, lp.b[n]);
    hipLaunchKernelGGL(k_sample, dim3(grid_of(samples)), dim3(256), 0, s, lp.coords[n], samples,
                       step, smp);
    HIPCHK(hipGetLastError());
    // the sampled rows in order, their runs (row, count), the runs by count,
    // most frequent first (equal counts keep ascending rows: the sort is stable)
    if ((rc = radix_sort_u32(smp, nullptr, sorted, nullptr, tk, nullptr, samples, bits, false, ws,
                             s)))
      return rc;
    hipLaunchKernelGGL(k_row_flags, dim3(grid_of(samples)), dim3(256), 0, s, sorted, samples,
                       flag);
    HIPCHK(hipGetLastError());
    int64_t nu = 0;
    if ((rc = select_flagged(flag, samples, starts, &nu, ws, s))) return rc;
    hipLaunchKernelGGL(k_runs, dim3(grid_of(nu)), dim3(256), 0, s, sorted, starts, nu, samples,
                       uniq, cnt);
    HIPCHK(hipGetLastError());
    if ((rc = radix_sort_u32(cnt, uniq, cnt2, row2, tk, tv, nu, 32, true, ws, s))) return rc;
    const size_t k = std::min<size_t>((size_t)nu, kHotMax + 1);
    std::vector<uint32_t> hc(k), hr(k);
    if (k) {
      HIPCHK(hipMemcpyAsync(hc.data(), cnt2, k * 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(hr.data(), row2, k * 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    int nh = 0;
    for (size_t j = 0; j < k; ++j) {
      t->hot_cnt[(size_t)n * (kHotMax + 1) + j] = (uint64_t)hc[j] * (uint64_t)step;
      if (j < (size_t)kHotMax && hc[j] >= need) t->hot[(size_t)n * kHotMax + nh++] = hr[j];
    }
    t->nhot[n] = nh;
  }
  return BLCO_OK;
}

int build_on_device(int nmodes, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
                    const float* values, int key_bits, int64_t cap, int64_t hot_min,
                    hipStream_t s, blco_tensor* t) {
  int rc = make_layout(nmodes, dims, key_bits, &t->lay);
  if (rc) return rc;
  const Layout& L = t->lay;
  t->nnz = nnz;
  t->max_block_nnz = cap;
  LinParams lp;
  memset(&lp, 0, sizeof(lp));
  lp.N = L.N;
  lp.K = L.K;
  lp.T = L.T;
  for (int m = 0; m < L.N; ++m) {
    lp.coords[m] = coords[m];
    lp.dims[m] = L.dims[m];
    lp.b[m] = L.b[m];
    lp.w[m] = L.w[m];
    lp.s[m] = L.s[m];
    for (int j = 0; j < L.b[m]; ++j) lp.pos[m][j] = (uint8_t)L.pos[m][j];
  }
  Pool pool;
  StageEvents stage;
  stage.mark(0, s);
  const bool wide = L.T > 64;
  // an index over 64 bits is sorted in two parts: the sort over the low 64 bits moves
  // the values and the high bits (32-bit words up to 96 bits, else 64-bit), the sort
  // over the high bits moves the values and the low bits; one of at most 64 bits
  // carries the values through its one sort
  const bool mid = wide && L.T <= 96;
  uint64_t *lo, *lo2, *hi = nullptr, *his = nullptr, *hif = nullptr, *bkey;
  uint32_t *h32 = nullptr, *h32s = nullptr, *h32f = nullptr, *vs = nullptr, *tv2 = nullptr;
  unsigned long long* bad;
  if ((rc = pool.get(&lo, nnz)) || (rc = pool.get(&lo2, nnz)) || (rc = pool.get(&bkey, nnz)) ||
      (rc = pool.get(&bad, 1)))
    return rc;
  if (wide && ((rc = pool.get(&vs, nnz)) || (rc = pool.get(&tv2, nnz))))
    return rc;
  if (mid && ((rc = pool.get(&h32, nnz)) || (rc = pool.get(&h32s, nnz)) ||
              (rc = pool.get(&h32f, nnz))))
    return rc;
  if (wide && !mid && ((rc = pool.get(&hi, nnz)) || (rc = pool.get(&his, nnz)) ||
                       (rc = pool.get(&hif, nnz))))
    return rc;
  // 1. linearize, through per-byte deposit tables
  std::vector<uint64_t> dep((size_t)L.N * 4 * 256 * 2, 0);
  for (int m = 0; m < L.N; ++m)
    for (int k = 0; k < 4; ++k)
      for (int v = 0; v < 256; ++v) {
        uint64_t xl = 0, xh = 0;
        for (int j = 0; j < 8; ++j) {
          const int bj = 8 * k + j;
          if (!((v >> j) & 1) || bj >= L.b[m]) continue;
          const int q = L.pos[m][bj];
          if (q < 64)
            xl |= 1ULL << q;
          else
            xh |= 1ULL << (q - 64);
        }
        dep[(((size_t)m * 4 + k) * 256 + v) * 2] = xl;
        dep[(((size_t)m * 4 + k) * 256 + v) * 2 + 1] = xh;
      }
  uint64_t* d_dep;
  if ((rc = pool.get(&d_dep, dep.size()))) return rc;
  HIPCHK(hipMemcpyAsync(d_dep, dep.data(), dep.size() * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, bad, ~0ULL);
  if (nnz > 0)
    hipLaunchKernelGGL(k_linearize, dim3(std::min<unsigned>(grid_of(nnz), kStrideGrid)), dim3(256),
                       wide ? 0 : (size_t)L.N * 4 * 256 * sizeof(uint64_t), s, lp, nnz, d_dep, lo,
                       mid ? nullptr : hi, h32, bad);
  HIPCHK(hipGetLastError());
  unsigned long long first_bad = ~0ULL;
  HIPCHK(hipMemcpyAsync(&first_bad, bad, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (first_bad != ~0ULL) {
    const int64_t i = (int64_t)first_bad;
    for (int m = 0; m < L.N; ++m) {
      uint32_t c = 0;
      HIPCHK(hipMemcpy(&c, coords[m] + i, 4, hipMemcpyDeviceToHost));
      if ((uint64_t)c >= L.dims[m])
        return set_error(BLCO_ERANGE, "coordinate %u of mode %d at non-zero %lld is >= %llu", c, m,
                         (long long)i, (unsigned long long)L.dims[m]);
    }
    return set_error(BLCO_ERANGE, "coordinate out of range at non-zero %lld", (long long)i);
  }
  // 2. stable sort along the encoding line
  stage.mark(1, s);
  size_t acc = 0;
  HIPCHK(hipMalloc((void**)&t->d_keys, sizeof(uint64_t) * std::max<int64_t>(nnz, 1)));
  HIPCHK(hipMalloc((void**)&t->d_vals, sizeof(float) * std::max<int64_t>(nnz, 1)));
  acc += (sizeof(uint64_t) + sizeof(float)) * (size_t)std::max<int64_t>(nnz, 1);
  if (nnz > 0) {
    const int nb0 = std::max(1, std::min(L.T, 64));
    uint64_t* tk;
    uint32_t* tv;
    unsigned int* ws;
    if ((rc = pool.get(&tk, nnz)) || (rc = pool.get(&tv, nnz)) ||
        (rc = pool.get(&ws, sort_workspace_words(nnz))))
      return rc;
    const uint32_t* v_in = reinterpret_cast<const uint32_t*>(values);
    uint32_t* v_out = reinterpret_cast<uint32_t*>(t->d_vals);
    if (!wide) {
      // at most 64 index bits: the values travel with the keys into the tensor
      if ((rc = radix_sort_u64(lo, v_in, lo2, v_out, tk, tv, nnz, nb0, ws, s))) return rc;
    } else {
      // the low 64 bits, moving the values and the high bits; then the high bits,
      // moving the values (into the tensor) and the low bits
      uint64_t* tk2;
      if (!mid && (rc = pool.get(&tk2, nnz))) return rc;
      SortVals v1 = {};
      v1.in32[0] = v_in;
      v1.out32[0] = vs;
      v1.tmp32[0] = tv;
      if (mid) {
        v1.in32[1] = h32;
        v1.out32[1] = h32s;
        v1.tmp32[1] = tv2;
      } else {
        v1.in64 = hi;
        v1.out64 = his;
        v1.tmp64 = tk2;
      }
      if ((rc = radix_sort_u64_vals(lo, lo2, tk, v1, nnz, nb0, ws, s))) return rc;
      SortVals v2 = {};
      v2.in32[0] = vs;
      v2.out32[0] = v_out;
      v2.tmp32[0] = tv2;
      v2.in64 = lo2;
      v2.out64 = lo;   // the unsorted low bits are no longer needed
      v2.tmp64 = tk;
      if (mid) {
        if ((rc = radix_sort_u32_vals(h32s, h32f, tv, v2, nnz, L.T - 64, ws, s))) return rc;
      } else {
        if ((rc = radix_sort_u64_vals(his, hif, tk2, v2, nnz, L.T - 64, ws, s))) return rc;
      }
      std::swap(lo, lo2);   // lo2: the low bits in the final order
    }
  }
  // 3. re-encode in sorted order; keys and values go straight into the tensor
  stage.mark(2, s);
  std::vector<uint64_t> enc((size_t)kEncBytes * 256, 0);
  {
    int owner_mode[128], owner_bit[128];
    for (int m = 0; m < L.N; ++m)
      for (int j = 0; j < L.b[m]; ++j) {
        owner_mode[L.pos[m][j]] = m;
        owner_bit[L.pos[m][j]] = j;
      }
    for (int k = 0; k < kEncBytes; ++k)
      for (int v = 0; v < 256; ++v) {
        uint64_t x = 0;
        for (int j = 0; j < 8; ++j) {
          const int q = 8 * k + j;
          if (!((v >> j) & 1) || q >= L.K) continue;
          x |= 1ULL << (L.s[owner_mode[q]] + owner_bit[q]);
        }
        enc[(size_t)k * 256 + v] = x;
      }
  }
  uint64_t* d_enc;
  if ((rc = pool.get(&d_enc, enc.size()))) return rc;
  HIPCHK(hipMemcpyAsync(d_enc, enc.data(), enc.size() * 8, hipMemcpyHostToDevice, s));
  // without block bits every block key is 0: no block keys to write or scan
  const bool blocked = L.S > 0;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_encode, dim3(grid_of(nnz)), dim3(256), 0, s, nnz, L.K, d_enc, lo2,
                       wide && !mid ? hif : nullptr, mid ? h32f : nullptr, t->d_keys,
                       blocked ? bkey : nullptr);
    HIPCHK(hipGetLastError());
  }
  // 4. runs of equal block key
  stage.mark(3, s);
  std::vector<int64_t> run_start;
  std::vector<uint64_t> run_key;
  if (nnz > 0 && !blocked) {
    run_start.assign(1, 0);
    run_key.assign(1, 0);
  } else if (nnz > 0) {
    uint8_t* flag;
    int64_t* starts;
    uint64_t* keys_at;
    if ((rc = pool.get(&flag, nnz)) || (rc = pool.get(&starts, nnz))) return rc;
    hipLaunchKernelGGL(k_run_flags, dim3(grid_of(nnz)), dim3(256), 0, s, bkey, nnz, flag);
    HIPCHK(hipGetLastError());
    unsigned int* ws;
    if ((rc = pool.get(&ws, select_workspace_words(nnz)))) return rc;
    int64_t nruns = 0;
    if ((rc = select_flagged(flag, nnz, starts, &nruns, ws, s))) return rc;
    if ((rc = pool.get(&keys_at, nruns))) return rc;
    hipLaunchKernelGGL(k_gather_keys, dim3(grid_of(nruns)), dim3(256), 0, s, bkey, starts, nruns,
                       keys_at);
    HIPCHK(hipGetLastError());
    run_start.resize((size_t)nruns);
    run_key.resize((size_t)nruns);
    HIPCHK(hipMemcpyAsync(run_start.data(), starts, 8 * nruns, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(run_key.data(), keys_at, 8 * nruns, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  finish_runs(L, nnz, run_start, run_key, cap, t);
  // 5. frequent rows
  stage.mark(4, s);
  if ((rc = gpu_hot_rows(lp, nnz, hot_min, pool, s, t))) return rc;
  stage.mark(5, s);
  if ((rc = upload_to(&t->d_run_start, t->run_start.data(), t->run_start.size(), s, &acc)) ||
      (rc = upload_to(&t->d_run_base, t->run_base.data(), t->run_base.size(), s, &acc)) ||
      (rc = upload_to(&t->d_tile_run, t->tile_run.data(), t->tile_run.size(), s, &acc)) ||
      (rc = upload_to(&t->d_hot, t->hot.data(), t->hot.size(), s, &acc)))
    return rc;
  HIPCHK(hipStreamSynchronize(s));
  stage.read(t->build_stage_ms);
  t->device_bytes = acc;
  return BLCO_OK;
}

}  // namespace

extern "C" int blco_build_device(int nmodes, const uint64_t* dims, int64_t nnz,
                                 const uint32_t* const* coords, const float* values,
                                 const blco_build_opts* opts, void* stream, blco_tensor** out) {
  clear_error();
  if (!out) return set_error(BLCO_EINVAL, "out is NULL");
  *out = nullptr;
  if (nmodes < 1 || nmodes > BLCO_MAX_MODES)
    return set_error(BLCO_EUNSUPPORTED, "nmodes %d outside 1..%d", nmodes, BLCO_MAX_MODES);
  if (!dims) return set_error(BLCO_EINVAL, "dims is NULL");
  if (nnz < 0) return set_error(BLCO_EINVAL, "nnz %lld < 0", (long long)nnz);
  if (nnz >= ((int64_t)1 << 31) - 1)
    return set_error(BLCO_EUNSUPPORTED, "the GPU builder takes fewer than 2^31 - 1 non-zeros");
  if (nnz > 0 && (!coords || !values)) return set_error(BLCO_EINVAL, "coords or values is NULL");
  for (int n = 0; n < nmodes; ++n) {
    if (dims[n] < 1) return set_error(BLCO_EINVAL, "dims[%d] = 0", n);
    if (dims[n] > (1ULL << 32))
      return set_error(BLCO_EUNSUPPORTED, "dims[%d] = %llu > 2^32", n, (unsigned long long)dims[n]);
    if (nnz > 0 && !coords[n]) return set_error(BLCO_EINVAL, "coords[%d] is NULL", n);
  }
  int key_bits = 64;
  int64_t cap = (int64_t)1 << 27;
  int placement = BLCO_PLACE_DEVICE;
  int64_t hot_min = kHotMinCount;
  if (opts) {
    key_bits = opts->key_bits;
    cap = opts->max_block_nnz;
    placement = opts->placement;
    if (opts->hot_min_count != 0) hot_min = opts->hot_min_count;
  }
  if (key_bits < 1 || key_bits > 64) return set_error(BLCO_EINVAL, "key_bits %d outside 1..64", key_bits);
  if (cap < 1) return set_error(BLCO_EINVAL, "max_block_nnz < 1");
  if (placement != BLCO_PLACE_DEVICE && placement != BLCO_PLACE_PINNED)
    return set_error(BLCO_EINVAL, "the GPU builder places the tensor on the device or in pinned memory");
  blco_tensor* t = new (std::nothrow) blco_tensor();
  if (!t) return set_error(BLCO_ENOMEM, "host allocation failed");
  t->placement = placement;
  t->hot_forced = opts && opts->hot_min_count > 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return set_error(BLCO_EDEVICE, "hipGetDevice failed");
  }
  int rc = build_on_device(nmodes, dims, nnz, coords, values, key_bits, cap, hot_min, s, t);
  if (rc == BLCO_OK && placement == BLCO_PLACE_PINNED) {
    // the non-zeros move to pinned host memory for streaming
    const size_t n1 = (size_t)std::max<int64_t>(nnz, 1);
    if (hipHostMalloc((void**)&t->h_keys, n1 * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&t->h_vals, n1 * 4, hipHostMallocDefault) != hipSuccess) {
      rc = set_error(BLCO_ENOMEM, "pinned allocation of %lld non-zeros failed", (long long)nnz);
    } else {
      t->host_free = pinned_release;
      if (hipMemcpy(t->h_keys, t->d_keys, (size_t)nnz * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(t->h_vals, t->d_vals, (size_t)nnz * 4, hipMemcpyDeviceToHost) != hipSuccess) {
        rc = set_error(BLCO_EDEVICE, "copy of the non-zeros to pinned memory failed");
      } else {
        (void)hipFree(t->d_keys);
        (void)hipFree(t->d_vals);
        t->d_keys = nullptr;
        t->d_vals = nullptr;
        t->device_bytes -= n1 * 12;
      }
    }
  }
  if (rc != BLCO_OK) {
    release_tensor_arrays(t);
    delete t;
    return rc;
  }
  *out = t;
  return BLCO_OK;
}
