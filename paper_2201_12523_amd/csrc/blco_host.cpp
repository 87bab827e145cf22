// Host-side BLCO construction (Section 4 of Nguyen et al., ICS '22).
//
// COO -> ALTO linear index (Section 4.1, Figure 6a) -> stable radix sort
// along the encoding line -> re-encoded keys with contiguous per-mode fields
// (Figure 6b) -> blocks on the uppermost T - K bits, split to a non-zero cap
// (Section 4.2) -> per-tile run table for the kernels.
//
// This file makes no GPU call, so a tensor with host placement can be built
// and inspected on a machine without a GPU.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "blco_internal.h"

namespace blco {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

// ------------------------------------------------------------------ threads

static int num_threads() {
  const char* e = getenv("BLCO_THREADS");
  long n = e ? atol(e) : (long)std::thread::hardware_concurrency();
  if (n < 1) n = 1;
  if (n > 16) n = 16;
  return (int)n;
}

// f(tid, lo, hi) over nt contiguous chunks of [0, n)
template <class F>
static void parallel_chunks(int64_t n, int nt, F f) {
  if (n < (1 << 16)) nt = 1;
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(f, t, n * t / nt, n * (t + 1) / nt);
  f(0, (int64_t)0, n / nt);
  for (auto& x : th) x.join();
}

// ------------------------------------------------------------------ layout

int make_layout(int N, const uint64_t* dims, int key_bits, Layout* L) {
  L->N = N;
  L->T = 0;
  int maxb = 0;
  for (int n = 0; n < N; ++n) {
    L->dims[n] = dims[n];
    int b = 0;
    while ((1ULL << b) < dims[n]) ++b;
    L->b[n] = b;
    L->T += b;
    maxb = std::max(maxb, b);
  }
  L->K = std::min(L->T, key_bits);
  L->S = L->T - L->K;
  if (L->S > 64)
    return set_error(BLCO_EUNSUPPORTED, "block key needs %d bits (> 64); raise key_bits", L->S);
  // ALTO order: round robin over the modes from the least significant bit
  int p = 0;
  for (int j = 0; j < maxb; ++j)
    for (int n = 0; n < N; ++n)
      if (j < L->b[n]) L->pos[n][j] = p++;
  int acc = 0;
  for (int n = 0; n < N; ++n) {
    int h = 0;
    for (int j = 0; j < L->b[n]; ++j) h += L->pos[n][j] >= L->K;
    L->h[n] = h;
    L->w[n] = L->b[n] - h;
    L->s[n] = acc;
    acc += L->w[n];
  }
  return BLCO_OK;
}

// ------------------------------------------------------------- records

#pragma pack(push, 4)
struct Rec64 {   // encoding line of at most 64 bits
  uint64_t lo;
  float v;
};
struct Rec128 {  // encoding line of 65..128 bits
  uint64_t lo;
  uint64_t hi;
  float v;
};
#pragma pack(pop)

static inline uint32_t digit_of(const Rec64& r, int off, uint32_t mask) {
  return (uint32_t)(r.lo >> off) & mask;
}
static inline uint32_t digit_of(const Rec128& r, int off, uint32_t mask) {
  if (off >= 64) return (uint32_t)(r.hi >> (off - 64)) & mask;
  uint64_t x = r.lo >> off;
  if (off > 0) x |= r.hi << (64 - off);
  return (uint32_t)x & mask;
}
static inline uint64_t shr(const Rec64& r, int K) { return K >= 64 ? 0 : (r.lo >> K); }
static inline uint64_t shr(const Rec128& r, int K) {
  if (K >= 64) return r.hi >> (K - 64);
  if (K == 0) return r.lo;
  return (r.lo >> K) | (r.hi << (64 - K));
}

struct U128 {
  uint64_t lo, hi;
};

// Stable LSD radix sort on the low T bits of the line, digits of <= 11 bits.
template <class Rec>
static Rec* radix_sort(Rec* a, Rec* b, int64_t n, int T, int nt) {
  if (n < 2 || T == 0) return a;
  if (n < (1 << 16)) nt = 1;
  int passes = (T + 10) / 11;
  int dbits = (T + passes - 1) / passes;
  uint32_t mask = (1u << dbits) - 1;
  int nb = 1 << dbits;
  std::vector<int64_t> hist((size_t)nt * nb);
  for (int pass = 0; pass < passes; ++pass) {
    int off = pass * dbits;
    parallel_chunks(n, nt, [&](int tid, int64_t lo, int64_t hi) {
      int64_t* h = &hist[(size_t)tid * nb];
      std::fill(h, h + nb, 0);
      for (int64_t i = lo; i < hi; ++i) h[digit_of(a[i], off, mask)]++;
    });
    // skip a digit that every record shares
    int64_t nonzero = 0;
    for (int d = 0; d < nb; ++d) {
      int64_t c = 0;
      for (int t = 0; t < nt; ++t) c += hist[(size_t)t * nb + d];
      nonzero += c != 0;
    }
    if (nonzero <= 1) continue;
    int64_t run = 0;
    for (int d = 0; d < nb; ++d)
      for (int t = 0; t < nt; ++t) {
        int64_t c = hist[(size_t)t * nb + d];
        hist[(size_t)t * nb + d] = run;
        run += c;
      }
    parallel_chunks(n, nt, [&](int tid, int64_t lo, int64_t hi) {
      int64_t* h = &hist[(size_t)tid * nb];
      for (int64_t i = lo; i < hi; ++i) b[h[digit_of(a[i], off, mask)]++] = a[i];
    });
    std::swap(a, b);
  }
  return a;
}

// Blocks (runs split to max_block_nnz), per-run high bits of every mode, and
// the tile -> run table, from the runs of equal block key (Section 4.2).
void finish_runs(const Layout& L, int64_t nnz, const std::vector<int64_t>& run_start,
                 const std::vector<uint64_t>& run_key, int64_t max_block_nnz, blco_tensor* t) {
  const int N = L.N;
  t->run_start = run_start;
  t->run_start.push_back(nnz);
  t->block_id.clear();
  t->block_start.clear();
  const int64_t nruns = (int64_t)run_key.size();
  for (int64_t r = 0; r < nruns; ++r)
    for (int64_t c = t->run_start[r]; c < t->run_start[r + 1]; c += max_block_nnz) {
      t->block_id.push_back(run_key[r]);
      t->block_start.push_back(c);
    }
  t->block_start.push_back(nnz);
  // high bits of every mode held by each run's block key, pre-shifted to their place
  t->run_base.assign((size_t)nruns * N, 0);
  for (int64_t r = 0; r < nruns; ++r)
    for (int n = 0; n < N; ++n) {
      uint64_t hi = 0;
      for (int j = 0; j < L.h[n]; ++j) hi |= ((run_key[r] >> (L.pos[n][L.w[n] + j] - L.K)) & 1ULL) << j;
      t->run_base[(size_t)r * N + n] = (uint32_t)(hi << L.w[n]);
    }
  // tile -> run of its first non-zero
  int64_t ntiles = (nnz + kTile - 1) / kTile;
  t->tile_run.resize((size_t)ntiles);
  int64_t r = 0;
  for (int64_t tl = 0; tl < ntiles; ++tl) {
    int64_t e = tl * kTile;
    while (t->run_start[r + 1] <= e) ++r;
    t->tile_run[(size_t)tl] = (int32_t)r;
  }
}

template <class Rec>
static int build_with(const Layout& L, int64_t nnz, const uint32_t* const* coords,
                      const float* values, int64_t max_block_nnz, blco_tensor* t) {
  const int N = L.N;
  const int nt = num_threads();
  // bit-deposit tables: byte k of a mode-n index -> its bits on the encoding line
  std::vector<U128> dep((size_t)N * 4 * 256);
  for (int n = 0; n < N; ++n)
    for (int k = 0; k < 4; ++k)
      for (int v = 0; v < 256; ++v) {
        U128 x{0, 0};
        for (int j = 0; j < 8; ++j) {
          int bj = 8 * k + j;
          if (!((v >> j) & 1) || bj >= L.b[n]) continue;
          int p = L.pos[n][bj];
          if (p < 64) x.lo |= 1ULL << p; else x.hi |= 1ULL << (p - 64);
        }
        dep[((size_t)n * 4 + k) * 256 + v] = x;
      }
  Rec* a = (Rec*)malloc(sizeof(Rec) * (size_t)std::max<int64_t>(nnz, 1));
  Rec* b = (Rec*)malloc(sizeof(Rec) * (size_t)std::max<int64_t>(nnz, 1));
  if (!a || !b) {
    free(a);
    free(b);
    return set_error(BLCO_ENOMEM, "host allocation of %lld sort records failed", (long long)nnz);
  }
  std::atomic<int64_t> bad{-1};
  parallel_chunks(nnz, nt, [&](int tid, int64_t lo, int64_t hi) {
    (void)tid;
    for (int64_t i = lo; i < hi; ++i) {
      U128 x{0, 0};
      for (int n = 0; n < N; ++n) {
        uint32_t c = coords[n][i];
        if ((uint64_t)c >= L.dims[n]) {
          int64_t e = -1;
          bad.compare_exchange_strong(e, i);
          c = 0;
        }
        const U128* d = &dep[(size_t)n * 4 * 256];
        for (int k = 0; k < 4; ++k) {
          const U128& y = d[k * 256 + ((c >> (8 * k)) & 255)];
          x.lo |= y.lo;
          x.hi |= y.hi;
        }
      }
      Rec r;
      r.lo = x.lo;
      if constexpr (sizeof(Rec) == sizeof(Rec128)) ((Rec128&)r).hi = x.hi;
      r.v = values[i];
      a[i] = r;
    }
  });
  if (bad.load() >= 0) {
    int64_t i = bad.load();
    int n = 0;
    for (; n < N; ++n)
      if ((uint64_t)coords[n][i] >= L.dims[n]) break;
    free(a);
    free(b);
    return set_error(BLCO_ERANGE, "coordinate %u of mode %d at non-zero %lld is >= %llu",
                     coords[n][i], n, (long long)i, (unsigned long long)L.dims[n]);
  }
  Rec* s = radix_sort(a, b, nnz, L.T, nt);
  Rec* spare = (s == a) ? b : a;
  free(spare);

  // runs of equal block key
  std::vector<int64_t> run_start;
  std::vector<uint64_t> run_key;
  for (int64_t i = 0; i < nnz; ++i) {
    uint64_t B = shr(s[i], L.K);
    if (i == 0 || B != run_key.back()) {
      run_key.push_back(B);
      run_start.push_back(i);
    }
  }
  finish_runs(L, nnz, run_start, run_key, max_block_nnz, t);
  // re-encode: every ALTO bit below K moves to its mode's field
  std::vector<uint64_t> enc(16 * 256, 0);
  {
    int owner_mode[128], owner_bit[128];
    for (int n = 0; n < N; ++n)
      for (int j = 0; j < L.b[n]; ++j) {
        owner_mode[L.pos[n][j]] = n;
        owner_bit[L.pos[n][j]] = j;
      }
    for (int k = 0; k < 16; ++k)
      for (int v = 0; v < 256; ++v) {
        uint64_t x = 0;
        for (int j = 0; j < 8; ++j) {
          int p = 8 * k + j;
          if (!((v >> j) & 1) || p >= L.K) continue;
          int n = owner_mode[p], bj = owner_bit[p];
          x |= 1ULL << (L.s[n] + bj);
        }
        enc[(size_t)k * 256 + v] = x;
      }
  }
  const int kbytes = (L.K + 7) / 8;
  parallel_chunks(nnz, nt, [&](int tid, int64_t lo, int64_t hi) {
    (void)tid;
    for (int64_t i = lo; i < hi; ++i) {
      const Rec& r = s[i];
      uint64_t key = 0;
      for (int k = 0; k < kbytes; ++k) {
        uint32_t byte = digit_of(r, 8 * k, 255);
        key |= enc[(size_t)k * 256 + byte];
      }
      t->h_keys[i] = key;
      t->h_vals[i] = r.v;
    }
  });
  free(s);
  return BLCO_OK;
}

int host_build(int nmodes, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
               const float* values, int key_bits, int64_t max_block_nnz, HostAlloc alloc,
               HostFree release, blco_tensor* t) {
  if (nmodes < 1 || nmodes > BLCO_MAX_MODES)
    return set_error(BLCO_EUNSUPPORTED, "nmodes %d outside 1..%d", nmodes, BLCO_MAX_MODES);
  if (!dims) return set_error(BLCO_EINVAL, "dims is NULL");
  if (nnz < 0) return set_error(BLCO_EINVAL, "nnz %lld < 0", (long long)nnz);
  if (nnz > 0 && (!coords || !values)) return set_error(BLCO_EINVAL, "coords or values is NULL");
  for (int n = 0; n < nmodes; ++n) {
    if (dims[n] < 1) return set_error(BLCO_EINVAL, "dims[%d] = 0", n);
    if (dims[n] > (1ULL << 32))
      return set_error(BLCO_EUNSUPPORTED, "dims[%d] = %llu > 2^32", n, (unsigned long long)dims[n]);
    if (nnz > 0 && !coords[n]) return set_error(BLCO_EINVAL, "coords[%d] is NULL", n);
  }
  if (key_bits < 1 || key_bits > 64) return set_error(BLCO_EINVAL, "key_bits %d outside 1..64", key_bits);
  if (max_block_nnz < 1) return set_error(BLCO_EINVAL, "max_block_nnz < 1");
  int rc = make_layout(nmodes, dims, key_bits, &t->lay);
  if (rc) return rc;
  t->nnz = nnz;
  t->max_block_nnz = max_block_nnz;
  t->host_free = release ? release : free;
  if (!alloc) alloc = malloc;
  t->h_keys = (uint64_t*)alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(nnz, 1));
  t->h_vals = (float*)alloc(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
  if (!t->h_keys || !t->h_vals) {
    free_host_arrays(t);
    return set_error(BLCO_ENOMEM, "host allocation of the BLCO arrays (%lld non-zeros) failed",
                     (long long)nnz);
  }
  if (t->lay.T <= 64)
    rc = build_with<Rec64>(t->lay, nnz, coords, values, max_block_nnz, t);
  else
    rc = build_with<Rec128>(t->lay, nnz, coords, values, max_block_nnz, t);
  if (rc) free_host_arrays(t);
  return rc;
}

void find_hot_rows(const uint32_t* const* coords, int64_t nnz, int64_t min_count, blco_tensor* t) {
  const int N = t->lay.N;
  t->hot.assign((size_t)N * kHotMax, 0xFFFFFFFFu);
  t->hot_cnt.assign((size_t)N * (kHotMax + 1), 0);
  for (int n = 0; n < N; ++n) t->nhot[n] = 0;
  if (nnz <= 0 || min_count < 0) return;
  const int64_t step = std::max<int64_t>(1, nnz / ((int64_t)1 << 22));
  std::vector<std::thread> th;
  for (int n = 0; n < N; ++n) {
    if (t->lay.dims[n] > ((uint64_t)1 << 26)) continue;
    th.emplace_back([=]() {
      const uint64_t I = t->lay.dims[n];
      std::vector<uint32_t> cnt((size_t)I, 0);
      for (int64_t i = 0; i < nnz; i += step) ++cnt[coords[n][i]];
      // the kHotMax + 1 most frequent rows; those reaching the sampled
      // threshold are the frequent rows, and all their counts are kept
      const uint64_t need = (uint64_t)std::max<int64_t>(1, (min_count + step - 1) / step);
      std::vector<std::pair<uint32_t, uint32_t>> c;
      for (uint64_t r = 0; r < I; ++r)
        if (cnt[r] > 0) c.push_back({cnt[r], (uint32_t)r});
      const size_t k = std::min<size_t>(c.size(), kHotMax + 1);
      std::partial_sort(c.begin(), c.begin() + k, c.end(),
                        [](const std::pair<uint32_t, uint32_t>& a,
                           const std::pair<uint32_t, uint32_t>& b) {
                          return a.first != b.first ? a.first > b.first : a.second < b.second;
                        });
      int nh = 0;
      for (size_t j = 0; j < k; ++j) {
        t->hot_cnt[(size_t)n * (kHotMax + 1) + j] = (uint64_t)c[j].first * (uint64_t)step;
        if (j < (size_t)kHotMax && c[j].first >= need) t->hot[(size_t)n * kHotMax + nh++] = c[j].second;
      }
      t->nhot[n] = nh;
    });
  }
  for (auto& x : th) x.join();
}

void free_host_arrays(blco_tensor* t) {
  if (t->host_free) {
    if (t->h_keys) t->host_free(t->h_keys);
    if (t->h_vals) t->host_free(t->h_vals);
  }
  t->h_keys = nullptr;
  t->h_vals = nullptr;
}

}  // namespace blco

extern "C" const char* blco_last_error(void) { return blco::g_err.c_str(); }
