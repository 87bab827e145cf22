// Sorting and compaction primitives of the GPU builder (Section 4.2: the
// non-zeros are ordered along the encoding line), written for gfx950.
//
// radix_sort: stable least-significant-digit radix sort of keys (u32 or u64)
// with up to two u32 value arrays and one u64 value array moved along, over key
// bits [0, bits), 8-bit digits:
//   * one pass over the keys forms their bitwise AND and OR: a pass whose digit
//     is the same for every key (the two agree on its bits) is skipped;
//   * per pass, over tiles of kSortTile keys: k_sort_count counts the tile's
//     digits (each wave's lanes that share a digit add their number once);
//     k_sort_scan turns the counts into each tile's start inside its digit
//     (digit-major, so tiles keep their order inside a digit) and each
//     digit's total, k_digit_base the digits' starts; k_sort_scatter
//     ranks each key among the tile's keys of its digit in input order (each
//     wave ranks its own consecutive keys with ballots and per-wave LDS
//     counters; the waves' counts then give each wave's offset), stages the
//     tile in LDS in digit order and writes it out, so keys of one digit leave
//     a tile as one contiguous run.
// Input order decides among equal digits in every pass, so the sort is
// stable; a descending variant sorts on the complemented key.
//
// select_flagged: the indices i with flag[i] != 0, in increasing order (a
// stream compaction: per-tile counts, a scan, per-tile writes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "blco_internal.h"

namespace blco {

#define SORT_HIPCHK(expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(BLCO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

namespace {

constexpr int kSortThreads = 256;                       // 4 waves
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = 16;                         // keys per thread
constexpr int kWaveKeys = 64 * kSortRounds;             // consecutive keys of one wave
constexpr int kSortTile = kSortThreads * kSortRounds;   // 4096 keys per tile
constexpr int kDigits = 256;
constexpr int kMaxPasses = 8;                           // 64-bit keys

template <typename K, bool DESC>
__device__ __forceinline__ uint32_t digit_of(K key, int shift) {
  if constexpr (DESC) key = ~key;
  return (uint32_t)(key >> shift) & 255u;
}

// Lanes of the wave whose digit equals this lane's (8 ballots).
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t set = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? set : ~set;
  }
  return m;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Bitwise AND and OR of all keys (as u64): a digit is the same for every key
// exactly where the two agree on its bits, and such a pass is skipped.
template <typename K>
__global__ __launch_bounds__(256) void k_sort_bits(const K* __restrict__ keys, int64_t n,
                                                   unsigned long long* __restrict__ andor) {
  __shared__ unsigned long long s_a[4], s_o[4];
  unsigned long long a = ~0ull, o = 0ull;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const unsigned long long k = (unsigned long long)keys[i];
    a &= k;
    o |= k;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a &= __shfl_xor(a, off, 64);
    o |= __shfl_xor(o, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_a[threadIdx.x >> 6] = a;
    s_o[threadIdx.x >> 6] = o;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < 4; ++j) {
      a &= s_a[j];
      o |= s_o[j];
    }
    atomicAnd(&andor[0], s_a[0] & a);
    atomicOr(&andor[1], s_o[0] | o);
  }
}

// Digit counts of each tile: tc[d * ntiles + tile].  Wave w of a tile takes its
// keys [w * kWaveKeys, (w + 1) * kWaveKeys), 64 at a time.
template <typename K, bool DESC>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const K* __restrict__ keys, int64_t n,
                                                             int shift, int64_t ntiles,
                                                             unsigned int* __restrict__ tc) {
  __shared__ unsigned int s[kDigits];
  for (int i = threadIdx.x; i < kDigits; i += kSortThreads) s[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t wb = (int64_t)blockIdx.x * kSortTile + (int64_t)w * kWaveKeys;
  uint32_t dg[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {   // every load in flight before the counting
    const int64_t i = wb + r * 64 + lane;
    dg[r] = digit_of<K, DESC>(i < n ? keys[i] : K(0), shift);
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool ok = wb + r * 64 + lane < n;
    const uint64_t peers = same_digit_lanes(dg[r]) & __ballot(ok);
    if (ok && !(peers & lanes_below(lane))) atomicAdd(&s[dg[r]], (unsigned int)__popcll(peers));
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kDigits; d += kSortThreads)
    tc[(int64_t)d * ntiles + blockIdx.x] = s[d];
}

// In place: tc[d * ntiles + t] becomes base + sum of tc[d * ntiles + t'] over
// t' < t, base = dbase[d] (0 when dbase is NULL); tot[d] (when given) receives the
// row's sum.  One workgroup per digit, ntiles entries each, in chunks of 1024.
__global__ __launch_bounds__(1024) void k_sort_scan(unsigned int* __restrict__ tc, int64_t ntiles,
                                                    const unsigned int* __restrict__ dbase,
                                                    unsigned int* __restrict__ tot) {
  __shared__ unsigned int s_w[16];
  __shared__ unsigned int s_carry;
  const int d = blockIdx.x;
  unsigned int* row = tc + (int64_t)d * ntiles;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_carry = dbase ? dbase[d] : 0u;
  __syncthreads();
  for (int64_t c0 = 0; c0 < ntiles; c0 += 1024) {
    const int64_t i = c0 + tid;
    const unsigned int v = i < ntiles ? row[i] : 0u;
    // inclusive scan inside the wave
    unsigned int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (tid < 64) {
      unsigned int t = tid < 16 ? s_w[tid] : 0u;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const unsigned int y = __shfl_up(t, off, 64);
        if (lane >= off) t += y;
      }
      if (tid < 16) s_w[tid] = t;   // inclusive over waves
    }
    __syncthreads();
    const unsigned int before = s_carry + (w > 0 ? s_w[w - 1] : 0u) + x - v;
    if (i < ntiles) row[i] = before;
    __syncthreads();
    if (tid == 0) s_carry += s_w[15];
    __syncthreads();
  }
  if (tot && tid == 0) tot[d] = s_carry;
}

// dbase[d] = sum of tot[d'] over d' < d (one workgroup of 256 threads).
__global__ __launch_bounds__(256) void k_digit_base(const unsigned int* __restrict__ tot,
                                                    unsigned int* __restrict__ dbase) {
  __shared__ unsigned int s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const unsigned int v = tot[tid];
  unsigned int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  unsigned int before = x - v;
  for (int j = 0; j < w; ++j) before += s_w[j];
  dbase[tid] = before;
}

// The value arrays one scatter pass reads and writes: NV u32 arrays and, with V64,
// one u64 array.
struct PassVals {
  const uint32_t* in[2];
  uint32_t* out[2];
  const uint64_t* in64;
  uint64_t* out64;
};

// One pass: every key (and its values) of a tile to its place.  Wave w ranks its
// kWaveKeys keys among themselves, 64 at a time in input order: a key's rank is
// the wave's earlier keys of the same digit (an LDS counter per wave and digit,
// read by every lane and advanced by the lowest lane of each digit group) plus
// its lanes below with that digit.  Then the waves' counts give each wave's
// offset inside each digit, the tile's digit counts their starts, and the tile
// is staged in LDS in digit order and written out, each digit's keys as one
// contiguous run starting at the (digit, tile) start from k_sort_scan.
template <typename K, int NV, bool V64, bool DESC>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const K* __restrict__ kin, K* __restrict__ kout, PassVals pv, int64_t n, int shift,
    int64_t ntiles, const unsigned int* __restrict__ tstart,
    const unsigned int* __restrict__ dbase) {
  __shared__ unsigned int s_cnt[kSortWaves][kDigits];   // per-wave counts, then wave offsets
  __shared__ unsigned int s_start[kDigits];             // tile's first position per digit
  __shared__ unsigned int s_gpos[kDigits];              // global start per digit
  __shared__ K s_k[kSortTile];
  __shared__ uint32_t s_v[NV > 0 ? NV : 1][NV > 0 ? kSortTile : 1];
  __shared__ uint64_t s_v64[V64 ? kSortTile : 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int d = tid; d < kDigits; d += kSortThreads) {
    s_gpos[d] = dbase[d] + tstart[(int64_t)d * ntiles + blockIdx.x];
#pragma unroll
    for (int j = 0; j < kSortWaves; ++j) s_cnt[j][d] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int64_t wb = base + (int64_t)w * kWaveKeys;
  K key[kSortRounds];
  uint32_t val[NV > 0 ? NV : 1][kSortRounds];
  uint64_t val64[V64 ? kSortRounds : 1];
  uint32_t rank[kSortRounds];   // rank among this wave's keys of the same digit
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {   // every load in flight before the ranking
    const int64_t i = wb + r * 64 + lane;
    const bool ok = i < n;
    key[r] = ok ? kin[i] : K(0);
#pragma unroll
    for (int j = 0; j < NV; ++j) val[j][r] = ok ? pv.in[j][i] : 0u;
    if constexpr (V64) val64[r] = ok ? pv.in64[i] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool ok = wb + r * 64 + lane < n;
    const uint32_t d = digit_of<K, DESC>(key[r], shift);
    const uint64_t peers = same_digit_lanes(d) & __ballot(ok);
    const unsigned int c = s_cnt[w][d];
    rank[r] = c + (unsigned int)__popcll(peers & lanes_below(lane));
    // every lane has read the counter before its group's lowest lane advances it
    // (one wave: the read and the write are issued in this order)
    if (ok && !(peers & lanes_below(lane))) s_cnt[w][d] = c + (unsigned int)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: each wave's offset, and the tile's count (into s_start)
  for (int d = tid; d < kDigits; d += kSortThreads) {
    unsigned int run = 0;
#pragma unroll
    for (int j = 0; j < kSortWaves; ++j) {
      const unsigned int c = s_cnt[j][d];
      s_cnt[j][d] = run;
      run += c;
    }
    s_start[d] = run;
  }
  __syncthreads();
  // exclusive sum of the tile's digit counts
  if (tid < 64) {
    unsigned int c[kDigits / 64];
    unsigned int tot = 0;
#pragma unroll
    for (int q = 0; q < kDigits / 64; ++q) {
      c[q] = s_start[tid * (kDigits / 64) + q];
      tot += c[q];
    }
    unsigned int x = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    unsigned int run = x - tot;
#pragma unroll
    for (int q = 0; q < kDigits / 64; ++q) {
      s_start[tid * (kDigits / 64) + q] = run;
      run += c[q];
    }
  }
  __syncthreads();
  // stage the tile in digit order
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    if (wb + r * 64 + lane < n) {
      const uint32_t d = digit_of<K, DESC>(key[r], shift);
      const uint32_t p = s_start[d] + s_cnt[w][d] + rank[r];
      s_k[p] = key[r];
#pragma unroll
      for (int j = 0; j < NV; ++j) s_v[j][p] = val[j][r];
      if constexpr (V64) s_v64[p] = val64[r];
    }
  }
  __syncthreads();
  // write runs of equal digit to their global places
  const int nt = (int)min<int64_t>(kSortTile, n - base);
  for (int j = tid; j < nt; j += kSortThreads) {
    const K k = s_k[j];
    const uint32_t d = digit_of<K, DESC>(k, shift);
    const int64_t g = (int64_t)s_gpos[d] + (j - (int)s_start[d]);
    kout[g] = k;
#pragma unroll
    for (int q = 0; q < NV; ++q) pv.out[q][g] = s_v[q][j];
    if constexpr (V64) pv.out64[g] = s_v64[j];
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(unsigned int* __restrict__ p, int64_t n,
                                                  unsigned int v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ a, T* __restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// ---- stream compaction
constexpr int kSelThreads = 256;
constexpr int kSelRounds = 8;
constexpr int kSelTile = kSelThreads * kSelRounds;

__global__ __launch_bounds__(kSelThreads) void k_sel_count(const uint8_t* __restrict__ flag,
                                                           int64_t n,
                                                           unsigned int* __restrict__ tc) {
  __shared__ unsigned int s_c[kSelThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kSelTile;
  unsigned int c = 0;
#pragma unroll
  for (int r = 0; r < kSelRounds; ++r) {
    const int64_t i = base + r * kSelThreads + threadIdx.x;
    c += (i < n && flag[i]) ? 1u : 0u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int t = 0;
#pragma unroll
    for (int j = 0; j < kSelThreads / 64; ++j) t += s_c[j];
    tc[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kSelThreads) void k_sel_write(const uint8_t* __restrict__ flag,
                                                           int64_t n,
                                                           const unsigned int* __restrict__ tstart,
                                                           int64_t* __restrict__ out) {
  __shared__ unsigned int s_w[kSelThreads / 64];
  __shared__ unsigned int s_base;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kSelTile;
  if (tid == 0) s_base = tstart[blockIdx.x];
  __syncthreads();
  for (int r = 0; r < kSelRounds; ++r) {
    const int64_t i = base + r * kSelThreads + tid;
    const bool f = i < n && flag[i];
    const uint64_t m = __ballot(f);
    if (lane == 0) s_w[w] = (unsigned int)__popcll(m);
    __syncthreads();
    unsigned int before = s_base;
    for (int j = 0; j < w; ++j) before += s_w[j];
    if (f) out[before + __popcll(m & ((1ull << lane) - 1ull))] = i;
    __syncthreads();
    if (tid == 0) {
      unsigned int t = 0;
      for (int j = 0; j < kSelThreads / 64; ++j) t += s_w[j];
      s_base += t;
    }
    __syncthreads();
  }
}

unsigned grid256(int64_t n) { return (unsigned)std::max<int64_t>((n + 255) / 256, 1); }

template <typename K, bool DESC>
int sort_impl(const K* kin, K* kout, K* ktmp, const SortVals& v, int64_t n, int bits,
              unsigned int* ws, hipStream_t s) {
  const int nv = v.in32[0] ? (v.in32[1] ? 2 : 1) : 0;
  const bool v64 = v.in64 != nullptr;
  if (n <= 0) return BLCO_OK;
  if (n >= ((int64_t)1 << 31))
    return set_error(BLCO_EUNSUPPORTED, "radix sort of %lld keys (at most 2^31 - 1)", (long long)n);
  if (v.in32[1] && !v.in32[0])
    return set_error(BLCO_EINVAL, "radix sort: second u32 value array without a first");
  if (v64 && nv > 1)
    return set_error(BLCO_EUNSUPPORTED, "radix sort: two u32 and one u64 value arrays");
  const int npass = std::min(kMaxPasses, (std::max(bits, 1) + 7) / 8);
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  unsigned long long* andor = reinterpret_cast<unsigned long long*>(ws);   // 2 x u64
  unsigned int* tot = ws + 4;                                             // 256
  unsigned int* dbase = tot + kDigits;                                    // 256
  unsigned int* tc = dbase + kDigits;                                     // 256 * ntiles
  // which digits vary: AND and OR of every key
  const unsigned long long init[2] = {~0ull, 0ull};
  SORT_HIPCHK(hipMemcpyAsync(andor, init, sizeof(init), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((k_sort_bits<K>), dim3((unsigned)std::min<int64_t>(grid256(n), 1024)),
                     dim3(256), 0, s, kin, n, andor);
  SORT_HIPCHK(hipGetLastError());
  unsigned long long ao[2] = {0, 0};
  SORT_HIPCHK(hipMemcpyAsync(ao, andor, sizeof(ao), hipMemcpyDeviceToHost, s));
  SORT_HIPCHK(hipStreamSynchronize(s));
  std::vector<int> passes;
  for (int p = 0; p < npass; ++p)
    if (((ao[0] ^ ao[1]) >> (8 * p)) & 255ull) passes.push_back(p);
  const unsigned cgrid = (unsigned)std::min<int64_t>(grid256(n), 8192);
  if (passes.empty()) {
    hipLaunchKernelGGL((k_copy<K>), dim3(cgrid), dim3(256), 0, s, kin, kout, n);
    SORT_HIPCHK(hipGetLastError());
    for (int j = 0; j < nv; ++j) {
      hipLaunchKernelGGL((k_copy<uint32_t>), dim3(cgrid), dim3(256), 0, s, v.in32[j], v.out32[j], n);
      SORT_HIPCHK(hipGetLastError());
    }
    if (v64) {
      hipLaunchKernelGGL((k_copy<uint64_t>), dim3(cgrid), dim3(256), 0, s, v.in64, v.out64, n);
      SORT_HIPCHK(hipGetLastError());
    }
    return BLCO_OK;
  }
  // the passes alternate between the output and the spare buffers so that the
  // last one writes the output; the inputs are only read
  const int P = (int)passes.size();
  for (int q = 0; q < P; ++q) {
    const int p = passes[q];
    const bool from_in = q == 0, from_out = ((P - q) % 2 == 0), to_out = ((P - 1 - q) % 2 == 0);
    const K* ki = from_in ? kin : (from_out ? kout : ktmp);
    K* ko = to_out ? kout : ktmp;
    PassVals pv = {};
    for (int j = 0; j < nv; ++j) {
      pv.in[j] = from_in ? v.in32[j] : (from_out ? v.out32[j] : v.tmp32[j]);
      pv.out[j] = to_out ? v.out32[j] : v.tmp32[j];
    }
    if (v64) {
      pv.in64 = from_in ? v.in64 : (from_out ? v.out64 : v.tmp64);
      pv.out64 = to_out ? v.out64 : v.tmp64;
    }
    hipLaunchKernelGGL((k_sort_count<K, DESC>), dim3((unsigned)ntiles), dim3(kSortThreads), 0, s,
                       ki, n, 8 * p, ntiles, tc);
    SORT_HIPCHK(hipGetLastError());
    // each (digit, tile) start inside its digit, each digit's total, the digits' starts
    hipLaunchKernelGGL(k_sort_scan, dim3(kDigits), dim3(1024), 0, s, tc, ntiles,
                       (const unsigned int*)nullptr, tot);
    SORT_HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_digit_base, dim3(1), dim3(kDigits), 0, s, (const unsigned int*)tot,
                       dbase);
    SORT_HIPCHK(hipGetLastError());
    const dim3 g((unsigned)ntiles), b(kSortThreads);
    const unsigned int* ts = tc;
    const unsigned int* db = dbase;
    if (v64)
      hipLaunchKernelGGL((k_sort_scatter<K, 1, true, DESC>), g, b, 0, s, ki, ko, pv, n, 8 * p,
                         ntiles, ts, db);
    else if (nv == 2)
      hipLaunchKernelGGL((k_sort_scatter<K, 2, false, DESC>), g, b, 0, s, ki, ko, pv, n, 8 * p,
                         ntiles, ts, db);
    else if (nv == 1)
      hipLaunchKernelGGL((k_sort_scatter<K, 1, false, DESC>), g, b, 0, s, ki, ko, pv, n, 8 * p,
                         ntiles, ts, db);
    else
      hipLaunchKernelGGL((k_sort_scatter<K, 0, false, DESC>), g, b, 0, s, ki, ko, pv, n, 8 * p,
                         ntiles, ts, db);
    SORT_HIPCHK(hipGetLastError());
  }
  return BLCO_OK;
}

}  // namespace

size_t sort_workspace_words(int64_t n) {
  const int64_t ntiles = (std::max<int64_t>(n, 1) + kSortTile - 1) / kSortTile;
  return (size_t)4 + 2 * kDigits + (size_t)kDigits * ntiles;
}

static SortVals one_value(const uint32_t* vin, uint32_t* vout, uint32_t* vtmp) {
  SortVals v = {};
  v.in32[0] = vin;
  v.out32[0] = vout;
  v.tmp32[0] = vtmp;
  return v;
}

int radix_sort_u64(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                   uint64_t* ktmp, uint32_t* vtmp, int64_t n, int bits, unsigned int* ws,
                   void* s) {
  return sort_impl<uint64_t, false>(kin, kout, ktmp, one_value(vin, vout, vtmp), n, bits, ws,
                                    (hipStream_t)s);
}

int radix_sort_u32(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                   uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits, bool descending,
                   unsigned int* ws, void* sv) {
  hipStream_t s = (hipStream_t)sv;
  const SortVals v = one_value(vin, vout, vtmp);
  return descending ? sort_impl<uint32_t, true>(kin, kout, ktmp, v, n, bits, ws, s)
                    : sort_impl<uint32_t, false>(kin, kout, ktmp, v, n, bits, ws, s);
}

int radix_sort_u64_vals(const uint64_t* kin, uint64_t* kout, uint64_t* ktmp, const SortVals& v,
                        int64_t n, int bits, unsigned int* ws, void* s) {
  return sort_impl<uint64_t, false>(kin, kout, ktmp, v, n, bits, ws, (hipStream_t)s);
}

int radix_sort_u32_vals(const uint32_t* kin, uint32_t* kout, uint32_t* ktmp, const SortVals& v,
                        int64_t n, int bits, unsigned int* ws, void* s) {
  return sort_impl<uint32_t, false>(kin, kout, ktmp, v, n, bits, ws, (hipStream_t)s);
}

size_t select_workspace_words(int64_t n) {
  return (size_t)(std::max<int64_t>(n, 1) + kSelTile - 1) / kSelTile;
}

int select_flagged(const uint8_t* flag, int64_t n, int64_t* out, int64_t* count,
                   unsigned int* ws, void* sv) {
  hipStream_t s = (hipStream_t)sv;
  *count = 0;
  if (n <= 0) return BLCO_OK;
  if (n >= ((int64_t)1 << 31))
    return set_error(BLCO_EUNSUPPORTED, "selection over %lld flags (at most 2^31 - 1)", (long long)n);
  const int64_t ntiles = (n + kSelTile - 1) / kSelTile;
  unsigned int* tc = ws;   // ntiles
  hipLaunchKernelGGL(k_sel_count, dim3((unsigned)ntiles), dim3(kSelThreads), 0, s, flag, n, tc);
  SORT_HIPCHK(hipGetLastError());
  // the tiles' starts: an exclusive sum over the tile counts (one row of the
  // digit scan kernel, base 0)
  unsigned int last = 0;   // the last tile's count, read before the scan replaces it
  SORT_HIPCHK(hipMemcpyAsync(&last, tc + ntiles - 1, sizeof(unsigned int),
                             hipMemcpyDeviceToHost, s));
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, tc, ntiles,
                     (const unsigned int*)nullptr, (unsigned int*)nullptr);
  SORT_HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_sel_write, dim3((unsigned)ntiles), dim3(kSelThreads), 0, s, flag, n,
                     (const unsigned int*)tc, out);
  SORT_HIPCHK(hipGetLastError());
  unsigned int start_last = 0;
  SORT_HIPCHK(hipMemcpyAsync(&start_last, tc + ntiles - 1, sizeof(unsigned int),
                             hipMemcpyDeviceToHost, s));
  SORT_HIPCHK(hipStreamSynchronize(s));
  *count = (int64_t)start_last + last;
  return BLCO_OK;
}

}  // namespace blco
