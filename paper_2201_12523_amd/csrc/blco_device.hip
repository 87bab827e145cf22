// Device runtime and gfx950 kernels of the BLCO sparse MTTKRP library.
//
// Method: Nguyen et al., "Efficient, Out-of-Memory Sparse MTTKRP on Massively
// Parallel Architectures", ICS '22.  Two MTTKRP kernels follow the processing /
// computing split of Section 5.1 (Figure 7), re-designed for wave64 and the
// memory-side atomics of MI355X:
//   k_mttkrp_win (register-based resolution, Section 5.2): one 1024-thread
//     workgroup per window of 1024 consecutive non-zeros (2048 or 4096 on modes
//     without frequent rows).  Processing: each thread loads one, two or four
//     (key, value) pairs (coalesced), decodes the coordinates
//     by shift and mask (Figure 6b), and the window is grouped by target row
//     with a counting sort on a hash of the target (LDS histogram, workgroup
//     scan, scatter), so each target forms one segment; every grouped position
//     gets a record (byte offsets of the other modes' rows, target, value).
//     Computing: groups of 16 lanes (1-4 ranks per lane) walk the records,
//     gather the factor rows with raw buffer loads, sum the scaled Hadamard
//     products in registers while the target repeats, and add each finished
//     segment to the output with one atomic per rank.  A mode's frequent rows
//     (found at build time) are summed in an LDS stash instead and flushed
//     once per persistent workgroup.
//   k_mttkrp_short (hierarchical resolution, Section 5.1), which the Section
//     5.3 heuristic picks for modes shorter than the compute-unit count: each
//     workgroup keeps a private LDS copy of all target rows (a rank slice) and
//     adds it to the output once at its end.
// Also here: the sampled CP model / residual / fp64 loss kernels, the bf16
// cast, the out-of-memory streaming runtime and the C ABI of include/blco.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "blco_internal.h"
#include "blco_kernels.h"

using namespace blco;

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(BLCO_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// ====================================================================== device code

template <typename FT>
__device__ __forceinline__ float ld_factor(const void* A, size_t i);

template <>
__device__ __forceinline__ float ld_factor<float>(const void* A, size_t i) {
  return static_cast<const float*>(A)[i];
}

template <>
__device__ __forceinline__ float ld_factor<uint16_t>(const void* A, size_t i) {
  return __uint_as_float((uint32_t)static_cast<const uint16_t*>(A)[i] << 16);
}

// Coordinates of one non-zero: kept bits by shift and mask, the rest from
// the block key of the run that holds it (Figure 6b).
template <int N>
__device__ __forceinline__ void decode(const KParams& p, uint64_t key, int64_t gidx,
                                       uint32_t (&c)[N]) {
  uint32_t base[N];
#pragma unroll
  for (int m = 0; m < N; ++m) base[m] = 0;
  if (p.multi) {
    int run = p.tile_run[gidx >> 6];
    while (gidx >= p.run_start[run + 1]) ++run;
#pragma unroll
    for (int m = 0; m < N; ++m) base[m] = p.run_base[(size_t)run * N + m];
  }
#pragma unroll
  for (int m = 0; m < N; ++m) c[m] = ((uint32_t)(key >> p.shift[m]) & p.mask[m]) | base[m];
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float term_scale(const KParams& p) {
  return p.scale_dev ? (float)((double)p.scale * p.scale_dev[0]) : p.scale;
}

// Zero-fill of an output (a kernel rather than a memset so the call can be captured).
__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
    float4* q = reinterpret_cast<float4*>(p);
    int64_t n4 = n >> 2;
    for (int64_t j = i; j < n4; j += stride) q[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t j = (n4 << 2) + i; j < n; j += stride) p[j] = 0.f;
  } else {
    for (int64_t j = i; j < n; j += stride) p[j] = 0.f;
  }
}

constexpr int kWin = 1024;     // threads of the window kernel (non-zeros per window / WPT)
constexpr int kWinRounds = 4;  // dispatch rounds of the persistent window kernel
constexpr int kWinBits = 10;
#ifndef BLCO_WIN_U
#define BLCO_WIN_U 8
#endif
// minimum waves per SIMD requested from the compiler: 8 lets two 1024-thread
// workgroups share a CU (measured about 1.7x faster than one)
#ifndef BLCO_WIN_OCC
#define BLCO_WIN_OCC 8
#endif

constexpr int kBucketBits = 12;
constexpr int kBuckets = 1 << kBucketBits;   // hash buckets per 1024-non-zero window

// In-place exclusive prefix sum of NB counters in LDS by a workgroup of NT
// threads (NB a multiple of NT): per-thread serial sums, a wave scan by
// cross-lane shifts, and one LDS pass over the per-wave totals.
template <int NB, int NT>
__device__ __forceinline__ void block_exclusive_scan(uint32_t* a, int tid, uint32_t* wsum) {
  constexpr int PER = NB / NT;
  uint32_t v[PER];
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    v[i] = a[tid * PER + i];
    tot += v[i];
  }
  const int lane = tid & 63;
  uint32_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[tid >> 6] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < (tid >> 6); ++w) wbase += wsum[w];
  uint32_t run = wbase + inc - tot;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    a[tid * PER + i] = run;
    run += v[i];
  }
  __syncthreads();
}

// Lane q of this lane's 16-lane row (DPP row_newbcast), and the value of the
// lane q places further along the row (DPP row_shl).  q must fold to a
// constant where they are called (unrolled loops).
__device__ __forceinline__ uint32_t row_bcast(uint32_t v, int q) {
  switch (q) {
    case 0: return __builtin_amdgcn_update_dpp(0u, v, 0x150, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(0u, v, 0x151, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0u, v, 0x152, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_update_dpp(0u, v, 0x153, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_update_dpp(0u, v, 0x154, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_update_dpp(0u, v, 0x155, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_update_dpp(0u, v, 0x156, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_update_dpp(0u, v, 0x157, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_update_dpp(0u, v, 0x158, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_update_dpp(0u, v, 0x159, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_update_dpp(0u, v, 0x15A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_update_dpp(0u, v, 0x15B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_update_dpp(0u, v, 0x15C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_update_dpp(0u, v, 0x15D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_update_dpp(0u, v, 0x15E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0u, v, 0x15F, 0xF, 0xF, false);
  }
}
__device__ __forceinline__ uint32_t row_shl(uint32_t v, int q) {
  switch (q) {
    case 1: return __builtin_amdgcn_update_dpp(0u, v, 0x101, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0u, v, 0x102, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_update_dpp(0u, v, 0x103, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_update_dpp(0u, v, 0x104, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_update_dpp(0u, v, 0x105, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_update_dpp(0u, v, 0x106, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_update_dpp(0u, v, 0x107, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_update_dpp(0u, v, 0x108, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_update_dpp(0u, v, 0x109, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_update_dpp(0u, v, 0x10A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_update_dpp(0u, v, 0x10B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_update_dpp(0u, v, 0x10C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_update_dpp(0u, v, 0x10D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_update_dpp(0u, v, 0x10E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0u, v, 0x10F, 0xF, 0xF, false);
  }
}

// target row of a record (field N - 1 of the record at LDS offset `at`)
__device__ __forceinline__ uint32_t seg_target(const uint32_t* rec, int at, int mode, int N) {
  (void)mode;
  return rec[at + N - 1];
}
constexpr uint32_t kBufFlags = 0x00020000u;  // raw buffer resource word 3 (gfx9 family)

// Factor-row gathers.  Raw buffer loads with a 32-bit byte offset (row * row
// bytes + rank offset) when every factor is below 4 GiB: no 64-bit address
// arithmetic, and the descriptor's size bound drops stray offsets.  Larger
// factors take 64-bit global addresses (BIG).  (Structured, index-scaled
// buffer loads would cover both but measured 1.5-2x slower on gfx950.)
template <typename FT>
__device__ __forceinline__ float ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float ld_buf<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ float ld_buf<uint16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0) << 16);
}

// fp32 gathers of the window kernel at four ranks per lane (33-64 ranks): a global load
// from the factor's base (uniform, in scalar registers) plus the zero-extended 32-bit
// byte offset.  That reaches all of 4 GiB, so a factor of exactly 4 GiB (2^24 rows of 64
// ranks) keeps 32-bit offsets, where a buffer descriptor's 32-bit size stops one byte
// short.  Measured on the 4-mode 200M-non-zero workload at R = 64: 17.5 -> 15.1 ms on the
// mode that gathers such a factor (it took 64-bit addresses before), 15.7 -> 15.2 ms on
// its other frequent-row mode; at two ranks per lane the same loads were 5% slower on the
// frequent-row modes, so R <= 32 keeps buffer loads.
__device__ __forceinline__ float ld_base(const void* A, uint32_t off) {
  return *reinterpret_cast<const float*>(static_cast<const char*>(A) + off);
}

// RPL consecutive bf16 factor elements from byte offset off, widened to fp32: one
// 4- or 8-byte buffer load when VEC (every run starts 4-byte aligned: R is even), else
// RPL 2-byte loads.  Element k sits at the lower address, in the low half of its word.
template <int RPL, bool VEC>
__device__ __forceinline__ void ld_bf16_run(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                            float (&t)[RPL]) {
  if constexpr (RPL == 2 && VEC) {
    {
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
      t[0] = __uint_as_float(v << 16);
      t[1] = __uint_as_float(v & 0xFFFF0000u);
      return;
    }
  } else if constexpr (RPL == 4 && VEC) {
    {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
      t[0] = __uint_as_float(v[0] << 16);
      t[1] = __uint_as_float(v[0] & 0xFFFF0000u);
      t[2] = __uint_as_float(v[1] << 16);
      t[3] = __uint_as_float(v[1] & 0xFFFF0000u);
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < RPL; ++k) t[k] = ld_buf<uint16_t>(r, off + 2u * (uint32_t)k);
}

// The same run through a 64-bit address (a factor of 4 GiB or more), which has no
// bounds check: only elements with act[k] set (ranks below R) are read, so a run that
// ends past the last row stays inside the factor.  VEC reads RPL / 2 four-byte words
// (runs start 4-byte aligned and R is even, so a word is read whole or not at all).
template <int RPL, bool VEC>
__device__ __forceinline__ void ld_bf16_run_ptr(const uint16_t* src, const bool (&act)[RPL],
                                                float (&t)[RPL]) {
  if constexpr (VEC && RPL % 2 == 0) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
#pragma unroll
    for (int q = 0; q < RPL / 2; ++q) {
      const uint32_t v = act[2 * q] ? w[q] : 0u;
      t[2 * q] = __uint_as_float(v << 16);
      t[2 * q + 1] = __uint_as_float(v & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < RPL; ++k) t[k] = act[k] ? ld_factor<uint16_t>(src, (size_t)k) : 0.f;
  }
}

// Adds a lane group's segment sums to one output row with contiguous-rank atomics
// when each lane holds RPL consecutive ranks (lane l: ranks RPL*l .. RPL*l + RPL - 1 of
// the slice): the j-th atomic of lane l adds rank l + j*LPN, fetched from the lane
// holding it, so every atomic instruction covers LPN consecutive floats.  dst points
// at the slice's first rank; ranks from nvalid on are not written.
template <int RPL, int LPN>
__device__ __forceinline__ void flush_packed(float* dst, const float (&a)[RPL], float scale,
                                             int rl, int nvalid) {
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int q = rl + j * LPN;
    float v = 0.f;
#pragma unroll
    for (int s2 = 0; s2 < RPL; ++s2) {
      const float t2 = __shfl(a[s2], q / RPL, LPN);
      if (s2 == rl % RPL) v = t2;
    }
    if (q < nvalid) unsafeAtomicAdd(dst + q, v * scale);
  }
}

// Frequent-row lookup of the window kernel: open addressing over kHotSlots
// LDS slots holding (row, stash index); at most half full.
constexpr int kHotSlots = 2 * blco::kHotMax;
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
constexpr uint32_t kHotFlag = 0x80000000u;   // record target field: stash index follows

__device__ __forceinline__ uint32_t hot_hash(uint32_t row) {
  return (row * 0x9E3779B1u) >> (32 - 9);   // 9 bits: kHotSlots = 512
}

__device__ __forceinline__ int hot_lookup(const uint32_t* keys, const uint32_t* idx, uint32_t row) {
  uint32_t h = hot_hash(row);
  for (int probe = 0; probe < kHotSlots; ++probe) {
    const uint32_t k = keys[h];
    if (k == row) return (int)idx[h];
    if (k == kNoRow) return -1;
    h = (h + 1) & (kHotSlots - 1);
  }
  return -1;
}

// BLCO MTTKRP with register-based conflict resolution (Sections 5.1-5.2) over
// windows of 1024 * WPT consecutive non-zeros; persistent workgroups take windows
// in turn (see below)
//   processing: WPT non-zeros per thread are loaded (the next window's load is
//     issued before the current walk) and decoded by shift and mask; the
//     window is grouped by target with a counting sort (LDS histogram with
//     atomic ranks, exclusive scan, scatter) on a hash of the target, so each
//     target's terms form one contiguous segment, and each grouped position
//     gets a record: byte offsets of the other modes' factor rows, target,
//     value;
//   computing: groups of LPN lanes (RPL ranks per lane) walk LPN consecutive
//     grouped positions each (records read from LDS, or for N = 3 held one
//     per lane and passed along the group by DPP row broadcasts),
//     gathering factor rows with buffer loads and
//     summing the scaled Hadamard products in registers; a segment that ends
//     inside the group is flushed once per rank; a segment that crosses into
//     later groups is completed by the group it started in, from partial sums
//     the later groups leave in LDS.
// A flush is a device-scope atomic into the output, which MI355X performs at
// the memory side (same-address updates serialise at about 32 ns), except for
// the mode's frequent rows (found at build time): those get buckets of their
// own, so each has exactly one segment per window, and its flush is a plain
// add into the workgroup's LDS stash row; the stash goes to the output with
// one atomic per (row, rank) when the workgroup ends.
//
// RES (the fused CP-gradient walk, one rank slice): the values are the data x_k,
// and each position also gathers its target row, so the walk forms the model
// xhat_k = sum_r prod_m A^(m)[i_m^k, r] (a sum over the 16 lanes of the group),
// the residual e_k = x_k - xhat_k, which it writes to p.resid in BLCO order, and
// sums e_k * prod_{m != mode} A^(m) instead of x_k * prod_{m != mode} A^(m).
//
// WPT: non-zeros per thread, so a window holds kWin * WPT non-zeros.  Two (for modes
// without a stash) merge more terms per flush: on the 2^20-row and 1024-row modes of
// the 4-mode 200M-non-zero tensor, 16% and 32% fewer row flushes than at one.  Four
// (at R > 32) merge more again but need 145 KiB of LDS, one workgroup per CU: faster
// at R = 64, where the walk has four ranks per lane to cover the gathers, slower at 32.
template <int LPN, int RPL, typename FT, int N, bool BIG, bool STASH, bool RES = false,
          bool VEC = false, int WPT = 1>
__global__ __launch_bounds__(kWin, WPT >= 4 ? 4 : BLCO_WIN_OCC) void k_mttkrp_win(KParams p) {
  constexpr int W = kWin * WPT;                 // non-zeros per window
  constexpr int G = kWin / LPN;                 // groups of LPN lanes
  constexpr int PPG = W / G;                    // grouped positions per group (= LPN * WPT)
  static_assert(PPG <= 64, "a group's segment ends must fit one 64-bit word");
  static_assert(WPT == 1 || (!STASH && !RES), "multi-non-zero windows: plain MTTKRP, no stash");
  // hash buckets: 4096 per 1024 non-zeros, 6144 per 2048 (two workgroups per CU keep
  // fitting in LDS), 12288 per 4096
  constexpr int NB = WPT == 1 ? kBuckets : WPT == 2 ? kBuckets * 3 / 2 : kBuckets * 3;
  // positions whose gathers are issued together: BLCO_WIN_U / RPL, except for
  // 3-mode tensors at one or four ranks per lane, where 4 and 1 positions keep
  // the registers from spilling and measured 8% and 3% faster; the fused
  // residual walk also gathers the target row and keeps the value, the
  // residual and the position of each, so it takes half as many (at four it
  // spilled about 45 registers per lane; 4-mode 80M-non-zero CP gradient step
  // 13.1 -> 12.0 ms)
  constexpr int UW0 = (N == 3 && RPL == 1) ? 4 : (N == 3 && RPL == 4) ? 1 : BLCO_WIN_U / RPL;
  constexpr int UW = RES ? (UW0 > 1 ? UW0 / 2 : 1) : UW0;
  constexpr int U = PPG < UW ? PPG : UW;
  // record fields: the other modes' row offsets, target, value; with RES also
  // the target row's offset and the position in the window
  constexpr int NF = RES ? N + 3 : N + 1;
  constexpr int NP = NF <= 4 ? 4 : ((NF + 1) / 2) * 2;
  static_assert(!RES || (LPN == 16 && !BIG), "fused residual walk: 16-lane groups, 32-bit offsets");
  // bf16 factors: each lane holds RPL consecutive ranks, so one 4- or 8-byte load
  // gathers them when R is even (VEC; measured 14% faster per mode on 200M
  // non-zeros), 2-byte loads otherwise; fp32 keeps ranks LPN apart, whose 4-byte
  // loads measured faster than 8- and 16-byte ones
  constexpr bool PACKED = sizeof(FT) == 2 && RPL > 1;
  static_assert(!VEC || PACKED, "vector gathers are for packed bf16 ranks");
  // fp32 gathers at four ranks per lane: ld_base instead of buffer loads
  constexpr bool BASE32 = sizeof(FT) == 4 && LPN == 16 && RPL == 4 && !RES && !BIG;
  __shared__ __align__(16) uint32_t s_rec[W * NP];  // records by grouped position
  __shared__ uint64_t s_end[W / 64];
  // the histogram (processing) and the carry partial sums (computing) are never
  // live at once: they share one array
  constexpr int NHH = NB > kWin * RPL ? NB : kWin * RPL;
  __shared__ __align__(16) uint32_t s_hist[NHH];
  float* s_head = reinterpret_cast<float*>(s_hist);
  __shared__ uint32_t s_wsum[kWin / 64];
  extern __shared__ __align__(16) unsigned char s_dyn_win[];
  // frequent rows in the stash; without STASH one window per workgroup
  const int K = STASH ? p.nhot : 0;
  const int R = p.R;
  float* s_stash = reinterpret_cast<float*>(s_dyn_win);   // K x R
  uint32_t* s_hkey = reinterpret_cast<uint32_t*>(s_stash + (size_t)K * R);
  uint32_t* s_hidx = s_hkey + kHotSlots;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int64_t nwin = (p.n + W - 1) / W;
  if (K > 0) {
    for (int i = tid; i < K * R; i += kWin) s_stash[i] = 0.f;
    for (int i = tid; i < kHotSlots; i += kWin) s_hkey[i] = kNoRow;
    __syncthreads();
    if (tid < K) {
      const uint32_t row = p.hot[tid];
      uint32_t h = hot_hash(row);
      for (int probe = 0; probe < kHotSlots; ++probe) {
        if (atomicCAS(&s_hkey[h], kNoRow, row) == kNoRow) {
          s_hidx[h] = (uint32_t)tid;
          break;
        }
        h = (h + 1) & (kHotSlots - 1);
      }
    }
  }
  // windows of this workgroup: blockIdx.x, blockIdx.x + gridDim.x, ...
  const int64_t wstep = gridDim.x;
  // the first window's non-zeros of this thread: window positions tid + i * kWin
  uint64_t nkey[WPT];
  float nx[WPT];
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    nkey[i] = 0;
    nx[i] = 0.f;
    const int64_t k = (int64_t)blockIdx.x * W + tid + i * kWin;
    if ((int64_t)blockIdx.x < nwin && k < p.n) {
      nkey[i] = p.keys[k];
      nx[i] = p.vals[k];
    }
  }
  constexpr int NO = N > 1 ? N - 1 : 1;          // other modes
  __amdgpu_buffer_rsrc_t rs[NO];
  const void* ap[NO];
#pragma unroll
  for (int j = 0; j + 1 < N; ++j) {
    const int m = (j < p.mode) ? j : j + 1;
    ap[j] = p.A[m];
    rs[j] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.A[m]), 0, (int)p.abytes[m],
                                              (int)kBufFlags);
  }
  // the target mode's factor (read by the fused residual walk only)
  const __amdgpu_buffer_rsrc_t rs_t = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(p.A[RES ? p.mode : 0]), 0, RES ? (int)p.abytes[p.mode] : 0,
      (int)kBufFlags);
  const float scale = term_scale(p);
  const int g = tid / LPN;
  const int rl = tid % LPN;
  const int p0 = g * PPG;
  const uint64_t gmask = PPG >= 64 ? ~0ULL : ((1ULL << PPG) - 1);

  for (int64_t win = blockIdx.x; win < nwin; win += wstep) {
    const int64_t k0 = win * W;
    const int nvalid = (int)min((int64_t)W, p.n - k0);

    // ---- processing: decode, group by target
    uint32_t c[WPT][N], tgt[WPT], tfield[WPT], bkt[WPT], rank[WPT];
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int wp = tid + i * kWin;   // position in the window
      if (wp < nvalid) {
        decode<N>(p, nkey[i], p.base + k0 + wp, c[i]);
      } else {
#pragma unroll
        for (int m = 0; m < N; ++m) c[i][m] = 0;
      }
      tgt[i] = 0;
#pragma unroll
      for (int m = 0; m < N; ++m)
        if (m == p.mode) tgt[i] = c[i][m];
    }
    for (int i = tid; i < NB; i += kWin) s_hist[i] = 0;
    __syncthreads();   // also: the stash lookup is built, the previous window is done
    // counting sort on a hash of the target; a frequent row has bucket = its
    // stash index, the other targets share the remaining buckets (two targets
    // sharing a bucket may interleave, which only splits a segment)
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const bool valid = tid + i * kWin < nvalid;
      tfield[i] = tgt[i];
      const int hs = (K > 0 && valid) ? hot_lookup(s_hkey, s_hidx, tgt[i]) : -1;
      if (hs >= 0) {
        bkt[i] = (uint32_t)hs;
        tfield[i] = kHotFlag | (uint32_t)hs;
      } else {
        const uint32_t h = tgt[i] * 0x9E3779B1u;
        bkt[i] = (uint32_t)K + (uint32_t)(((uint64_t)h * (uint32_t)(NB - K)) >> 32);
      }
      rank[i] = valid ? atomicAdd(&s_hist[bkt[i]], 1u) : 0u;
    }
    __syncthreads();
    block_exclusive_scan<NB, kWin>(s_hist, tid, s_wsum);
    // record at the grouped position: fields 0..N-2 the byte offsets (row
    // indices when BIG) of the other modes' factor rows in ascending mode
    // order, field N-1 the target field, field N the value; padding positions
    // (nvalid and above) stay where they are
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int wp = tid + i * kWin;
      const int pos = wp < nvalid ? (int)(s_hist[bkt[i]] + rank[i]) : wp;
#pragma unroll
      for (int j = 0; j + 1 < N; ++j) {
        const uint32_t cj = (j < p.mode) ? c[i][j] : c[i][j + 1];
        s_rec[pos * NP + j] = BIG ? cj : cj * p.rowbytes;
      }
      s_rec[pos * NP + N - 1] = tfield[i];
      s_rec[pos * NP + N] = __float_as_uint(wp < nvalid ? nx[i] : 0.f);
      if constexpr (RES) {
        s_rec[pos * NP + N + 1] = tgt[i] * p.rowbytes;
        s_rec[pos * NP + N + 2] = (uint32_t)wp;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int wp = tid + i * kWin;
      const uint32_t t0 = s_rec[wp * NP + N - 1];
      const bool end = (wp < nvalid) && (wp == nvalid - 1 || s_rec[(wp + 1) * NP + N - 1] != t0);
      const uint64_t em = __ballot(end);
      if (lane == 0) s_end[wp >> 6] = em;
    }
    // the next window's non-zeros, in flight during this walk
    if constexpr (STASH) {
#pragma unroll
      for (int i = 0; i < WPT; ++i) {
        const int64_t k = (win + wstep) * W + tid + i * kWin;
        if (win + wstep < nwin && k < p.n) {
          nkey[i] = p.keys[k];
          nx[i] = p.vals[k];
        }
      }
    }
    __syncthreads();

    // ---- computing: LPN lanes per group, RPL ranks per lane (lane j holds
    // ranks j, j + LPN, ... for fp32 factors, ranks RPL*j .. RPL*j + RPL - 1 for
    // bf16), each group walking LPN consecutive positions
    const uint64_t endw = s_end[p0 >> 6] >> (p0 & 63);
    const bool starts_before =
        p0 > 0 && p0 < nvalid && !((s_end[(p0 - 1) >> 6] >> ((p0 - 1) & 63)) & 1);
    const bool can_carry = p0 + PPG <= nvalid;
    // 3-mode tensors with 16-lane groups (one DPP row per group): the walk
    // takes record fields from registers.  Lane rl of a group starts with the
    // record of the group's position rl; each step of U positions broadcasts
    // lanes 0..U-1 of the row and then shifts the row down by U lanes.  (For
    // other mode counts the extra registers cost more than the LDS reads save.)
    constexpr bool kRowB = (LPN == 16) && (N == 3);
    for (int r0 = 0; r0 < R; r0 += LPN * RPL) {
      uint32_t myrec[kRowB ? NF : 1];
      bool ract[RPL];
      uint32_t loff[RPL];
      float acc[RPL], carry[RPL];
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = PACKED ? r0 + rl * RPL + k : r0 + rl + k * LPN;
        ract[k] = r < R;
        loff[k] = (uint32_t)(ract[k] ? r : 0) * (uint32_t)sizeof(FT);
        acc[k] = 0.f;
        carry[k] = 0.f;
      }
      bool first = true, has_carry = false;
      for (int q0 = 0; q0 < PPG; q0 += U) {
        if constexpr (kRowB) {
          // the records of the next LPN positions, one per lane
          if (q0 % LPN == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) myrec[f] = s_rec[(p0 + q0 + rl) * NP + f];
          }
        }
        float pr[U][RPL];
        float ta[RES ? U : 1][RPL];
        float xs[RES ? U : 1];
        uint32_t wpos[RES ? U : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // the record of position q0 + u: from the row, or from LDS
          uint32_t e[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f)
            if (f != N - 1) {
              if constexpr (kRowB) e[f] = row_bcast(myrec[f], u);
            }
          const uint32_t* er = &s_rec[(p0 + q0 + u) * NP];
          const float xv = __uint_as_float(kRowB ? e[N] : er[N]);
#pragma unroll
          for (int k = 0; k < RPL; ++k) pr[u][k] = RES ? 1.f : xv;
          if constexpr (RES) {
            xs[u] = xv;
            const uint32_t toff = kRowB ? e[N + 1] : er[N + 1];
            wpos[u] = kRowB ? e[N + 2] : er[N + 2];
            if constexpr (PACKED) {
              ld_bf16_run<RPL, VEC>(rs_t, toff + loff[0], ta[u]);
            } else {
#pragma unroll
              for (int k = 0; k < RPL; ++k) ta[u][k] = ld_buf<FT>(rs_t, toff + loff[k]);
            }
          }
#pragma unroll
          for (int j = 0; j + 1 < N; ++j) {
            const uint32_t f = kRowB ? e[j] : er[j];
            if constexpr (BIG && PACKED) {
              const FT* rowp = static_cast<const FT*>(ap[j]) + (size_t)f * R;
              float t3[RPL];
              ld_bf16_run_ptr<RPL, VEC>(rowp + loff[0] / sizeof(FT), ract, t3);
#pragma unroll
              for (int k = 0; k < RPL; ++k) pr[u][k] *= t3[k];
            } else if constexpr (BIG) {
              const FT* rowp = static_cast<const FT*>(ap[j]) + (size_t)f * R;
#pragma unroll
              for (int k = 0; k < RPL; ++k)
                pr[u][k] *= ld_factor<FT>(rowp, (size_t)(loff[k] / sizeof(FT)));
            } else if constexpr (PACKED) {
              float t3[RPL];
              ld_bf16_run<RPL, VEC>(rs[j], f + loff[0], t3);
#pragma unroll
              for (int k = 0; k < RPL; ++k) pr[u][k] *= t3[k];
            } else if constexpr (BASE32) {
#pragma unroll
              for (int k = 0; k < RPL; ++k) pr[u][k] *= ld_base(ap[j], f + loff[k]);
            } else {
#pragma unroll
              for (int k = 0; k < RPL; ++k) pr[u][k] *= ld_buf<FT>(rs[j], f + loff[k]);
            }
          }
        }
        if constexpr (RES) {
          // model at each position (sum over the group's 16 lanes), residual, and
          // the residual-scaled product of the other modes' rows
#pragma unroll
          for (int u = 0; u < U; ++u) {
            float part = 0.f;
#pragma unroll
            for (int k = 0; k < RPL; ++k)
              if (ract[k]) part += pr[u][k] * ta[u][k];
#pragma unroll
            for (int off = LPN / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
            const float ev = xs[u] - part;
#pragma unroll
            for (int k = 0; k < RPL; ++k) pr[u][k] *= ev;
            if (rl == 0 && (int)wpos[u] < nvalid) p.resid[k0 + wpos[u]] = ev;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = q0 + u;
#pragma unroll
          for (int k = 0; k < RPL; ++k) acc[k] += pr[u][k];
          const bool seg_end = (endw >> q) & 1;
          if (seg_end || (q == PPG - 1 && can_carry)) {
            if (first && starts_before) {
#pragma unroll
              for (int k = 0; k < RPL; ++k) s_head[tid * RPL + k] = acc[k];
            } else if (seg_end) {
              const uint32_t tf = kRowB ? row_bcast(myrec[N - 1], u)
                                        : seg_target(s_rec, (p0 + q) * NP, p.mode, N);
              if (K > 0 && (tf & kHotFlag)) {
                float* srow = s_stash + (size_t)(tf & ~kHotFlag) * R + r0 + (PACKED ? rl * RPL : rl);
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                  if (ract[k]) srow[PACKED ? k : k * LPN] += acc[k];
              } else {
                const size_t row = (size_t)tf * R;
                if constexpr (PACKED) {
                  flush_packed<RPL, LPN>(p.out + row + r0, acc, scale, rl, R - r0);
                } else {
#pragma unroll
                  for (int k = 0; k < RPL; ++k)
                    if (ract[k]) unsafeAtomicAdd(p.out + row + r0 + rl + k * LPN, acc[k] * scale);
                }
              }
            } else {
#pragma unroll
              for (int k = 0; k < RPL; ++k) carry[k] = acc[k];
              has_carry = true;
            }
#pragma unroll
            for (int k = 0; k < RPL; ++k) acc[k] = 0.f;
            first = false;
          }
        }
        if constexpr (kRowB) {
#pragma unroll
          for (int f = 0; f < NF; ++f) myrec[f] = row_shl(myrec[f], U);
        }
      }
      __syncthreads();
      if (has_carry) {
        // this group owns a segment that continues into the next groups
        for (int g2 = g + 1; g2 < G; ++g2) {
          const int q2 = g2 * PPG;
#pragma unroll
          for (int k = 0; k < RPL; ++k) carry[k] += s_head[(g2 * LPN + rl) * RPL + k];
          if ((s_end[q2 >> 6] >> (q2 & 63)) & gmask) break;
        }
        const uint32_t tf = seg_target(s_rec, (p0 + PPG - 1) * NP, p.mode, N);
        if (K > 0 && (tf & kHotFlag)) {
          float* srow = s_stash + (size_t)(tf & ~kHotFlag) * R + r0 + (PACKED ? rl * RPL : rl);
#pragma unroll
          for (int k = 0; k < RPL; ++k)
            if (ract[k]) srow[PACKED ? k : k * LPN] += carry[k];
        } else {
          const size_t row = (size_t)tf * R;
          if constexpr (PACKED) {
            flush_packed<RPL, LPN>(p.out + row + r0, carry, scale, rl, R - r0);
          } else {
#pragma unroll
            for (int k = 0; k < RPL; ++k)
              if (ract[k]) unsafeAtomicAdd(p.out + row + r0 + rl + k * LPN, carry[k] * scale);
          }
        }
      }
      __syncthreads();
    }
    if constexpr (!STASH) break;
  }
  // ---- the stash of frequent rows: one atomic per (row, rank) that received a term
  if (K > 0) {
    __syncthreads();
    for (int i = tid; i < K * R; i += kWin) {
      const float v = s_stash[i];
      const int hr = i / R;
      if (v != 0.f) unsafeAtomicAdd(p.out + (size_t)p.hot[hr] * R + (i - hr * R), v * scale);
    }
  }
}

// ---------------------------------------------------------------------------
// BLCO MTTKRP with hierarchical conflict resolution (Section 5.1, steps 1-6),
// the mechanism the heuristic of Section 5.3 picks for short target modes.
//
// Each workgroup owns a contiguous range of the ALTO-ordered non-zeros and a
// slice of at most 64 ranks (blockIdx.y), and keeps a private copy of that
// slice of all I_n output rows in LDS (the stash; it covers every target row,
// so no lookup is needed).  Per batch of kShortB non-zeros:
//   processing: one non-zero per thread is loaded (coalesced) and decoded by
//     shift and mask; the batch is grouped by target row with a counting sort
//     (LDS histogram with atomic ranks, exclusive scan, scatter), and each
//     grouped position gets a record: byte offsets of the other modes' factor
//     rows, target row, value;
//   computing: each group of LPN lanes (RPL ranks per lane) walks LPN
//     consecutive grouped positions, kShortLoads / RPL at a time, gathering
//     the other modes' rows and summing the scaled Hadamard products in
//     registers while the target stays the same;
//   stash update: a target's positions form one run, so each run has one
//     owner, the group holding its first position.  A group whose first
//     segment continues a run from an earlier group leaves that partial sum
//     in a per-group carry slot; after a barrier the owner of a run that
//     crosses into later groups adds their carries.  Every owner then adds its
//     run's sum into the stash row with a plain LDS read-modify-write: no two
//     lanes touch one stash entry in a batch, so no LDS atomics are needed
//     (fp32 LDS atomics measured several times slower than this on gfx950).
// When the range is done the stash is added to the output with one global
// atomic per (row, rank) that received any term, so an output row sees one
// update per workgroup instead of one per window.
constexpr int kShortB = 1024;               // threads = non-zeros per batch
constexpr int kShortLPN = 16;               // lanes per position
constexpr int kShortNG = kShortB / kShortLPN;   // lane groups = positions per group
constexpr int kShortHist = 1024;            // histogram bins (>= I_n)
constexpr int kShortLds = 64 * 1024;        // records + histogram + carries + stash
constexpr int kShortLoads = 8;              // positions x ranks in flight per lane

// LDS bytes besides the stash: records, histogram, scan totals, carry slots
// (one per group, cls = 16, 32 or 64 floats: the ranks one group covers)
__host__ __device__ constexpr size_t short_fixed_lds(int N, int cls) {
  return (size_t)kShortB * (N + 1) * 4 + (size_t)kShortHist * 4 + (kShortB / 64) * 4 +
         (size_t)kShortNG * cls * 4;
}

//
// Rank layout as in the window kernel: with bf16 factors each lane holds RPL
// consecutive ranks of the slice (VEC: one 4- or 8-byte gather when R is even).
template <int RPL, typename FT, int N, bool BIG, bool VEC = false>
__global__ __launch_bounds__(kShortB, 8) void k_mttkrp_short(KParams p, int64_t per) {
  extern __shared__ __align__(16) unsigned char smem_short[];
  constexpr int LPN = kShortLPN;
  constexpr bool PACKED = sizeof(FT) == 2 && RPL > 1;
  static_assert(!VEC || PACKED, "vector gathers are for packed bf16 ranks");
  constexpr int NF = N + 1;
  constexpr int NG = kShortNG;
  constexpr int C = kShortB / NG;            // positions per group and batch
  constexpr int U = kShortLoads / RPL;       // positions in flight per group
  constexpr int CW = LPN * RPL;              // ranks one group covers (carry slot)
  const int I = (int)p.short_rows;
  const int SW = p.short_width;              // <= CW
  const int rlo = (int)blockIdx.y * SW;
  const int W = min(SW, p.R - rlo);
  uint32_t* s_rec = reinterpret_cast<uint32_t*>(smem_short);    // kShortB x NF
  uint32_t* s_hist = s_rec + kShortB * NF;                      // kShortHist
  uint32_t* s_wsum = s_hist + kShortHist;                       // kShortB / 64
  float* s_carry = reinterpret_cast<float*>(s_wsum + kShortB / 64);   // NG x CW
  float* s_out = s_carry + NG * CW;                             // I x SW
  const int tid = threadIdx.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(p.n, lo + per);
  if (lo >= hi || W <= 0) return;
  for (int i = tid; i < I * SW; i += kShortB) s_out[i] = 0.f;
  for (int i = tid; i < kShortHist; i += kShortB) s_hist[i] = 0;
  const int gi = tid / LPN, rl = tid % LPN;
  constexpr int NO = N > 1 ? N - 1 : 1;
  __amdgpu_buffer_rsrc_t rs[NO];
  const void* ap[NO];
#pragma unroll
  for (int j = 0; j + 1 < N; ++j) {
    const int m = (j < p.mode) ? j : j + 1;
    ap[j] = p.A[m];
    rs[j] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.A[m]), 0, (int)p.abytes[m],
                                              (int)kBufFlags);
  }
  uint32_t loff[RPL];
  bool ract[RPL];
  int rix[RPL];   // slice-relative rank of each of this lane's RPL values
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = PACKED ? rl * RPL + q : rl + q * LPN;
    rix[q] = r;
    ract[q] = r < W;
    loff[q] = (uint32_t)(rlo + (ract[q] ? r : 0)) * (uint32_t)sizeof(FT);
  }
  for (int64_t b0 = lo; b0 < hi; b0 += kShortB) {
    // ---- processing: load, decode, group by target
    __syncthreads();   // histogram cleared; the previous batch's records and carries consumed
    const int64_t k = b0 + tid;
    const bool valid = k < hi;
    uint32_t c[N];
    float x = 0.f;
    uint32_t tgt = 0, rank = 0;
    if (valid) {
      decode<N>(p, p.keys[k], p.base + k, c);
      x = p.vals[k];
#pragma unroll
      for (int m = 0; m < N; ++m)
        if (m == p.mode) tgt = c[m];
      rank = atomicAdd(&s_hist[tgt], 1u);
    }
    __syncthreads();
    block_exclusive_scan<kShortHist, kShortB>(s_hist, tid, s_wsum);
    if (valid) {
      const int pos = (int)(s_hist[tgt] + rank);
#pragma unroll
      for (int j = 0; j + 1 < N; ++j)
        s_rec[pos * NF + j] = ((j < p.mode) ? c[j] : c[j + 1]) * (BIG ? 1u : p.rowbytes);
      s_rec[pos * NF + N - 1] = tgt;
      s_rec[pos * NF + N] = __float_as_uint(x);
    }
    __syncthreads();
    // ---- computing: segment sums of this group's positions
    const int nb = (int)min<int64_t>(kShortB, hi - b0);
    const int q0 = gi * C;
    const int qe = min(q0 + C, nb);
    float acc[RPL];
    uint32_t cur = 0;
    bool pending = false;   // owner of a run that continues into later groups
    int run_end = 0;        // end of that run (grouped position)
    if (q0 < qe) {
      cur = s_rec[q0 * NF + N - 1];
      const bool first_shared = q0 > 0 && s_rec[(q0 - 1) * NF + N - 1] == cur;
      const bool last_cont = qe < nb && s_rec[qe * NF + N - 1] == s_rec[(qe - 1) * NF + N - 1];
      bool first = true;
#pragma unroll
      for (int q = 0; q < RPL; ++q) acc[q] = 0.f;
      for (int j0 = q0; j0 < qe; j0 += U) {
        float pr[U][RPL];
        uint32_t tg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = j0 + u;
          const uint32_t* e = &s_rec[(j < qe ? j : j0) * NF];
          const float xv = __uint_as_float(e[N]);
          tg[u] = e[N - 1];
#pragma unroll
          for (int q = 0; q < RPL; ++q) pr[u][q] = xv;
#pragma unroll
          for (int jj = 0; jj + 1 < N; ++jj) {
            if constexpr (BIG && PACKED) {
              const FT* rowp = static_cast<const FT*>(ap[jj]) + (size_t)e[jj] * p.R;
              float t3[RPL];
              ld_bf16_run_ptr<RPL, VEC>(rowp + loff[0] / sizeof(FT), ract, t3);
#pragma unroll
              for (int q = 0; q < RPL; ++q) pr[u][q] *= t3[q];
            } else if constexpr (BIG) {
              const FT* rowp = static_cast<const FT*>(ap[jj]) + (size_t)e[jj] * p.R;
#pragma unroll
              for (int q = 0; q < RPL; ++q)
                pr[u][q] *= ld_factor<FT>(rowp, (size_t)(loff[q] / sizeof(FT)));
            } else if constexpr (PACKED) {
              float t3[RPL];
              ld_bf16_run<RPL, VEC>(rs[jj], e[jj] + loff[0], t3);
#pragma unroll
              for (int q = 0; q < RPL; ++q) pr[u][q] *= t3[q];
            } else {
#pragma unroll
              for (int q = 0; q < RPL; ++q) pr[u][q] *= ld_buf<FT>(rs[jj], e[jj] + loff[q]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (j0 + u >= qe) break;
          if (tg[u] != cur) {
            // a finished segment that does not reach the end of this group
            if (first && first_shared) {
#pragma unroll
              for (int q = 0; q < RPL; ++q) s_carry[gi * CW + rix[q]] = acc[q];
            } else {
#pragma unroll
              for (int q = 0; q < RPL; ++q)
                if (ract[q]) s_out[cur * SW + rix[q]] += acc[q];
            }
            first = false;
            cur = tg[u];
#pragma unroll
            for (int q = 0; q < RPL; ++q) acc[q] = 0.f;
          }
#pragma unroll
          for (int q = 0; q < RPL; ++q) acc[q] += pr[u][q];
        }
      }
      // the segment that reaches the end of this group
      if (first && first_shared) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) s_carry[gi * CW + rix[q]] = acc[q];
      } else if (last_cont) {
        pending = true;
        // the scanned histogram holds each target's first position, so the
        // run of `cur` ends where the next target's begins
        run_end = cur + 1 < (uint32_t)kShortHist ? (int)s_hist[cur + 1] : nb;
      } else {
#pragma unroll
        for (int q = 0; q < RPL; ++q)
          if (ract[q]) s_out[cur * SW + rix[q]] += acc[q];
      }
    }
    __syncthreads();
    // ---- owners of runs that cross groups add the later groups' carries
    if (pending) {
#pragma unroll 4
      for (int g2 = gi + 1; g2 * C < run_end; ++g2) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) acc[q] += s_carry[g2 * CW + rix[q]];
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (ract[q]) s_out[cur * SW + rix[q]] += acc[q];
    }
    for (int i = tid; i < kShortHist; i += kShortB) s_hist[i] = 0;
  }
  __syncthreads();
  // ---- one global atomic per stash entry that received a term
  const float scale = term_scale(p);
  for (int i = tid; i < I * W; i += kShortB) {
    const int row = i / W, r = i - row * W;
    const float v = s_out[row * SW + r];
    if (v != 0.f) unsafeAtomicAdd(p.out + (size_t)row * p.R + rlo + r, v * scale);
  }
}

// Sampled CP model, residual and squared residual sums (Section 2.2 model):
// one wave per 64 consecutive non-zeros.  Each non-zero's record (byte offsets,
// or row indices when BIG, of its N factor rows, and its value) goes to LDS;
// groups of 16 lanes (RPL ranks per lane) then walk 16 records each,
// 8 / RPL at a time, issuing every gather of those records before the first
// use, and reduce the rank sum across the group.  The residual x - xhat is
// written in BLCO order; the squared residuals are summed in fp64 per
// workgroup (k_reduce_loss adds the partials in a fixed order).  bf16 factors take
// the packed rank layout of the MTTKRP kernels (VEC: one 4- or 8-byte gather).
template <int RPL, typename FT, int N, bool BIG, bool VEC = false>
__global__ __launch_bounds__(kBlock) void k_loss_tile(KParams p) {
  constexpr int LPN = 16;
  constexpr bool PACKED = sizeof(FT) == 2 && RPL > 1;
  static_assert(!VEC || PACKED, "vector gathers are for packed bf16 ranks");
  constexpr int G = 64 / LPN;                  // groups per wave
  constexpr int PPG = 64 / G;                  // records per group
  constexpr int NF = N + 1;
  constexpr int U = (8 / RPL) < PPG ? (8 / RPL) : PPG;
  __shared__ uint32_t s[kWaves][64][NF];
  __shared__ float s_e[kWaves][64];
  __shared__ double s_part[kWaves];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * kWaves + wv;
  const int64_t k = tile * 64 + lane;
  const bool valid = k < p.n;
  uint32_t c[N];
  float x = 0.f;
  if (valid) {
    uint64_t key = p.keys[k];
    x = p.vals[k];
    decode<N>(p, key, p.base + k, c);
  } else {
#pragma unroll
    for (int m = 0; m < N; ++m) c[m] = 0;
  }
#pragma unroll
  for (int m = 0; m < N; ++m) s[wv][lane][m] = BIG ? c[m] : c[m] * p.rowbytes;
  s[wv][lane][N] = __float_as_uint(x);
  s_e[wv][lane] = x;
  __amdgpu_buffer_rsrc_t rs[N];
#pragma unroll
  for (int m = 0; m < N; ++m)
    rs[m] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.A[m]), 0, (int)p.abytes[m],
                                              (int)kBufFlags);
  wave_sync_lds();
  const int g = lane / LPN;
  const int rl = lane % LPN;
  const int R = p.R;
  for (int r0 = 0; r0 < R; r0 += LPN * RPL) {
    uint32_t loff[RPL];
    bool ract[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = PACKED ? r0 + rl * RPL + q : r0 + rl + q * LPN;
      ract[q] = r < R;
      loff[q] = (uint32_t)(ract[q] ? r : 0) * (uint32_t)sizeof(FT);
    }
    for (int q0 = 0; q0 < PPG; q0 += U) {
      float v[U][RPL];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t* e = s[wv][g * PPG + q0 + u];
#pragma unroll
        for (int q = 0; q < RPL; ++q) v[u][q] = 1.f;
#pragma unroll
        for (int m = 0; m < N; ++m) {
          const uint32_t f = e[m];
          if constexpr (BIG && PACKED) {
            const FT* rowp = static_cast<const FT*>(p.A[m]) + (size_t)f * R;
            float t3[RPL];
            ld_bf16_run_ptr<RPL, VEC>(rowp + loff[0] / sizeof(FT), ract, t3);
#pragma unroll
            for (int q = 0; q < RPL; ++q) v[u][q] *= t3[q];
          } else if constexpr (BIG) {
            const FT* rowp = static_cast<const FT*>(p.A[m]) + (size_t)f * R;
#pragma unroll
            for (int q = 0; q < RPL; ++q)
              v[u][q] *= ld_factor<FT>(rowp, (size_t)(loff[q] / sizeof(FT)));
          } else if constexpr (PACKED) {
            float t3[RPL];
            ld_bf16_run<RPL, VEC>(rs[m], f + loff[0], t3);
#pragma unroll
            for (int q = 0; q < RPL; ++q) v[u][q] *= t3[q];
          } else {
#pragma unroll
            for (int q = 0; q < RPL; ++q) v[u][q] *= ld_buf<FT>(rs[m], f + loff[q]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float part = 0.f;
#pragma unroll
        for (int q = 0; q < RPL; ++q)
          if (ract[q]) part += v[u][q];
#pragma unroll
        for (int off = LPN / 2; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (rl == 0) s_e[wv][g * PPG + q0 + u] -= part;
      }
    }
  }
  wave_sync_lds();
  const float e = s_e[wv][lane];
  if (valid && p.out) p.out[k] = e;
  double e2 = valid ? (double)e * (double)e : 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
  if (lane == 0) s_part[wv] = e2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_part[w];
    p.partials[blockIdx.x] = t;
  }
}

// Sum of squares of a residual in fp64: workgroup b sums entries
// [b * kSqPer, (b + 1) * kSqPer) in a fixed order into part[b].
constexpr int kSqPer = 4096;
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ r, int64_t n,
                                               double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t lo = (int64_t)blockIdx.x * kSqPer;
  const int64_t hi = min(n, lo + (int64_t)kSqPer);
  double a = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double e = (double)r[i];
    a += e * e;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss = 1/2 * sum of the partials, in a fixed order (one workgroup).
__global__ __launch_bounds__(1024) void k_reduce_loss(const double* __restrict__ part, int64_t n,
                                                      double* __restrict__ loss) {
  __shared__ double sh[1024];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) a += part[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = 0.5 * sh[0];
}

// fp32 -> bf16, round to nearest even; NaN stays a (quiet) NaN.
__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src,
                                                   uint16_t* __restrict__ dst, int64_t n) {
  int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    uint32_t u = __float_as_uint(src[i]);
    uint16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      b = (uint16_t)((u >> 16) | 0x40u);
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      b = (uint16_t)(u >> 16);
    }
    dst[i] = b;
  }
}

// Calibration of the memory-side atomic rate: for each k < n, one row-op on
// out row rows[k]: 16 lanes add 1.0f to the row's R entries, lane l holding
// ranks l, l + 16, ..., as the window kernel flushes a finished segment.  Row
// ids at or past nrows are skipped.
__global__ __launch_bounds__(256) void k_atomic_probe(float* __restrict__ out, int64_t nrows,
                                                      const uint32_t* __restrict__ rows,
                                                      int64_t n, int R) {
  const int64_t g = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int rl = threadIdx.x & 15;
  if (g >= n) return;
  const uint32_t row = rows[g];
  if ((int64_t)row >= nrows) return;
  float* dst = out + (size_t)row * R;
  for (int r = rl; r < R; r += 16) unsafeAtomicAdd(dst + r, 1.0f);
}

// Measurement kernel: groups of 16 lanes read kGatherRows rows of table each (ranks
// l, l + 16, ... per lane, all loads of a group in flight together), as the MTTKRP
// kernels gather factor rows; lane 0 of a group stores its partial sum in sink[group].
constexpr int kGatherRows = 6;
__global__ __launch_bounds__(256) void k_gather_probe(const float* __restrict__ table,
                                                      int64_t nrows,
                                                      const uint32_t* __restrict__ rows,
                                                      int64_t n, int R, float* __restrict__ sink) {
  const int64_t g = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int rl = threadIdx.x & 15;
  const int64_t k0 = g * kGatherRows;
  if (k0 >= n) return;
  uint32_t rr[kGatherRows];
#pragma unroll
  for (int j = 0; j < kGatherRows; ++j) {
    rr[j] = k0 + j < n ? rows[k0 + j] : 0xFFFFFFFFu;
    if ((int64_t)rr[j] >= nrows) rr[j] = 0xFFFFFFFFu;
  }
  float s = 0.f;
#pragma unroll 4
  for (int r = rl; r < R; r += 16) {
    float v[kGatherRows];
#pragma unroll
    for (int j = 0; j < kGatherRows; ++j)
      v[j] = rr[j] != 0xFFFFFFFFu ? table[(size_t)rr[j] * R + r] : 0.f;
#pragma unroll
    for (int j = 0; j < kGatherRows; ++j) s += v[j];
  }
  if (rl == 0) sink[g] = s;
}

// x[i] *= (float)(alpha * scale[0]) (the chain-rule factor of an autograd backward).
__global__ __launch_bounds__(256) void k_scale(float* __restrict__ x, int64_t n,
                                               const double* __restrict__ scale, double alpha) {
  const float f = (float)(alpha * (scale ? scale[0] : 1.0));
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) x[i] *= f;
}

// ====================================================================== dispatch

typedef void (*KernelFn)(KParams);

template <int LPN, int RPL, typename FT, bool BIG, bool STASH, bool VEC>
static KernelFn pick_win_s(int N) {
  switch (N) {
    case 1: return k_mttkrp_win<LPN, RPL, FT, 1, BIG, STASH, false, VEC>;
    case 2: return k_mttkrp_win<LPN, RPL, FT, 2, BIG, STASH, false, VEC>;
    case 3: return k_mttkrp_win<LPN, RPL, FT, 3, BIG, STASH, false, VEC>;
    case 4: return k_mttkrp_win<LPN, RPL, FT, 4, BIG, STASH, false, VEC>;
    case 5: return k_mttkrp_win<LPN, RPL, FT, 5, BIG, STASH, false, VEC>;
    case 6: return k_mttkrp_win<LPN, RPL, FT, 6, BIG, STASH, false, VEC>;
    case 7: return k_mttkrp_win<LPN, RPL, FT, 7, BIG, STASH, false, VEC>;
    default: return k_mttkrp_win<LPN, RPL, FT, 8, BIG, STASH, false, VEC>;
  }
}

// windows of 2048 or 4096 non-zeros (two or four per thread; no stash), up to 5 modes
constexpr int kWideMaxN = 5;
template <int LPN, int RPL, typename FT, bool BIG, bool VEC, int WPT>
static KernelFn pick_win_wide(int N) {
  switch (N) {
    case 1: return k_mttkrp_win<LPN, RPL, FT, 1, BIG, false, false, VEC, WPT>;
    case 2: return k_mttkrp_win<LPN, RPL, FT, 2, BIG, false, false, VEC, WPT>;
    case 3: return k_mttkrp_win<LPN, RPL, FT, 3, BIG, false, false, VEC, WPT>;
    case 4: return k_mttkrp_win<LPN, RPL, FT, 4, BIG, false, false, VEC, WPT>;
    default: return k_mttkrp_win<LPN, RPL, FT, 5, BIG, false, false, VEC, WPT>;
  }
}

// Non-zeros per thread of the window kernel: for a plain MTTKRP without a stash over
// 16-lane groups and at most kWideMaxN modes, two at R <= 32 and four at 32 < R <= 64
// (four ranks per lane); else one.
static int win_wpt(int N, int R, bool stash, bool resid) {
  if (stash || resid || R > 64 || N > kWideMaxN) return 1;
  return R > 32 ? 4 : 2;
}

// VEC (vector gathers of packed bf16 ranks) only where the ranks are packed: bf16
// factors, two or more ranks per lane, and an even R
template <int LPN, int RPL, typename FT, bool BIG>
static KernelFn pick_win(int N, int R, bool stash) {
  // the wide window of this rank layout (win_wpt's rule: four ranks per lane take four)
  constexpr int WW = RPL == 4 ? 4 : 2;
  const bool wide = win_wpt(N, R, stash, false) > 1;
  if constexpr (sizeof(FT) == 2 && RPL > 1) {
    if (R % 2 == 0) {
      if constexpr (LPN == 16)
        if (wide) return pick_win_wide<LPN, RPL, FT, BIG, true, WW>(N);
      return stash ? pick_win_s<LPN, RPL, FT, BIG, true, true>(N)
                   : pick_win_s<LPN, RPL, FT, BIG, false, true>(N);
    }
  }
  if constexpr (LPN == 16)
    if (wide) return pick_win_wide<LPN, RPL, FT, BIG, false, WW>(N);
  return stash ? pick_win_s<LPN, RPL, FT, BIG, true, false>(N)
               : pick_win_s<LPN, RPL, FT, BIG, false, false>(N);
}

// the fused residual walk (16-lane groups, one rank slice of at most 64, 32-bit offsets)
template <int RPL, typename FT, bool STASH, bool VEC>
static KernelFn pick_res_s(int N) {
  switch (N) {
    case 1: return k_mttkrp_win<16, RPL, FT, 1, false, STASH, true, VEC>;
    case 2: return k_mttkrp_win<16, RPL, FT, 2, false, STASH, true, VEC>;
    case 3: return k_mttkrp_win<16, RPL, FT, 3, false, STASH, true, VEC>;
    case 4: return k_mttkrp_win<16, RPL, FT, 4, false, STASH, true, VEC>;
    case 5: return k_mttkrp_win<16, RPL, FT, 5, false, STASH, true, VEC>;
    case 6: return k_mttkrp_win<16, RPL, FT, 6, false, STASH, true, VEC>;
    case 7: return k_mttkrp_win<16, RPL, FT, 7, false, STASH, true, VEC>;
    default: return k_mttkrp_win<16, RPL, FT, 8, false, STASH, true, VEC>;
  }
}

template <int RPL, typename FT>
static KernelFn pick_res(int N, int R, bool stash) {
  if constexpr (sizeof(FT) == 2 && RPL > 1) {
    if (R % 2 == 0)
      return stash ? pick_res_s<RPL, FT, true, true>(N) : pick_res_s<RPL, FT, false, true>(N);
  }
  return stash ? pick_res_s<RPL, FT, true, false>(N) : pick_res_s<RPL, FT, false, false>(N);
}

template <typename FT>
static KernelFn select_res_t(int N, int R, bool stash) {
  if (R <= 16) return pick_res<1, FT>(N, R, stash);
  if (R <= 32) return pick_res<2, FT>(N, R, stash);
  return pick_res<4, FT>(N, R, stash);
}

static KernelFn select_res(int N, int R, int fdt, bool stash) {
  return fdt == BLCO_F32 ? select_res_t<float>(N, R, stash) : select_res_t<uint16_t>(N, R, stash);
}

typedef void (*ShortFn)(KParams, int64_t);

template <int RPL, typename FT, bool BIG, bool VEC>
static ShortFn pick_short_v(int N) {
  switch (N) {
    case 1: return k_mttkrp_short<RPL, FT, 1, BIG, VEC>;
    case 2: return k_mttkrp_short<RPL, FT, 2, BIG, VEC>;
    case 3: return k_mttkrp_short<RPL, FT, 3, BIG, VEC>;
    case 4: return k_mttkrp_short<RPL, FT, 4, BIG, VEC>;
    case 5: return k_mttkrp_short<RPL, FT, 5, BIG, VEC>;
    case 6: return k_mttkrp_short<RPL, FT, 6, BIG, VEC>;
    case 7: return k_mttkrp_short<RPL, FT, 7, BIG, VEC>;
    default: return k_mttkrp_short<RPL, FT, 8, BIG, VEC>;
  }
}

// VEC where the bf16 ranks are packed (two or more per lane) and R is even
template <int RPL, typename FT, bool BIG>
static ShortFn pick_short(int N, int R) {
  if constexpr (sizeof(FT) == 2 && RPL > 1) {
    if (R % 2 == 0) return pick_short_v<RPL, FT, BIG, true>(N);
  }
  return pick_short_v<RPL, FT, BIG, false>(N);
}

// ranks per lane of the hierarchical kernel for a slice width (<= 64)
static int short_rpl(int SW) { return SW <= 16 ? 1 : SW <= 32 ? 2 : 4; }

template <typename FT, bool BIG>
static ShortFn select_short_t(int N, int SW, int R) {
  const int rpl = short_rpl(SW);
  if (rpl == 1) return pick_short<1, FT, BIG>(N, R);
  if (rpl == 2) return pick_short<2, FT, BIG>(N, R);
  return pick_short<4, FT, BIG>(N, R);
}

static ShortFn select_short(int N, int SW, int R, int fdt, bool big) {
  if (fdt == BLCO_F32)
    return big ? select_short_t<float, true>(N, SW, R) : select_short_t<float, false>(N, SW, R);
  return big ? select_short_t<uint16_t, true>(N, SW, R)
             : select_short_t<uint16_t, false>(N, SW, R);
}

static size_t short_lds(int N, uint64_t rows, int SW) {
  return short_fixed_lds(N, kShortLPN * short_rpl(SW)) + (size_t)rows * SW * sizeof(float);
}

// Rank-slice width of the hierarchical kernel: slices of at most 64 ranks, as
// even as possible, in multiples of 16 when there are several, such that the
// stash (I_n x SW fp32), the records, the histogram and the carry slots fit in
// kShortLds bytes.  0 when even a 16-rank slice does not fit.
static int short_slice_width(int N, uint64_t rows, int R) {
  if (rows > (uint64_t)kShortHist) return 0;
  for (int slices = (R + 63) / 64; slices <= (R + 15) / 16; ++slices) {
    const int w = slices == 1 ? R : ((R + slices - 1) / slices + 15) / 16 * 16;
    if (short_lds(N, rows, w) <= (size_t)kShortLds) return w;
  }
  return 0;
}

// Compute units of the current device (the Section 5.3 threshold), read once per device.
static int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

template <int RPL, typename FT, bool BIG, bool VEC>
static KernelFn pick_loss_v(int N) {
  switch (N) {
    case 1: return k_loss_tile<RPL, FT, 1, BIG, VEC>;
    case 2: return k_loss_tile<RPL, FT, 2, BIG, VEC>;
    case 3: return k_loss_tile<RPL, FT, 3, BIG, VEC>;
    case 4: return k_loss_tile<RPL, FT, 4, BIG, VEC>;
    case 5: return k_loss_tile<RPL, FT, 5, BIG, VEC>;
    case 6: return k_loss_tile<RPL, FT, 6, BIG, VEC>;
    case 7: return k_loss_tile<RPL, FT, 7, BIG, VEC>;
    default: return k_loss_tile<RPL, FT, 8, BIG, VEC>;
  }
}

// VEC where the bf16 ranks are packed (two or more per lane) and R is even
template <int RPL, typename FT, bool BIG>
static KernelFn pick_loss(int N, int R) {
  if constexpr (sizeof(FT) == 2 && RPL > 1) {
    if (R % 2 == 0) return pick_loss_v<RPL, FT, BIG, true>(N);
  }
  return pick_loss_v<RPL, FT, BIG, false>(N);
}

// window kernel shape (lanes per non-zero x ranks per lane), chosen by measurement on
// the Zipf workloads: R <= 16: 16 x 1; R <= 32: 16 x 2 (8 x 4 was 1.8x slower);
// R <= 64: 16 x 4 (10% faster than 32 x 2); larger: 64 x 2 per pass over the rank
template <typename FT, bool BIG>
static KernelFn select_win_t(int N, int R, bool stash) {
  if (R <= 16) return pick_win<16, 1, FT, BIG>(N, R, stash);
  if (R <= 32) return pick_win<16, 2, FT, BIG>(N, R, stash);
  if (R <= 64) return pick_win<16, 4, FT, BIG>(N, R, stash);
  return pick_win<64, 2, FT, BIG>(N, R, stash);
}

static KernelFn select_win(int N, int R, int fdt, bool big, bool stash) {
  if (fdt == BLCO_F32)
    return big ? select_win_t<float, true>(N, R, stash) : select_win_t<float, false>(N, R, stash);
  return big ? select_win_t<uint16_t, true>(N, R, stash) : select_win_t<uint16_t, false>(N, R, stash);
}

template <typename FT, bool BIG>
static KernelFn select_loss_t(int N, int R) {
  if (R <= 16) return pick_loss<1, FT, BIG>(N, R);
  if (R <= 32) return pick_loss<2, FT, BIG>(N, R);
  return pick_loss<4, FT, BIG>(N, R);
}

static KernelFn select_loss(int N, int R, int fdt, bool big) {
  if (fdt == BLCO_F32)
    return big ? select_loss_t<float, true>(N, R) : select_loss_t<float, false>(N, R);
  return big ? select_loss_t<uint16_t, true>(N, R) : select_loss_t<uint16_t, false>(N, R);
}

// Conflict-resolution mechanism of a mode-`mode` MTTKRP at rank R (Section
// 5.3): the tensor's setting, where AUTO takes the hierarchical mechanism when
// the target mode is shorter than the device's compute units.  *sw receives
// the hierarchical kernel's rank-slice width.
static int resolve(const blco_tensor* t, int mode, int rank, int* sw) {
  const uint64_t rows = t->lay.dims[mode];
  const int w = short_slice_width(t->lay.N, rows, rank);
  *sw = w;
  if (t->resolution == BLCO_RES_REGISTER) return BLCO_RES_REGISTER;
  if (t->resolution == BLCO_RES_HIERARCHICAL) {
    if (!w)
      return set_error(BLCO_EUNSUPPORTED,
                       "hierarchical resolution: mode %d (%llu rows) does not fit the LDS stash",
                       mode, (unsigned long long)rows);
    return BLCO_RES_HIERARCHICAL;
  }
  return (w && rows < (uint64_t)device_cus()) ? BLCO_RES_HIERARCHICAL : BLCO_RES_REGISTER;
}

// Static LDS bytes of a kernel, read once per kernel.
static size_t kernel_static_lds(const void* f) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> cache;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : cache)
    if (e.first == f) return e.second;
  hipFuncAttributes a;
  size_t v = 64 * 1024;   // unknown: assume no room
  if (hipFuncGetAttributes(&a, f) == hipSuccess) v = a.sharedSizeBytes;
  cache.push_back({f, v});
  return v;
}

// LDS per window-kernel workgroup: half a CU's (two resident workgroups),
// at most the per-workgroup limit; read once per device.
static size_t win_lds_budget() {
  static size_t cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  if (!cached[dev]) {
    int cu = 0, blk = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess || cu <= 0)
      cu = 64 * 1024;
    if (hipDeviceGetAttribute(&blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        blk <= 0)
      blk = 64 * 1024;
    cached[dev] = std::min<size_t>((size_t)cu / 2, (size_t)blk);
  }
  return cached[dev];
}

// ====================================================================== host runtime

static size_t factor_elem_bytes(int fdt) { return fdt == BLCO_BF16 ? 2 : 4; }

static void fill_params(const blco_tensor* t, KParams* p) {
  memset(p, 0, sizeof(*p));
  const Layout& L = t->lay;
  for (int m = 0; m < L.N; ++m) {
    p->shift[m] = L.w[m] ? (uint32_t)L.s[m] : 0u;
    p->mask[m] = L.w[m] >= 32 ? 0xFFFFFFFFu : ((1u << L.w[m]) - 1u);
  }
  p->run_start = t->d_run_start;
  p->run_base = t->d_run_base;
  p->tile_run = t->d_tile_run;
  p->multi = (t->run_start.size() > 2) ? 1 : 0;
  if (t->run_start.size() == 2) {
    for (int m = 0; m < L.N; ++m)
      if (t->run_base[m]) p->multi = 1;
  }
  p->scale = 1.0f;
}

static int fill_zero(float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return BLCO_OK;
  int64_t blocks = std::min<int64_t>((n / 4 + 255) / 256 + 1, 8192);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, out, n);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

static int check_factor_args(const blco_tensor* t, int mode, const void* const* factors, int fdt,
                             int rank, const float* out, bool need_mode_factor) {
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  const int N = t->lay.N;
  if (mode < 0 || mode >= N) return set_error(BLCO_EINVAL, "mode %d outside 0..%d", mode, N - 1);
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  if (fdt != BLCO_F32 && fdt != BLCO_BF16) return set_error(BLCO_EINVAL, "factor dtype %d", fdt);
  if (!factors) return set_error(BLCO_EINVAL, "factors is NULL");
  for (int m = 0; m < N; ++m)
    if ((m != mode || need_mode_factor) && !factors[m] && t->nnz > 0)
      return set_error(BLCO_EINVAL, "factors[%d] is NULL", m);
  if (!out) return set_error(BLCO_EINVAL, "out is NULL");
  int sw = 0;
  const int res = resolve(t, mode, rank, &sw);
  return res < 0 ? res : BLCO_OK;
}

// Frequent rows of the target mode that the window kernel `f` keeps in its
// LDS stash: as many as fit beside the kernel's own LDS in one workgroup's
// share of a CU, or none when the rows left out would not be much less
// frequent than the most frequent one (a stash shortens the longest atomic
// chains only then: measured slower on a 1024-row uniform mode, where a fifth
// of the rows fit).  An explicit threshold at build time keeps the stash
// regardless.  The kernel's static LDS does not depend on the factor type.
static int stash_rows(const blco_tensor* t, int mode, int rank, KernelFn f) {
  if (t->nhot[mode] <= 0 || !t->d_hot) return 0;
  int K = 0;
  const size_t fixed = kernel_static_lds((const void*)f) + 2 * (size_t)kHotSlots * 4;
  const size_t budget = win_lds_budget();
  if (budget > fixed)
    K = (int)std::min<size_t>((size_t)t->nhot[mode], (budget - fixed) / ((size_t)rank * 4));
  if (K > 0 && !t->hot_forced) {
    const uint64_t* cnt = t->hot_cnt.data() + (size_t)mode * (kHotMax + 1);
    if (cnt[K] * 4 > cnt[0]) K = 0;
  }
  return K;
}

// Launch the MTTKRP kernel over [lo, lo + n) of the tensor given by keys/vals.
// With resid != nullptr the fused residual walk runs instead (the caller has
// checked fused_mode_ok): resid[0, n) receives the residual of each non-zero.
static int launch_mttkrp(const blco_tensor* t, const uint64_t* keys, const float* vals,
                         int64_t lo, int64_t n, int mode, const void* const* factors, int fdt,
                         int rank, float scale, const double* scale_dev, float* out,
                         hipStream_t s, float* resid = nullptr) {
  if (n <= 0) return BLCO_OK;
  KParams p;
  fill_params(t, &p);
  p.keys = keys;
  p.vals = vals;
  p.base = lo;
  p.n = n;
  for (int m = 0; m < t->lay.N; ++m) p.A[m] = factors[m];
  p.out = out;
  p.R = rank;
  p.mode = mode;
  p.scale = scale;
  p.scale_dev = scale_dev;
  const size_t fsz = factor_elem_bytes(fdt);
  p.rowbytes = (uint32_t)((size_t)rank * fsz);
  // factors below 4 GiB are gathered with 32-bit byte offsets, larger ones
  // with 64-bit addresses; the window kernel's fp32 gathers at 33-64 ranks
  // (ld_base) also take a factor of exactly 4 GiB with 32-bit offsets
  const bool row_big = (size_t)rank * fsz >= (1ULL << 31);
  size_t other = 0;
  for (int m = 0; m < t->lay.N; ++m) {
    const size_t bytes = (size_t)t->lay.dims[m] * rank * fsz;
    p.abytes[m] = (uint32_t)std::min<size_t>(bytes, 0xFFFFFFFFull);
    if (m != mode) other = std::max(other, bytes);
  }
  const bool big = row_big || other > 0xFFFFFFFFull;
  const bool base32 = fdt == BLCO_F32 && rank > 32 && rank <= 64 && !resid;
  const bool big_win = row_big || other > (base32 ? (1ULL << 32) : 0xFFFFFFFFull);
  int sw = 0;
  const int res = resolve(t, mode, rank, &sw);
  if (res < 0) return res;
  if (resid && (res != BLCO_RES_REGISTER || big || rank > 64 ||
                (size_t)t->lay.dims[mode] * rank * fsz > 0xFFFFFFFFull))
    return set_error(BLCO_EUNSUPPORTED, "fused residual walk on mode %d", mode);
  p.resid = resid;
  if (res == BLCO_RES_HIERARCHICAL) {
    p.short_rows = (uint32_t)t->lay.dims[mode];
    p.short_width = sw;
    const int slices = (rank + sw - 1) / sw;
    // two resident workgroups per CU over all slices; each takes an equal range
    const int64_t want = std::max<int64_t>(device_cus() * 2 / slices, 1);
    int64_t per = std::max<int64_t>((n + want - 1) / want, (int64_t)kShortB * 4);
    per = (per + kShortB - 1) / kShortB * kShortB;
    const int64_t nwg = (n + per - 1) / per;
    const size_t lds = short_lds(t->lay.N, t->lay.dims[mode], sw);
    ShortFn f = select_short(t->lay.N, sw, rank, fdt, big);
    hipLaunchKernelGGL(f, dim3((unsigned)nwg, (unsigned)slices), dim3(kShortB), lds, s, p, per);
    HIPCHK(hipGetLastError());
    return BLCO_OK;
  }
  {
    const int N = t->lay.N;
    KernelFn f = resid ? select_res(N, rank, fdt, true) : select_win(N, rank, fdt, big_win, true);
    const int K = stash_rows(t, mode, rank, f);
    p.hot = t->d_hot + (size_t)mode * kHotMax;
    p.nhot = K;
    if (K == 0) f = resid ? select_res(N, rank, fdt, false) : select_win(N, rank, fdt, big_win, false);
    const int64_t nwin = (n + (int64_t)kWin * win_wpt(N, rank, K > 0, resid) - 1) /
                         ((int64_t)kWin * win_wpt(N, rank, K > 0, resid));
    const size_t dyn = K > 0 ? (size_t)K * rank * 4 + 2 * (size_t)kHotSlots * 4 : 0;
    // with a stash: persistent workgroups, kWinRounds times the resident count
    // (two per CU), which balances the end of the launch (measured 1-2% faster
    // than one round) at the cost of more stash flushes; without one: a
    // workgroup per window (measured about 1% faster than persistent ones)
    const int64_t grid =
        K > 0 ? std::min<int64_t>(nwin, (int64_t)device_cus() * 2 * kWinRounds) : nwin;
    hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(kWin), dyn, s, p);
  }
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

static void* pinned_alloc(size_t n) {
  void* p = nullptr;
  if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
  return p;
}
static void pinned_free(void* p) { (void)hipHostFree(p); }


template <class T>
static int upload(T** dst, const T* src, size_t count, size_t* acc) {
  size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
  HIPCHK(hipMalloc((void**)dst, bytes));
  if (count) HIPCHK(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
  *acc += bytes;
  return BLCO_OK;
}

static void release_device(blco_tensor* t) {
  StreamState& st = t->st;
  if (st.copy_stream) {
    (void)hipStreamSynchronize((hipStream_t)st.copy_stream);
    for (int i = 0; i < 2; ++i) {
      if (st.ev_free[i]) (void)hipEventSynchronize((hipEvent_t)st.ev_free[i]);
    }
  }
  for (void* e : st.ev_t) {
    (void)hipEventSynchronize((hipEvent_t)e);
    (void)hipEventDestroy((hipEvent_t)e);
  }
  for (int i = 0; i < 2; ++i) {
    if (st.d_keys[i]) (void)hipFree(st.d_keys[i]);
    if (st.d_vals[i]) (void)hipFree(st.d_vals[i]);
    if (st.d_res[i]) (void)hipFree(st.d_res[i]);
    if (st.ev_ready[i]) (void)hipEventDestroy((hipEvent_t)st.ev_ready[i]);
    if (st.ev_free[i]) (void)hipEventDestroy((hipEvent_t)st.ev_free[i]);
  }
  if (st.copy_stream) (void)hipStreamDestroy((hipStream_t)st.copy_stream);
  st = StreamState();
  if (t->d_keys) (void)hipFree(t->d_keys);
  if (t->d_vals) (void)hipFree(t->d_vals);
  if (t->d_run_start) (void)hipFree(t->d_run_start);
  if (t->d_run_base) (void)hipFree(t->d_run_base);
  if (t->d_tile_run) (void)hipFree(t->d_tile_run);
  if (t->d_partials) (void)hipFree(t->d_partials);
  if (t->d_hot) (void)hipFree(t->d_hot);
  t->d_hot = nullptr;
  t->d_keys = nullptr;
  t->d_vals = nullptr;
  t->d_run_start = nullptr;
  t->d_run_base = nullptr;
  t->d_tile_run = nullptr;
  t->d_partials = nullptr;
}

// ====================================================================== C ABI

extern "C" int blco_build(int nmodes, const uint64_t* dims, int64_t nnz,
                          const uint32_t* const* coords, const float* values,
                          const blco_build_opts* opts, blco_tensor** out) {
  clear_error();
  if (!out) return set_error(BLCO_EINVAL, "out is NULL");
  *out = nullptr;
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
  const bool hot_forced = opts && opts->hot_min_count > 0;
  if (placement != BLCO_PLACE_DEVICE && placement != BLCO_PLACE_PINNED &&
      placement != BLCO_PLACE_HOST)
    return set_error(BLCO_EINVAL, "placement %d", placement);
  blco_tensor* t = new (std::nothrow) blco_tensor();
  if (!t) return set_error(BLCO_ENOMEM, "host allocation failed");
  t->placement = placement;
  HostAlloc ha = nullptr;
  HostFree hf = nullptr;
  if (placement == BLCO_PLACE_PINNED) {
    ha = pinned_alloc;
    hf = pinned_free;
  }
  int rc = host_build(nmodes, dims, nnz, coords, values, key_bits, cap, ha, hf, t);
  if (rc) {
    delete t;
    return rc;
  }
  find_hot_rows(coords, nnz, hot_min, t);
  t->hot_forced = hot_forced;
  if (placement == BLCO_PLACE_HOST) {
    *out = t;
    return BLCO_OK;
  }
  auto fail = [&](int code) {
    release_device(t);
    free_host_arrays(t);
    delete t;
    return code;
  };
  if (hipGetDevice(&t->device) != hipSuccess) {
    set_error(BLCO_EDEVICE, "hipGetDevice failed");
    return fail(BLCO_EDEVICE);
  }
  size_t acc = 0;
  if ((rc = upload(&t->d_run_start, t->run_start.data(), t->run_start.size(), &acc))) return fail(rc);
  if ((rc = upload(&t->d_run_base, t->run_base.data(), t->run_base.size(), &acc))) return fail(rc);
  if ((rc = upload(&t->d_tile_run, t->tile_run.data(), t->tile_run.size(), &acc))) return fail(rc);
  if ((rc = upload(&t->d_hot, t->hot.data(), t->hot.size(), &acc))) return fail(rc);
  if (placement == BLCO_PLACE_DEVICE) {
    if ((rc = upload(&t->d_keys, t->h_keys, (size_t)nnz, &acc))) return fail(rc);
    if ((rc = upload(&t->d_vals, t->h_vals, (size_t)nnz, &acc))) return fail(rc);
    free_host_arrays(t);
  }
  t->device_bytes = acc;
  *out = t;
  return BLCO_OK;
}

extern "C" int blco_mttkrp_v(blco_tensor* t, int mode, const float* values,
                             const void* const* factors, int factor_dtype, int rank,
                             const double* scale, double alpha, float* out, void* stream) {
  clear_error();
  int rc = check_factor_args(t, mode, factors, factor_dtype, rank, out, false);
  if (rc) return rc;
  if (t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "in-memory MTTKRP needs a tensor placed on the device");
  if (!values && t->nnz > 0) return set_error(BLCO_EINVAL, "values is NULL");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = fill_zero(out, (int64_t)t->lay.dims[mode] * rank, s))) return rc;
  return launch_mttkrp(t, t->d_keys, values, 0, t->nnz, mode, factors, factor_dtype, rank,
                       (float)alpha, scale, out, s);
}

extern "C" int blco_mttkrp(blco_tensor* t, int mode, const void* const* factors, int factor_dtype,
                           int rank, float* out, void* stream) {
  clear_error();
  int rc = check_factor_args(t, mode, factors, factor_dtype, rank, out, false);
  if (rc) return rc;
  if (t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "in-memory MTTKRP needs a tensor placed on the device; "
                                  "use blco_mttkrp_stream for a pinned tensor");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = fill_zero(out, (int64_t)t->lay.dims[mode] * rank, s))) return rc;
  return launch_mttkrp(t, t->d_keys, t->d_vals, 0, t->nnz, mode, factors, factor_dtype, rank,
                       1.0f, nullptr, out, s);
}

extern "C" int blco_mttkrp_acc(blco_tensor* t, int mode, const void* const* factors,
                               int factor_dtype, int rank, float* out, void* stream) {
  clear_error();
  int rc = check_factor_args(t, mode, factors, factor_dtype, rank, out, false);
  if (rc) return rc;
  if (t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "in-memory MTTKRP needs a tensor placed on the device");
  return launch_mttkrp(t, t->d_keys, t->d_vals, 0, t->nnz, mode, factors, factor_dtype, rank,
                       1.0f, nullptr, out, (hipStream_t)stream);
}

// Stream the pinned non-zeros once through two reused staging buffers and,
// for every chunk, run the MTTKRP of each selected mode (outs[m] != NULL) while
// the chunk is resident.  Device bytes: factors read + selected outputs +
// tensor tables + two staging buffers <= budget.
// Whether the fused residual walk can serve mode m: register-based resolution,
// one rank slice of 16-lane groups (R <= 64) and 32-bit gather offsets.
static bool fused_mode_ok(const blco_tensor* t, int m, int rank, int fdt) {
  int sw = 0;
  if (resolve(t, m, rank, &sw) != BLCO_RES_REGISTER) {
    clear_error();
    return false;
  }
  const size_t fsz = factor_elem_bytes(fdt);
  if (rank > 64 || (size_t)rank * fsz >= (1ULL << 31)) return false;
  for (int j = 0; j < t->lay.N; ++j)
    if ((size_t)t->lay.dims[j] * rank * fsz > 0xFFFFFFFFull) return false;
  return true;
}

// Partial sums the loss needs per launch of the sampled-loss kernel over n non-zeros.
static int64_t loss_blocks(int64_t n) { return ((n + 63) / 64 + kWaves - 1) / kWaves; }

// The sampled-loss kernel over [lo, lo + n) of the tensor given by keys/vals: the
// residual of each non-zero into resid (may be NULL) and one fp64 partial sum of
// squared residuals per workgroup into partials[0, loss_blocks(n)).
static int launch_loss(const blco_tensor* t, const uint64_t* keys, const float* vals, int64_t lo,
                       int64_t n, const void* const* factors, int fdt, int rank, float* resid,
                       double* partials, hipStream_t s) {
  if (n <= 0) return BLCO_OK;
  KParams p;
  fill_params(t, &p);
  p.keys = keys;
  p.vals = vals;
  p.base = lo;
  p.n = n;
  for (int m = 0; m < t->lay.N; ++m) p.A[m] = factors[m];
  p.out = resid;
  p.partials = partials;
  p.R = rank;
  p.mode = -1;
  // factors below 4 GiB are gathered with 32-bit byte offsets, larger ones
  // with 64-bit addresses
  const size_t fsz = factor_elem_bytes(fdt);
  p.rowbytes = (uint32_t)((size_t)rank * fsz);
  bool big = (size_t)rank * fsz >= (1ULL << 31);
  for (int m = 0; m < t->lay.N; ++m) {
    const size_t bytes = (size_t)t->lay.dims[m] * rank * fsz;
    p.abytes[m] = (uint32_t)std::min<size_t>(bytes, 0xFFFFFFFFull);
    if (bytes > 0xFFFFFFFFull) big = true;
  }
  KernelFn f = select_loss(t->lay.N, rank, fdt, big);
  hipLaunchKernelGGL(f, dim3((unsigned)loss_blocks(n)), dim3(kBlock), 0, s, p);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

// Device array of at least `count` fp64 partial sums held by the tensor.
static int ensure_partials(blco_tensor* t, int64_t count, hipStream_t s) {
  count = std::max<int64_t>(count, 1);
  if (t->partials_cap >= count) return BLCO_OK;
  if (t->d_partials) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipFree(t->d_partials));
    t->d_partials = nullptr;
    t->partials_cap = 0;
  }
  HIPCHK(hipMalloc((void**)&t->d_partials, sizeof(double) * (size_t)count));
  t->partials_cap = count;
  return BLCO_OK;
}

// The CP gradient of blco_cp_grad inside stream_modes: the residual comes from the
// fused walk of mode m0 (or, when no mode allows it, from the sampled-loss kernel)
// and feeds the other modes' MTTKRPs.
struct GradArgs {
  int m0;                   // mode of the fused residual walk, -1: sampled-loss kernel first
  float scale;              // host-side scale of every gradient term (-alpha)
  const double* scale_dev;  // optional device-side scale
  float* resid;             // DEVICE placement: the caller's residual (nnz)
  double* loss;             // device: 1/2 sum of squared residuals
  double* partials;         // DEVICE placement: workspace of partial sums, NULL: the tensor's
};

// Residual and gradients of one range [lo, lo + n) whose keys/vals are given;
// partial sums of squared residuals go to part[0, ...) and their count to *nparts.
static int grad_range(blco_tensor* t, const GradArgs& g, const uint64_t* keys, const float* vals,
                      int64_t lo, int64_t n, const void* const* factors, int fdt, int rank,
                      float* const* outs, float* resid, double* part, int64_t* nparts,
                      hipStream_t s) {
  int rc;
  *nparts = 0;
  if (n <= 0) return BLCO_OK;
  if (g.m0 >= 0) {
    if ((rc = launch_mttkrp(t, keys, vals, lo, n, g.m0, factors, fdt, rank, g.scale, g.scale_dev,
                            outs[g.m0], s, resid)))
      return rc;
    *nparts = (n + kSqPer - 1) / kSqPer;
    hipLaunchKernelGGL(k_sumsq, dim3((unsigned)*nparts), dim3(256), 0, s, (const float*)resid, n,
                       part);
    HIPCHK(hipGetLastError());
  } else {
    if ((rc = launch_loss(t, keys, vals, lo, n, factors, fdt, rank, resid, part, s))) return rc;
    *nparts = loss_blocks(n);
  }
  for (int m = 0; m < t->lay.N; ++m) {
    if (m == g.m0) continue;
    if ((rc = launch_mttkrp(t, keys, resid, lo, n, m, factors, fdt, rank, g.scale, g.scale_dev,
                            outs[m], s)))
      return rc;
  }
  return BLCO_OK;
}

// Partial sums per range of n non-zeros (the larger of the two kernels' counts).
static int64_t grad_parts(int64_t n) {
  return std::max<int64_t>((n + kSqPer - 1) / kSqPer, loss_blocks(n));
}

static int stream_modes(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                        float* const* outs, size_t device_budget_bytes, hipStream_t s,
                        const GradArgs* grad = nullptr) {
  const Layout& L = t->lay;
  bool need[BLCO_MAX_MODES] = {};
  int nsel = 0;
  for (int m = 0; m < L.N; ++m)
    if (outs[m]) {
      ++nsel;
      for (int j = 0; j < L.N; ++j)
        if (j != m || grad) need[j] = true;   // the residual reads every factor
    }
  if (nsel == 0) return set_error(BLCO_EINVAL, "no output given");
  size_t fixed = t->device_bytes;
  for (int m = 0; m < L.N; ++m) {
    if (outs[m]) fixed += (size_t)L.dims[m] * rank * sizeof(float);
    if (need[m]) fixed += (size_t)L.dims[m] * rank * factor_elem_bytes(factor_dtype);
  }
  int rc;
  if (t->placement == BLCO_PLACE_DEVICE && grad) {
    for (int m = 0; m < L.N; ++m)
      if ((rc = fill_zero(outs[m], (int64_t)L.dims[m] * rank, s))) return rc;
    double* part = grad->partials;
    if (!part) {
      if ((rc = ensure_partials(t, grad_parts(t->nnz), s))) return rc;
      part = t->d_partials;
    }
    int64_t np = 0;
    if ((rc = grad_range(t, *grad, t->d_keys, t->d_vals, 0, t->nnz, factors, factor_dtype, rank,
                         outs, grad->resid, part, &np, s)))
      return rc;
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(1024), 0, s, (const double*)part, np,
                       grad->loss);
    HIPCHK(hipGetLastError());
    t->stream_peak_bytes = fixed;
    t->stream_chunks = 0;
    t->st.timed_chunks = 0;
    return BLCO_OK;
  }
  if (t->placement == BLCO_PLACE_DEVICE) {
    if (fixed > device_budget_bytes)
      return set_error(BLCO_ENOMEM, "budget %zu below factors + outputs + tensor = %zu",
                       device_budget_bytes, fixed);
    for (int m = 0; m < L.N; ++m) {
      if (!outs[m]) continue;
      if ((rc = fill_zero(outs[m], (int64_t)L.dims[m] * rank, s))) return rc;
      if ((rc = launch_mttkrp(t, t->d_keys, t->d_vals, 0, t->nnz, m, factors, factor_dtype, rank,
                              1.0f, nullptr, outs[m], s)))
        return rc;
    }
    t->stream_peak_bytes = fixed;
    t->stream_chunks = 0;
    t->st.timed_chunks = 0;
    return BLCO_OK;
  }
  if (t->placement != BLCO_PLACE_PINNED)
    return set_error(BLCO_EINVAL, "streaming needs a tensor in pinned host memory");
  // staging per non-zero: key and value, and the chunk's residual for the gradient
  const size_t per_nnz = sizeof(uint64_t) + sizeof(float) + (grad ? sizeof(float) : 0);
  if (device_budget_bytes < fixed + 2 * 64 * per_nnz)
    return set_error(BLCO_ENOMEM, "budget %zu cannot hold factors + outputs + tables (%zu) and "
                                  "two staging buffers", device_budget_bytes, fixed);
  int64_t cap = (int64_t)((device_budget_bytes - fixed) / 2 / per_nnz);
  int64_t blk_cap = ((t->max_block_nnz + 63) / 64) * 64;
  cap = std::min(cap, blk_cap);
  cap = std::min(cap, ((t->nnz + 63) / 64) * 64);
  cap = (cap / 64) * 64;
  if (cap < 64) cap = 64;
  StreamState& st = t->st;
  if (!st.copy_stream) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    st.copy_stream = cs;
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e1, e2;
      HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
      st.ev_ready[i] = e1;
      st.ev_free[i] = e2;
    }
  }
  if (st.cap_nnz != cap) {
    // buffers of another size: wait until no kernel reads the old ones, then replace them
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipEventSynchronize((hipEvent_t)st.ev_free[i]));
      if (st.d_keys[i]) HIPCHK(hipFree(st.d_keys[i]));
      if (st.d_vals[i]) HIPCHK(hipFree(st.d_vals[i]));
      st.d_keys[i] = nullptr;
      st.d_vals[i] = nullptr;
    }
    st.cap_nnz = 0;
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipMalloc((void**)&st.d_keys[i], sizeof(uint64_t) * (size_t)cap));
      HIPCHK(hipMalloc((void**)&st.d_vals[i], sizeof(float) * (size_t)cap));
    }
    st.cap_nnz = cap;
  }
  if (grad && st.res_cap != cap) {
    for (int i = 0; i < 2; ++i) {
      HIPCHK(hipEventSynchronize((hipEvent_t)st.ev_free[i]));
      if (st.d_res[i]) HIPCHK(hipFree(st.d_res[i]));
      st.d_res[i] = nullptr;
    }
    st.res_cap = 0;
    for (int i = 0; i < 2; ++i) HIPCHK(hipMalloc((void**)&st.d_res[i], sizeof(float) * (size_t)cap));
    st.res_cap = cap;
  }
  for (int m = 0; m < L.N; ++m)
    if (outs[m] && (rc = fill_zero(outs[m], (int64_t)L.dims[m] * rank, s))) return rc;
  const int64_t nchunks = (t->nnz + cap - 1) / cap;
  if (grad && (rc = ensure_partials(t, nchunks * grad_parts(cap), s))) return rc;
  int64_t poff = 0;   // partial sums written so far (CP gradient)
  // the previous call's timing events must have fired before they are reused
  for (size_t i = 0; i < st.ev_t.size(); ++i) HIPCHK(hipEventSynchronize((hipEvent_t)st.ev_t[i]));
  while ((int64_t)st.ev_t.size() < 4 * nchunks) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    st.ev_t.push_back(e);
  }
  st.timed_chunks = 0;
  int64_t chunks = 0;
  for (int64_t lo = 0; lo < t->nnz; lo += cap, ++chunks) {
    const int b = (int)(chunks & 1);
    const int64_t cnt = std::min(cap, t->nnz - lo);
    hipStream_t cs = (hipStream_t)st.copy_stream;
    hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(&st.ev_t[4 * chunks]);
    HIPCHK(hipStreamWaitEvent(cs, (hipEvent_t)st.ev_free[b], 0));
    HIPCHK(hipEventRecord(ev[0], cs));
    HIPCHK(hipMemcpyAsync(st.d_keys[b], t->h_keys + lo, sizeof(uint64_t) * (size_t)cnt,
                          hipMemcpyHostToDevice, cs));
    HIPCHK(hipMemcpyAsync(st.d_vals[b], t->h_vals + lo, sizeof(float) * (size_t)cnt,
                          hipMemcpyHostToDevice, cs));
    HIPCHK(hipEventRecord(ev[1], cs));
    HIPCHK(hipEventRecord((hipEvent_t)st.ev_ready[b], cs));
    HIPCHK(hipStreamWaitEvent(s, (hipEvent_t)st.ev_ready[b], 0));
    HIPCHK(hipEventRecord(ev[2], s));
    if (grad) {
      int64_t np = 0;
      if ((rc = grad_range(t, *grad, st.d_keys[b], st.d_vals[b], lo, cnt, factors, factor_dtype,
                           rank, outs, st.d_res[b], t->d_partials + poff, &np, s)))
        return rc;
      poff += np;
    } else {
      for (int m = 0; m < L.N; ++m) {
        if (!outs[m]) continue;
        if ((rc = launch_mttkrp(t, st.d_keys[b], st.d_vals[b], lo, cnt, m, factors, factor_dtype,
                                rank, 1.0f, nullptr, outs[m], s)))
          return rc;
      }
    }
    HIPCHK(hipEventRecord(ev[3], s));
    HIPCHK(hipEventRecord((hipEvent_t)st.ev_free[b], s));
  }
  if (grad) {
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(1024), 0, s, (const double*)t->d_partials,
                       poff, grad->loss);
    HIPCHK(hipGetLastError());
  }
  st.timed_chunks = chunks;
  t->stream_peak_bytes = fixed + 2 * (size_t)cap * per_nnz;
  t->stream_chunks = chunks;
  return BLCO_OK;
}

extern "C" int blco_mttkrp_stream(blco_tensor* t, int mode, const void* const* factors,
                                  int factor_dtype, int rank, float* out,
                                  size_t device_budget_bytes, void* stream) {
  clear_error();
  int rc = check_factor_args(t, mode, factors, factor_dtype, rank, out, false);
  if (rc) return rc;
  float* outs[BLCO_MAX_MODES] = {};
  outs[mode] = out;
  return stream_modes(t, factors, factor_dtype, rank, outs, device_budget_bytes,
                      (hipStream_t)stream);
}

extern "C" int blco_mttkrp_stream_all(blco_tensor* t, const void* const* factors,
                                      int factor_dtype, int rank, float* const* outs,
                                      size_t device_budget_bytes, void* stream) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (!outs) return set_error(BLCO_EINVAL, "outs is NULL");
  float* o[BLCO_MAX_MODES] = {};
  int first = -1;
  for (int m = 0; m < t->lay.N; ++m) {
    o[m] = outs[m];
    if (o[m] && first < 0) first = m;
  }
  if (first < 0) return set_error(BLCO_EINVAL, "no output given");
  for (int m = 0; m < t->lay.N; ++m) {
    if (!o[m]) continue;
    int rc = check_factor_args(t, m, factors, factor_dtype, rank, o[m], false);
    if (rc) return rc;
    for (int j = 0; j < t->lay.N; ++j) {
      if (j == m || !o[j]) continue;
      const float* a = o[m];
      const float* b = o[j];
      const size_t na = (size_t)t->lay.dims[m] * rank, nb = (size_t)t->lay.dims[j] * rank;
      if (a < b + nb && b < a + na) return set_error(BLCO_EINVAL, "outs[%d] overlaps outs[%d]", m, j);
    }
  }
  return stream_modes(t, factors, factor_dtype, rank, o, device_budget_bytes,
                      (hipStream_t)stream);
}

// ---- workspace of blco_cp_grad_noalloc: the fp64 partial sums of the loss live in
// a static device array instead of memory the tensor allocates.  Each device holds
// its own copy; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is not a device address there).
constexpr int64_t kScratchParts = 1 << 19;   // 4 MiB of fp64 partial sums per device
static __device__ __align__(256) double scratch[kScratchParts];
constexpr int kScratchDevs = 64;

// Device address of `scratch` on the current device, looked up once per device.
static int scratch_ptr(double** out) {
  static std::mutex mu;
  static double* addr[kScratchDevs] = {};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevs)
    return set_error(BLCO_EDEVICE, "device %d outside 0..%d", dev, kScratchDevs - 1);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(BLCO_EDEVICE, "no device address for the workspace on device %d", dev);
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return BLCO_OK;
}

// blco_cp_grad and blco_cp_grad_noalloc; with noalloc the tensor must be on the
// device and the partial sums go to the static workspace.
static int cp_grad_impl(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                        const double* scale, double alpha, float* residual, double* loss,
                        float* const* grads, size_t device_budget_bytes, void* stream,
                        bool noalloc) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (!loss) return set_error(BLCO_EINVAL, "loss is NULL");
  if (!grads) return set_error(BLCO_EINVAL, "grads is NULL");
  if (!factors) return set_error(BLCO_EINVAL, "factors is NULL");
  if (noalloc && t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "the allocation-free CP gradient needs a tensor on the device");
  const int N = t->lay.N;
  float* o[BLCO_MAX_MODES] = {};
  for (int m = 0; m < N; ++m) {
    o[m] = grads[m];
    if (!o[m]) return set_error(BLCO_EINVAL, "grads[%d] is NULL", m);
    if (!factors[m]) return set_error(BLCO_EINVAL, "factors[%d] is NULL", m);
    int rc = check_factor_args(t, m, factors, factor_dtype, rank, o[m], true);
    if (rc) return rc;
  }
  for (int m = 0; m < N; ++m)
    for (int j = 0; j < N; ++j) {
      if (j == m) continue;
      const size_t na = (size_t)t->lay.dims[m] * rank, nb = (size_t)t->lay.dims[j] * rank;
      if (o[m] < o[j] + nb && o[j] < o[m] + na)
        return set_error(BLCO_EINVAL, "grads[%d] overlaps grads[%d]", m, j);
    }
  if (t->placement == BLCO_PLACE_DEVICE) {
    if (!residual && t->nnz > 0) return set_error(BLCO_EINVAL, "residual is NULL");
  } else if (t->placement == BLCO_PLACE_PINNED) {
    if (residual)
      return set_error(BLCO_EINVAL, "residual must be NULL for a tensor in pinned host memory");
  } else {
    return set_error(BLCO_EINVAL, "the CP gradient needs a tensor on the device or in pinned "
                                  "host memory");
  }
  if (noalloc && grad_parts(t->nnz) > kScratchParts)
    return set_error(BLCO_EUNSUPPORTED, "%lld non-zeros need %lld partial sums; the static workspace "
                                  "holds %lld (at most %lld non-zeros are always accepted)",
                     (long long)t->nnz, (long long)grad_parts(t->nnz), (long long)kScratchParts,
                     (long long)kScratchParts * kBlock);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  double* ws = nullptr;
  if (noalloc && (rc = scratch_ptr(&ws))) return rc;
  if (t->nnz == 0) {
    for (int m = 0; m < N; ++m)
      if ((rc = fill_zero(o[m], (int64_t)t->lay.dims[m] * rank, s))) return rc;
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(1024), 0, s, (const double*)nullptr,
                       (int64_t)0, loss);
    HIPCHK(hipGetLastError());
    return BLCO_OK;
  }
  GradArgs g;
  g.m0 = -1;
  for (int m = 0; m < N && g.m0 < 0; ++m)
    if (fused_mode_ok(t, m, rank, factor_dtype)) g.m0 = m;
  g.scale = (float)(-alpha);
  g.scale_dev = scale;
  g.resid = residual;
  g.loss = loss;
  g.partials = ws;
  return stream_modes(t, factors, factor_dtype, rank, o, device_budget_bytes, s, &g);
}

extern "C" int blco_cp_grad(blco_tensor* t, const void* const* factors, int factor_dtype,
                            int rank, const double* scale, double alpha, float* residual,
                            double* loss, float* const* grads, size_t device_budget_bytes,
                            void* stream) {
  return cp_grad_impl(t, factors, factor_dtype, rank, scale, alpha, residual, loss, grads,
                      device_budget_bytes, stream, false);
}

extern "C" int blco_cp_grad_noalloc(blco_tensor* t, const void* const* factors, int factor_dtype,
                                    int rank, const double* scale, double alpha, float* residual,
                                    double* loss, float* const* grads, void* stream) {
  return cp_grad_impl(t, factors, factor_dtype, rank, scale, alpha, residual, loss, grads, 0,
                      stream, true);
}

extern "C" int blco_sampled_loss(blco_tensor* t, const void* const* factors, int factor_dtype,
                                 int rank, float* residual, double* loss, void* stream) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (!loss) return set_error(BLCO_EINVAL, "loss is NULL");
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  if (factor_dtype != BLCO_F32 && factor_dtype != BLCO_BF16)
    return set_error(BLCO_EINVAL, "factor dtype %d", factor_dtype);
  if (!factors) return set_error(BLCO_EINVAL, "factors is NULL");
  for (int m = 0; m < t->lay.N; ++m)
    if (!factors[m]) return set_error(BLCO_EINVAL, "factors[%d] is NULL", m);
  if (t->placement != BLCO_PLACE_DEVICE)
    return set_error(BLCO_EINVAL, "the sampled loss needs a tensor placed on the device");
  hipStream_t s = (hipStream_t)stream;
  if (t->nnz == 0) {
    // no non-zeros: the loss is 0 (the reduction over zero partials writes it),
    // and no factor row is gathered
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(1024), 0, s, (const double*)nullptr,
                       (int64_t)0, loss);
    HIPCHK(hipGetLastError());
    return BLCO_OK;
  }
  const int64_t blocks = loss_blocks(t->nnz);
  int rc;
  if ((rc = ensure_partials(t, blocks, s))) return rc;
  if ((rc = launch_loss(t, t->d_keys, t->d_vals, 0, t->nnz, factors, factor_dtype, rank, residual,
                        t->d_partials, s)))
    return rc;
  hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(1024), 0, s, (const double*)t->d_partials,
                     blocks, loss);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

extern "C" int blco_atomic_probe(float* out, int64_t nrows, int rank, const uint32_t* rows,
                                 int64_t n, void* stream) {
  clear_error();
  if (n < 0 || nrows < 0) return set_error(BLCO_EINVAL, "negative size");
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  if (n == 0) return BLCO_OK;
  if (!out || !rows) return set_error(BLCO_EINVAL, "out or rows is NULL");
  const int64_t blocks = (n * 16 + 255) / 256;
  if (blocks > 0x7FFFFFFF) return set_error(BLCO_EINVAL, "n = %lld too large", (long long)n);
  hipLaunchKernelGGL(k_atomic_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     out, nrows, rows, n, rank);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

extern "C" int blco_gather_probe(const float* table, int64_t nrows, int rank,
                                 const uint32_t* rows, int64_t n, float* sink, void* stream) {
  clear_error();
  if (n < 0 || nrows < 0) return set_error(BLCO_EINVAL, "negative size");
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  if (n == 0) return BLCO_OK;
  if (!table || !rows || !sink) return set_error(BLCO_EINVAL, "table, rows or sink is NULL");
  const int64_t groups = (n + kGatherRows - 1) / kGatherRows;
  const int64_t blocks = (groups * 16 + 255) / 256;
  if (blocks > 0x7FFFFFFF) return set_error(BLCO_EINVAL, "n = %lld too large", (long long)n);
  hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     table, nrows, rows, n, rank, sink);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

extern "C" int blco_scale(float* x, int64_t n, const double* scale, double alpha,
                          void* stream) {
  clear_error();
  if (n < 0) return set_error(BLCO_EINVAL, "n = %lld < 0", (long long)n);
  if (n == 0) return BLCO_OK;
  if (!x) return set_error(BLCO_EINVAL, "x is NULL");
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, x, n,
                     scale, alpha);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

extern "C" int blco_set_resolution(blco_tensor* t, int resolution) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (resolution != BLCO_RES_AUTO && resolution != BLCO_RES_REGISTER &&
      resolution != BLCO_RES_HIERARCHICAL)
    return set_error(BLCO_EINVAL, "resolution %d", resolution);
  t->resolution = resolution;
  return BLCO_OK;
}

extern "C" int blco_resolution(const blco_tensor* t, int mode, int rank, int* chosen) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  if (mode < 0 || mode >= t->lay.N)
    return set_error(BLCO_EINVAL, "mode %d outside 0..%d", mode, t->lay.N - 1);
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  if (!chosen) return set_error(BLCO_EINVAL, "chosen is NULL");
  int sw = 0;
  const int res = resolve(t, mode, rank, &sw);
  if (res < 0) return res;
  *chosen = res;
  return BLCO_OK;
}

extern "C" int blco_frequent_rows(const blco_tensor* t, int mode, int rank, int* rows) {
  clear_error();
  if (!t || !rows) return set_error(BLCO_EINVAL, "tensor or rows is NULL");
  if (mode < 0 || mode >= t->lay.N)
    return set_error(BLCO_EINVAL, "mode %d outside 0..%d", mode, t->lay.N - 1);
  if (rank < 1) return set_error(BLCO_EINVAL, "rank %d < 1", rank);
  *rows = stash_rows(t, mode, rank, select_win(t->lay.N, rank, BLCO_F32, false, true));
  return BLCO_OK;
}

extern "C" int blco_cast_bf16(const float* src, uint16_t* dst, int64_t n, void* stream) {
  clear_error();
  if (n < 0) return set_error(BLCO_EINVAL, "n < 0");
  if (n == 0) return BLCO_OK;
  if (!src || !dst) return set_error(BLCO_EINVAL, "src or dst is NULL");
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, src,
                     dst, n);
  HIPCHK(hipGetLastError());
  return BLCO_OK;
}

extern "C" int blco_info(const blco_tensor* t, blco_info_t* info) {
  clear_error();
  if (!t || !info) return set_error(BLCO_EINVAL, "tensor or info is NULL");
  memset(info, 0, sizeof(*info));
  const Layout& L = t->lay;
  info->nmodes = L.N;
  info->nnz = t->nnz;
  info->total_bits = L.T;
  info->key_bits = L.K;
  info->block_bits = L.S;
  for (int m = 0; m < L.N; ++m) {
    info->bits[m] = L.b[m];
    info->kept[m] = L.w[m];
    info->shift[m] = L.s[m];
    info->high[m] = L.h[m];
    info->dims[m] = L.dims[m];
    info->hot_rows[m] = t->nhot[m];
  }
  for (int k = 0; k < 5; ++k) info->build_stage_ms[k] = t->build_stage_ms[k];
  info->nblocks = (int64_t)t->block_id.size();
  info->nruns = (int64_t)t->run_start.size() - 1;
  info->placement = t->placement;
  info->device_bytes = t->device_bytes;
  info->host_bytes = (t->h_keys ? (size_t)t->nnz * (sizeof(uint64_t) + sizeof(float)) : 0);
  info->stream_peak_bytes = t->stream_peak_bytes;
  info->stream_chunks = t->stream_chunks;
  info->stream_chunk_nnz = t->st.cap_nnz;
  const StreamState& st = t->st;
  if (st.timed_chunks > 0) {
    hipEvent_t* ev = reinterpret_cast<hipEvent_t*>(const_cast<void**>(st.ev_t.data()));
    const int64_t n = st.timed_chunks;
    HIPCHK(hipEventSynchronize(ev[4 * (n - 1) + 3]));
    double copy = 0.0, kern = 0.0;
    for (int64_t c = 0; c < n; ++c) {
      float a = 0.f, b = 0.f;
      HIPCHK(hipEventElapsedTime(&a, ev[4 * c], ev[4 * c + 1]));
      HIPCHK(hipEventElapsedTime(&b, ev[4 * c + 2], ev[4 * c + 3]));
      copy += a;
      kern += b;
    }
    float tot = 0.f;
    HIPCHK(hipEventElapsedTime(&tot, ev[0], ev[4 * (n - 1) + 3]));
    info->stream_copy_ms = copy;
    info->stream_kernel_ms = kern;
    info->stream_total_ms = tot;
  }
  return BLCO_OK;
}

extern "C" int blco_export(const blco_tensor* t, uint64_t* keys, float* values,
                           uint64_t* block_ids, int64_t* block_starts) {
  clear_error();
  if (!t) return set_error(BLCO_EINVAL, "tensor is NULL");
  const size_t n = (size_t)t->nnz;
  if (keys && n) {
    if (t->h_keys) memcpy(keys, t->h_keys, n * sizeof(uint64_t));
    else HIPCHK(hipMemcpy(keys, t->d_keys, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
  }
  if (values && n) {
    if (t->h_vals) memcpy(values, t->h_vals, n * sizeof(float));
    else HIPCHK(hipMemcpy(values, t->d_vals, n * sizeof(float), hipMemcpyDeviceToHost));
  }
  if (block_ids && !t->block_id.empty())
    memcpy(block_ids, t->block_id.data(), t->block_id.size() * sizeof(uint64_t));
  if (block_starts) memcpy(block_starts, t->block_start.data(), t->block_start.size() * sizeof(int64_t));
  return BLCO_OK;
}

extern "C" void blco_free(blco_tensor* t) {
  if (!t) return;
  if (t->placement != BLCO_PLACE_HOST) release_device(t);
  free_host_arrays(t);
  delete t;
}
