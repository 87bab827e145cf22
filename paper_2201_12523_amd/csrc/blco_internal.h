// Internal definitions shared by the host builder and the device runtime of
// the BLCO library.  Not installed; the public interface is include/blco.h.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/blco.h"

namespace blco {

constexpr int kTile = 64;  // non-zeros per wave tile (one per lane of a wave64)
constexpr int kHotMax = 256;  // frequent rows kept per mode
constexpr int64_t kHotMinCount = 2048;  // default: a frequent row holds at least this many non-zeros

// The bit map of a tensor (Sections 4.1-4.2).
struct Layout {
  int N = 0;
  uint64_t dims[BLCO_MAX_MODES] = {};
  int b[BLCO_MAX_MODES] = {};        // bits per mode
  int pos[BLCO_MAX_MODES][32] = {};  // ALTO position of bit j of mode n
  int T = 0, K = 0, S = 0;           // total bits, kept bits, block-key bits
  int w[BLCO_MAX_MODES] = {};        // kept bits of mode n
  int s[BLCO_MAX_MODES] = {};        // field shift of mode n in the key
  int h[BLCO_MAX_MODES] = {};        // bits of mode n in the block key
};

// Device-side state used only by blco_mttkrp_stream (owned by the tensor).
struct StreamState {
  void* copy_stream = nullptr;     // hipStream_t, library-owned, default priority
  void* ev_ready[2] = {nullptr, nullptr};
  void* ev_free[2] = {nullptr, nullptr};
  uint64_t* d_keys[2] = {nullptr, nullptr};
  float* d_vals[2] = {nullptr, nullptr};
  float* d_res[2] = {nullptr, nullptr};   // residual of each staged chunk (CP gradient)
  int64_t cap_nnz = 0;             // non-zeros per staging buffer
  int64_t res_cap = 0;             // non-zeros per residual buffer
  // timing events of the last call: per chunk copy start/end (copy stream)
  // and kernel start/end (caller's stream)
  std::vector<void*> ev_t;         // 4 per chunk
  int64_t timed_chunks = 0;
};

}  // namespace blco

struct blco_tensor {
  blco::Layout lay;
  int64_t nnz = 0;
  int placement = BLCO_PLACE_DEVICE;
  int64_t max_block_nnz = 0;
  // blocks after splitting (export / info), and runs of equal block key (kernels)
  std::vector<uint64_t> block_id;
  std::vector<int64_t> block_start;  // nblocks + 1
  std::vector<int64_t> run_start;    // nruns + 1
  std::vector<uint32_t> run_base;    // nruns * N: high bits of mode n of the run, already shifted by w_n
  std::vector<int32_t> tile_run;     // per 64-non-zero tile: run holding its first non-zero
  // host arrays (HOST: malloc, PINNED: hipHostMalloc; DEVICE: released after upload)
  uint64_t* h_keys = nullptr;
  float* h_vals = nullptr;
  void (*host_free)(void*) = nullptr;
  // device arrays
  uint64_t* d_keys = nullptr;
  float* d_vals = nullptr;
  int64_t* d_run_start = nullptr;
  uint32_t* d_run_base = nullptr;
  int32_t* d_tile_run = nullptr;
  double* d_partials = nullptr;  // sampled-loss partial sums (one per tile group)
  int64_t partials_cap = 0;
  size_t device_bytes = 0;
  blco::StreamState st;
  size_t stream_peak_bytes = 0;
  int64_t stream_chunks = 0;
  int device = -1;
  int resolution = BLCO_RES_AUTO;   // conflict resolution (blco_set_resolution)
  // frequent rows of each mode (kHotMax per mode, most frequent first, padded
  // with 0xFFFFFFFF): the register-based kernel sums them per workgroup in LDS
  std::vector<uint32_t> hot;         // N * kHotMax
  std::vector<uint64_t> hot_cnt;     // N * (kHotMax + 1): estimated counts of the most frequent rows
  int nhot[BLCO_MAX_MODES] = {};
  bool hot_forced = false;           // an explicit threshold: stash whatever fits
  double build_stage_ms[5] = {};     // blco_build_device stage times (blco_info_t)
  uint32_t* d_hot = nullptr;
};

namespace blco {

int set_error(int code, const char* fmt, ...);
void clear_error();

typedef void* (*HostAlloc)(size_t);
typedef void (*HostFree)(void*);

// Host half of blco_build: validates, linearizes, sorts, re-encodes, blocks.
// Fills everything but the device arrays.  h_keys/h_vals come from `alloc`
// and are released with `release` (NULL: malloc/free).
int host_build(int nmodes, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
               const float* values, int key_bits, int64_t max_block_nnz, HostAlloc alloc,
               HostFree release, blco_tensor* t);

// Frequent rows of every mode (t->hot, t->nhot): rows counted over at most
// 2^22 evenly spaced non-zeros, the kHotMax most frequent whose estimated count
// reaches min_count (< 0: none).  Modes longer than 2^26 get none.
void find_hot_rows(const uint32_t* const* coords, int64_t nnz, int64_t min_count, blco_tensor* t);

void free_host_arrays(blco_tensor* t);

// Bit map of a tensor (Sections 4.1-4.2); EUNSUPPORTED when the block key
// would need more than 64 bits.
int make_layout(int N, const uint64_t* dims, int key_bits, Layout* L);

// Blocks, per-run high bits and tile -> run table from the runs of equal
// block key (run_start without the final nnz; run_key their block keys).
void finish_runs(const Layout& L, int64_t nnz, const std::vector<int64_t>& run_start,
                 const std::vector<uint64_t>& run_key, int64_t max_block_nnz, blco_tensor* t);

// Device sorting and compaction of the GPU builder (blco_sort.hip), ordered on
// stream s (a hipStream_t, void* here so the host builder needs no HIP header).
// The sort waits for s once (to read its digit counts) and returns with its
// passes queued; the selection waits for s to return the count.
//
// Stable ascending radix sort of n < 2^31 keys over bits [0, bits) (bits beyond
// them must be zero), with u32 values when vin != NULL: (kin, vin) -> (kout, vout),
// the input is only read, (ktmp, vtmp) are spares of n entries, ws holds
// sort_workspace_words(n) words.  The u32 form can sort descending (on the
// complemented key, still stable).
size_t sort_workspace_words(int64_t n);
int radix_sort_u64(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                   uint64_t* ktmp, uint32_t* vtmp, int64_t n, int bits, unsigned int* ws,
                   void* s);
int radix_sort_u32(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                   uint32_t* ktmp, uint32_t* vtmp, int64_t n, int bits, bool descending,
                   unsigned int* ws, void* s);

// The same sort with more values moved along: up to two u32 arrays (in32[0], then
// in32[1]) and one u64 array, at most three words per key (two u32 arrays exclude the
// u64 one); each output and spare array holds n entries, unused entries are NULL.
struct SortVals {
  const uint32_t* in32[2];
  uint32_t* out32[2];
  uint32_t* tmp32[2];
  const uint64_t* in64;
  uint64_t* out64;
  uint64_t* tmp64;
};
int radix_sort_u64_vals(const uint64_t* kin, uint64_t* kout, uint64_t* ktmp, const SortVals& v,
                        int64_t n, int bits, unsigned int* ws, void* s);
int radix_sort_u32_vals(const uint32_t* kin, uint32_t* kout, uint32_t* ktmp, const SortVals& v,
                        int64_t n, int bits, unsigned int* ws, void* s);

// The indices i < n with flag[i] != 0, ascending, into out; their number into
// *count (host).  ws holds select_workspace_words(n) words.
size_t select_workspace_words(int64_t n);
int select_flagged(const uint8_t* flag, int64_t n, int64_t* out, int64_t* count,
                   unsigned int* ws, void* s);

}  // namespace blco
