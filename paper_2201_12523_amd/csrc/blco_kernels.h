// Device kernels of the BLCO library (gfx950, wave64).  Included by
// blco_device.hip only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace blco {

constexpr int kWaves = 4;             // waves per workgroup
constexpr int kBlock = kWaves * 64;   // threads per workgroup

// Everything a launch over one contiguous range of non-zeros needs.
struct KParams {
  const uint64_t* keys;   // keys[0] is global non-zero `base`
  const float* vals;
  int64_t base;           // global index of keys[0]; a multiple of 64
  int64_t n;              // non-zeros in this launch
  const int64_t* run_start;   // runs of equal block key (global indices)
  const uint32_t* run_base;   // nruns x N: high bits of each mode, in place
  const int32_t* tile_run;    // global tile -> run of its first non-zero
  int multi;                  // more than one run (else every base is 0)
  const void* A[8];           // factor matrices (A[mode] unused by MTTKRP)
  float* out;                 // MTTKRP: I_mode x R; loss: residual (nnz)
  float* resid;               // fused residual walk: residual of each non-zero (n)
  double* partials;           // loss: one fp64 partial sum per workgroup
  int R;
  int mode;
  uint32_t shift[8];
  uint32_t mask[8];
  const uint32_t* hot;        // window kernel: frequent rows of the target mode
  int nhot;                   // window kernel: frequent rows held in the LDS stash
  uint32_t short_rows;        // hierarchical kernel: target mode length
  int short_width;            // hierarchical kernel: ranks per slice
  uint32_t rowbytes;          // bytes of one factor row (R x element size)
  uint32_t abytes[8];         // bytes of each factor matrix (clamped to 2^32 - 1)
  float scale;                // host-side scale of every term
  const double* scale_dev;    // optional device-side scale (one double)
};

}  // namespace blco
