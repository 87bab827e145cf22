/*
 * blco.h — C ABI of a sparse MTTKRP library over the Blocked Linearized
 * CoOrdinate (BLCO) format for AMD Instinct MI355X (gfx950).
 *
 * Method: Nguyen et al., "Efficient, Out-of-Memory Sparse MTTKRP on Massively
 * Parallel Architectures", ICS '22 (arXiv 2201.12523).
 *
 * Conventions shared by every call
 *   - Modes are 0-based (the paper counts from 1).  Coordinates are 0-based.
 *   - A tensor has N = nmodes modes, 1 <= N <= BLCO_MAX_MODES, mode lengths
 *     1 <= I_n <= 2^32.
 *   - A factor matrix A^(m) is a dense I_m x R row-major array (row i holds
 *     R contiguous elements) in device memory, fp32 or bf16 (BLCO_F32 /
 *     BLCO_BF16), owned by the caller.  `factors` is a host array of N device
 *     pointers; factors[mode] is not read and may be NULL.
 *   - Outputs are dense I_n x R row-major fp32 in device memory, owned by the
 *     caller, and OVERWRITTEN (Algorithm 1 assigns M).  An output must not
 *     overlap a factor.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued on it and the call returns without waiting; pointers passed in
 *     must stay valid until that work has run.  Every argument is checked
 *     before any device work is enqueued: on an error return nothing has
 *     been written.  Errors raised while the work runs surface at the
 *     caller's next synchronisation.
 *   - Every call returns BLCO_OK (0) or a negative status; blco_last_error()
 *     gives a message for the calling thread's last failure.
 *   - Floating-point outputs of the MTTKRP calls depend on the order in which
 *     atomic additions land, so they are not bitwise reproducible; keys,
 *     blocks and every integer result are.
 *   - Calls on one tensor may run concurrently only when they are in-memory
 *     MTTKRP calls; blco_mttkrp_stream and blco_sampled_loss use buffers held
 *     by the tensor and must not overlap another call on the same tensor.
 */
#ifndef BLCO_H
#define BLCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLCO_MAX_MODES 8

/* status codes */
#define BLCO_OK 0
#define BLCO_EINVAL (-1)       /* bad argument: null pointer, mode or rank out of range, ... */
#define BLCO_ENOMEM (-2)       /* host or device allocation failed, or a budget is too small */
#define BLCO_EDEVICE (-3)      /* a HIP call failed; the message holds hipGetErrorString */
#define BLCO_ERANGE (-4)       /* a coordinate is >= its mode length */
#define BLCO_EUNSUPPORTED (-5) /* N outside 1..8, a mode longer than 2^32, or a block key over 64 bits */

/* factor storage */
#define BLCO_F32 0
#define BLCO_BF16 1

/* conflict resolution of the MTTKRP calls (Sections 5.1-5.3) */
#define BLCO_RES_AUTO 0         /* Section 5.3: HIERARCHICAL when I_mode < compute units, else REGISTER */
#define BLCO_RES_REGISTER 1     /* Section 5.2: segment sums in registers, one atomic per segment */
#define BLCO_RES_HIERARCHICAL 2 /* Section 5.1: segment sums into a per-workgroup LDS stash */

/* where blco_build places the non-zeros */
#define BLCO_PLACE_DEVICE 0 /* device memory: in-memory MTTKRP */
#define BLCO_PLACE_PINNED 1 /* pinned host memory: streamed by blco_mttkrp_stream */
#define BLCO_PLACE_HOST 2   /* pageable host memory only; no GPU call is made (inspection) */

typedef struct blco_tensor blco_tensor;

typedef struct {
  int key_bits;          /* target integer width of a key, 1..64 (default 64), Section 4.2 */
  int64_t max_block_nnz; /* cap on the non-zeros of a block, >= 1 (default 2^27), Section 4.2 */
  int placement;         /* BLCO_PLACE_* (default BLCO_PLACE_DEVICE) */
  int64_t hot_min_count; /* frequent-row threshold (0: default 2048; < 0: none; > 0: this one,
                            and the stash is used whenever rows are found), see blco_build */
} blco_build_opts;

typedef struct {
  int nmodes;
  int64_t nnz;
  int total_bits;            /* T = sum of b_n */
  int key_bits;              /* K = min(T, key_bits option): bits kept in a key */
  int block_bits;            /* T - K: uppermost bits that form the block key */
  int bits[BLCO_MAX_MODES];  /* b_n = ceil(log2 I_n) */
  int kept[BLCO_MAX_MODES];  /* w_n: bits of mode n kept in the key */
  int shift[BLCO_MAX_MODES]; /* s_n: position of mode n's field in the key */
  int high[BLCO_MAX_MODES];  /* h_n: bits of mode n moved into the block key */
  uint64_t dims[BLCO_MAX_MODES];
  int64_t nblocks;           /* blocks after splitting to max_block_nnz */
  int64_t nruns;             /* distinct block keys */
  int placement;
  size_t device_bytes;       /* device memory held by the tensor itself */
  size_t host_bytes;         /* host memory held by the tensor */
  size_t stream_peak_bytes;  /* last blco_mttkrp_stream call: factors + out + staging + tables */
  int64_t stream_chunks;     /* last blco_mttkrp_stream call: chunks transferred */
  int64_t stream_chunk_nnz;  /* last blco_mttkrp_stream call: non-zeros per staging buffer */
  double stream_copy_ms;     /* last streaming call: host-to-device copy time, summed over chunks */
  double stream_kernel_ms;   /* last streaming call: MTTKRP kernel time, summed over chunks */
  double stream_total_ms;    /* last streaming call: first copy start to last kernel end */
  int hot_rows[BLCO_MAX_MODES]; /* frequent rows recorded per mode (see blco_build) */
  double build_stage_ms[5];  /* blco_build_device: stream time of its stages (linearize,
                                sort, re-encode, runs of block keys, frequent rows), host
                                work in between included; 0 for blco_build */
} blco_info_t;

/*
 * Build a BLCO tensor from a COO tensor (Section 4; Figure 6).
 *   nmodes, dims[nmodes]: the shape.  nnz >= 0 non-zeros.
 *   coords[nmodes]: host arrays of nnz 0-based indices; values: host, nnz.
 *   opts: NULL for the defaults.
 * Steps: ALTO linearization of every coordinate (Section 4.1), a stable sort
 * along the encoding line, re-encoding into per-mode bit fields decoded by
 * shift and mask (Figure 6b), blocks on the uppermost T - K bits, split to
 * at most max_block_nnz non-zeros (Section 4.2).  Also records, per mode of
 * at most 2^26 rows, up to 256 frequent rows (estimated from at most 2^22
 * evenly spaced non-zeros; at least hot_min_count non-zeros each, most
 * frequent first): the register-based MTTKRP sums their updates per
 * workgroup in LDS instead of once per window (not a mode-specific copy:
 * 1 KiB per mode).  With the default threshold a mode uses them only when
 * the most frequent row left out of the LDS stash is at most a quarter as
 * frequent as the most frequent row; a threshold given in opts uses them
 * whenever rows are found.  The inputs are copied: the
 * caller may free them on return.  Duplicate coordinates are kept (their
 * terms add up).  On success *out owns every buffer; release it with
 * blco_free.  Errors: EINVAL, ERANGE, EUNSUPPORTED, ENOMEM, EDEVICE.
 * This call is synchronous.
 */
int blco_build(int nmodes, const uint64_t* dims, int64_t nnz, const uint32_t* const* coords,
               const float* values, const blco_build_opts* opts, blco_tensor** out);

/*
 * blco_build on the GPU: coords is a host array of nmodes DEVICE pointers
 * (nnz 0-based indices each), values a DEVICE array of nnz; both stay owned by
 * the caller and may be freed on return.  Linearization, a stable radix sort
 * along the encoding line, re-encoding, run detection and the frequent-row
 * counts run on `stream`; the block list and per-run tables are finished on
 * the host.  The result equals blco_build's for the same input, bit for bit.
 * Placement DEVICE or PINNED (the non-zeros are copied to pinned memory).
 * nnz < 2^31 - 1.  Synchronous.  Errors: as blco_build, EUNSUPPORTED for
 * larger nnz, EINVAL for placement HOST.
 */
int blco_build_device(int nmodes, const uint64_t* dims, int64_t nnz,
                      const uint32_t* const* coords, const float* values,
                      const blco_build_opts* opts, void* stream, blco_tensor** out);

/*
 * Mode-`mode` MTTKRP (Eq. (1); Figure 3; Sections 5.1-5.2) of an in-memory
 * tensor (placement DEVICE):
 *   out[i, r] = sum over non-zeros k with i_mode = i of x_k * prod_{m != mode} A^(m)[i_m, r]
 * factor_dtype: BLCO_F32 or BLCO_BF16 (products and sums are fp32 either way).
 * rank R >= 1.  out: device, I_mode x R fp32, overwritten.
 * Errors: EINVAL (null handle/pointer, mode, rank, dtype, placement).
 */
int blco_mttkrp(blco_tensor* t, int mode, const void* const* factors, int factor_dtype, int rank,
                float* out, void* stream);

/*
 * As blco_mttkrp but accumulating: out += MTTKRP_mode (out is not cleared).
 * For summing the MTTKRPs of several tensors that share factor matrices (for
 * instance one tensor split over several BLCO copies).
 */
int blco_mttkrp_acc(blco_tensor* t, int mode, const void* const* factors, int factor_dtype,
                    int rank, float* out, void* stream);

/*
 * As blco_mttkrp with the tensor's values replaced by `values` (device, nnz
 * fp32, in the tensor's BLCO order, e.g. the residual written by
 * blco_sampled_loss) and the result scaled:
 *   out = alpha * (scale ? *scale : 1) * MTTKRP_mode(values)
 * scale: device pointer to one double, or NULL.  This is the gradient of the
 * sparse CP fit loss when values are the residuals and alpha = -1.
 */
int blco_mttkrp_v(blco_tensor* t, int mode, const float* values, const void* const* factors,
                  int factor_dtype, int rank, const double* scale, double alpha, float* out,
                  void* stream);

/*
 * Out-of-memory MTTKRP (Section 4.2): the non-zeros stay in pinned host
 * memory (placement PINNED) and are streamed through at least two device
 * staging buffers reused in turn; the copy of one chunk overlaps the kernel of
 * the previous one.  device_budget_bytes bounds factors + out + staging +
 * tables; the staging size is what remains, split in two (capped at
 * max_block_nnz non-zeros each).  Result as blco_mttkrp.  A DEVICE tensor is
 * computed in memory (the budget must still cover factors, out and tensor).
 * Errors: as blco_mttkrp, plus ENOMEM when the budget cannot hold two
 * staging buffers of one 64-non-zero tile each.  The staging buffers
 * are allocated on the first call and kept by the tensor.  The copies and
 * kernels of each chunk are bracketed by timing events; blco_info reports
 * their busy times (and waits for the call to finish to do so).
 */
int blco_mttkrp_stream(blco_tensor* t, int mode, const void* const* factors, int factor_dtype,
                       int rank, float* out, size_t device_budget_bytes, void* stream);

/*
 * Out-of-memory MTTKRP of several modes in one pass over the non-zeros: each
 * chunk is copied to the device once and, while resident, the MTTKRP of every
 * mode m with outs[m] != NULL is computed into outs[m] (device, I_m x R fp32,
 * overwritten; outputs must not overlap each other or a factor).  `outs` is a
 * host array of N pointers.  The budget covers the factors the selected modes
 * read, all selected outputs, the tensor's tables and the two staging buffers.
 * With N modes this moves the non-zeros over the host link once instead of N
 * times (the per-mode form is the paper's, Section 4.2).  Errors: as
 * blco_mttkrp_stream, EINVAL when no output is given or outputs overlap.
 */
int blco_mttkrp_stream_all(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                           float* const* outs, size_t device_budget_bytes, void* stream);

/*
 * Sparse CP fit loss at the non-zeros (model of Section 2.2):
 *   xhat_k = sum_r prod_{m} A^(m)[i_m^k, r],  e_k = x_k - xhat_k,
 *   *loss = 1/2 sum_k e_k^2
 * residual: device, nnz fp32, written in the tensor's BLCO order (may be NULL).
 * loss: device pointer to one double.  Products are fp32; the residual norm
 * is accumulated in fp64 in a fixed order (deterministic).  Placement DEVICE.
 * Every factors[m] must be non-NULL.  A tensor without non-zeros gets
 * *loss = 0 and no factor row is read.  Errors: EINVAL (null handle, loss or
 * factor pointer, rank, dtype, placement).
 */
int blco_sampled_loss(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                      float* residual, double* loss, void* stream);

/*
 * Sparse CP fit loss and its gradient with respect to every factor in one call
 * (model of Section 2.2; the gradient of 1/2 sum_k e_k^2 with respect to A^(m)
 * is -MTTKRP_m(E), E the tensor of residuals e_k = x_k - xhat_k at the
 * non-zeros, since d xhat_k / d A^(m)[i, r] = prod_{j != m} A^(j)[i_j^k, r]):
 *   *loss    = 1/2 sum_k e_k^2  (fp64, fixed summation order)
 *   grads[m] = -alpha * (scale ? *scale : 1) * MTTKRP_m(E)  for every mode m
 * grads: host array of N device pointers, I_m x R fp32 each, overwritten, not
 * overlapping.  factors: all N non-NULL.  The residual is formed inside the
 * MTTKRP walk of one mode (the first whose register-based kernel takes R <= 64
 * with 32-bit gather offsets), which also gathers the target row, so no
 * separate pass over the non-zeros computes the model; the other modes' MTTKRPs
 * read that residual.  (When no mode qualifies, the sampled-loss kernel forms
 * the residual first.)
 * DEVICE placement: residual (device, nnz fp32) receives e in BLCO order;
 *   device_budget_bytes is not used.
 * PINNED placement: residual must be NULL; the non-zeros are streamed as in
 *   blco_mttkrp_stream_all, each chunk crossing the host link once for the loss
 *   and all N gradients; the budget covers the tensor's tables, every factor,
 *   every gradient and two staging buffers of 16 bytes per non-zero (key,
 *   value, residual).
 * Products are fp32 (factors fp32 or bf16); the result equals blco_sampled_loss
 * followed by blco_mttkrp_v of its residual in every mode, up to rounding.
 * Uses buffers held by the tensor (no concurrent call on the same tensor).
 * Errors: EINVAL (null pointers, rank, dtype, placement, overlapping grads),
 * ENOMEM (budget), EUNSUPPORTED (a forced hierarchical mode too long).
 */
int blco_cp_grad(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                 const double* scale, double alpha, float* residual, double* loss,
                 float* const* grads, size_t device_budget_bytes, void* stream);

/*
 * blco_cp_grad without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as blco_cp_grad for a tensor with DEVICE
 * placement (there is no budget: nothing is staged).  The loss's fp64 partial
 * sums live in a static device array of 2^19 doubles (4 MiB, held by every GPU
 * the library runs on until the process ends) instead of memory the tensor
 * allocates; the call reserves ceil(nnz / 256) of them (the most either of its
 * loss reductions writes), so a tensor of at most 2^27 non-zeros is accepted and
 * a larger one gets EUNSUPPORTED before any device work.  The array is shared by
 * every call on a GPU and keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap on one GPU, from any stream or thread, race.
 * Errors: those of blco_cp_grad, EINVAL for a tensor not on the device,
 * EUNSUPPORTED (workspace size), EDEVICE (workspace address lookup).
 */
int blco_cp_grad_noalloc(blco_tensor* t, const void* const* factors, int factor_dtype, int rank,
                         const double* scale, double alpha, float* residual, double* loss,
                         float* const* grads, void* stream);

/*
 * x[i] *= alpha * (scale ? *scale : 1) for i < n (x device fp32, scale a device
 * double or NULL): the chain-rule factor of an autograd backward applied to
 * gradients computed ahead by blco_cp_grad.  Errors: EINVAL.
 */
int blco_scale(float* x, int64_t n, const double* scale, double alpha, void* stream);

/*
 * Choose the conflict-resolution mechanism of every later MTTKRP call on t
 * (blco_mttkrp*, blco_mttkrp_stream*, the CP gradient), Sections 5.1-5.3:
 *   BLCO_RES_REGISTER: each window of non-zeros is sorted by target row and
 *     every segment is summed in registers and added to the output with one
 *     atomic per rank (Section 5.2);
 *   BLCO_RES_HIERARCHICAL: each workgroup adds its segment sums into a private
 *     copy of the output rows in LDS and adds that copy to the output once, at
 *     its end (Section 5.1).  The copy holds I_mode rows of a slice of at least 16
 *     ranks in 64 KiB of LDS next to the records of a 1024-non-zero batch: a
 *     mode longer than 895 - 64 (N + 1) rows cannot use it, and its calls then
 *     fail with EUNSUPPORTED;
 *   BLCO_RES_AUTO (the default): the heuristic of Section 5.3, HIERARCHICAL
 *     when the target mode is shorter than the device's compute units (256 on
 *     MI355X), REGISTER otherwise.
 * Results agree to rounding (the order of additions differs).  Errors: EINVAL.
 */
int blco_set_resolution(blco_tensor* t, int resolution);

/* The mechanism (BLCO_RES_REGISTER or BLCO_RES_HIERARCHICAL) a mode-`mode`
   MTTKRP call at rank `rank` on the current device uses, in *chosen.
   Errors: EINVAL, EUNSUPPORTED (HIERARCHICAL forced on a mode too long). */
int blco_resolution(const blco_tensor* t, int mode, int rank, int* chosen);

/*
 * Measurement kernel, not part of the method: for each k < n, adds 1.0f to the
 * `rank` entries of row rows[k] of out (device, nrows x rank fp32), with one
 * device-scope fp32 atomic per entry, issued by groups of 16 lanes exactly as
 * the MTTKRP kernels flush a finished segment.  Timed over distinct random
 * rows it calibrates the memory-side atomic rate that bounds the
 * register-based MTTKRP.  rows: device, n uint32; ids >= nrows are skipped.
 * Errors: EINVAL (negative size, rank < 1, null pointer with n > 0).
 */
int blco_atomic_probe(float* out, int64_t nrows, int rank, const uint32_t* rows, int64_t n,
                      void* stream);

/*
 * Measurement kernel, not part of the method: reads rows rows[0..n) of table
 * (device, nrows x rank fp32) by groups of 16 lanes, six rows per group with all
 * of a group's loads in flight together (lane l reads ranks l, l + 16, ...), as
 * the MTTKRP kernels gather factor rows, and stores one partial sum per group in
 * sink (device, at least ceil(n / 6) floats, overwritten).  Timed over distinct
 * random rows of a table far larger than L2 it calibrates the random-row gather
 * rate that, beside the atomic rate, bounds the register-based MTTKRP.  rows:
 * device, n uint32; ids >= nrows are skipped.
 * Errors: EINVAL (negative size, rank < 1, null pointer with n > 0).
 */
int blco_gather_probe(const float* table, int64_t nrows, int rank, const uint32_t* rows,
                      int64_t n, float* sink, void* stream);

/* Rows of mode `mode` whose segment sums a register-based MTTKRP at rank
   `rank` on the current device adds into its LDS stash of frequent rows (found
   at build time) instead of the output, in *rows (0: none).  For inspection.
   Errors: EINVAL. */
int blco_frequent_rows(const blco_tensor* t, int mode, int rank, int* rows);

/* dst[i] = bf16(src[i]), round to nearest even (NaN stays NaN); device arrays. */
int blco_cast_bf16(const float* src, uint16_t* dst, int64_t n, void* stream);

/*
 * Gram matrix G = A^T A of a factor matrix (the factors of V in Algorithm 1):
 * A device, rows x rank, fp32 or bf16 (dtype); G device, rank x rank fp64,
 * overwritten.  Products are fp32 over 64 rows at a time, sums fp64; the
 * workgroups add their sums with fp64 atomics, so G is not bitwise
 * reproducible.  1 <= rank <= 64.  Errors: EINVAL.
 */
int blco_gram(const void* A, int dtype, int64_t rows, int rank, double* G, void* stream);

typedef struct {
  int max_iters;    /* iteration cap, >= 1 (NULL options: 25) */
  double tol;       /* stop once an iteration raises the fit by less than tol (1e-5); a
                       negative tol only stops on a fit drop larger than |tol| */
  int factor_dtype; /* what the MTTKRP reads: BLCO_F32, or BLCO_BF16 copies refreshed from the
                       fp32 factors after every update (BLCO_F32) */
} blco_cpals_opts;

typedef struct {
  int iters;           /* iterations run */
  int pinv_fallbacks;  /* updates whose V was singular to working precision */
} blco_cpals_report;

/*
 * CP-ALS (Algorithm 1) on an in-memory tensor (placement DEVICE).  For each
 * iteration and each mode n in turn:
 *   V = Hadamard product of A^(m)T A^(m) over m != n (fp64),
 *   M = mode-n MTTKRP (blco_mttkrp, the tensor's conflict resolution),
 *   A^(n) = M V^+ (fp64 sums, stored fp32),
 * then the fit 1 - ||X - [[A^(1..N)]]||_F / ||X||_F from the norm identity
 * ||X||^2 - 2 <X, Xhat> + ||Xhat||^2 (<X, Xhat> from the last mode's M).
 * Iterations stop after max_iters or once the fit rises by less than tol.
 * V^+ is V^-1 by Gauss-Jordan elimination when every pivot exceeds
 * 1e-13 * max diag(V); otherwise a rank-revealing pivoted Cholesky
 * P^T V P = L L^T gives V^+ = P L (L^T L)^-2 L^T P^T (counted in the report).
 * factors: host array of N device pointers to fp32 I_m x R matrices, the
 * initial values, overwritten with the result.  fits: host array of
 * max_iters doubles (may be NULL) receiving the fit after each iteration;
 * report may be NULL.  1 <= rank <= 64.  Device workspace (largest I_m x R
 * fp32, N + 4 R x R fp64, bf16 copies if asked) is allocated and freed by the
 * call.  Synchronous: waits on `stream` once per iteration for the fit.
 * The fit identity loses digits to cancellation once the residual is small:
 * with fp32 MTTKRP outputs it is good to about 1e-4 near a fit of 1.
 * Errors: EINVAL (placement, rank, options, empty tensor), ENOMEM, EDEVICE.
 */
int blco_cp_als(blco_tensor* t, float* const* factors, int rank, const blco_cpals_opts* opts,
                double* fits, blco_cpals_report* report, void* stream);

/* Layout, sizes and last streaming call statistics of a tensor (waits for the
   last streaming call to finish when it has not been measured yet). */
int blco_info(const blco_tensor* t, blco_info_t* info);

/*
 * Copy the BLCO arrays to host memory (any placement; synchronous):
 * keys[nnz], values[nnz], block_ids[nblocks], block_starts[nblocks + 1].
 * Any pointer may be NULL to skip that array.
 */
int blco_export(const blco_tensor* t, uint64_t* keys, float* values, uint64_t* block_ids,
                int64_t* block_starts);

/* Release a tensor (NULL is ignored).  Waits for the tensor's own streams. */
void blco_free(blco_tensor* t);

/* Message of the calling thread's last failed call ("" if none). */
const char* blco_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BLCO_H */
