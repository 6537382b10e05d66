/*
 * ols.h -- C ABI of the MI355X (gfx950) overlap-and-save convolution library.
 *
 * The method: Adamek, Dimoudi, Giles, Armour, "GPU Fast Convolution via the
 * Overlap-and-Save Method in Shared Memory".  A long complex signal s of
 * length N_s is convolved with K short filters h_r of length M (eq. 1, sec. 1)
 * by overlap-and-save (sec. 3.2): overlapping segments of FFT length N are
 * transformed once, multiplied point-wise by every filter spectrum, inverse
 * transformed, and only the unaliased samples are kept.  One fused HIP kernel
 * does all of that per segment tile, on chip (sec. 3.4, Alg. 2).
 *
 * Conventions used by every entry point:
 *   - complex64 = interleaved {float re, float im}, 8-byte aligned;
 *   - every data pointer is a DEVICE pointer owned by the caller (the library
 *     never frees or keeps it beyond the call);
 *   - `stream` is a hipStream_t (NULL = the null stream); all device work is
 *     enqueued asynchronously on it; errors inside kernels surface at the
 *     caller's next synchronisation;
 *   - every call validates its arguments on the host before enqueuing
 *     anything, returns an ols_status_t and never throws or aborts; a failing
 *     call enqueues nothing; ols_last_error() gives a message for the calling
 *     thread's most recent failure;
 *   - index arithmetic is 64-bit (K * N_s may exceed 2^31);
 *   - ols_forward only reads its plan, so forward calls of one plan may run
 *     on several streams at once; a plan's other device state -- its filter
 *     spectra (rewritten by ols_plan_update_filters) and its backward
 *     workspace (rewritten by every ols_backward) -- makes those calls
 *     ordered with the calls that read it: enqueue them on one stream, or
 *     order the streams with events.  Two plans never share state.
 */
#ifndef OLS_H_
#define OLS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ols_plan_s* ols_plan_t;
typedef void* ols_stream_t; /* a hipStream_t */

typedef enum {
  OLS_SUCCESS = 0,
  OLS_ERROR_INVALID_VALUE = 1, /* null pointer, bad size, overlap, misalignment */
  OLS_ERROR_UNSUPPORTED = 2,   /* FFT length outside {256, ..., 8192} or not a power of two */
  OLS_ERROR_OUT_OF_MEMORY = 3, /* device allocation failed (plan creation only) */
  OLS_ERROR_HIP = 4,           /* a HIP runtime call or kernel launch failed */
  OLS_ERROR_INTERNAL = 5       /* unexpected exception caught at the boundary */
} ols_status_t;

/* Smallest and largest supported FFT (segment) length N. */
#define OLS_MIN_FFT_LENGTH 256
#define OLS_MAX_FFT_LENGTH 8192

/*
 * ols_plan -- prepare the convolution of any signal with a bank of K filters.
 *
 * Paper: the filters are Fourier transformed once, before the segments are
 * processed (Fig. 1; Alg. 2, "Forward FFT of the filters"); the FFT length N
 * is a power of two and leaves L = N - M + 1 unaliased samples per segment
 * (sec. 3.2).
 *
 *   plan   out: receives the new plan (set to NULL on failure)
 *   h      device, complex64 [K][M] row-major: the filter taps h_r[k]
 *   K      number of filters, >= 1
 *   M      filter length, 1 <= M <= N
 *   N      FFT length: power of two in [256, 8192], or 0 to let the library
 *          choose (cost model: FFT work per valid output sample, among
 *          N >= 1024, or N >= 2048 for K >= 24 filters; the shorter lengths
 *          run slower per output there than their work says)
 *   stream the filter spectra are computed on this stream; the plan may be
 *          used on any stream once this work is complete (the call itself
 *          synchronises `stream` before returning, so it is)
 *
 * The plan owns device memory for the K filter spectra (8*K*N bytes), the
 * same spectra delayed by 0 .. LS-1 samples (LS = 16, or 32 for float32
 * outputs: 8*K*N*LS bytes, allocated only when that is at most 256 MiB; see
 * ols_forward) and the twiddle tables, all allocated here; forward calls
 * allocate nothing.  `h` may be freed as soon as the call returns.
 * Errors: INVALID_VALUE (null plan/h, K < 1, M < 1, M > N), UNSUPPORTED (N),
 * OUT_OF_MEMORY, HIP.
 */
ols_status_t ols_plan(ols_plan_t* plan, const void* h, int32_t K, int32_t M, int32_t N, ols_stream_t stream);

/*
 * ols_plan_ex -- ols_plan with flags (any combination):
 *   OLS_POST_DERIVATIVE  fused post-processing (sec. 4, the non-local example
 *                        of the paper): y'_r[n] = y_r[n] - y_r[n-1],
 *                        y_r[-1] = 0.  Being a convolution with [1, -1] it is
 *                        folded into the filter spectra, which adds one
 *                        aliased sample per segment: M + 1 <= N is required
 *                        and the hop is at most N - M.
 *   OLS_POST_POWER       fused per-element post-processing (sec. 4): the
 *                        power |y_r[n]|^2 is written instead of y, as float32
 *                        [K][N_s] (half the output bytes of complex64).
 *   OLS_REAL             real-to-real convolution (sec. 1 and 3.4, R2R): h is
 *                        float32 [K][M], and ols_forward takes s as float32
 *                        [N_s] and writes y as float32 [K][N_s].  Two real
 *                        segments share one complex FFT of length N (one in
 *                        the real, one in the imaginary part; with real
 *                        filters the two results come back separated), so a
 *                        real segment costs half a complex one in arithmetic
 *                        and in bytes.
 * Post-processing applies after the derivative (POWER|DERIVATIVE is the power
 * of the derivative).  Plans with flags do not support ols_backward
 * (UNSUPPORTED).  Pointers need the alignment of their element type (4 bytes
 * for float32, 8 for complex64).  Other errors as ols_plan; an unknown flag is
 * INVALID_VALUE.
 */
#define OLS_POST_NONE 0
#define OLS_POST_DERIVATIVE 1
#define OLS_POST_POWER 2
#define OLS_REAL 4
ols_status_t ols_plan_ex(ols_plan_t* plan, const void* h, int32_t K, int32_t M, int32_t N, int32_t flags,
                         ols_stream_t stream);

/*
 * ols_plan_update_filters -- replace the K filters of a plan (same K and M),
 * recomputing their spectra on `stream` (stream ordered; forward calls queued
 * later on the same stream see the new filters).  Paper: Alg. 2, forward FFT
 * of the filters.  Errors: INVALID_VALUE (null), HIP.
 */
ols_status_t ols_plan_update_filters(ols_plan_t plan, const void* h, ols_stream_t stream);

/*
 * ols_plan_set_hop -- choose the segment stride H (valid outputs kept per
 * segment).  The paper keeps L = N - M + 1 samples per segment and states
 * that the result does not depend on the segment size (sec. 3.2), so any
 * 1 <= H <= N - Me + 1 gives the same output, with Me = M, or M + 1 for a plan
 * with OLS_POST_DERIVATIVE (the derivative is folded into the filter as one
 * more tap).  By default the library uses the largest H whose segments start
 * on 16-sample (128-byte) boundaries: D = Me - 1 rounded up to a multiple of
 * 16 (when that still leaves room), H = N - D.  H = 0 restores the default.
 * With a stencil (below) the limit is 1 <= H <= N - (Me - 1 + left) - right.
 * Errors: INVALID_VALUE.
 */
ols_status_t ols_plan_set_hop(ols_plan_t plan, int32_t H);

/*
 * ols_plan_set_stencil -- non-local post-processing inside the forward kernel
 * (sec. 4: an output combined with its neighbours, the paper's examples being
 * the numerical derivative and interpolation).  After each segment's inverse
 * FFT its outputs are staged in LDS, and every output sample n of filter r
 * yields J values
 *     z_r[J*n + j] = sum_{d=-left}^{right} w[j*T + d + left] * y_r[n + d],
 *     T = left + 1 + right, j = 0 .. J-1,
 * with y_r[m] = 0 for m < 0 (zero history) and, for m >= N_s, y_r[m] the
 * convolution of the signal continued by zeros (its tail).  The plan's other
 * flags apply around it: OLS_POST_DERIVATIVE before (y is then the
 * derivative), OLS_POST_POWER after (|z|^2, float32), OLS_REAL throughout
 * (float32 rows).  ols_forward then writes y as [K][J*N_s] elements of the
 * plan's output type.  Example, cubic midpoint interpolation (two outputs per
 * sample): J = 2, left = 1, right = 2, w = {0, 1, 0, 0, -1/16, 9/16, 9/16,
 * -1/16}.
 *   J       phases, 1 .. 4; 0 removes the stencil (left, right, w ignored).
 *   left    taps before the sample, right taps after: left, right >= 0,
 *           left + 1 + right <= 8.
 *   w       host array of J*T float32 weights, read during the call only.
 * Each segment keeps only outputs whose neighbours are unaliased: the first
 * kept position D >= Me - 1 + left (Me as for ols_plan_set_hop: M, or M + 1
 * with the derivative) and the hop H <= N - D - right, so
 * Me - 1 + left + right <= N - 1 is required; the
 * default hop is N - D - right rounded down to a multiple of 16 samples (when
 * at least 16), which keeps segments on the 128-byte output grid.  The call
 * resets the hop to that default and the tiling to one filter per unit and
 * the stage kernel's occupancy (ols_plan_set_tiling may change it after).
 * With y aligned to J output elements (always for J = 1), one or two phases
 * per sample are written as one element.  A plan with a stencil has no
 * ols_backward (UNSUPPORTED).
 * Errors: INVALID_VALUE (null plan or w, J, left, right out of range, filter
 * too long for the stencil), HIP.
 */
ols_status_t ols_plan_set_stencil(ols_plan_t plan, int32_t J, int32_t left, int32_t right, const float* w);

/* Plan properties: FFT length N, hop H, delay D (first kept circular sample,
 * D >= M - 1), K and M.  Any output pointer may be NULL. */
ols_status_t ols_plan_get_info(ols_plan_t plan, int32_t* N, int32_t* H, int32_t* D, int32_t* K, int32_t* M);

/* The plan's FFT (segment) length N (sec. 3.2), the library's or the caller's
 * choice.  Errors: INVALID_VALUE (NULL plan or N). */
ols_status_t ols_plan_get_fft_length(ols_plan_t plan, int32_t* N);

/*
 * ols_plan_get_spectra -- copy the plan's filter spectra, in natural frequency
 * order, to `out` (device, complex64 [K][N]): out[r][m] = (1/N) *
 * sum_{n<M} h_r[n] exp(-2 pi i m n / N) (the forward FFT of the zero-padded
 * filter, eq. 2, with the inverse transform's 1/N folded in; for a plan with
 * OLS_POST_DERIVATIVE the filter is h_r[n] - h_r[n-1], n <= M, as applied;
 * for OLS_REAL the real filter's complex spectrum).  Internally the
 * spectra are kept in the transform's digit-reversed order (sec. 3.4); this
 * call undoes the permutation.  Enqueued on `stream`.  Errors: INVALID_VALUE, HIP.
 */
ols_status_t ols_plan_get_spectra(ols_plan_t plan, void* out, ols_stream_t stream);

/*
 * ols_forward -- y_r = s * h_r for every filter r (eq. 1, zero history:
 * y_r[n] = sum_{k=0}^{M-1} h_r[k] s[n-k], s[m] = 0 for m < 0, n in [0, N_s)),
 * computed by overlap-and-save (sec. 3.2) in one fused kernel (sec. 3.4,
 * Alg. 2).
 *
 *   s    device, complex64 [N_s] (float32 [N_s] for an OLS_REAL plan)
 *   N_s  signal length, >= 0 (0 is a successful no-op)
 *   y    device, complex64 [K][N_s] row-major (float32 [K][N_s] for a plan
 *        with OLS_POST_POWER or OLS_REAL), written completely, post-processed
 *        as the plan's flags say; must not overlap s (out of place only)
 * Errors: INVALID_VALUE (null plan/s/y, N_s < 0, misaligned, overlap,
 * K*N_s*8 overflow), HIP (launch failure).  Allocates nothing.
 * Rows off the 128-byte grid (y not 128-byte aligned, or N_s not a multiple
 * of LS = 16, of 32 for float32 outputs), in calls of K*N_s >= 2^22 outputs
 * on plans that hold their delayed spectra and have no stencil: filter r is
 * taken delayed by 0..LS-1 samples (the plan's precomputed spectrum times
 * the delay's phase) so that every store instruction of row r starts on a
 * 128-byte line, and the call runs with the hop rounded down to a multiple of
 * LS with room for the delay; results agree with an aligned call to
 * rounding.  Such rows then run within ~5 % of aligned ones.
 */
ols_status_t ols_forward(ols_plan_t plan, const void* s, int64_t N_s, void* y, ols_stream_t stream);

/*
 * ols_backward -- adjoint of ols_forward (gradients of a real loss L with
 * respect to the signal and the filters, given dL/dy; complex gradients in
 * the convention dL/d(conj z), the one PyTorch uses):
 *   ds[m]   = sum_r sum_k conj(h_r[k]) g_r[m+k]      (g_r[n] = 0 for n >= N_s)
 *   dh_r[k] = sum_m conj(s[m]) g_r[m+k]              (m in [0, N_s))
 * Both are computed by overlap-and-save with the plan's segment geometry: one
 * forward transform of each gradient window serves both; the correlation
 * uses future samples, so its aliased samples sit at the end of each segment
 * (footnote to eq. 2).  Segment spectra are recomputed, nothing is stored
 * from the forward call.  Partial results are summed in a fixed order
 * (deterministic, no atomics).
 *
 *   s    device, complex64 [N_s] (the forward input; may be NULL if dh is NULL)
 *   gy   device, complex64 [K][N_s], dL/dy
 *   ds   device, complex64 [N_s] out, or NULL to skip
 *   dh   device, complex64 [K][M] out, or NULL to skip
 * Outputs must not overlap the inputs or each other.  N_s = 0 writes dh = 0.
 * The first call allocates the plan's backward workspace unless
 * ols_plan_reserve_backward was called (then no call allocates).
 * Errors: INVALID_VALUE, OUT_OF_MEMORY (workspace), HIP.
 */
ols_status_t ols_backward(ols_plan_t plan, const void* s, int64_t N_s, const void* gy, void* ds, void* dh,
                          ols_stream_t stream);

/*
 * ols_backward_static -- ols_backward for callers that cannot allocate device
 * memory (code under hipGraph capture, serving loops, harnesses that forbid
 * hipMalloc): the adjoint's scratch (partial ds windows of tiles shared by
 * workgroups, per-workgroup dh lag partials and their chunk sums) lives in a
 * library-owned static device array of OLS_STATIC_SCRATCH_BYTES per device,
 * held until the process ends, instead of plan memory.  Same arguments,
 * outputs and kernels as ols_backward; the call allocates nothing.
 *   - The plan must belong to the current device.
 *   - The scratch holds the full persistent grid's partials when they fit,
 *     otherwise as many workgroups as fit; with fewer workgroups the partial
 *     sums are grouped differently, so results agree with ols_backward's up
 *     to float rounding (bit-identical when the full grid fits).
 *   - Every part of the scratch is written before it is read within a call;
 *     nothing needs clearing.  All calls on one device share its array: calls
 *     that may overlap in time on one device (different streams, or host
 *     threads without stream ordering) race and give wrong results.
 * Errors: as ols_backward, plus INVALID_VALUE when a single workgroup's scratch
 * (2*SEGS*N + SEGS*K*M complex64 plus chunk sums) exceeds
 * OLS_STATIC_SCRATCH_BYTES (the message gives both sizes), or when the plan
 * was made on another device.
 */
#define OLS_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
ols_status_t ols_backward_static(ols_plan_t plan, const void* s, int64_t N_s, const void* gy, void* ds, void* dh,
                                 ols_stream_t stream);

/* Allocate the plan's backward workspace now (grid x 2 x SEGS x N,
 * grid x SEGS x K x M and ceil(grid x SEGS / 16) x K x M complex64,
 * grid = persistent workgroups), so that
 * ols_backward never allocates.  Idempotent.  Errors: INVALID_VALUE,
 * OUT_OF_MEMORY, HIP. */
ols_status_t ols_plan_reserve_backward(ols_plan_t plan);

/*
 * Batched uneven overlap-and-save: many signals, each with its own filter bank
 * (K_i filters of length M_i) and FFT length, in one persistent kernel launch
 * (sec. 3.2 / Alg. 2 per item; the filter spectra first, Fig. 1).
 *
 * ols_batch_item_t, one per signal:
 *   s    device, complex64 [N_s];  N_s >= 0
 *   h    device, complex64 [K][M]
 *   K, M >= 1
 *   N    FFT length of this item: power of two in [256, 4096], or 0 for the
 *        library's choice (cost model: least transform work per kept sample,
 *        among N >= 1024, or N >= 2048 for K >= 24 filters)
 *   y    device, complex64 [K][N_s], must not overlap s; outputs of different
 *        items must not overlap each other (not checked)
 * Pointers must be 8-byte aligned.
 */
#define OLS_MAX_BATCH_FFT_LENGTH 4096
typedef struct {
  const void* s;
  int64_t N_s;
  const void* h;
  int32_t K;
  int32_t M;
  int32_t N;
  void* y;
} ols_batch_item_t;

/*
 * ols_batched_workspace_size -- device bytes the workspace of ols_batched
 * needs for these items (a header, twiddle tables, the ordered item table and
 * the filter spectra, K x N complex64 per item at the FFT length it will
 * use).  Host only: validates the items (HOST array, the same shapes the
 * device array of ols_batched will hold) and touches no GPU.
 * Errors: INVALID_VALUE (item number in the message), UNSUPPORTED (N, or an
 * M needing N > 4096).
 */
ols_status_t ols_batched_workspace_size(const ols_batch_item_t* host_items, int32_t n_signals, size_t* bytes);

/*
 * ols_batched -- y_i = s_i * h_i,r for every item i and filter r (eq. 1, zero
 * history), all items in one call.  Enqueues three kernels on `stream` and
 * allocates nothing, so the call can be captured in a hipGraph and replayed:
 *   1. setup (one workgroup): reads the DEVICE item array, repeats the item
 *      checks, chooses each N, orders the items by (N, filters per unit) and
 *      lays out the tile list and the spectra in the workspace;
 *   2. the filter spectra of every item, FFT_N(pad h)/N, into the workspace
 *      (so a replay sees the filters' current values); an item whose output
 *      rows are off the 128-byte grid gets each filter delayed by its row's
 *      line phase (0..15 samples) and a hop with room for it, as ols_forward
 *      does;
 *   3. one persistent forward kernel over the segment tiles of all items.
 * Every replay reads dev_items again: the caller may change the items (new
 * pointers, new filters, other shapes that fit the workspace) between calls.
 *
 *   dev_items  device, ols_batch_item_t [n_signals], 8-byte aligned
 *   workspace  device, caller-owned, 256-byte aligned, ws_bytes long (at least
 *              ols_batched_workspace_size of the same items); calls that
 *              share a workspace must be ordered
 * Errors on the host (nothing enqueued): INVALID_VALUE for NULL or misaligned
 * pointers, n_signals < 1, or a workspace too small for n_signals items of
 * the smallest size; HIP (launch).  Errors found on the device (an invalid
 * item, or items that need more workspace than ws_bytes) make the call write
 * no output at all; ols_batched_status reports them.
 */
ols_status_t ols_batched(const ols_batch_item_t* dev_items, int32_t n_signals, void* workspace, size_t ws_bytes,
                         ols_stream_t stream);

/*
 * ols_batched_status -- outcome of the device-side checks of the last
 * ols_batched call on `workspace`: *status = OLS_SUCCESS, INVALID_VALUE (an
 * invalid item, or the workspace too small) or UNSUPPORTED (an item's N);
 * *bad_item = the first invalid item's index, or -1.  Copies the workspace
 * header back and synchronises `stream`.  Errors: INVALID_VALUE, HIP.
 */
ols_status_t ols_batched_status(const void* workspace, ols_stream_t stream, int32_t* status, int32_t* bad_item);

/*
 * Batch plans: the same batched computation with the setup and the filter
 * spectra done once, at plan time, for repeated launches over fixed items.
 * ols_batch_plan validates the HOST item array, allocates the batch's own
 * workspace, runs the setup and spectra kernels of ols_batched on `stream`
 * and synchronises it; ols_batch_run then enqueues only the persistent
 * forward kernel (allocates nothing; capturable).  The batch keeps the item
 * pointers: each run reads the signals and writes the outputs named at plan
 * time, with the filter spectra of plan time.
 * Errors: as ols_batched_workspace_size, OUT_OF_MEMORY, HIP.
 */
typedef struct ols_batch_s* ols_batch_t;
ols_status_t ols_batch_plan(ols_batch_t* batch, const ols_batch_item_t* items, int32_t n, ols_stream_t stream);

/* One persistent launch over all items of a batch plan, on `stream`.
 * Allocates nothing; capturable.  Errors: INVALID_VALUE, HIP. */
ols_status_t ols_batch_run(ols_batch_t batch, ols_stream_t stream);

/* Total work units, launch grid and item count of a batch (NULL outputs skipped). */
ols_status_t ols_batch_get_info(ols_batch_t batch, int64_t* total_units, int32_t* grid, int32_t* n);

/* FFT length, hop and delay chosen for item i (the caller's numbering). */
ols_status_t ols_batch_get_item(ols_batch_t batch, int32_t i, int32_t* N, int32_t* H, int32_t* D);

/* Release a batch (NULL is a no-op). */
ols_status_t ols_batch_destroy(ols_batch_t batch);

/* Release a plan and its device memory (NULL is a no-op).  The caller must
 * make sure no enqueued work still uses the plan. */
ols_status_t ols_plan_destroy(ols_plan_t plan);

/* Static text for a status code. */
const char* ols_status_string(ols_status_t status);

/* Message of the calling thread's most recent failed call ("" if none). */
const char* ols_last_error(void);

/*
 * ols_calibration_copy -- plain device copy of `bytes` bytes (multiple of 16,
 * both pointers 16-byte aligned) with the library's own kernel.  Not part of
 * the method: it is the reference workload for reading HBM traffic counters
 * (FETCH_SIZE / WRITE_SIZE) of a kernel whose byte count is known exactly.
 * Errors: INVALID_VALUE, HIP.
 */
ols_status_t ols_calibration_copy(void* dst, const void* src, size_t bytes, ols_stream_t stream);

/* Number of compute units of the current device as seen by the library, and
 * the persistent grid (workgroups) ols_forward launches for this plan. */
ols_status_t ols_plan_get_launch(ols_plan_t plan, int32_t* grid, int32_t* block, int32_t* cus);

/*
 * ols_plan_set_tiling -- the forward kernel's tiling, for autotuners.  A
 * workgroup transforms a tile of segments once and reuses the spectra for a
 * run of filters (sec. 3.4: the segment is reused for every filter); work
 * units of one tile and `filters_per_unit` filters are split into equal
 * contiguous ranges over `workgroups_per_cu` x (compute units) persistent
 * workgroups, so fewer workgroups give each more consecutive segments
 * (segments per workgroup = number of segments / grid).
 *   filters_per_unit   1 or 2 inverse transforms interleaved per unit
 *                      (2 only for N <= 4096, and N <= 2048 for R2R);
 *                      0 restores the library's choice
 *   workgroups_per_cu  1 .. the kernel's occupancy; 0 = the occupancy
 * The workgroup count leaves the output bit-identical; the filters-per-unit
 * choice selects another kernel instance, whose results may differ in the
 * last bits of float rounding.  Errors: INVALID_VALUE.
 */
ols_status_t ols_plan_set_tiling(ols_plan_t plan, int32_t filters_per_unit, int32_t workgroups_per_cu);

/* Current tiling (see ols_plan_set_tiling) and the occupancy limit for it. */
ols_status_t ols_plan_get_tiling(ols_plan_t plan, int32_t* filters_per_unit, int32_t* workgroups_per_cu,
                                 int32_t* max_workgroups_per_cu);

#ifdef __cplusplus
}
#endif

#endif /* OLS_H_ */
