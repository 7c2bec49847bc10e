/*
 * sidwt.h -- C ABI of libsidwt, multiresolution correlation of complex
 * radar signals in the shift-invariant DWT (SIDWT) domain on AMD MI355X
 * (gfx950).
 *
 * Method: C. Bhattacharya and P.R. Mahapatra, "A Novel Application of
 * Lifting Scheme for Multiresolution Correlation of Complex Radar Signals".
 *
 * What one call computes (notation of the paper, Sec. II and IV):
 *   N = 2^J * ceil(n / 2^J); the reference x (length m <= N) and the
 *   received pulse y (length n) are zero-padded to N and treated as
 *   circular.  For every scale j = 0..J-1 and every lag s = 0..N-1
 *
 *       R_j[s] = sum_k conj(a~_{j+1,k}^{(s)}) c_{j+1,k}
 *              + sum_k conj(b~_{j+1,k}^{(s)}) d_{j+1,k}
 *
 *   (eq. (15), eq. (20)/(20a)): a~, b~ are the level-(j+1) approximation
 *   and detail coefficients of x delayed by s, obtained by lifting with the
 *   analysis matrix P~(z^-1); c, d those of y, obtained by lifting with the
 *   dual analysis matrix P^T(z^-1) (eq. (13)).  By shift-circulance (Sec. II)
 *   a~^{(s)} is a circular shift of one of 2^{j+1} stored phase vectors, so
 *   the plan stores those phases once (Fig. 5 tree) and each call lifts y
 *   (Fig. 7) and correlates.  For float filters R_j equals, up to rounding,
 *   the plain circular correlation of the level-j approximations; plane 0 is
 *   the matched-filter output  R_0[s] = sum_n conj(x[n - s]) y[n].
 *
 * Conventions for every entry point:
 *   - Return value: SIDWT_OK (0) or a negative SIDWT_E_* code.  Argument
 *     errors are detected on the host and returned before anything is
 *     enqueued; nothing is written in that case.
 *   - Device pointers are plain HIP device addresses (for instance a
 *     PyTorch tensor's data_ptr()); the caller owns them.  Host pointers are
 *     read during the call only.
 *   - Work is enqueued asynchronously on a stream and the call returns;
 *     results are ready when the stream is synchronised.  Faults of earlier
 *     device work surface as SIDWT_E_DEVICE.  The entry points ending in
 *     _on take the stream as their last argument (a hipStream_t; NULL = the
 *     null stream); the older plan-stream forms (sidwt_correlate,
 *     sidwt_correlate_many, sidwt_correlate_planes, sidwt_correlate_swapped)
 *     use the stream stored in the plan by sidwt_set_stream.
 *   - Concurrency: the _on entry points read the plan and never modify it,
 *     so any number of them may run at once with one plan on different
 *     streams (from different host threads too).  sidwt_set_stream modifies
 *     the plan, and the plan-stream forms keep the tiled path's buffers in
 *     the plan (see sidwt_correlate): calls of those forms on one plan must
 *     not overlap each other or sidwt_set_stream.
 *
 * Data types:
 *   - Float filters (SIDWT_LEGALL53, SIDWT_CDF97, SIDWT_D4_CAUSAL): the
 *     reference (host) and received pulses (device) are complex64,
 *     interleaved (re, im) float32.  Output: complex64 [J][N], plane-major.
 *   - Integer filter (SIDWT_LEGALL53_INT): reference (host) and received
 *     pulses (device) are int16 interleaved (I, Q).  Output: int64
 *     [J][N][2] (re, im).  Results are exact (no rounding beyond the
 *     integer lifting itself).
 */
#ifndef SIDWT_H
#define SIDWT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sidwt_plan sidwt_plan;
typedef struct sidwt_lifting sidwt_lifting;

/* Lifting factorisations (Sec. III).
 * SIDWT_LEGALL53:     5/3 in dual analysis bases, Sec. III-C Case I.
 * SIDWT_CDF97:        9/7 with the rational Table I constants, Case II.
 * SIDWT_D4_CAUSAL:    causal Daubechies-4, eq. (17); both sides (Sec. III-B).
 * SIDWT_LEGALL53_INT: reversible integer-to-integer 5/3 (Sec. I, V-B cite
 *                     integer lifting; the rounding rule used is
 *                     x-side  o -= (e[k]+e[k+1])>>1, e += (o[k-1]+o[k]+2)>>2;
 *                     y-side  e += (o[k-1]+o[k]+1)>>1, o -= (e[k]+e[k+1]+2)>>2,
 *                     detail scalings 1/2 and 2 dropped as they cancel). */
typedef enum {
  SIDWT_LEGALL53 = 1,
  SIDWT_CDF97 = 2,
  SIDWT_D4_CAUSAL = 3,
  SIDWT_LEGALL53_INT = 4
} sidwt_filter;

enum {
  SIDWT_OK = 0,
  SIDWT_E_INVAL = -1,   /* NULL pointer, n<1, m<1, J<1 or J>16, N/2^J<2,
                           unknown filter, negative count                 */
  SIDWT_E_SIZE = -2,    /* m > N; integer plan support would wrap at this N;
                           integer plan whose sums could reach 2^53; or a
                           size beyond the library's limits               */
  SIDWT_E_NOMEM = -3,   /* device allocation failed                       */
  SIDWT_E_DEVICE = -4,  /* a HIP runtime error (including earlier faults) */
  SIDWT_E_UNSUPPORTED = -5, /* valid request the library does not handle */
  SIDWT_E_SCRATCH = -6  /* request needs more than the library's static
                           scratch (SIDWT_NOALLOC_SCRATCH_BYTES)          */
};

#define SIDWT_MAX_LEVELS 16

/* Create a plan: copies the host reference (m samples, type per filter),
 * builds on the current device the even/odd shift-circulant phase pyramid
 * of the reference, a~_l^{(r)} and b~_l^{(r)} for l = 1..J and
 * r = 0..2^l-1 (Sec. II "even and odd shifts"; Fig. 5), on their linear
 * support.  The plan owns its device memory until sidwt_free; it belongs to
 * the device current at creation, and correlation calls made with another
 * device current return SIDWT_E_INVAL.  The call is synchronous.  *out is
 * set only on success.
 * Integer plans (int16 I/Q reference) are exact for every int16 pulse: the
 * plan is refused with SIDWT_E_SIZE, before any device work, when a bound
 * on the partial sums of some level reaches 2^53, the limit of exact
 * integers in the FP64 accumulation.  The bound takes a full-scale pulse,
 * whose approximation bound doubles per level (the y-side lowpass
 * (1/2, 1, 1/2) has l1 norm 2), and this reference's peak, whose
 * approximation bound grows by 3/2 per level (x-side lowpass l1 norm 3/2);
 * details stay within 2X + 1 of their level's input bound X. */
int sidwt_plan_create(int filter, int J, const void *ref, int64_t m,
                      sidwt_plan **out);

/* Release a plan (waits for the plan's device memory to be idle).  NULL is a
 * no-op. */
void sidwt_free(sidwt_plan *p);

/* Number of output elements (complex values) for a pulse of n samples:
 * J * N with N = 2^J * ceil(n / 2^J); -1 if p is NULL or n < 1. */
int64_t sidwt_out_len(const sidwt_plan *p, int64_t n);

/* Stream for the plan's subsequent calls (a hipStream_t; NULL = null
 * stream). */
int sidwt_set_stream(sidwt_plan *p, void *hip_stream);

/* One pulse: rx (device, n samples) -> out (device, sidwt_out_len
 * elements).  Fused kernel: y-side lifting of all J levels in LDS, each
 * level correlated against the plan's phases as soon as it exists
 * (eq. (20)/(20a)).  A pulse too long for one workgroup's LDS goes through
 * the tiled path instead (levels lifted into an HBM scratch pyramid, then
 * lag tiles on every CU, as in the uneven batch); the plan keeps that
 * path's device buffers for the last (n, count) it saw, so calls on one
 * plan must not overlap.  An integer pulse too long for one workgroup is
 * lifted into a temporary HBM pyramid and correlated in blocks of lag rows
 * on int8 matrix cores (plans up to J = 7; the call synchronises its stream
 * before it returns); deeper integer plans return SIDWT_E_UNSUPPORTED
 * there. */
int sidwt_correlate(const sidwt_plan *p, const void *rx, int64_t n, void *out);

/* sidwt_correlate on `hip_stream`, leaving the plan untouched: safe to call
 * concurrently with one plan from several streams and threads.  A pulse
 * that needs the tiled path gets its own temporary buffers (allocated,
 * used, the stream synchronised, freed) instead of the plan's. */
int sidwt_correlate_on(const sidwt_plan *p, const void *rx, int64_t n, void *out,
                       void *hip_stream);

/* A uniform batch in one launch: `count` pulses of n samples each, pulse i
 * at rx + i * rx_stride samples; its planes at out + i * out_stride
 * elements (elements are complex64 or int64 pairs).  rx_stride >= n and
 * out_stride >= sidwt_out_len(p, n).  count = 0 checks the sizes and
 * launches nothing (rx and out may then be NULL). */
int sidwt_correlate_many(const sidwt_plan *p, const void *rx, int64_t n,
                         int64_t count, int64_t rx_stride, void *out,
                         int64_t out_stride);

/* Scale mask (Sec. V: the coarse scales can be correlated on their own):
 * as sidwt_correlate_many, but only the planes j with bit j of plane_mask
 * set are computed (every level is still lifted); the other planes of out
 * are left untouched.  Bits at or above J are ignored; no plane left ->
 * SIDWT_E_INVAL.  Pulses that need the tiled path (longer than one
 * workgroup's LDS) take only the full mask (else SIDWT_E_UNSUPPORTED). */
int sidwt_correlate_planes(const sidwt_plan *p, const void *rx, int64_t n,
                           int64_t count, int64_t rx_stride, void *out,
                           int64_t out_stride, unsigned plane_mask);

/* sidwt_correlate_planes on `hip_stream` (plane_mask ~0u: every plane, the
 * work of sidwt_correlate_many), leaving the plan untouched as
 * sidwt_correlate_on does (pulses on the tiled path: temporary buffers and
 * a synchronised stream). */
int sidwt_correlate_many_on(const sidwt_plan *p, const void *rx, int64_t n,
                            int64_t count, int64_t rx_stride, void *out,
                            int64_t out_stride, unsigned plane_mask,
                            void *hip_stream);

/* Lifting only (a1 + a2 of the path, for bandwidth measurement and for
 * callers that correlate elsewhere): `count` pulses of n samples, pulse i
 * at rx + i*rx_stride; writes the critical y-side pyramid of each pulse,
 * N elements at pyr + i*N in the order  d_1 | d_2 | ... | d_J | c_J
 * (lengths N/2, N/4, ..., N/2^J, N/2^J).  Element type = output element
 * type of the lifting (complex64 for float filters, int32 pairs for the
 * integer filter).  count = 0 checks the sizes and launches nothing. */
int sidwt_lift_many(int filter, int J, const void *rx, int64_t n,
                    int64_t count, int64_t rx_stride, void *pyr,
                    void *hip_stream);

/* Coarse-to-fine formation (eq. (21), Sec. V): the inverse of the y-side
 * lifting, level by level, from a critical pyramid laid out as
 * sidwt_lift_many writes it (pyr + i*N: d_1 | ... | d_J | c_J, N elements
 * of the lifting's element type) to the approximation c_to of each pulse
 * (out + i*(N >> to), N >> to elements; to = 0 gives the zero-padded pulse
 * back, to < J).  N is a transform length (a multiple of 2^J with
 * N/2^J >= 2); one workgroup per pulse holds 1.5 (N >> (to+1)) elements
 * in LDS, so SIDWT_E_UNSUPPORTED beyond 160 KB.  Float filters reconstruct to
 * FP32 rounding; the integer filter exactly.  count = 0 launches nothing. */
int sidwt_synth_many(int filter, int J, int to, const void *pyr, int64_t N,
                     int64_t count, void *out, void *hip_stream);

/* Roles exchanged (Sec. I: the redundant, all-shift analysis may sit on
 * either signal; eq. (20a)'s approximation form at every scale): each
 * received pulse gets the redundant y-side tree and the plan's reference
 * only its critical x-side approximations.  Plane j, lag s (0 <= j < J,
 * 0 <= s < N): sum_k conj(a_j[k]) * Y_{j,p}[k + s / 2^j] with p = s mod 2^j,
 * a_j the level-j x-side approximation of the reference (a_0 = the
 * reference) and Y_{j,p} the level-j y-side approximation of the pulse
 * advanced by p samples.  A shift of the pulse shifts every plane by
 * exactly as many lags; at lags that are multiples of 2^j plane j equals
 * sidwt_correlate_many's.  Layout and strides as sidwt_correlate_many
 * (complex64 in and out).  `workspace` (device, caller-owned, at least
 * sidwt_swap_workspace_bytes(p, n, count) bytes; may be NULL when J = 1)
 * holds levels 1 .. J-1 of the pulses' trees; the plan's stream orders the
 * launches, and calls that share a workspace must not overlap.  One
 * workgroup per (pulse, plane) holds that plane's phases in LDS (about
 * N + 2^j (len_j + 31) complex elements); when that exceeds 160 KB for some
 * plane, every plane goes in chunks (one workgroup per pulse, plane, phase
 * and group of up to 8192 lags: about 8192 + 2 len_j + 63 elements).
 * SIDWT_E_UNSUPPORTED when even a chunk exceeds 160 KB and for the integer
 * filter; SIDWT_E_INVAL for a short workspace; SIDWT_E_SIZE when the
 * launch grid (count 2^(J-1) tree workgroups, or the chunks) exceeds 2^31
 * or the workspace 2^63 bytes (sidwt_swap_workspace_bytes then returns -1).
 * count = 0 checks the sizes and launches nothing. */
int64_t sidwt_swap_workspace_bytes(const sidwt_plan *p, int64_t n, int64_t count);
int sidwt_correlate_swapped(const sidwt_plan *p, const void *rx, int64_t n,
                            int64_t count, int64_t rx_stride, void *out,
                            int64_t out_stride, void *workspace,
                            int64_t workspace_bytes);
/* The same on `hip_stream`, leaving the plan untouched (calls in flight at
 * once need their own workspaces). */
int sidwt_correlate_swapped_on(const sidwt_plan *p, const void *rx, int64_t n,
                               int64_t count, int64_t rx_stride, void *out,
                               int64_t out_stride, void *workspace,
                               int64_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * sidwt_correlate_swapped_on, with the tree levels kept in a scratch array
 * that the library holds in each GPU's memory from its first use until the
 * process ends (SIDWT_NOALLOC_SCRATCH_BYTES per device, looked up on the
 * first call on each device), instead of a caller workspace.  The call
 * allocates and frees nothing.  The caller passes inputs and outputs as for
 * sidwt_correlate_swapped_on.  Requests whose tree needs more than the
 * scratch holds (sidwt_swap_workspace_bytes(p, n, count) above
 * SIDWT_NOALLOC_SCRATCH_BYTES) return SIDWT_E_SCRATCH before anything is
 * enqueued.  Every call on one GPU uses that GPU's one array: calls that can
 * run at the same time on one GPU (other streams, other threads) race and
 * must be ordered by the caller.  The array needs no clearing: each call
 * writes the tree levels it reads. */
#define SIDWT_NOALLOC_SCRATCH_BYTES (64ll << 20)
int sidwt_correlate_swapped_noalloc(const sidwt_plan *p, const void *rx, int64_t n,
                                    int64_t count, int64_t rx_stride, void *out,
                                    int64_t out_stride, void *hip_stream);

/* Target declaration (Sec. V-A, Fig. 6: targets read off |R| in dB at each
 * scale as peaks above a level).  planes: device complex64, pulse i's plane
 * j at planes + i*pulse_stride + j*N elements (the layout of
 * sidwt_correlate_many).  Lag s of a plane is a peak when its power
 * p[s] = Re^2 + Im^2 exceeds p[s-1], is not below p[s+1] (circular lags;
 * the first sample of a flat top) and is not below rel_power * max(p)
 * (rel_power = 10^(level_dB / 10), e.g. 0.1 for -10 dB); single precision,
 * one rounding per operation.  For item k = i*J + j: found[k] = number of
 * peaks; the first min(found[k], max_peaks) in increasing lag order go to
 * lags[k*max_peaks ...] (int32) with db[...] = 10 log10(p / max p) (float).
 * All arrays are device memory; lags and db may be NULL when max_peaks = 0.
 * SIDWT_E_INVAL for a negative or NaN rel_power or inconsistent sizes;
 * count = 0 launches nothing. */
int sidwt_detect_peaks(const void *planes, int64_t count, int J, int64_t N,
                       int64_t pulse_stride, float rel_power, int max_peaks,
                       int32_t *lags, float *db, int32_t *found,
                       void *hip_stream);

/* Lifting factorization (Sec. III-A, eq. (16): Euclid on the polyphase
 * components of the lowpass, one last step for the highpass) of any
 * perfect-reconstruction analysis pair given by taps (host doubles):
 * lowpass out[k] = sum_t lo[t] u[2k + lo_first + t], highpass likewise.
 * With e[k] = u[2k], o[k] = u[2k+1] the result is a list of steps applied
 * in order, step s: kind 0 (predict) o[k] += sum_t coef[t] e[k + first + t],
 * kind 1 (update) e[k] += sum_t coef[t] o[k + first + t]; then
 * c[k] = ke e[k + se], d[k] = ko o[k + so].  Each division is balanced
 * (the quotient cancels as many low as high terms), so symmetric pairs give
 * symmetric steps.  SIDWT_E_INVAL when the polyphase determinant is not a
 * monomial (no perfect reconstruction) or an argument is out of range (at
 * most 64 taps, first in [-64, 64]); SIDWT_E_UNSUPPORTED beyond 16 steps or
 * 8 taps per step.  Host only; the object is freed with
 * sidwt_lifting_free. */
int sidwt_lifting_factorize(const double *lo, int lo_first, int lo_len,
                            const double *hi, int hi_first, int hi_len,
                            sidwt_lifting **out);
/* Number of steps (SIDWT_E_INVAL for NULL). */
int sidwt_lifting_count(const sidwt_lifting *f);
/* Step i (0 <= i < count): kind, first offset, number of taps; coef (may be
 * NULL) receives the len coefficients (at most 8). */
int sidwt_lifting_step(const sidwt_lifting *f, int i, int *kind, int *first,
                       int *len, double *coef);
/* Final scaling and shifts: c[k] = ke e[k + se], d[k] = ko o[k + so]. */
int sidwt_lifting_scaling(const sidwt_lifting *f, double *ke, int *se,
                          double *ko, int *so);
void sidwt_lifting_free(sidwt_lifting *f);   /* NULL is a no-op */

/* Critical lifting of a batch with a factorized pair (its steps taken at
 * run time, in single precision): as sidwt_lift_many (same pyramid layout
 * d_1 | ... | d_J | c_J, complex64 in and out, I and Q alike), for pairs the
 * compiled filters do not cover.  SIDWT_E_UNSUPPORTED when the steps' reach
 * exceeds 48 lanes per 64-lane window or the pulse exceeds the LDS. */
int sidwt_lift_generic(const sidwt_lifting *f, int J, const void *rx, int64_t n,
                       int64_t count, int64_t rx_stride, void *pyr,
                       void *hip_stream);

/* ---- Uneven batches (one persistent launch) ------------------------------
 * A batch fixes `count` pulses, each with its own plan (float filters; the
 * filter and J may differ per pulse) and length n[i].  Short pulses are
 * processed whole in LDS; long ones are lifted, several levels per pass,
 * into a library-owned HBM scratch pyramid and split into lag tiles of one
 * level.
 * All items are sorted by estimated cost (largest first) and pulled from a
 * device work counter by one persistent kernel.  The launch sequence
 * (counter reset, lifting passes of long pulses, persistent kernels) is
 * captured in a HIP graph on first run and replayed afterwards; a run only
 * uploads the pulse / output pointers.  Plans must outlive the batch.
 * Calls that use one batch object must not overlap (they share its
 * descriptors, scratch and counter); different batch objects are
 * independent. */
typedef struct sidwt_batch sidwt_batch;

/* plans[i], n[i] for i < count (host arrays).  Builds descriptors and
 * allocates device scratch; synchronous.
 * Integer batches: when every plan is the integer filter the batch takes
 * int16 I/Q pulses and int64 (re, im) outputs, exact as sidwt_correlate.
 * Its pulses are grouped by (plan, n); a group of a plan up to J = 7 is one
 * launch of the int8 whole-pulse kernel, or (pulses beyond one workgroup's
 * LDS) one lifting launch per level into the batch's HBM pyramid plus one
 * launch over blocks of lag rows, reading the group's per-pulse pointers
 * (uploaded only when they change); deeper plans run one FP64 whole-pulse
 * launch per pulse.  No graph capture; sidwt_batch_config / _configure
 * change nothing and sidwt_batch_tune only runs the batch once.
 * SIDWT_E_INVAL when integer and float plans are mixed;
 * SIDWT_E_UNSUPPORTED for an integer pulse no path can hold (a plan with
 * J >= 8 whose pulse exceeds one workgroup's LDS). */
int sidwt_batch_create(const sidwt_plan *const *plans, const int64_t *n, int count,
                       sidwt_batch **out);

/* Enqueue one pass on `hip_stream`: rx[i] (device, n[i] complex64 samples,
 * or n[i] int16 (re, im) pairs in an integer batch) -> out[i] (device,
 * J_i x N_i complex64, or int64 (re, im) pairs).  rx and out are host arrays
 * of device pointers, read during the call. */
int sidwt_batch_run(sidwt_batch *b, const void *const *rx, void *const *out, void *hip_stream);

/* Autotuner: times candidate tile windows, then fused/tiled splits, then
 * lifting depths (see sidwt_batch_configure) by running the batch on these
 * buffers (events on `hip_stream`), keeps the fastest.  The outputs hold a
 * valid result afterwards.  Synchronous. */
int sidwt_batch_tune(sidwt_batch *b, const void *const *rx, void *const *out, void *hip_stream);

/* Set the split explicitly: pulses with N <= fused_max_N run whole in LDS
 * (when their layout fits); a tile of a long pulse's level covers as many
 * lag-block rows (a multiple of 64, at least 64) as keep its band window
 * near tile_window elements (64..32768).  Synchronous. */
int sidwt_batch_config(sidwt_batch *b, int64_t fused_max_N, int tile_window);

/* As sidwt_batch_config, plus the scale-fusion depth of the long pulses'
 * lifting: each pass lifts lift_depth consecutive levels (1..8) from one
 * read of its input level (blocks of 4096 input samples with halos that
 * cover every level of the pass; a level of at most 4096 samples is one
 * block), and writes every level's bands to the scratch pyramid.  The
 * default depth is 4.  Synchronous. */
int sidwt_batch_configure(sidwt_batch *b, int64_t fused_max_N, int tile_window, int lift_depth);

/* values[0..nvalues): fused_max_N, tile_window, items, whole-pulse items,
 * tile items, LDS bytes per workgroup, persistent grid size, scratch
 * bytes, tuned (0/1), best tuned time in microseconds, lifting depth,
 * lifting passes (launches). */
int sidwt_batch_info(const sidwt_batch *b, int64_t *values, int nvalues);

/* NULL is a no-op; waits for the device to be idle. */
void sidwt_batch_free(sidwt_batch *b);

/* One-shot form: builds a temporary batch, runs it without graph capture,
 * synchronises `hip_stream` and frees the batch before returning. */
int sidwt_correlate_batch(const sidwt_plan *const *plans,
                          const void *const *rx, const int64_t *n,
                          void *const *out, int count, void *hip_stream);

/* ---- Reference banks (16-bit MFMA with hi+lo correction) -----------------
 * A bank holds `count` references of one float filter, in ascending length
 * m[0] <= m[1] <= ..., each with a phase pyramid of Jmax levels.  For a pulse
 * of n samples the eligible references are those with m <= n (a prefix).
 * One request computes, for every eligible reference e, the same planes as
 * sidwt_correlate with that reference's plan: out = E x J x N complex64
 * (reference-major, then plane, then lag).  The dense step (eq. (20)/(20a)
 * for all references at once, a GEMM whose data operand is shared) runs on
 * v_mfma_f32_32x32x16_{f16,bf16}: every operand x is split into
 * hi = h(x s), lo = h(x s - hi) with power-of-two scales s and a product is
 * accumulated in FP32 as hi*hi + hi*lo + lo*hi.  Relative error against the
 * exact planes: about 1e-6 (FP16) or 1e-5 (BF16) per plane.
 * Calls through one workspace (below) reuse its device descriptors and
 * scratch: issue them on one stream (or synchronise in between). */
typedef struct sidwt_bank sidwt_bank;

enum { SIDWT_BANK_FP32 = 0, SIDWT_BANK_FP16 = 1, SIDWT_BANK_BF16 = 2 };

/* refs[e]: host complex64 arrays of m[e] samples (ascending m).  Builds one
 * plan per reference and, for FP16/BF16, the split weights; synchronous.
 * SIDWT_BANK_FP32 keeps the FP32 path instead: a call runs every (request,
 * eligible reference) pair as one pulse of a one-shot uneven batch (the
 * kernels of sidwt_correlate_batch, FP32 MFMA, same output layout and
 * tolerance as sidwt_correlate); such calls synchronise `hip_stream` before
 * returning, record no workspace timing, and use no workspace scratch.
 * SIDWT_E_UNSUPPORTED for the integer filter; SIDWT_E_INVAL if m is not
 * ascending. */
int sidwt_bank_create(int filter, int Jmax, const void *const *refs, const int64_t *m,
                      int count, int precision, sidwt_bank **out);

/* `count` requests: rx[i] (device, n[i] complex64), J[i] <= Jmax scales,
 * out[i] (device, sidwt_bank_out_len(bank, n[i], J[i]) complex64, laid out
 * [e][j][k] for eligible reference e, scale j, lag k; 16-byte aligned, else
 * SIDWT_E_INVAL; NULL allowed for a request with no eligible reference).
 * All requests go through the lifting passes (four levels per launch) and
 * the GEMM launches (for a call large enough to fill the device, levels 1-3
 * and then the deeper levels on a kernel instance of their own; otherwise
 * one launch) on `hip_stream`; returns once they are queued.  count = 0 is a
 * no-op (nothing launched or timed). */
int sidwt_bank_correlate(sidwt_bank *bank, const void *const *rx, const int64_t *n,
                         const int *J, void *const *out, int count, void *hip_stream);

/* Workspaces: the device buffers of one call in flight (descriptors and the
 * scratch pyramids, grown on demand and kept).  sidwt_bank_correlate uses
 * the bank's own workspace; callers that overlap requests on several
 * streams give each stream its own workspace.  A workspace must not be used
 * by two calls that can run at the same time. */
typedef struct sidwt_bank_ws sidwt_bank_ws;
int sidwt_bank_ws_create(const sidwt_bank *bank, sidwt_bank_ws **out);
void sidwt_bank_ws_free(sidwt_bank_ws *ws);   /* NULL is a no-op; waits for the device */
int sidwt_bank_correlate_ws(sidwt_bank *bank, sidwt_bank_ws *ws, const void *const *rx,
                            const int64_t *n, const int *J, void *const *out, int count,
                            void *hip_stream);

/* Kernel timing of the calls through a workspace (benchmarks): with timing
 * on, every call records HIP events on its stream before the lifting
 * launches, between lifting and the GEMM launches, and after them.
 * sidwt_bank_ws_times waits for the last call and returns both durations
 * in milliseconds; SIDWT_E_INVAL if no call was timed since timing was
 * switched on. */
int sidwt_bank_ws_timing(sidwt_bank_ws *ws, int on);
int sidwt_bank_ws_times(sidwt_bank_ws *ws, float *lift_ms, float *gemm_ms);

/* Device scratch one request needs inside a workspace (bytes; -1 on bad
 * arguments); for SIDWT_BANK_FP32, the most its one-shot batch may hold
 * (one pyramid per eligible reference). */
int64_t sidwt_bank_scratch_bytes(const sidwt_bank *bank, int64_t n, int J);

/* Eligible references for a pulse of n samples (-1 on bad arguments). */
int64_t sidwt_bank_eligible(const sidwt_bank *bank, int64_t n);

/* Output elements for one request: eligible(n) * J * N (-1 on bad arguments). */
int64_t sidwt_bank_out_len(const sidwt_bank *bank, int64_t n, int J);

/* The bank's FP32 plan of reference e (owned by the bank; Jmax levels). */
const sidwt_plan *sidwt_bank_plan(const sidwt_bank *bank, int e);

/* values[0..nvalues): references, Jmax, precision, weight bytes, longest
 * padded lag window. */
int sidwt_bank_info(const sidwt_bank *bank, int64_t *values, int nvalues);

/* NULL is a no-op; waits for the device to be idle. */
void sidwt_bank_free(sidwt_bank *bank);

/* Introspection for tests: copy phase r of band b (0 = approximation,
 * 1 = detail) at level l (1..J) to host memory.  Writes *lo (first index of
 * the stored linear support) and *len; dst must hold *len elements of the
 * plan's coefficient type (complex64, or int32 pairs for the integer
 * filter).  With dst == NULL only lo and len are returned. */
int sidwt_plan_phase(const sidwt_plan *p, int level, int band, int r,
                     int32_t *lo, int32_t *len, void *dst);

/* values[0..nvalues): filter, J, m, bytes of the stored phase pyramid, and
 * for integer plans the int8 matrix-core path's weight digits per phase
 * entry (1..3; 0 when that path does not apply and the FP64 form is used)
 * and the bytes of its digit panels.  Host only. */
int sidwt_plan_info(const sidwt_plan *p, int64_t *values, int nvalues);

/* Short description of an error code (static string). */
const char *sidwt_strerror(int code);

/* Library version string. */
const char *sidwt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SIDWT_H */
