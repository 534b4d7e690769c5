/*
 * pafc.h -- permutation-avoiding FFT-based circular convolution on AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The operation (Venkovic & Anzt, arXiv 2506.12718, Sec. "1D problem",
 * eq. convolution, and Sec. "Multi-dimensional problem",
 * eq. convolution-multi-dimensional): for complex arrays X, H of shape
 * n_1 x ... x n_d (d = 1, 2, 3), row-major with the last index fastest
 * (definition of vec in Sec. "Multi-dimensional problem"),
 *
 *     Y = DFT^{-1}( DFT(H) o DFT(X) ),   i.e.  Y_j = sum_k X_k H_{(j-k) mod n}
 *
 * with DFT sign w_n = exp(-2 pi i / n).  It is evaluated without any index
 * reversal (eq. 35 and the d-way form of Sec. "Permutation-avoiding
 * multi-dimensional convolution"; mixed radix: Sec. "Mixed-radix
 * framework"):
 *
 *     vec(Y) = (conj A_1 (x) ... (x) conj A_d) [ Hdr o (A_1^T (x) ... (x) A_d^T) vec(X) ]
 *
 * where A_i^T is a decimation-in-frequency transform that leaves its output
 * in digit-reversed order, Hdr = (A_1^T (x) ... (x) A_d^T) vec(H) / N is the
 * filter spectrum held in that same order on the device (kept as A^T h; the
 * 1/N is applied with the product), and conj A_i is a decimation-in-time
 * inverse that takes digit-reversed input and returns natural order.
 * N = n_1 ... n_d.
 *
 * Conventions for every call:
 *   - Complex data are interleaved (re, im): PAFC_C64 = 2 x float (8 bytes
 *     per element, torch.complex64), PAFC_C128 = 2 x double (16 bytes,
 *     torch.complex128).
 *   - Pointers named *_dev are device pointers (hipMalloc or equivalent) on
 *     the device that was current when the plan was created.  The caller
 *     owns them.
 *   - hip_stream is a hipStream_t passed as void*; NULL means the default
 *     stream.  Every call that takes a stream is stream-ordered and
 *     asynchronous: it enqueues work and returns without a host sync.
 *   - No exception crosses the ABI; every call returns a pafc_status.
 *   - A plan owns device memory (twiddles, filter spectrum, scratch) that is
 *     shared by all calls on that plan.  pafc_convolve on a PAFC_PERM_FREE or
 *     PAFC_PERM_FREE_UNFUSED plan only reads plan-owned memory, so such a
 *     plan may run convolutions concurrently on several streams, provided
 *     pafc_set_filter does not overlap them; a PAFC_EXPLICIT_PERM plan
 *     writes its scratch array and must be used on one stream at a time.
 *     Distinct plans are independent.
 */
#ifndef PAFC_H
#define PAFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every enum below ends in a *_MAX_ENUM member: it keeps each non-negative
   int a value of the enum type, so an out-of-range value passed across the
   C ABI is rejected by the library's checks (INVALID_VALUE) instead of being
   undefined in its C++ implementation.  *_MAX_ENUM is never a valid
   argument. */
typedef enum pafc_status {
  PAFC_SUCCESS = 0,
  PAFC_ERROR_INVALID_VALUE = 1,    /* null/misaligned pointer, bad ndim, n_i < 2, bad enum */
  PAFC_ERROR_UNSUPPORTED_SIZE = 2, /* prime factor outside {2,3,5} in a 2-D/3-D shape or with an explicit radix,
                                      a 1-D length above 2^29 with such a factor (Rader's primes: 2^30), or
                                      n_i != r^t for an explicit uniform radix */
  PAFC_ERROR_OUT_OF_MEMORY = 3,    /* device allocation failed */
  PAFC_ERROR_DEVICE = 4,           /* HIP runtime or launch error */
  PAFC_ERROR_FILTER_NOT_SET = 5,   /* pafc_convolve before pafc_set_filter */
  PAFC_STATUS_MAX_ENUM = 0x7FFFFFFF
} pafc_status;

typedef enum pafc_dtype {
  PAFC_C64 = 1,  /* complex float32, interleaved */
  PAFC_C128 = 2, /* complex float64, interleaved */
  PAFC_DTYPE_MAX_ENUM = 0x7FFFFFFF
} pafc_dtype;

typedef enum pafc_variant {
  /* The paper's method: forward DIF left digit-reversed, product with the
     digit-reversed spectrum, DIT inverse to natural order; no index reversal
     is executed.  The product is fused between the last forward and the
     first inverse stage of one axis pass (Alg. alg:permutation-avoiding-
     convolution). */
  PAFC_PERM_FREE = 0,
  /* Comparison: the standard route with explicit index reversals executed as
     device passes (Alg. alg:fft-based-convolution with FFT2 of
     Alg. alg:forward-fft and Alg. alg:backward-fft): forward transforms,
     reversal to natural order fused with the product by the natural-order
     spectrum, reversal back, inverse transforms. */
  PAFC_EXPLICIT_PERM = 1,
  /* Ablation: permutation-free, but every axis transform is its own pass and
     the product is a separate elementwise pass (no fusion). */
  PAFC_PERM_FREE_UNFUSED = 2,
  /* Prime-factor route for a 1-D length n = N_1 N_2 (N_3) with pairwise
     coprime factors (the powers of 2, 3 and 5 in n; at least two of them),
     Sec. "Prime factor framework": the input map Gamma^T (Chinese-remainder
     reindexing) turns the length-n circular convolution into one on the
     N_1 x N_2 (x N_3) grid, which runs permutation-free; Gamma maps the
     result back.  Three index permutations per evaluation counting the
     filter's, which is done once at pafc_set_filter.  Radix: NULL or 0. */
  PAFC_PRIME_FACTOR = 3,
  /* Comparison: the same route with the grid convolution done by the
     explicit-permutation variant (the standard prime-factor FFT
     convolution, six permutations). */
  PAFC_PRIME_FACTOR_EXPLICIT = 4,
  PAFC_VARIANT_MAX_ENUM = 0x7FFFFFFF
} pafc_variant;

typedef enum pafc_filter_domain {
  PAFC_FILTER_SPATIAL = 0,          /* h given in the spatial domain, natural order */
  PAFC_FILTER_SPECTRAL_NATURAL = 1, /* the DFT of h given, natural frequency order */
  PAFC_FILTER_DOMAIN_MAX_ENUM = 0x7FFFFFFF
} pafc_filter_domain;

typedef struct pafc_plan_s* pafc_plan_t;

/*
 * pafc_plan -- build a convolution plan for one grid shape.
 *
 * ndim:   1, 2 or 3.
 * dims:   host array of ndim sizes n_1..n_d (n_d is the fastest axis); each
 *         n_i >= 2 and a product of factors in {2, 3, 5}, except for ndim = 1:
 *         a length n with a prime factor above 5 is planned on an inner
 *         plan of smooth length with the requested variant (PAFC_PERM_FREE,
 *         PAFC_EXPLICIT_PERM or PAFC_PERM_FREE_UNFUSED; radix NULL or 0),
 *         Sec. "Rader's and Bluestein's frameworks":
 *         - a prime n <= 2^30 with n - 1 {2,3,5}-smooth by Rader's method:
 *           the DFT at the nonzero frequencies, reindexed by powers of a
 *           generator g, is a circular convolution of length n - 1.  The
 *           filter's spectrum is kept in generator order, so one evaluation
 *           permutes twice (gather, scatter).  The plan owns an inner plan of
 *           length n - 1, an (n - 1)-element scratch array, the n-element
 *           spectrum, 8n bytes of index tables and 32 KiB of block sums;
 *         - any other such n <= 2^29 by Bluestein's method: the DFT is a
 *           circular convolution of length m, the smallest {2,3,5}-smooth
 *           m >= 2n - 1, between elementwise chirp products.  The plan owns
 *           an inner plan of length m, an m-element scratch array, the
 *           n-element chirp and the n-element natural-order spectrum.
 *         The environment variable PAFC_BLUESTEIN=1, read at planning, sends
 *         Rader's primes to Bluestein's method too.  Either way one
 *         convolution is two inner convolutions (the forward DFT of x, and
 *         the inverse DFT through conjugation on the same inner filter); the
 *         filter's spectrum is taken once, at pafc_set_filter.
 *         pafc_forward, pafc_inverse, pafc_set_symbol and pafc_plan_radices
 *         return INVALID_VALUE for such a plan (its spectrum has no
 *         digit-reversed layout of its own); so they do for a
 *         PAFC_PRIME_FACTOR(_EXPLICIT) plan.
 * radix:  NULL, or host array of ndim entries.  radix[i] = 0 lets the
 *         planner choose the radix sequence of axis i (over {2,3,4,5,8});
 *         radix[i] = r in {2,3,4,5,8} requests the uniform radix-r
 *         factorization of Sec. "General radix Cooley-Tukey framework" and
 *         requires n_i = r^t.  The radix sequence fixes the digit-reversed
 *         layout of the spectrum (the mixed-radix reversal of Sec. "Mixed-
 *         radix framework"), never the result.
 * dtype:  PAFC_C64 or PAFC_C128: the element type of x, y, h and of all
 *         arithmetic.  Twiddles are generated in FP64 on the host; PAFC_C64
 *         plans use their round-to-nearest FP32 values.
 * variant: see pafc_variant.
 * hip_stream: stream on which the twiddle uploads are enqueued.
 *
 * On success *out receives the plan, which owns device memory for the
 * twiddles, the filter spectrum (N elements, or the slots of the middle
 * pass's tiles when its last tile is partial) and one N-element scratch
 * array for PAFC_EXPLICIT_PERM, and for PAFC_PERM_FREE plans whose strided
 * middle pass reads the spectrum tile-major (each tile's values in one
 * contiguous block, written by the filter's last forward pass from that
 * scratch array); it allocates with hipMalloc (PAFC_HTM=0 in the environment
 * at planning keeps the plan layout).  On failure *out is set to NULL and
 * nothing is leaked.
 * Errors: INVALID_VALUE (out == NULL, ndim outside 1..3, dims == NULL,
 * n_i < 2, bad dtype/variant), UNSUPPORTED_SIZE, OUT_OF_MEMORY, DEVICE.
 */
pafc_status pafc_plan(pafc_plan_t* out, int ndim, const int64_t* dims,
                      const int* radix, pafc_dtype dtype, pafc_variant variant,
                      void* hip_stream);

/*
 * pafc_set_filter -- set the convolution kernel h of a plan.
 *
 * h_dev: device array of N elements of the plan dtype in the plan's shape
 *        (row-major).  SPATIAL: h itself.  SPECTRAL_NATURAL: DFT(h) in
 *        natural frequency order.  The library copies what it needs (h is
 *        read only by work enqueued on hip_stream, so the caller may free or
 *        overwrite it once the stream has passed this call).
 * The plan keeps the unscaled spectrum in the digit-reversed order of its
 * forward transform (PAFC_EXPLICIT_PERM plans keep natural order); the single
 * normalisation 1/N of the inverse transform is applied in the product with
 * it, so setting a filter costs exactly one forward transform.  The spatial
 * filter is transformed with the plan's own forward passes
 * (Alg. alg:permutation-avoiding-convolution, first step); a natural-order
 * spectrum is reordered once, here, and never again.  Replaces any previous
 * filter.
 * Errors: INVALID_VALUE (p or h_dev NULL, h_dev not aligned to 8 bytes for
 * C64 / 16 bytes for C128, bad domain), DEVICE.
 */
pafc_status pafc_set_filter(pafc_plan_t p, const void* h_dev,
                            pafc_filter_domain domain, void* hip_stream);

/*
 * pafc_convolve -- y = x * h (circular), stream-ordered on hip_stream.
 *
 * x_dev: device array of N elements (read only, unless y_dev == x_dev).
 * y_dev: device array of N elements; y_dev == x_dev (in place) is allowed;
 *        other overlap is not.
 * Deterministic: the same inputs give the same bits, whatever else runs on
 * the device.  Asynchronous faults surface at the caller's next
 * synchronisation.
 * Errors: INVALID_VALUE (NULL or misaligned pointers), FILTER_NOT_SET,
 * DEVICE (launch error).
 */
pafc_status pafc_convolve(pafc_plan_t p, const void* x_dev, void* y_dev,
                          void* hip_stream);

/*
 * Diagonal operators of the DFT for pafc_set_symbol.  S(k) is evaluated at
 * the signed frequency kt_i = k_i (2 k_i <= n_i) or k_i - n_i of each axis,
 * with w_i = 2 pi kt_i / n_i (unit grid spacing, period n_i):
 *   INV_LAPLACIAN     -1 / sum_i w_i^2, 0 at k = 0: the periodic Poisson
 *                     solve of the spectral Laplacian (mean removed)
 *   INV_LAPLACIAN_FD  -1 / sum_i 4 sin^2(pi k_i / n_i), 0 at k = 0: the
 *                     inverse of the (2d+1)-point finite-difference Laplacian
 *   HEAT              exp(-t sum_i w_i^2), params[0] = t >= 0
 *   DERIVATIVE        i w_a along axis a = params[0] (0 at the Nyquist
 *                     frequency of an even axis): the spectral derivative
 *   GAUSSIAN          the DFT of the unit-sum periodic Gaussian of width
 *                     sigma = params[0] (0.05 <= sigma <= 1e6), whose spatial
 *                     form is h_j = prod_i g_i(j_i) / sum_j g_i(j) with
 *                     g_i(j) = sum_{p in Z} exp(-(j + p n_i)^2 / (2 sigma^2)):
 *                     by Poisson summation its spectrum is the product over
 *                     the axes of theta_i(kt_i) / theta_i(0), theta_i(kt) =
 *                     sum_{m in Z} exp(-2 pi^2 sigma^2 (kt / n_i + m)^2), so
 *                     pafc_convolve computes y = x * h without h ever being
 *                     formed or transformed
 */
typedef enum pafc_symbol {
  PAFC_SYMBOL_INV_LAPLACIAN = 0,
  PAFC_SYMBOL_INV_LAPLACIAN_FD = 1,
  PAFC_SYMBOL_HEAT = 2,
  PAFC_SYMBOL_DERIVATIVE = 3,
  PAFC_SYMBOL_GAUSSIAN = 4,
  PAFC_SYMBOL_MAX_ENUM = 0x7FFFFFFF
} pafc_symbol;

/*
 * pafc_set_symbol -- make the plan's spectrum a diagonal operator given by
 * its symbol, so that pafc_convolve computes y = DFT^{-1}(S o DFT(x)): the
 * unordered transforms with a general diagonal operator between them.  The
 * scheme of Sec. "Permutation-avoiding convolution" only needs that operator
 * to be elementwise in the frequency basis, held in the same digit-reversed
 * order as the data (fast Poisson solvers are among the applications the
 * Introduction names).  No array is passed: the
 * per-axis factors are tabulated on the host (long double, rounded once to
 * FP64, at most sum n_i entries) and combined on the device, where each
 * position of the plan's layout finds its frequency through the inverse
 * digit-reversal map.  Replaces any filter.  Synchronises hip_stream once
 * (the table upload).
 * params / nparams: as the symbol requires (NULL and 0 when none).
 * Errors: INVALID_VALUE (bad kind, parameter count or value: t < 0 or not
 * finite, axis not an integer in [0, ndim), sigma outside [0.05, 1e6]),
 * DEVICE.
 */
pafc_status pafc_set_symbol(pafc_plan_t p, pafc_symbol kind, const double* params,
                            int nparams, void* hip_stream);

/*
 * pafc_convolve_with_filter -- y = x * h with the filter transformed inside
 * the call: the evaluation of Alg. alg:permutation-avoiding-convolution as
 * the paper times it, three transforms per call (forward of h, forward of
 * x, inverse), for callers whose filter changes every call.  Equivalent to
 * pafc_set_filter(p, h_dev, SPATIAL) followed by pafc_convolve, and leaves
 * h as the plan's filter.
 * h_dev: spatial filter, N elements, read only; x_dev, y_dev as for
 * pafc_convolve (h_dev may not overlap y_dev).  Writes the plan's spectrum,
 * so it must not overlap other work on the same plan.
 * Errors: INVALID_VALUE (NULL or misaligned pointers), DEVICE.
 */
pafc_status pafc_convolve_with_filter(pafc_plan_t p, const void* x_dev,
                                      const void* h_dev, void* y_dev,
                                      void* hip_stream);

/*
 * pafc_convolve_with_filter_noalloc -- for callers that cannot allocate
 * device memory at call time (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same y = x * h as
 * pafc_convolve_with_filter (same kernels, same results), but the per-call
 * filter spectrum lives in a fixed array that the library holds on every
 * device it runs on (PAFC_NOALLOC_MAX_BYTES, from module load to process
 * exit), not in the plan's spectrum, which this call leaves unchanged (a
 * filter set with pafc_set_filter stays in effect for pafc_convolve).
 * The call allocates nothing and calls no allocating routine; everything
 * else it needs was prepared when the plan was made.
 * Every call on one device shares that one array, which keeps the last
 * call's spectrum: calls that overlap on one device (other streams, other
 * plans, other threads) race and give wrong results.  Serialise them.
 * The plan's staging array is also written (tile-major plans), so the call
 * must not overlap other work on the same plan either.
 * p: a PAFC_PERM_FREE plan of a {2,3,5}-smooth shape; x_dev, h_dev, y_dev
 * as for pafc_convolve_with_filter.
 * Errors: INVALID_VALUE (NULL or misaligned pointers; a plan of another
 * variant or of a prime-length or prime-factor route), UNSUPPORTED_SIZE (the
 * plan's spectrum, N elements or, for tile-major plans, every slot of the
 * middle pass's tiles, exceeds PAFC_NOALLOC_MAX_BYTES: 2^21 complex128 or
 * 2^22 complex64 elements), DEVICE.
 */
#define PAFC_NOALLOC_MAX_BYTES ((size_t)32 << 20)
pafc_status pafc_convolve_with_filter_noalloc(pafc_plan_t p, const void* x_dev,
                                              const void* h_dev, void* y_dev,
                                              void* hip_stream);

/*
 * pafc_forward -- z = (A_1^T (x) ... (x) A_d^T) x: the forward transform
 * without permutation (Alg. alg:uFFT1D..alg:uFFT3D, uFFT2 branch): the DFT
 * of x in digit-reversed order along every axis, unscaled.  Entry
 * (pos_1(k_1), ..., pos_d(k_d)) of z is DFT(x)[k_1, ..., k_d], where pos_i is
 * the mixed-radix digit reversal of axis i's radix sequence (see
 * pafc_plan_radices).  z_dev == x_dev allowed.  Same conventions and errors
 * as pafc_convolve (no filter needed).
 */
pafc_status pafc_forward(pafc_plan_t p, const void* x_dev, void* z_dev,
                         void* hip_stream);

/*
 * pafc_inverse -- y = (conj A_1 (x) ... (x) conj A_d) z / N: the inverse
 * transform without permutation (Alg. alg:uiFFT1D..alg:uiFFT3D): z in
 * digit-reversed order in, natural order out, scaled once by 1/N.
 * pafc_inverse(pafc_forward(x)) = x.  y_dev == z_dev allowed.
 */
pafc_status pafc_inverse(pafc_plan_t p, const void* z_dev, void* y_dev,
                         void* hip_stream);

/*
 * pafc_destroy -- free everything the plan owns.  NULL is a no-op.  The
 * caller must ensure no work on the plan is still pending (synchronise the
 * stream first).
 * Errors: DEVICE.
 */
pafc_status pafc_destroy(pafc_plan_t p);

/* Static, NUL-terminated description of a status code. */
const char* pafc_status_string(pafc_status s);

/* Device bytes owned by the plan (for HBM-budget admission). */
pafc_status pafc_plan_device_bytes(pafc_plan_t p, size_t* bytes);

/*
 * pafc_plan_radices -- the radix sequence the plan uses on axis `axis`
 * (0-based), listed r_1 first (the innermost stage, Sec. "Mixed-radix
 * framework"), written to rho[0..*len-1]; *len is set to the sequence
 * length.  Host only.  Errors: INVALID_VALUE (NULL pointers, bad axis,
 * capacity < length: *len then holds the length needed).
 */
pafc_status pafc_plan_radices(pafc_plan_t p, int axis, int* rho, int* len);

/*
 * pafc_describe -- plan the given problem on the host only (no device call,
 * no allocation on the device) and write a JSON description of the chosen
 * radix sequences, passes, tiles and algorithmic HBM bytes per convolution
 * into buf (NUL-terminated, truncated to cap bytes).  Arguments as for
 * pafc_plan.  *needed (if not NULL) receives the full length + 1.
 * Errors: as pafc_plan, except OUT_OF_MEMORY and DEVICE.
 */
pafc_status pafc_describe(int ndim, const int64_t* dims, const int* radix,
                          pafc_dtype dtype, pafc_variant variant, char* buf,
                          size_t cap, size_t* needed);

/*
 * pafc_profile_passes -- run pafc_convolve `reps` times on hip_stream with a
 * hipEvent recorded around every kernel the convolution launches (timing-only
 * events, created with hipEventDisableSystemFence so that recording them
 * writes back and invalidates no cache), synchronise,
 * and report the mean duration of each launch position in ms_per_pass[]
 * (capacity *npass on entry; the number of launches per convolution on
 * exit) and the algorithmic HBM bytes of each launch in bytes_per_pass[]
 * (may be NULL), and the time from the first to the last event of every
 * repetition in ms_per_rep[0..reps-1] (may be NULL).  Same buffer rules as
 * pafc_convolve.  Blocks the host.
 * Errors: INVALID_VALUE (capacity too small: *npass then holds the count),
 * FILTER_NOT_SET, DEVICE.
 */
pafc_status pafc_profile_passes(pafc_plan_t p, const void* x_dev, void* y_dev,
                                void* hip_stream, int reps, double* ms_per_pass,
                                int64_t* bytes_per_pass, double* ms_per_rep,
                                int* npass);

/*
 * pafc_profile_launch -- the same measurement with fewer events: run
 * pafc_convolve `reps` times on hip_stream, with timing-only events around
 * launch `launch` only (its position in pafc_profile_passes' order,
 * 0 <= launch < *npass there) and, when ms_per_rep is not NULL, at the start
 * of every repetition and the end of the last.  Where that launch is a
 * pipelined pass kernel of a plain (not prime-length or prime-factor) plan,
 * its two events are bound to the launch itself (hipExtLaunchKernel) and
 * take the dispatch's own start and end timestamps, so that no event packet
 * enters the stream around it; elsewhere they are marker packets.  A plan
 * of a single launch timed with ms_per_rep NULL and reps > 1 takes one pair
 * over the whole sequence (the start of the first launch and the end of the
 * last), and *ms_launch is its span over reps, gaps between launches
 * included.  Otherwise *ms_launch receives the mean duration of that launch;
 * ms_per_rep[0..reps-1] (may be NULL) the time from the start of each
 * repetition to the start of the next (the end, for the last).  Same buffer
 * rules as pafc_convolve.  Blocks the host.
 * Errors: INVALID_VALUE (NULL pointers, reps < 1, launch out of range),
 * FILTER_NOT_SET, DEVICE.
 */
pafc_status pafc_profile_launch(pafc_plan_t p, const void* x_dev, void* y_dev,
                                void* hip_stream, int reps, int launch,
                                double* ms_launch, double* ms_per_rep);

/*
 * pafc_twiddle -- the FP64 twiddle the planner uploads for w_n^e =
 * exp(-2 pi i e / n) (host only): evaluated in long double with exact
 * reduction of 8e/n to an octant, so that +-1, +-i and (+-1 +-i)/sqrt(2) are
 * exact, then rounded once to double.  PAFC_C64 plans use the float rounding
 * of these values.  Errors: INVALID_VALUE (n < 1, NULL outputs).
 */
pafc_status pafc_twiddle(int64_t n, int64_t e, double* re, double* im);

/*
 * pafc_stream_copy -- a reference kernel of known traffic over `bytes`
 * bytes (multiple of 16) on hip_stream, used to calibrate hardware byte
 * counters; not part of the convolution.  kind 0: streaming copy src_dev ->
 * dst_dev with 16 bytes per lane (one read and one write of every byte);
 * kind 1: the same copy with 8 bytes per lane; kind 2: read-only sweep of
 * src_dev (every byte read once), writing one 16-byte partial sum per block
 * of 256 lanes at the start of dst_dev (at most bytes / 256 + 16 bytes).
 * Both arrays hold `bytes` bytes and are 16-byte aligned.  kinds 3 and 4
 * probe the access pattern of a strided middle pass: the arrays are 256 rows
 * of bytes / 4096 16-byte elements, walked in tiles of all rows x 16 columns
 * (256-byte row segments); kind 3 copies src_dev to dst_dev that way, kind 4
 * writes x * h, where src_dev holds x (`bytes`) followed by h (`bytes`, read
 * contiguously in tile order).  bytes must then be a multiple of 65536.
 * Errors: INVALID_VALUE (NULL, misaligned, bytes not a multiple of 16 (of
 * 65536 for kinds 3 and 4), kind not 0..4), DEVICE.
 */
pafc_status pafc_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, int kind,
                             void* hip_stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent 1-D convolutions of uneven sizes.
 *
 * pafc_batch_plan -- count problems; problem i has length sizes[i] (each a
 * {2,3,5}-smooth size >= 2) and uses filter filter_ids[i] in
 * [0, nfilters).  Every problem that uses filter f must have the same
 * length (one filter per size class).  Inputs and outputs are packed: the
 * elements of problem i start at offset sum_{j<i} sizes[j] of one device
 * array.  The batch owns per-size-class plans (radix splits and tiles chosen
 * by the planner, or from the table set by pafc_set_tuning) and a device
 * work list, in one of three forms:
 *   PAFC_BATCH_PERSISTENT: pafc_batch_convolve enqueues ONE launch.  Its
 *     blocks (as many as fit the device at once) claim whole problems from
 *     a device counter, largest first, and each runs every pass of its
 *     problem in order; blocks never wait for one another.  The size-class
 *     plans are made for that one kernel: 256 threads, register groups of
 *     at most 16 points, tiles within one LDS size (80 KB in FP64, 32 KB in
 *     FP32 by default), and without the pafc_set_tuning table.  The
 *     launch leaves its two control words zero, so it can be replayed from a
 *     captured hipGraph; two launches of one batch must not overlap.
 *   PAFC_BATCH_LEVELS: pafc_batch_convolve enqueues, for each pass level in
 *     turn (at most five), one launch per register class and LDS-bound
 *     occupancy present (up to 18 launches for the mixed workload of
 *     powers of 2, 3 and 5), with the size-class plans of pafc_plan.
 *   PAFC_BATCH_CLASSES: as LEVELS, except that each pass of a size class
 *     that its plan runs on the pipelined kernel is one launch of that
 *     kernel over every problem of the class (a device table gives each
 *     problem's offset), and each size class's launches form a chain: the
 *     chains run on 6 streams (PAFC_BATCH_STREAMS), five of them the
 *     batch's own, forked from the caller's stream and joined back into it
 *     by events (capturable).  The packed arrays and the spectra must each
 *     stay within 4 GiB.
 *   PAFC_BATCH_AUTO: the fastest of the three (below).
 * Any form may be captured in a hipGraph.  All arguments are checked before
 * any device call.
 * Errors: INVALID_VALUE (out, sizes or filter_ids NULL, count < 1,
 * nfilters < 1, a length < 2, a filter id out of range, two lengths on one
 * filter, bad dtype or form), UNSUPPORTED_SIZE (a length with a prime factor
 * above 5, one that no plan within the persistent form's limits holds, or
 * the classes form's 4 GiB bound exceeded), OUT_OF_MEMORY, DEVICE.
 */
typedef struct pafc_batch_s* pafc_batch_t;

typedef enum pafc_batch_form {
  PAFC_BATCH_PERSISTENT = 0,
  PAFC_BATCH_LEVELS = 1,
  /* the form measured fastest on MI355X (the mixed workload of 4096
     problems, both element types): classes, which falls back to levels
     where the classes form's 4 GiB bound is exceeded */
  PAFC_BATCH_AUTO = 2,
  PAFC_BATCH_CLASSES = 3,
  PAFC_BATCH_FORM_MAX_ENUM = 0x7FFFFFFF
} pafc_batch_form;

pafc_status pafc_batch_plan(pafc_batch_t* out, int count, const int64_t* sizes,
                            const int* filter_ids, int nfilters,
                            pafc_dtype dtype, pafc_batch_form form,
                            void* hip_stream);

/* Set filter f (length = the size class of f) from a device array. */
pafc_status pafc_batch_set_filter(pafc_batch_t b, int filter_id,
                                  const void* h_dev, pafc_filter_domain domain,
                                  void* hip_stream);

/* y = x * h for every problem; x_dev and y_dev are packed arrays of
   sum(sizes) elements; y_dev == x_dev allowed.  A batch is used on one
   stream at a time (its control words, and in the classes form its own
   streams and events, are shared by its calls).
   Errors: INVALID_VALUE, FILTER_NOT_SET (some filter used but not set), DEVICE. */
pafc_status pafc_batch_convolve(pafc_batch_t b, const void* x_dev, void* y_dev,
                                void* hip_stream);

pafc_status pafc_batch_destroy(pafc_batch_t b);

pafc_status pafc_batch_device_bytes(pafc_batch_t b, size_t* bytes);

/*
 * pafc_batch_profile -- run pafc_batch_convolve `reps` times with a hipEvent
 * around every launch, all on hip_stream (so the classes form's launches do
 * not overlap here), synchronise, and report the mean ms of
 * each launch, its algorithmic HBM bytes (one read and one write of every
 * element of every problem in the launch, plus each filter spectrum once in
 * the launch that multiplies by it), and the ms of every repetition
 * (ms_per_rep may be NULL).  *nlevel: capacity in, count out.
 * Errors: as pafc_batch_convolve; INVALID_VALUE if the capacity is too small
 * (with *nlevel set to the count and nothing launched).
 */
pafc_status pafc_batch_profile(pafc_batch_t b, const void* x_dev, void* y_dev,
                               void* hip_stream, int reps, double* ms_per_level,
                               int64_t* bytes_per_level, double* ms_per_rep,
                               int* nlevel);

/* JSON description of a batch plan (host only). */
pafc_status pafc_batch_describe(pafc_batch_t b, char* buf, size_t cap,
                                size_t* needed);

/*
 * pafc_set_tuning -- install planner overrides for plans created afterwards.
 * text: lines "<c64|c128> <n> <split> <W>",
 * "<c64|c128> <n> <split> <W> <Wo> <g3> <g5>" or the same with <g3i> after
 * <g5> ('#' starts a comment), keyed by element type and axis length n:
 *   split  inner length of a 1-D transform cut into an outer (strided) and an
 *          inner (contiguous) pass; 0 = planner default
 *   W, Wo  tile width of the axis pass (of the inner piece when split) and
 *          of the outer piece; 0 = default
 *   g3, g5 largest number of radix-3 (<= 3) and radix-5 (<= 2) stages fused
 *          into one register group; 0 = default (3 and 2)
 *   g3i    the same as g3 for the inner pieces of an axis cut into pieces
 *          (the piece that carries the fused product); 0 = g3
 * None of these changes the result, only the pass and register schedule.
 * An entry applies to every axis of length n; a plan that its choices make
 * infeasible (more ops in one pass than a pass holds) is made with the
 * planner defaults instead.  NULL clears the table.  Errors: INVALID_VALUE (unparsable text; the
 * previous table stays).
 */
pafc_status pafc_set_tuning(const char* text);

#ifdef __cplusplus
}
#endif

#endif /* PAFC_H */
