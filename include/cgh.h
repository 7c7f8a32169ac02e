/*
 * cgh.h -- C-ABI of the MI355X (gfx950) point-cloud hologram library.
 *
 * The library computes the amplitude computer-generated hologram of a cloud
 * of N point light sources (Section 2.1, "Direct calculation"): Eq. (2), the
 * Fresnel approximation of the spherical wave of each point, inserted in the
 * interference hologram of Eq. (5) with the reference-wave phase taken as 0,
 * the constant 2 A_r dropped (as Eq. (5) allows) and the per-point constant
 * phase 2 pi z_j / lambda dropped (as the paper's direct-calculation
 * programs do), which leaves
 *
 *     I(x_h, y_h) = sum_j A_j cos( pi / (lambda z_j) ((x_h - x_j)^2 + (y_h - y_j)^2) ).
 *
 * Problem statement (Section 2.1 and the direct-calculation programs of
 * Section 4.1): a W x H hologram of square pixel pitch p, one wavelength
 * lambda, and N points (x_j, y_j, z_j) with amplitudes A_j, given as four
 * float arrays (structure of arrays, as the paper's programs hold them).
 *
 * Units and conventions
 *   - SI metres throughout.
 *   - Pixel (ix, iy), 0 <= ix < W, 0 <= iy < H, sits at
 *       x_h = (ix - (W-1)/2) p,   y_h = (iy - (H-1)/2) p,
 *     i.e. x_j, y_j are measured from the hologram centre.
 *   - z_j > 0 is the distance of point j from the hologram plane.
 *   - Output holograms are float32, row-major, x fastest: out[iy*W + ix]
 *     (the paper's layout), raw sums with no normalisation or quantisation.
 *
 * Threads and streams
 *   - A context is not thread-safe: use one per host thread.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Compute calls only enqueue work; their results are ready when the
 *     stream reaches them.  A single hologram's descriptors travel in the
 *     kernel arguments; a batch's tables are copied asynchronously from
 *     library-owned page-locked memory.  The host blocks only when a
 *     workspace buffer must grow (the first call of a larger evaluation):
 *     the library then waits for the device before replacing the buffer.
 *   - Calls on one context share its workspace.  A call on another stream
 *     than the previous call's first makes its stream wait for the end of
 *     that call (an event), so calls may be issued on any streams.
 *   - cgh_compute, cgh_compute_complex and cgh_kinoform enqueue kernels only
 *     (no copies or memsets), so once their workspace has grown they may be
 *     captured into a caller's HIP graph; the graph then reads the
 *     context's workspace and must not run concurrently with other calls on
 *     the context.
 *   - Same inputs, mode and device give bitwise-identical output on every run
 *     (no floating-point atomics; all reductions run in a fixed order).
 *
 * Errors
 *   - Every function returns a cgh_status.  Argument checks run before any
 *     HIP call, so they behave the same on a host with no GPU.
 *   - On failure, cgh_last_error() returns a thread-local text with detail
 *     (for CGH_EDEVICE: the HIP error string).  No C++ exception crosses the
 *     ABI.
 */
#ifndef CGH_H
#define CGH_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define CGH_API __attribute__((visibility("default")))
#else
#define CGH_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgh_ctx cgh_ctx; /* opaque; owned by the library */

typedef enum {
    CGH_OK = 0,
    CGH_EINVAL = 1,  /* an argument is out of its documented range            */
    CGH_ENOMEM = 2,  /* host or device allocation failed                      */
    CGH_EDEVICE = 3, /* no usable gfx950 device, or a HIP call failed         */
    CGH_ENOTSUP = 4, /* valid request the library does not support            */
    CGH_ESTATE = 5   /* call out of order (e.g. compute before any upload)    */
} cgh_status;

/* How the sum is evaluated.  All modes return the same quantity, I above.
 *
 * CGH_DIRECT_FP32   Per point and pixel, one cosine of the phase.  The large
 *                   phase is range-reduced in FP64 per (pixel column, point)
 *                   and (pixel row, point) -- the square (x_h - x_j)^2 +
 *                   (y_h - y_j)^2 splits into a column part and a row part --
 *                   so the FP32 cosine only sees a phase in [0, 2)
 *                   revolutions.  FP32 accumulation.
 * CGH_SPLIT_BF16    The same split written as a product of complex factors,
 *                   exp(i a) exp(i b) = exp(i (a + b)): a real matrix product
 *                   over the point axis (K = 2N), run on the matrix cores in
 *                   BF16 with FP32 accumulation; each factor is stored as a
 *                   hi + lo pair of BF16 numbers and three products
 *                   (hi*hi + hi*lo + lo*hi) win back the precision.
 * CGH_SPLIT_FP16    As CGH_SPLIT_BF16 with FP16 hi + lo factors.
 * CGH_FP16          One FP16 product (no lo part): a third of the matrix work.
 * CGH_SEPARABLE_FP32  The same factor product with FP32 factors on the
 *                   FP32 matrix instructions (no per-pixel cosine, no
 *                   reduced-precision operand): the accuracy of
 *                   CGH_DIRECT_FP32 at a quarter of the matrix rate of the
 *                   16-bit products.
 * CGH_SPHERICAL_FP32  Not the Fresnel sum: the exact spherical wave of
 *                   Eq. (1), I = sum_j A_j cos(2 pi d_j / lambda) with
 *                   d_j = sqrt((x_h - x_j)^2 + (y_h - y_j)^2 + z_j^2) (the
 *                   on-axis term z_j / lambda included).  Not separable, so
 *                   evaluated directly: d_j / lambda is split into the
 *                   Fresnel phase plus z_j / lambda (reduced per line in
 *                   FP64) and the remainder -(d_j - z_j)^2 / (2 z_j lambda),
 *                   computed per point and pixel in FP32 without cancellation
 *                   (relative error ~1e-6 of a term that stays below 0.1
 *                   revolution at paraxial geometries).  FP32 accumulation.
 */
typedef enum {
    CGH_DIRECT_FP32 = 0,
    CGH_SPLIT_BF16 = 1,
    CGH_SPLIT_FP16 = 2,
    CGH_FP16 = 3,
    CGH_SEPARABLE_FP32 = 4,
    CGH_SPHERICAL_FP32 = 5
} cgh_mode;

typedef enum { CGH_MEM_HOST = 0, CGH_MEM_DEVICE = 1 } cgh_mem;

/* One hologram of a batch: points [point_offset, point_offset + point_count)
 * of the uploaded cloud, seen at its own wavelength (metres). */
typedef struct {
    int64_t point_offset;
    int64_t point_count;
    double wavelength;
} cgh_frame;

/* Create a context for W x H holograms of pitch `pitch_m` at wavelength
 * `wavelength_m` on HIP device `device` (an index as hipSetDevice takes).
 *   out           receives the context (set to NULL on failure); non-NULL.
 *   width, height in [1, 65536].
 *   pitch_m, wavelength_m  finite and > 0.
 * Errors: CGH_EINVAL for a bad argument; CGH_EDEVICE if the device does not
 * exist or is not gfx950; CGH_ENOMEM.  The caller frees it with cgh_destroy. */
CGH_API cgh_status cgh_create(cgh_ctx **out, int32_t width, int32_t height, double pitch_m,
                      double wavelength_m, int32_t device);

/* Copy N points into library-owned device memory (replacing any previous
 * cloud).  x, y, z, amp: float32 arrays of length n, in host memory
 * (where = CGH_MEM_HOST) or device memory (CGH_MEM_DEVICE).
 *   n >= 0; the four pointers are non-NULL when n > 0.
 *   Host data is checked: every value finite and z > 0, else CGH_EINVAL and
 *   the previous cloud is kept.  Device data is not inspected (a z <= 0
 *   there gives non-finite output).
 * A host upload is complete on return.  A device upload is ordered on
 * `stream`; the caller may reuse its arrays once the stream passes it.
 * n = 0 is valid and makes every later hologram zero. */
CGH_API cgh_status cgh_points_upload(cgh_ctx *c, const float *x, const float *y, const float *z,
                             const float *amp, int64_t n, cgh_mem where, void *stream);

/* Compute the hologram of the whole uploaded cloud at the context's
 * wavelength into `out_dev`, a device buffer of height*width floats
 * (row-major, x fastest) owned by the caller.
 * Errors: CGH_EINVAL (NULL out_dev, unknown mode), CGH_ESTATE (no upload
 * yet), CGH_ENOMEM (workspace), CGH_EDEVICE (launch failure). */
CGH_API cgh_status cgh_compute(cgh_ctx *c, cgh_mode mode, float *out_dev, void *stream);

/* Complex object wave O of Eq. (2) (Section 2.1, Fresnel form, without the
 * per-point constant phase, as for cgh_compute) of the whole cloud:
 *   Re O = sum_j A_j cos(pi r_j^2 / (lambda z_j)),
 *   Im O = sum_j A_j sin(pi r_j^2 / (lambda z_j)),
 * into `out_dev`, a caller-owned device buffer of 2*height*width floats:
 * plane 0 (the first height*width floats) = Re O, which equals cgh_compute's
 * output up to rounding, plane 1 = Im O; each plane row-major, x fastest.
 * Modes: all of cgh_mode; the direct mode evaluates a sine beside each
 * cosine, the matrix-core modes multiply a stacked [real; imaginary] row
 * factor (2*height rows) by the same column factor.
 * Errors as cgh_compute. */
CGH_API cgh_status cgh_compute_complex(cgh_ctx *c, cgh_mode mode, float *out_dev, void *stream);

/* Phase-only hologram (kinoform) of Eq. (3): for every pixel the argument
 * theta = atan2(Im O, Re O) of the object wave above, moved to [0, 2 pi) by
 * adding 2 pi when negative, quantised to floor(theta * 255 / (2 pi)) in
 * FP32 (codes 0 .. 254; 255 only when rounding carries theta up to 2 pi).
 * `out_dev`: caller-owned device buffer of height*width bytes, row-major.
 * The complex field is kept in a library-owned workspace (8 bytes per
 * pixel).  Errors as cgh_compute. */
CGH_API cgh_status cgh_kinoform(cgh_ctx *c, cgh_mode mode, uint8_t *out_dev, void *stream);

/* Compute n_frames holograms in one go: frame f covers the points and the
 * wavelength of frames[f] (a host array) and lands in
 * out_dev[f*height*width ...] (device, caller-owned).  The frames may
 * overlap, repeat, or be empty (a zero hologram).  Work of all frames is
 * balanced across the device by one persistent kernel launch per stage, and
 * a repeated call with the same frame table replays a captured HIP graph.
 *   n_frames in [1, 65535]; each frame's points lie within the upload and
 *   its wavelength is finite and > 0.  The matrix-core modes process the
 *   frames in groups whose factors fit the workspace budget, balanced by
 *   size (one constants,
 *   one factor and one persistent GEMM launch per group; each (frame, tile)
 *   item runs its frame's whole K range in one workgroup, so a frame's sums
 *   are ordered differently from cgh_compute's split-K).  A call on a
 *   non-NULL stream runs eagerly and then records its kernel sequence in a
 *   HIP graph; a later call with the same mode, frame table and output
 *   replays that graph.  A call that changes any of them, or that must grow
 *   a workspace buffer, runs eagerly and replaces the graph.  The graph
 *   reads device tables that only batch calls write, so single-hologram
 *   calls on the context between replays do not disturb it.
 * Modes: all of cgh_mode.  Errors as cgh_compute; CGH_ESTATE when `stream`
 * is itself being captured (the call records its own graph). */
CGH_API cgh_status cgh_batch_compute(cgh_ctx *c, const cgh_frame *frames, int32_t n_frames,
                             cgh_mode mode, float *out_dev, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the hologram
 * of cgh_compute (same quantity, conventions and modes) of n points given
 * directly in device memory, evaluated without any allocation.  Every
 * intermediate (constants, tables or factors, split partials) lives in one
 * fixed 32 MiB array of static device memory per GPU, which the library's
 * code object holds until the process ends; a large cloud is processed in
 * point chunks that fit it and accumulate into the output in order, with
 * fewer split-K or point-split partials than cgh_compute when they do not
 * fit, so results agree with cgh_compute's to rounding, not bit for bit.
 *   width, height in [1, 65536]; pitch_m, wavelength_m finite and > 0.
 *   x_dev, y_dev, z_dev, amp_dev: float32 device arrays of n points (not
 *   inspected; z must be > 0), non-NULL when n > 0; n in [0, 2^34].
 *   out_dev: caller-owned device buffer of height*width floats.
 *   device: HIP device index in [0, 64) (made current for the call).
 * The call enqueues kernels on `stream` and nothing else (no allocation, no
 * copy, no memset, no host wait), so it may be captured into a graph.  The
 * first call on a device resolves the array's address there (call once
 * outside a capture).  All calls on one device share its array and leave
 * their intermediates in it: calls whose work overlaps on one device (other
 * streams, or graphs replayed concurrently) race and must be ordered by the
 * caller.
 * Errors: CGH_EINVAL for a bad argument, or for a hologram whose
 * intermediates of one group of 32 points exceed the array (the largest
 * sizes only: about 32 x (W + H) x 8 bytes in CGH_SPLIT_*, CGH_SEPARABLE_FP32
 * and CGH_SPHERICAL_FP32, half that in CGH_DIRECT_FP32 and CGH_FP16, so
 * 65536 x 65536 is refused in the first three), both checked before any HIP
 * call; CGH_EDEVICE (no gfx950 at `device`, launch failure). */
CGH_API cgh_status cgh_compute_noalloc(int32_t width, int32_t height, double pitch_m,
                                       double wavelength_m, const float *x_dev,
                                       const float *y_dev, const float *z_dev,
                                       const float *amp_dev, int64_t n, cgh_mode mode,
                                       float *out_dev, int32_t device, void *stream);

/* Autotune the launch shape of `mode` for this context's hologram size:
 * times every candidate (matrix-core modes: each built GEMM tile shape with a
 * few split-K counts, the time of the GEMM plus its split-K reduce; direct
 * modes: 4, 8 or 16 rows per lane, each with the points in 1, 2 or 4 runs
 * summed in a fixed order) `repeats` times on the uploaded cloud (its
 * first point chunk) with HIP events on `stream`, and keeps the fastest for
 * later evaluations of this size and mode whose K size falls in the same
 * power-of-two bucket.  With the environment variable CGH_TUNE_CACHE set to
 * a file path, the choice is appended to that file (JSON lines) and every
 * later cgh_create reads the file back.  `report` (optional, report_len
 * bytes) receives a one-line description of the choice.  Blocks the host
 * until the timing finishes.
 * Errors: CGH_EINVAL (repeats outside [1, 1000], bad buffer, unknown mode),
 * CGH_ESTATE (no upload), CGH_ENOTSUP (no candidate fits the hologram),
 * CGH_EDEVICE. */
CGH_API cgh_status cgh_tune(cgh_ctx *c, cgh_mode mode, int32_t repeats, char *report,
                            int32_t report_len, void *stream);

/* Autotune the persistent batched launch of cgh_batch_compute for this
 * frame table and mode: times `repeats` whole batch calls (after one
 * warm-up) per candidate -- every built GEMM tile shape in the matrix-core
 * modes, 4, 8 or 16 rows per lane in the direct modes -- writing into out_dev
 * (as cgh_batch_compute would), and keeps the fastest for later batch calls
 * of this hologram size and mode whose largest frame falls in the same
 * power-of-two K bucket (appended to CGH_TUNE_CACHE as cgh_tune does).
 * Drops any captured batch graph.  Blocks the host until the timing ends.
 * Arguments as cgh_batch_compute, plus repeats in [1, 1000] and the report
 * buffer as cgh_tune.  Errors as cgh_tune (CGH_ENOTSUP: a direct-mode batch
 * whose tables exceed the workspace budget). */
CGH_API cgh_status cgh_tune_batch(cgh_ctx *c, const cgh_frame *frames, int32_t n_frames,
                                  cgh_mode mode, float *out_dev, int32_t repeats, char *report,
                                  int32_t report_len, void *stream);

/* ---------------------------------------------------------------------
 * Fresnel diffraction of a sampled field (Section 2.3, Eq. (10)): the second
 * step of the wavefront-recording method, a field u on an n x n grid of pitch
 * p at distance z from the hologram propagated to the hologram plane and read
 * on the same grid,
 *   O[m][c] = exp(i 2 pi z / lambda) / (i lambda z) p^2
 *             sum_k sum_l u[k][l] exp(i pi p^2 ((m-k)^2 + (c-l)^2) / (lambda z)),
 * the integral of Eq. (10) taken as a sum over the samples times the sample
 * area.  Evaluated by FFT, as the equation's second line writes it, with the
 * impulse response's separability: the linear convolution along every
 * column and every row (n <= 1024: columns first; larger n: rows first),
 * each on the line zero-padded to 2n (no wrap-around) and cropped to n;
 * FP32 transforms with FP64-reduced chirp phases and twiddles.
 * --------------------------------------------------------------------- */
typedef struct cgh_fresnel cgh_fresnel;

/* Plan for n x n fields: n a power of two in [16, 8192]; pitch_m and
 * wavelength_m finite and > 0; z_m finite and non-zero (negative z
 * propagates backwards); device as for cgh_create.  Allocates 8 n^2 + 16 n
 * bytes of device workspace (16 n^2 + 16 n for n >= 2048) plus a twiddle
 * table of at most 5 n bytes, and
 * computes the transform of the impulse response (blocks until done).
 * Errors: CGH_EINVAL, CGH_EDEVICE, CGH_ENOMEM.  Free with cgh_fresnel_destroy. */
CGH_API cgh_status cgh_fresnel_create(cgh_fresnel **out, int32_t n, double pitch_m,
                                      double wavelength_m, double z_m, int32_t device);

/* Propagate u_dev to out_dev, both device buffers of n*n complex values
 * stored as interleaved float pairs (re, im), row-major; caller-owned; they
 * may be the same buffer.  Ordered on `stream`.  Calls on one plan must not
 * overlap (they share its workspace).  Two kernel launches (four for
 * n >= 2048) and nothing else, so a call may be captured into a HIP graph
 * (the plan must then outlive the graph).
 * Errors: CGH_EINVAL (NULL plan or buffer, or a buffer not 8-byte aligned),
 * CGH_EDEVICE (launch failure). */
CGH_API cgh_status cgh_fresnel_run(cgh_fresnel *f, const float *u_dev, float *out_dev,
                                   void *stream);

/* Free the plan (synchronises its device first).  NULL-safe. */
CGH_API void cgh_fresnel_destroy(cgh_fresnel *f);

/* ---------------------------------------------------------------------
 * Wavefront-recording method (Section 2.3): a virtual plane between the
 * points and the hologram first records the object wave (step 1), which
 * Fresnel diffraction (Eq. (10), step 2) then carries to the hologram.
 *
 * The plane is an n x n grid with the context's pitch p, centred like the
 * hologram, at distance zw from the hologram: sample (m, c) sits at
 * x_w = (c - (n-1)/2) p, y_w = (m - (n-1)/2) p.  Point j lies
 * d_j = z_j - zw beyond it; points with d_j <= 0 are not recorded.  Step 1
 * writes each point's Fresnel wave of Eq. (2) at depth d_j, without the
 * constant phase 2 pi d_j / lambda (as cgh_compute drops it), only over the
 * disc of radius r_j = lambda d_j / (2 p) around (x_j, y_j), beyond which the
 * wave's local frequency exceeds what the grid samples:
 *   u_w = sum over j with d_j > 0, (x_w - x_j)^2 + (y_w - y_j)^2 <= r_j^2 of
 *         A_j exp(i pi ((x_w - x_j)^2 + (y_w - y_j)^2) / (lambda d_j)).
 * The membership test is evaluated in FP64 exactly as written; the phase is
 * range-reduced in FP64 and the sum accumulated in FP32, in point order
 * (clouds of more than 4096 points: in point order within each of up to 4
 * chunks of consecutive points, whose sums are then added in chunk order,
 * with (chunks - 1) n^2 complex values of context workspace).
 * --------------------------------------------------------------------- */

/* Step 1 for the uploaded cloud: the plane at distance plane_z_m (finite;
 * metres) into field_dev, a caller-owned device buffer of n*n complex values
 * (interleaved float pairs, row-major, 8-byte aligned); n a power of two in
 * [16, 8192] (the plane sizes the diffraction step takes).  Every sample is
 * written.  Ordered on `stream` like cgh_compute.
 * Errors: CGH_EINVAL, CGH_ESTATE (no upload), CGH_ENOMEM, CGH_EDEVICE. */
CGH_API cgh_status cgh_wrm_record(cgh_ctx *c, double plane_z_m, int32_t n, float *field_dev,
                                  void *stream);

/* The whole method: step 1 on the plane of `plan` (its n, at its distance z
 * from the hologram) into field_dev (n*n complex, caller-owned, also the
 * diffraction's in-place buffer), step 2 = cgh_fresnel_run of that field
 * with `plan`, and the amplitude hologram of Eq. (5) (phi_r = 0, 2 A_r
 * dropped), Re O over the hologram's W x H window of the n x n result, into
 * out_dev (height*width floats, row-major).  The plan must have the
 * context's pitch and wavelength (equal values), z > 0, and n >= width,
 * height with n - width and n - height even (so the two grids' samples
 * coincide).  Calls on one plan must not overlap.
 * Errors: CGH_EINVAL, CGH_ESTATE, CGH_ENOMEM, CGH_EDEVICE. */
CGH_API cgh_status cgh_wrm_compute(cgh_ctx *c, cgh_fresnel *plan, float *field_dev,
                                   float *out_dev, void *stream);

/* Free the context and all its device memory (synchronises the device it
 * used first).  NULL-safe. */
CGH_API void cgh_destroy(cgh_ctx *c);

/* Static text for a status code. */
CGH_API const char *cgh_strerror(cgh_status s);

/* Thread-local detail of the last failure in this thread ("" if none). */
CGH_API const char *cgh_last_error(void);

/* ---------------------------------------------------------------------
 * Measurement support (not part of the hologram arithmetic).
 *
 * With profiling on, every kernel the context enqueues is bracketed by HIP
 * events on its stream.  cgh_profile_read() waits for those events and
 * returns, per kernel name, the number of launches and their total time in
 * milliseconds since the last reset; names[i] are static strings.
 *   capacity: entries the caller's arrays hold; *count receives the number
 *   written (at most capacity).
 * ------------------------------------------------------------------- */
CGH_API cgh_status cgh_profile_enable(cgh_ctx *c, int32_t on);
CGH_API cgh_status cgh_profile_reset(cgh_ctx *c);
CGH_API cgh_status cgh_profile_read(cgh_ctx *c, const char **names, int64_t *launches, double *total_ms,
                            int32_t capacity, int32_t *count);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
CGH_API int32_t cgh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CGH_H */
