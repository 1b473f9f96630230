/*
 * sobel4x5.h -- C ABI of the MI355X (gfx950) four-directional 5x5 Sobel library.
 *
 * The operator (Chang et al., "Multi-directional Sobel operator kernel on
 * GPUs", Sec. 3.1): four fixed 5x5 integer filters, Eq. (sobel5_1) --
 * 0 deg (Gx), 45 deg (Gd), 90 deg (Gy), 135 deg (Gdt) -- are applied to every
 * pixel of an 8-bit grayscale image as a correlation (tap (i, j) of a printed
 * matrix multiplies the pixel at row offset i-2, column offset j-2, the way
 * the row filters Eq. (Fx) and Eq. (Gd+) of Sec. 4.3 index the pixels), and
 * combined into the root-sum-of-squares magnitude of Eq. (sobel5_2).
 *
 * Conventions shared by every entry point
 *   - Buffers named src/dst/mag/dir/grad are DEVICE pointers owned by the
 *     caller.  Nothing here frees them.  Descriptor arrays and the outputs
 *     struct are HOST memory, read during the call only.
 *   - Pitches and strides are in BYTES.  A row pitch must be at least the
 *     row's width in bytes; any larger value is accepted.  Input images
 *     with 16-byte aligned rows (base and pitch) take the fast path; any
 *     other input takes a slower path with identical results.  Output rows
 *     need no alignment.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; device faults surface at the
 *     caller's next synchronisation.
 *   - Every argument is checked on the host before anything is enqueued, so
 *     an error return means no work was queued.  Launch failures map to
 *     SOBEL4X5_EHIP.  sobel4x5_last_error() gives a human-readable detail
 *     for the calling thread's last failed call.
 *   - Inputs and outputs must not overlap (the stencil reads neighbours).
 *   - Calls are thread-safe.  A plan's work queue admits one launch at a
 *     time: launches of one plan must be ordered (one stream, or streams
 *     joined by events), never overlapping.  One-shot batched calls keep a
 *     separate cached plan per stream, so they may run on several streams.
 *
 * Borders (Sec. 4.3 leaves the padding rule to an earlier work)
 *   SOBEL4X5_BORDER_REPLICATE : clamp-to-edge; output is H x W; any H, W >= 1.
 *   SOBEL4X5_BORDER_VALID     : the paper's shrink by 2r = 4 (Sec. 4.3, data
 *                               flow); output is (H-4) x (W-4) and
 *                               out(y, x) = replicate(y+2, x+2); H, W >= 5.
 *   SOBEL4X5_BORDER_ZERO      : pixels outside the image read 0; H x W.
 *   SOBEL4X5_BORDER_REFLECT101: pixels outside the image read their mirror
 *                               image about the edge pixel, which is not
 *                               repeated (index -1 -> 1, -2 -> 2, W -> W-2,
 *                               W+1 -> W-3); an axis of 1 or 2 pixels
 *                               reflects again until the index lands inside
 *                               (period 2(n-1)).  H x W; any H, W >= 1.
 *   Every entry point serves all four (uint8 single, operators, run-time
 *   weights, batched, pipeline, and the fp32 pair).
 *
 * uint8 magnitude: min(255, round-to-nearest(sqrt(S))), S = Gx^2 + Gd^2 +
 * Gy^2 + Gdt^2 -- exact (integer S never sits on a half-way point).
 */
#ifndef SOBEL4X5_H
#define SOBEL4X5_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOBEL4X5_VERSION 111

/* status codes */
#define SOBEL4X5_OK 0
#define SOBEL4X5_EINVAL 1          /* bad argument; nothing enqueued          */
#define SOBEL4X5_EUNSUPPORTED 2    /* valid request this build cannot serve   */
#define SOBEL4X5_EHIP 3            /* a HIP runtime call or launch failed     */
#define SOBEL4X5_ENOMEM 4          /* device or host allocation failed        */

/* border rules */
#define SOBEL4X5_BORDER_REPLICATE 0
#define SOBEL4X5_BORDER_VALID 1
#define SOBEL4X5_BORDER_ZERO 2
#define SOBEL4X5_BORDER_REFLECT101 3

/* directional output element types */
#define SOBEL4X5_DIR_NONE 0
#define SOBEL4X5_DIR_S16 1         /* int16 planes (exact: |G| <= 12240)      */
#define SOBEL4X5_DIR_S32 2         /* int32 planes                            */

/*
 * Outputs of one uint8 image.  Host struct.
 *   mag       : Ho rows of Wo bytes, row r at mag + r*mag_pitch; NULL = none.
 *   dir[k]    : plane k (0 = 0 deg Gx, 1 = 45 deg Gd, 2 = 90 deg Gy,
 *               3 = 135 deg Gdt), Ho rows of Wo elements of dir_type, row r at
 *               (char*)dir[k] + r*dir_pitch.  Used iff dir_type != DIR_NONE,
 *               and then all four must be non-NULL.
 * At least one of mag / dir must be requested.
 */
typedef struct sobel4x5_outputs {
    uint8_t *mag;
    int64_t mag_pitch;
    void *dir[4];
    int64_t dir_pitch;
    int32_t dir_type;
} sobel4x5_outputs;

/*
 * sobel4x5_u8 -- Eq. (sobel5_1) + Eq. (sobel5_2) on one uint8 image.
 *   src        : H rows of W bytes, row r at src + r*src_pitch (device).
 *   width      : W >= 1 (>= 5 for VALID); height: H likewise.
 *   border     : SOBEL4X5_BORDER_*.
 *   out        : host struct, see above.
 * Integer arithmetic throughout; results are bit-exact.
 */
int sobel4x5_u8(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch,
                int32_t border, const sobel4x5_outputs *out, void *stream);

/* Host-only argument check of sobel4x5_u8 (never touches the GPU). */
int sobel4x5_validate_u8(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch,
                         int32_t border, const sobel4x5_outputs *out);

/*
 * Operators.  Besides its four-directional 5x5 operator the paper defines
 * the classic two-directional 3x3 Sobel pair, Eq. (sobel3_1) with the
 * magnitude of Eq. (sobel3_2), and measures its kernels against the 3x3
 * operator (Sec. 5, Table 1).
 *   SOBEL4X5_OP_4DIR_5X5 : Eq. (sobel5_1) + Eq. (sobel5_2) (= sobel4x5_u8).
 *   SOBEL4X5_OP_2DIR_5X5 : the 0 and 90 deg filters of Eq. (sobel5_1) alone,
 *                          S = Gx^2 + Gy^2.
 *   SOBEL4X5_OP_2DIR_3X3 : Eq. (sobel3_1) + Eq. (sobel3_2), tap (i, j)
 *                          multiplying the pixel at offset (i-1, j-1); its
 *                          radius is 1, so VALID shrinks the image by 2:
 *                          output (H-2) x (W-2), out(y, x) =
 *                          replicate(y+1, x+1), H, W >= 3.
 */
#define SOBEL4X5_OP_4DIR_5X5 0
#define SOBEL4X5_OP_2DIR_5X5 1
#define SOBEL4X5_OP_2DIR_3X3 2

/*
 * sobel4x5_u8_op -- sobel4x5_u8 for the operator `op` (SOBEL4X5_OP_*).
 *   The two-directional operators write directional planes dir[0] (Gx,
 *   0 deg) and dir[2] (Gy, 90 deg) only; dir[1] and dir[3] are ignored and
 *   may be NULL.  Their int16 planes are exact (|G| <= 1020 for 3x3,
 *   12240 for 5x5).  Magnitude min(255, round(sqrt(S))), exact.  Other
 *   arguments, errors and layouts as for sobel4x5_u8; op 0 is sobel4x5_u8.
 *   An unknown op is SOBEL4X5_EINVAL.
 */
int sobel4x5_u8_op(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t op,
                   int32_t border, const sobel4x5_outputs *out, void *stream);

/* Host-only argument check of sobel4x5_u8_op (never touches the GPU). */
int sobel4x5_validate_u8_op(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch,
                            int32_t op, int32_t border, const sobel4x5_outputs *out);

/*
 * Generalised weights (Sec. 3.2, Eq. (sobel5_param)).
 *
 * sobel4x5_u8_weighted -- sobel4x5_u8 with run-time integer kernels.
 *   weights : HOST array of 4*25 int32: four 5x5 kernels in plane order
 *             (0 deg, 45 deg, 90 deg, 135 deg), each row-major; tap (i, j)
 *             multiplies the pixel at offset (i-2, j-2) (correlation, as for
 *             the default operator).  Read during the call only.
 *   Every kernel must be antisymmetric under a half turn
 *   (k[4-i][4-j] == -k[i][j], so k[2][2] == 0; the family K(a, b, n, m) is)
 *   and have sum |k_ij| <= 32768 (then |G| < 2^23 and int32 planes are
 *   exact); with dir_type DIR_S16, sum |k_ij| <= 128 (|G| <= 32767).
 *   Anything else is SOBEL4X5_EINVAL.  Other arguments, outputs and the
 *   uint8 rounding min(255, round(sqrt(S))) are as for sobel4x5_u8.  The
 *   default weights of Eq. (sobel5_1) give the same results as sobel4x5_u8,
 *   which runs them on a faster path.  Magnitude-only calls whose weights
 *   all lie in [-128, 127] run on the matrix cores (same results; the
 *   environment variable SOBEL4X5_W_MFMA=0 selects the vector kernel).
 */
int sobel4x5_u8_weighted(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch,
                         int32_t border, const int32_t *weights, const sobel4x5_outputs *out,
                         void *stream);

/* Host-only check of a weights array for sobel4x5_u8_weighted with the
 * given dir_type (never touches the GPU). */
int sobel4x5_validate_weights(const int32_t *weights, int32_t dir_type);

/*
 * sobel4x5_family_weights -- the four kernels of the family K(a, b, n, m)
 * of Eq. (sobel5_param) (K_x, K_d, K_y = K_x transposed, K_dt = K_d mirrored
 * left-right), written to weights_out (HOST, 4*25 int32, the layout of
 * sobel4x5_u8_weighted).  The family is given by its six distinct integer
 * weights a, a*b, a*n, a*m, a*n*b, a*m*b, which must be positive and
 * consistent: (a*n)(a*b) == a(a*n*b) and (a*m)(a*b) == a(a*m*b).
 * Eq. (sobel5_1) is (1, 2, 4, 6, 8, 12).  EINVAL otherwise.
 */
int sobel4x5_family_weights(int32_t a, int32_t ab, int32_t an, int32_t am, int32_t anb, int32_t amb,
                            int32_t *weights_out);

/*
 * Batched uint8 magnitudes: many images of uneven sizes in ONE launch of a
 * persistent work-queue kernel (not in the paper; it applies the same integer
 * arithmetic per image).
 *   sobel4x5_image : host descriptor; src/mag device pointers, pitches in bytes.
 */
typedef struct sobel4x5_image {
    const uint8_t *src;
    uint8_t *mag;
    int32_t width;
    int32_t height;
    int64_t src_pitch;
    int64_t mag_pitch;
} sobel4x5_image;

typedef struct sobel4x5_plan_s *sobel4x5_plan;

#define SOBEL4X5_PLAN_AUTOTUNE 1u  /* time candidate tile shapes, keep the fastest
                                      that is bit-exact against the default   */
#define SOBEL4X5_PLAN_NO_GRAPH 2u  /* launch the kernel directly, no hipGraph */

/*
 * sobel4x5_plan_create -- build a reusable plan for a fixed set of images.
 *   imgs/count : host array of count >= 1 descriptors (copied).
 *   border     : SOBEL4X5_BORDER_*.
 *   flags      : SOBEL4X5_PLAN_* bits.
 *   out        : receives the plan handle.
 * Allocates device memory for the tile table and queue counters (ENOMEM on
 * failure), uploads them, selects the tile shape (autotuned with
 * SOBEL4X5_PLAN_AUTOTUNE, which runs and synchronises the device), and
 * captures the launch in a hipGraph.  The images' contents are not read here
 * except during autotuning, which writes the mag buffers.
 */
int sobel4x5_plan_create(const sobel4x5_image *imgs, int32_t count, int32_t border,
                         uint32_t flags, sobel4x5_plan *out);

/* Enqueue the plan's work on `stream` (graph launch).  The queue counters
 * reset themselves at the end of every launch, so launches can repeat. */
int sobel4x5_plan_launch(sobel4x5_plan plan, void *stream);

/* Tile shape the plan uses: pixels per lane, rows per tile, waves per
 * workgroup, and the persistent grid size.  Any pointer may be NULL. */
int sobel4x5_plan_info(sobel4x5_plan plan, int32_t *px_per_lane, int32_t *rows_per_tile,
                       int32_t *waves_per_group, int32_t *grid);

/*
 * sobel4x5_debug_plan_claims -- work-queue check: one launch of the plan that
 * also counts, per tile of its work table, how many waves took that tile.
 *   plan     : a plan from sobel4x5_plan_create(_ex).
 *   claims   : device array of `capacity` uint32 counters, or NULL to only
 *              query the tile count.
 *   capacity : counters in `claims`; must be >= *ntiles (EINVAL otherwise).
 *   ntiles   : receives the plan's tile count (always, also with claims NULL).
 *   stream   : HIP stream.
 * Clears claims[0 .. ntiles) and launches the plan's kernel once, directly
 * (not through its graph), on `stream`; the outputs are written as by
 * sobel4x5_plan_launch.  In a correct launch every counter ends at 1 (none
 * skipped, none taken twice), in the persistent and in the static grid form.
 * Must not overlap another launch of the same plan.  For tests and
 * diagnostics: it checks the batched work queue, which is this library's own
 * scheduling of many images and has no counterpart in the paper.
 */
int sobel4x5_debug_plan_claims(sobel4x5_plan plan, uint32_t *claims, int64_t capacity, int64_t *ntiles,
                               void *stream);

/* Free the plan (device memory, graph).  Waits for nothing: the caller must
 * make sure no launch of it is still running. */
int sobel4x5_plan_destroy(sobel4x5_plan plan);

/* One-shot batched call: builds (or reuses a cached) plan for these images
 * and launches it on `stream`.  Equivalent to plan_create + plan_launch.
 * The cache (8 plans, least recently used first out) is keyed by every
 * descriptor field, the border, the device and the stream; evicting a plan
 * waits for its stream. */
int sobel4x5_batched(const sobel4x5_image *imgs, int32_t count, int32_t border, void *stream);

/* Host-only argument check of a batch (never touches the GPU). */
int sobel4x5_validate_batch(const sobel4x5_image *imgs, int32_t count, int32_t border);

/*
 * sobel4x5_batched_noalloc -- sobel4x5_batched for callers that cannot
 * allocate memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  The same batched kernel (magnitudes
 * only, the default tile shape and grid form, no autotuning, no graph), but
 * its job table, tile table and queue counters live in a fixed device buffer
 * of the library, one per device, held until the process ends; the call
 * allocates no memory, device or host (it builds the tables in fixed
 * static host buffers, one call at a time per process, then copies them
 * into that device buffer and launches, both on `stream`).
 *   imgs/count/border : as for sobel4x5_batched (magnitudes only).
 *   Limits: count <= SOBEL4X5_NOALLOC_MAX_IMAGES and at most
 *   SOBEL4X5_NOALLOC_MAX_TILES wave-tiles (about 150 per 2048x2048 image);
 *   a batch beyond either is SOBEL4X5_EINVAL, with nothing enqueued.
 *   Every call on one device uses that device's one buffer, which keeps the
 *   last call's tables: calls on one stream are ordered and safe, but calls
 *   that overlap in time on one device (different streams not joined by
 *   events, or different threads) race and give wrong results.
 */
#define SOBEL4X5_NOALLOC_MAX_IMAGES 1024
#define SOBEL4X5_NOALLOC_MAX_TILES 65536
int sobel4x5_batched_noalloc(const sobel4x5_image *imgs, int32_t count, int32_t border, void *stream);

/*
 * Batches with per-image outputs: the calls above with `outs`, a HOST array
 * of `count` sobel4x5_outputs (copied), image i writing outs[i] -- its
 * magnitude (mag may be NULL) and/or its directional planes (dir_type, four
 * planes, as for sobel4x5_u8).  imgs[i].mag and mag_pitch are ignored.
 * outs == NULL is the plain call.  Outputs of all images must not overlap
 * each other or any input.  The autotuner checks every output plane.
 */
int sobel4x5_plan_create_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count,
                            int32_t border, uint32_t flags, sobel4x5_plan *out);
int sobel4x5_batched_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count,
                        int32_t border, void *stream);
int sobel4x5_validate_batch_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count,
                               int32_t border);

/*
 * Host pipeline: uint8 images in HOST memory -> magnitudes in HOST memory.
 * The paper measures host<->device transfer as the dominant cost of the
 * whole operation (Table 1, IO column; Sec. 5) and names overlapping it as
 * future work (Sec. 6).  A pipeline holds `depth` slots, each with device
 * buffers for the largest image, pinned staging buffers and a stream of its
 * own; image i uses slot i % depth, so the copy to the device of one image,
 * the kernel of another and the copy back of a third run at the same time.
 *
 * sobel4x5_pipe_create -- allocate a pipeline for images of at most
 *   max_width x max_height (device: 2 * depth * round_up(max_width, 256) *
 *   max_height bytes; pinned host: the same).  depth in [1, 16].
 * sobel4x5_pipe_run -- process `count` images (sobel4x5_image descriptors
 *   whose src and mag point to HOST memory, pageable or pinned; pinned
 *   buffers are copied directly, pageable ones through the staging
 *   buffers) with the given border; magnitude only.  Synchronous: returns
 *   when every magnitude is in host memory.  A pipeline must not be run by
 *   two threads at once.  On an EHIP return every copy and kernel the call
 *   queued has finished (nothing writes a caller buffer afterwards), the
 *   magnitudes of this call's images are unspecified, and the pipeline is
 *   idle and reusable with any other image array.
 * sobel4x5_pipe_destroy -- wait for nothing, free everything.
 */
typedef struct sobel4x5_pipe_s *sobel4x5_pipe;
int sobel4x5_pipe_create(int32_t max_width, int32_t max_height, int32_t depth, sobel4x5_pipe *out);
int sobel4x5_pipe_run(sobel4x5_pipe pipe, const sobel4x5_image *host_imgs, int32_t count, int32_t border);
int sobel4x5_pipe_destroy(sobel4x5_pipe pipe);

/*
 * Real-valued path (not in the paper): the same correlation in fp32 on a
 * batch of images, for use as a differentiable edge loss.
 *
 * sobel4x5_f32_fwd -- M = sqrt(Gx^2 + Gd^2 + Gy^2 + Gdt^2) per pixel, fp32
 * arithmetic.  Each response is summed as differences of opposite taps, so a
 * flat 5x5 window gives exactly M = 0.
 *   src  : batch images of height rows x width floats; image b, row r at
 *          (char*)src + b*src_bstride + r*src_pitch.
 *   mag  : batch images of Ho x Wo floats, same addressing with mag_* strides.
 */
int sobel4x5_f32_fwd(const float *src, int32_t batch, int32_t width, int32_t height,
                     int64_t src_pitch, int64_t src_bstride, int32_t border,
                     float *mag, int64_t mag_pitch, int64_t mag_bstride, void *stream);

/*
 * sobel4x5_f32_bwd -- adjoint of sobel4x5_f32_fwd: given grad_mag = dL/dM
 * (Ho x Wo per image), writes grad_src = dL/dsrc (H x W per image,
 * overwritten).  u_k = grad_mag * G_k / M where M > 0 and 0 where M = 0; each
 * u_k is spread back through the transposed filter.  The contributions that
 * fell on positions outside the image go to the pixel the border rule read
 * there: the edge pixel (REPLICATE), the mirror pixel (REFLECT101), or
 * nowhere (ZERO: those taps read a constant).  G is recomputed from src (no
 * saved state).
 */
int sobel4x5_f32_bwd(const float *src, int64_t src_pitch, int64_t src_bstride,
                     const float *grad_mag, int64_t g_pitch, int64_t g_bstride,
                     int32_t batch, int32_t width, int32_t height, int32_t border,
                     float *grad_src, int64_t gs_pitch, int64_t gs_bstride, void *stream);

/* Host-only argument check shared by the two fp32 calls (never touches the
 * GPU).  Pass grad pointers as NULL and their strides as 0 to check a
 * forward call. */
int sobel4x5_validate_f32(const float *src, int32_t batch, int32_t width, int32_t height,
                          int64_t src_pitch, int64_t src_bstride, int32_t border,
                          const float *out, int64_t out_pitch, int64_t out_bstride);

/*
 * Diagnostic: the library's uint8 rounding of the magnitude, applied to n
 * given values of S (the sum of the four squared responses, 0 <= S < 2^31).
 * out[i] = min(255, round(sqrt(S[i]))).  Device pointers; n >= 0.
 */
int sobel4x5_debug_round_mag(const int32_t *S, uint8_t *out, int64_t n, void *stream);

/*
 * The same with a choice of the two implementations of that rounding in
 * the two-directional operators' kernels: method 0 converts S to fp32 and
 * rounds its square root (kernels that run three waves per SIMD); method 1
 * reads a table of the rounded value of every S below 2^16, held in LDS, at
 * min(S, 65535) (kernels that run two waves per SIMD).  Both must give the
 * same byte for every S.  EINVAL for another method.
 */
int sobel4x5_debug_round_mag_ex(const int32_t *S, uint8_t *out, int64_t n, int32_t method, void *stream);

/*
 * Diagnostic: the rounding of the four-directional kernels, step for step.
 * They never form S; they form E1 = (Gx + Gy)/2, E2 = (Gx - Gy)/2,
 * Hp = (Gd + Gdt)/2 and Hm = (Gd - Gdt)/2 (all int16), for which
 * S = 2 (E1^2 + E2^2 + Hp^2 + Hm^2) (Eq. (sobel5_2)), sum the four squares
 * on int16 lanes saturating at 32767, and read min(255, round(sqrt(2 T)))
 * from a table in LDS.  q: n quadruples (E1, E2, Hp, Hm) of int16 (device,
 * 8 bytes each); out[i] (device) receives the byte of quadruple i, which
 * must equal min(255, round(sqrt(S))) for every int16 quadruple.
 * EINVAL for n < 0 or NULL pointers with n > 0.
 */
int sobel4x5_debug_round_quad(const int16_t *q, uint8_t *out, int64_t n, void *stream);

/*
 * Diagnostic: plain device-to-device copy of nbytes (a multiple of 16;
 * 16-byte aligned device pointers) with 128-bit accesses, each workgroup
 * copying one contiguous 16 KiB block.  It is the measured reference for
 * the achievable HBM bandwidth and the calibration of memory-traffic
 * counters.
 */
int sobel4x5_debug_copy(const void *src, void *dst, int64_t nbytes, void *stream);

/*
 * Test hook for the error paths: with nth_call = n > 0, the n-th HIP call
 * made after this one through the library's guarded call sites (the uint8
 * launch, plan launches, and every copy, launch and wait of
 * sobel4x5_pipe_run) reports a runtime failure, so the caller gets
 * SOBEL4X5_EHIP although the call itself ran; 0 disarms.  Process-wide.
 * EINVAL for n < 0.
 */
int sobel4x5_debug_inject_failure(int32_t nth_call);

const char *sobel4x5_status_string(int status);
const char *sobel4x5_last_error(void);
int sobel4x5_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SOBEL4X5_H */
