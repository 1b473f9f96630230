/*
 * Host-side checks of the C ABI, built with the address and undefined-
 * behaviour sanitizers (tests/test_sanitizers.py).  Every call here is an
 * argument check or a host-only helper: nothing reaches a GPU.  Exits 0 when
 * every return code is the expected one; the sanitizers abort on any memory
 * or undefined-behaviour error.  Pointers are fake device addresses, never
 * dereferenced.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sobel4x5.h"

static int failures = 0;

#define EXPECT(expr, want)                                                                      \
    do {                                                                                        \
        const int got_ = (expr);                                                                \
        if (got_ != (want)) {                                                                   \
            fprintf(stderr, "%s:%d: %s = %d, expected %d (%s)\n", __FILE__, __LINE__, #expr,    \
                    got_, (want), sobel4x5_last_error());                                      \
            ++failures;                                                                         \
        }                                                                                       \
    } while (0)

#define FAKE ((uintptr_t)0x10000000u)
#define P(x) ((void *)(uintptr_t)(x))

static int v_u8(uintptr_t src, int w, int h, int64_t pitch, int border, uintptr_t mag, int64_t mag_pitch,
                int dir_type, const uintptr_t *dirs, int64_t dir_pitch)
{
    sobel4x5_outputs o;
    memset(&o, 0, sizeof o);
    o.mag = (uint8_t *)P(mag);
    o.mag_pitch = mag_pitch;
    o.dir_type = dir_type;
    o.dir_pitch = dir_pitch;
    for (int k = 0; k < 4; ++k) o.dir[k] = dirs ? P(dirs[k]) : NULL;
    return sobel4x5_validate_u8((const uint8_t *)P(src), w, h, pitch, border, &o);
}

static void check_u8(void)
{
    const uintptr_t mag = FAKE + (1u << 24);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, mag, 64, 0, NULL, 0), SOBEL4X5_OK);
    EXPECT(v_u8(0, 64, 32, 64, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 0, 32, 64, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, -1, 64, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 63, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, 4, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, -1, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 4, 32, 64, 1, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 5, 5, 5, 1, mag, 1, 0, NULL, 0), SOBEL4X5_OK);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, FAKE + 100, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 1, 1, 1, 3, mag, 1, 0, NULL, 0), SOBEL4X5_OK);
    EXPECT(v_u8(FAKE, 1 << 30, 1, (int64_t)1 << 30, 0, FAKE + ((uintptr_t)1 << 33), (int64_t)1 << 30, 0, NULL, 0),
           SOBEL4X5_OK);
    EXPECT(v_u8(FAKE, (1 << 30) + 1, 1, (int64_t)1 << 31, 0, mag, (int64_t)1 << 31, 0, NULL, 0), SOBEL4X5_EINVAL);
    /* pitches near the int64 limit must be rejected without overflowing */
    EXPECT(v_u8(FAKE, 64, 32, INT64_MAX, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 1 << 30, INT64_MAX / 4, 0, mag, 64, 0, NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, mag, INT64_MAX, 0, NULL, 0), SOBEL4X5_EINVAL);
    const uintptr_t dirs[4] = {FAKE + 2 * (1u << 24), FAKE + 3 * (1u << 24), FAKE + 4 * (1u << 24),
                               FAKE + 5 * (1u << 24)};
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 1, dirs, 128), SOBEL4X5_OK);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 2, dirs, 128), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 3, dirs, 256), SOBEL4X5_EINVAL);
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 1, dirs, INT64_MAX), SOBEL4X5_EINVAL);
    const uintptr_t same[4] = {dirs[0], dirs[0], dirs[0], dirs[0]};
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 1, same, 128), SOBEL4X5_EINVAL);
    const uintptr_t odd[4] = {dirs[0] + 1, dirs[1], dirs[2], dirs[3]};
    EXPECT(v_u8(FAKE, 64, 32, 64, 0, 0, 64, 1, odd, 128), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_u8((const uint8_t *)P(FAKE), 64, 32, 64, 0, NULL), SOBEL4X5_EINVAL);
    /* operators */
    sobel4x5_outputs o;
    memset(&o, 0, sizeof o);
    o.mag = (uint8_t *)P(mag);
    o.mag_pitch = 64;
    for (int op = 0; op < 3; ++op) EXPECT(sobel4x5_validate_u8_op((const uint8_t *)P(FAKE), 64, 32, 64, op, 0, &o), 0);
    EXPECT(sobel4x5_validate_u8_op((const uint8_t *)P(FAKE), 64, 32, 64, 3, 0, &o), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_u8_op((const uint8_t *)P(FAKE), 3, 3, 3, 2, 1, &o), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_u8_op((const uint8_t *)P(FAKE), 2, 3, 3, 2, 1, &o), SOBEL4X5_EINVAL);
    /* the last error is a readable string */
    if (strlen(sobel4x5_last_error()) == 0) {
        fprintf(stderr, "empty last error\n");
        ++failures;
    }
}

static void check_batch(void)
{
    sobel4x5_image im[3];
    memset(im, 0, sizeof im);
    for (int i = 0; i < 3; ++i) {
        im[i].src = (const uint8_t *)P(FAKE + (uintptr_t)i * (1u << 24));
        im[i].mag = (uint8_t *)P(FAKE + (uintptr_t)(10 + i) * (1u << 24));
        im[i].width = 100 + i;
        im[i].height = 50;
        im[i].src_pitch = 256;
        im[i].mag_pitch = 256;
    }
    EXPECT(sobel4x5_validate_batch(im, 3, 0), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_batch(im, 0, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_batch(NULL, 3, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_batch(im, 3, 5), SOBEL4X5_EINVAL);
    im[1].mag = im[0].mag + 10;
    EXPECT(sobel4x5_validate_batch(im, 3, 0), SOBEL4X5_EINVAL);
    im[1].mag = (uint8_t *)im[2].src;
    EXPECT(sobel4x5_validate_batch(im, 3, 0), SOBEL4X5_EINVAL);
    im[1].mag = (uint8_t *)P(FAKE + 11 * (1u << 24));
    im[2].width = 300;
    EXPECT(sobel4x5_validate_batch(im, 3, 0), SOBEL4X5_EINVAL);
    im[2].width = 102;
    for (int b = 2; b < 4; ++b) EXPECT(sobel4x5_validate_batch(im, 3, b), SOBEL4X5_OK);
    sobel4x5_outputs outs[3];
    memset(outs, 0, sizeof outs);
    for (int i = 0; i < 3; ++i) {
        outs[i].mag = (uint8_t *)P(FAKE + (uintptr_t)(20 + i) * (1u << 24));
        outs[i].mag_pitch = 128;
        outs[i].dir_type = SOBEL4X5_DIR_S16;
        outs[i].dir_pitch = 256;
        for (int k = 0; k < 4; ++k) outs[i].dir[k] = P(FAKE + (uintptr_t)(30 + 4 * i + k) * (1u << 24));
    }
    EXPECT(sobel4x5_validate_batch_ex(im, outs, 3, 0), SOBEL4X5_OK);
    outs[2].dir[3] = (char *)outs[0].dir[1] + 64;
    EXPECT(sobel4x5_validate_batch_ex(im, outs, 3, 0), SOBEL4X5_EINVAL);
    sobel4x5_plan plan = (sobel4x5_plan)P(1);
    EXPECT(sobel4x5_plan_create(im, 0, 0, 0, &plan), SOBEL4X5_EINVAL);
    if (plan != NULL) {
        fprintf(stderr, "plan handle not cleared on error\n");
        ++failures;
    }
    EXPECT(sobel4x5_plan_create(im, 3, 0, 0x80u, NULL), SOBEL4X5_EINVAL);
    /* allocation-free batched call: host checks before any HIP call */
    EXPECT(sobel4x5_batched_noalloc(NULL, 3, 0, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_batched_noalloc(im, 0, 0, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_batched_noalloc(im, 3, 7, NULL), SOBEL4X5_EINVAL);
    {
        const int n = SOBEL4X5_NOALLOC_MAX_IMAGES + 1;
        sobel4x5_image *many = (sobel4x5_image *)calloc((size_t)n, sizeof *many);
        for (int i = 0; many && i < n; ++i) {
            many[i].src = (const uint8_t *)P(FAKE + (uintptr_t)i * 512u);
            many[i].mag = (uint8_t *)P(FAKE + (uintptr_t)(n + i) * 512u);
            many[i].width = many[i].height = 16;
            many[i].src_pitch = many[i].mag_pitch = 16;
        }
        if (many) EXPECT(sobel4x5_batched_noalloc(many, n, 0, NULL), SOBEL4X5_EINVAL);
        free(many);
    }
    EXPECT(sobel4x5_plan_launch(NULL, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_plan_destroy(NULL), SOBEL4X5_EINVAL);
    char bogus[256];
    memset(bogus, 0x11, sizeof bogus);
    EXPECT(sobel4x5_plan_destroy((sobel4x5_plan)(void *)bogus), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_plan_info(NULL, NULL, NULL, NULL, NULL), SOBEL4X5_EINVAL);
    {
        int64_t nt = -1;
        EXPECT(sobel4x5_debug_plan_claims(NULL, NULL, 0, &nt, NULL), SOBEL4X5_EINVAL);
    }
}

static void check_f32(void)
{
    const float *src = (const float *)P(FAKE);
    const float *out = (const float *)P(FAKE + (1u << 26));
    EXPECT(sobel4x5_validate_f32(src, 2, 64, 32, 256, 256 * 32, 0, out, 256, 256 * 32), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_f32(src, 2, 64, 32, 256, 256 * 31, 0, out, 256, 256 * 32), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_f32(src, 2, 64, 32, 255, 256 * 32, 0, out, 256, 256 * 32), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_f32(src, 1, 4, 4, 16, 0, 1, out, 16, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_f32(src, 0, 8, 8, 32, 0, 0, out, 32, 0), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_f32(src, 1 << 30, 64, 32, 256, INT64_MAX / 2, 0, out, 256, 256 * 32), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_f32(src, 3, 64, 32, INT64_MAX - 3, 0, 0, out, 256, 256 * 32), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_f32_fwd(src, 2, 64, 32, 255, 256 * 32, 0, (float *)out, 256, 256 * 32, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_f32_bwd(src, 256, 256 * 32, NULL, 256, 256 * 32, 2, 64, 32, 0, (float *)out, 256, 256 * 32,
                            NULL),
           SOBEL4X5_EINVAL);
}

static void check_weights_and_misc(void)
{
    int32_t w[100];
    EXPECT(sobel4x5_family_weights(1, 2, 4, 6, 8, 12, w), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_weights(w, 0), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_weights(w, SOBEL4X5_DIR_S16), SOBEL4X5_OK);
    EXPECT(sobel4x5_family_weights(1, 2, 4, 6, 8, 13, w), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_family_weights(0, 2, 4, 6, 8, 12, w), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_family_weights(1, 2, 4, 6, 8, 12, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_family_weights(1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, 1 << 30, w), SOBEL4X5_OK);
    EXPECT(sobel4x5_validate_weights(w, 0), SOBEL4X5_EINVAL);   /* sum of |w| overflows int32: rejected */
    for (int i = 0; i < 100; ++i) w[i] = 0;
    w[0] = 1;
    EXPECT(sobel4x5_validate_weights(w, 0), SOBEL4X5_EINVAL);   /* not antisymmetric */
    w[0] = INT32_MIN;
    w[24] = INT32_MIN;
    EXPECT(sobel4x5_validate_weights(w, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_validate_weights(NULL, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_debug_round_mag(NULL, NULL, 5, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_debug_copy(P(FAKE + 1), P(FAKE), 16, NULL), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_debug_inject_failure(-1), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_debug_inject_failure(0), SOBEL4X5_OK);
    sobel4x5_pipe pipe = (sobel4x5_pipe)P(1);
    EXPECT(sobel4x5_pipe_create(64, 64, 0, &pipe), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_pipe_create(64, 64, 17, &pipe), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_pipe_create(0, 64, 2, &pipe), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_pipe_run(NULL, NULL, 0, 0), SOBEL4X5_EINVAL);
    EXPECT(sobel4x5_pipe_destroy(NULL), SOBEL4X5_EINVAL);
    for (int s = -1; s < 7; ++s)
        if (!sobel4x5_status_string(s) || !*sobel4x5_status_string(s)) {
            fprintf(stderr, "status string %d empty\n", s);
            ++failures;
        }
    if (sobel4x5_version() != SOBEL4X5_VERSION) {
        fprintf(stderr, "version mismatch\n");
        ++failures;
    }
}

int main(void)
{
    check_u8();
    check_batch();
    check_f32();
    check_weights_and_misc();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("abi checks ok\n");
    return 0;
}
