/*
 * The CPU oracle run under the address and undefined-behaviour sanitizers
 * (tests/test_sanitizers.py): every entry point on tiny and odd shapes under
 * every border rule (axes of 1 to 9 pixels, where the reflect-101 mirror
 * folds repeatedly), row pitches wider than the row, and rejected
 * arguments.  A few exact properties are checked on the way (a constant
 * image has zero responses under the edge-preserving rules; an impulse at c
 * gives tap (2-dy, 2-dx) of each filter at c + (dy, dx)), but the point is
 * that nothing reads or writes outside its buffers and no arithmetic
 * overflows.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_u8(const uint8_t *src, int W, int H, long pitch, int border, uint8_t *mag, long mag_pitch,
              int32_t *dir, const int32_t *weights, int nthreads);
int oracle_u8_points(const uint8_t *src, int W, int H, long pitch, int border, const int32_t *ys,
                     const int32_t *xs, long n, uint8_t *mag, int32_t *dir, const int32_t *weights);
int oracle_f64_fwd(const double *x, int B, int H, int W, int border, double *mag, double *dir,
                   const int32_t *weights, int nthreads);
int oracle_f64_bwd(const double *x, const double *g, int B, int H, int W, int border, double *dx,
                   const int32_t *weights, int nthreads);
int oracle_f64_bwd_scale(const double *x, const double *g, int B, int H, int W, int border, double *A,
                         const int32_t *weights, int nthreads);
int oracle_f64_fwd_scale(const double *x, int B, int H, int W, int border, double *scale, const int32_t *weights,
                         int nthreads);
int oracle_u8_2dir(const uint8_t *src, int W, int H, long pitch, int border, int size, uint8_t *mag,
                   long mag_pitch, int32_t *dir, int nthreads);
void oracle_weights(int32_t *out);
int64_t oracle_round_sqrt(int64_t S);

static int failures = 0;
#define CHECK(cond)                                                            \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static uint32_t rng_state = 12345u;
static uint32_t rnd(void)
{
    rng_state = rng_state * 1664525u + 1013904223u;
    return rng_state >> 8;
}

/* exact-size heap buffers, so that the sanitizer sees every overrun */
static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) abort();
    return p;
}

static void u8_shapes(void)
{
    int32_t K[100];
    oracle_weights(K);
    for (int border = 0; border < 4; ++border)
        for (int H = 1; H <= 9; ++H)
            for (int W = 1; W <= 9; ++W) {
                const long pitch = W + (long)(rnd() % 3);
                const int valid = border == 1;
                const int Ho = valid ? H - 4 : H, Wo = valid ? W - 4 : W;
                uint8_t *src = xmalloc((size_t)((H - 1) * pitch + W));
                for (long i = 0; i < (H - 1) * pitch + W; ++i) src[i] = (uint8_t)rnd();
                if (valid && (H < 5 || W < 5)) {
                    CHECK(oracle_u8(src, W, H, pitch, border, NULL, 1, NULL, NULL, 1) != 0);
                    free(src);
                    continue;
                }
                uint8_t *mag = xmalloc((size_t)Ho * Wo);
                int32_t *dir = xmalloc(sizeof(int32_t) * 4 * (size_t)Ho * Wo);
                CHECK(oracle_u8(src, W, H, pitch, border, mag, Wo, dir, NULL, 1) == 0);
                CHECK(oracle_u8(src, W, H, pitch, border, mag, Wo, NULL, K, 2) == 0);
                CHECK(oracle_u8_2dir(src, W, H, pitch, border, 5, mag, Wo, NULL, 1) == 0);
                if (!valid || (H >= 3 && W >= 3)) {
                    const int o3h = valid ? H - 2 : H, o3w = valid ? W - 2 : W;
                    uint8_t *m3 = xmalloc((size_t)o3h * o3w);
                    int32_t *d3 = xmalloc(sizeof(int32_t) * 2 * (size_t)o3h * o3w);
                    CHECK(oracle_u8_2dir(src, W, H, pitch, border, 3, m3, o3w, d3, 1) == 0);
                    free(m3);
                    free(d3);
                }
                int32_t ys[3] = {0, Ho - 1, Ho / 2}, xs[3] = {Wo - 1, 0, Wo / 2};
                int32_t pd[12];
                uint8_t pm[3];
                CHECK(oracle_u8_points(src, W, H, pitch, border, ys, xs, 3, pm, pd, NULL) == 0);
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 4; ++k) CHECK(pd[4 * i + k] == dir[(size_t)k * Ho * Wo + (size_t)ys[i] * Wo + xs[i]]);
                /* a constant image: zero responses except under ZERO */
                memset(src, 77, (size_t)((H - 1) * pitch + W));
                CHECK(oracle_u8(src, W, H, pitch, border, mag, Wo, dir, NULL, 1) == 0);
                if (border != 2)
                    for (long i = 0; i < 4L * Ho * Wo; ++i) CHECK(dir[i] == 0);
                free(src);
                free(mag);
                free(dir);
            }
    /* the impulse response under REPLICATE, away from the edges */
    {
        enum { N = 11 };
        uint8_t img[N * N];
        memset(img, 0, sizeof img);
        img[5 * N + 5] = 1;
        int32_t dir[4 * N * N];
        CHECK(oracle_u8(img, N, N, N, 0, NULL, 1, dir, NULL, 1) == 0);
        for (int k = 0; k < 4; ++k)
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx)
                    CHECK(dir[k * N * N + (5 + dy) * N + (5 + dx)] == K[k * 25 + (2 - dy) * 5 + (2 - dx)]);
    }
    /* rejected arguments */
    uint8_t b[64];
    memset(b, 0, sizeof b);
    CHECK(oracle_u8(NULL, 8, 8, 8, 0, NULL, 1, NULL, NULL, 1) != 0);
    CHECK(oracle_u8(b, 8, 8, 7, 0, NULL, 1, NULL, NULL, 1) != 0);
    CHECK(oracle_u8(b, 8, 8, 8, 4, NULL, 1, NULL, NULL, 1) != 0);
    CHECK(oracle_u8(b, 0, 8, 8, 0, NULL, 1, NULL, NULL, 1) != 0);
    CHECK(oracle_u8(b, 8, 8, 8, 0, b, 7, NULL, NULL, 1) != 0);
    int32_t bad_y = 8, ok_x = 0;
    CHECK(oracle_u8_points(b, 8, 8, 8, 0, &bad_y, &ok_x, 1, NULL, NULL, NULL) != 0);
    CHECK(oracle_u8_2dir(b, 8, 8, 8, 0, 4, NULL, 1, NULL, 1) != 0);
}

static void f64_shapes(void)
{
    for (int border = 0; border < 4; ++border)
        for (int H = 1; H <= 8; ++H)
            for (int W = 1; W <= 8; W += (W < 4 ? 1 : 3)) {
                const int B = 2;
                const int valid = border == 1;
                if (valid && (H < 5 || W < 5)) {
                    double x1[1] = {0};
                    double m1[1];
                    CHECK(oracle_f64_fwd(x1, 1, H, W, border, m1, NULL, NULL, 1) != 0);
                    continue;
                }
                const int Ho = valid ? H - 4 : H, Wo = valid ? W - 4 : W;
                const size_t nin = (size_t)B * H * W, nout = (size_t)B * Ho * Wo;
                double *x = xmalloc(sizeof(double) * nin), *g = xmalloc(sizeof(double) * nout);
                double *M = xmalloc(sizeof(double) * nout), *D = xmalloc(sizeof(double) * 4 * nout);
                double *dx = xmalloc(sizeof(double) * nin), *A = xmalloc(sizeof(double) * nin);
                double *sf = xmalloc(sizeof(double) * nout);
                for (size_t i = 0; i < nin; ++i) x[i] = (rnd() % 1000) / 997.0;
                for (size_t i = 0; i < nout; ++i) g[i] = ((int)(rnd() % 2001) - 1000) / 1000.0;
                CHECK(oracle_f64_fwd(x, B, H, W, border, M, D, NULL, 1) == 0);
                CHECK(oracle_f64_fwd_scale(x, B, H, W, border, sf, NULL, 1) == 0);
                CHECK(oracle_f64_bwd(x, g, B, H, W, border, dx, NULL, 1) == 0);
                CHECK(oracle_f64_bwd_scale(x, g, B, H, W, border, A, NULL, 1) == 0);
                for (size_t i = 0; i < nout; ++i) CHECK(isfinite(M[i]) && M[i] >= 0 && sf[i] >= 0);
                for (size_t i = 0; i < nin; ++i) CHECK(isfinite(dx[i]) && fabs(dx[i]) <= A[i] + 1e-12);
                free(x);
                free(g);
                free(M);
                free(D);
                free(dx);
                free(A);
                free(sf);
            }
    double x[4] = {0, 0, 0, 0};
    CHECK(oracle_f64_fwd(NULL, 1, 2, 2, 0, x, NULL, NULL, 1) != 0);
    CHECK(oracle_f64_bwd(x, NULL, 1, 2, 2, 0, x, NULL, 1) != 0);
    CHECK(oracle_f64_fwd_scale(x, -1, 2, 2, 0, x, NULL, 1) != 0);
}

static void rounding(void)
{
    for (int64_t S = 0; S <= 70000; ++S) {
        const int64_t r = oracle_round_sqrt(S);
        /* r = round(sqrt(S)) <=> (r - 1/2)^2 < S < (r + 1/2)^2, i.e. r^2 - r < S <= r^2 + r
           for r >= 1, and S = 0 for r = 0 */
        CHECK(r == 0 ? S == 0 : (r * r - r < S && S <= r * r + r));
    }
    const int64_t big[] = {599270400, 64770, 64771, (int64_t)1 << 40, ((int64_t)1 << 62) - 1};
    for (size_t i = 0; i < sizeof big / sizeof big[0]; ++i) {
        const int64_t r = oracle_round_sqrt(big[i]);
        CHECK(r >= 0 && r * r - r < big[i] && big[i] <= r * r + r);
    }
    CHECK(oracle_round_sqrt(-1) == -1);
    CHECK(oracle_round_sqrt(INT64_MAX) == -1);
}

int main(void)
{
    u8_shapes();
    f64_shapes();
    rounding();
    if (failures) {
        fprintf(stderr, "%d oracle check(s) failed\n", failures);
        return 1;
    }
    printf("oracle checks ok\n");
    return 0;
}
