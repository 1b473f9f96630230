/*
 * Plain CPU oracle for the four-directional 5x5 Sobel operator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * library and its Python binding never do.  It shares no code, header, table
 * or helper with the GPU path.
 *
 * What it computes (Chang et al., "Multi-directional Sobel operator kernel on
 * GPUs", Sec. 3.1):
 *   - four fixed 5x5 integer filters, Eq. (sobel5_1): 0 deg (Gx), 45 deg (Gd),
 *     90 deg (Gy), 135 deg (Gdt), each applied to every pixel;
 *   - the root-sum-of-squares magnitude, Eq. (sobel5_2);
 *   - the two-directional operators the paper compares against: the 3x3
 *     Sobel pair of Eq. (sobel3_1) with Eq. (sobel3_2), and the 0 / 90 deg
 *     pair of Eq. (sobel5_1) alone (oracle_u8_2dir).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - the filters are applied as a correlation: tap (i, j) of the printed
 *     matrix multiplies the pixel at row offset i-2 and column offset j-2
 *     (this is how the paper's own row filters, Eq. (Fx) and Eq. (Gd+), index
 *     the pixels in Sec. 4.3);
 *   - border REPLICATE (clamp-to-edge) keeps the output at HxW; border VALID
 *     is the paper-native shrink by 2r = 4 rows and columns (Sec. 4.3, data
 *     flow), out(y, x) = full(y + 2, x + 2); ZERO (pixels outside read 0)
 *     and REFLECT101 (mirror about the edge pixel, see border_index) keep
 *     H x W as well;
 *   - the uint8 magnitude is min(255, round-to-nearest(sqrt(S))), computed
 *     exactly in integers (ties cannot occur for integer S);
 *   - the real-valued path (not in the paper) is the same correlation in fp64,
 *     summed as differences of opposite taps (see responses_f64), with
 *     M = sqrt(S); its adjoint is the literal scatter of every tap
 *     through the same border index (a tap that reads 0 under ZERO
 *     scatters nothing), with the subgradient u_k = 0 where M = 0.
 *
 * Every loop below is the plain definition: no separable factoring, no
 * blocking, no reordering beyond pairing opposite taps in the real-valued
 * path (see responses_f64).  OpenMP only splits independent output rows (or,
 * for the adjoint, independent images).
 */
#include <stddef.h>
#include <stdint.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
static int omp_default_threads(void) { return omp_get_max_threads(); }
#else
static int omp_default_threads(void) { return 1; }
#endif

#define OR_OK 0
#define OR_EINVAL 1

#define OR_BORDER_REPLICATE 0
#define OR_BORDER_VALID 1
#define OR_BORDER_ZERO 2
#define OR_BORDER_REFLECT101 3

/* Eq. (sobel5_1), typed in row by row from the printed matrices, in plane
 * order 0 deg (Gx), 45 deg (Gd), 90 deg (Gy), 135 deg (Gdt). */
static const int32_t K_PAPER[4][5][5] = {
    /* Gx */
    {{-1, -2, 0, 2, 1},
     {-4, -8, 0, 8, 4},
     {-6, -12, 0, 12, 6},
     {-4, -8, 0, 8, 4},
     {-1, -2, 0, 2, 1}},
    /* Gd */
    {{-6, -4, -1, -2, 0},
     {-4, -12, -8, 0, 2},
     {-1, -8, 0, 8, 1},
     {-2, 0, 8, 12, 4},
     {0, 2, 1, 4, 6}},
    /* Gy */
    {{-1, -4, -6, -4, -1},
     {-2, -8, -12, -8, -2},
     {0, 0, 0, 0, 0},
     {2, 8, 12, 8, 2},
     {1, 4, 6, 4, 1}},
    /* Gdt */
    {{0, -2, -1, -4, -6},
     {2, 0, -8, -12, -4},
     {1, 8, 0, -8, -1},
     {4, 12, 8, 0, -2},
     {6, 4, 1, 2, 0}},
};

/* Copy of the literal table, so that tests can compare it with the paper's
 * second printing of the same weights (Eq. (sobel5_param)). */
void oracle_weights(int32_t *out /* [4][5][5] */)
{
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j)
                out[(k * 5 + i) * 5 + j] = K_PAPER[k][i][j];
}

static const int32_t *pick_weights(const int32_t *w)
{
    return w ? w : &K_PAPER[0][0][0];
}

static inline long clampl(long v, long lo, long hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/*
 * Index of the pixel that stands in for position i of an axis of n pixels
 * (0 <= i < n maps to itself), or -1 where the border reads zero.
 *   REPLICATE / VALID : the nearest pixel (clamp to [0, n-1]);
 *   ZERO              : -1 (the pixel reads 0);
 *   REFLECT101        : the mirror image about the edge pixel, without
 *                       repeating it (..., 2, 1 | 0, 1, ..., n-1 | n-2, ...),
 *                       applied until the index lands inside: the extended
 *                       axis is periodic with period 2(n-1); n = 1 gives 0.
 */
static long border_index(long i, long n, int border)
{
    if (i >= 0 && i < n)
        return i;
    if (border == OR_BORDER_ZERO)
        return -1;
    if (border == OR_BORDER_REFLECT101) {
        if (n == 1)
            return 0;
        const long p = 2 * (n - 1);
        long m = i % p;
        if (m < 0)
            m += p;
        return m < n ? m : p - m;
    }
    return clampl(i, 0, n - 1);
}

/* Pixel value at (y, x) under the border rule. */
static inline int64_t pixel_u8(const uint8_t *src, int W, int H, long pitch, int border, long y, long x)
{
    const long yy = border_index(y, H, border), xx = border_index(x, W, border);
    return (yy < 0 || xx < 0) ? 0 : (int64_t)src[yy * pitch + xx];
}

/* round(sqrt(S)) for S >= 0, exactly, by integer square root.
 * r = floor(sqrt(S)); sqrt(S) >= r + 1/2  <=>  S > r*r + r (S integer). */
static int64_t round_sqrt_i64(int64_t S)
{
    int64_t r = (int64_t)sqrt((double)S);
    while (r > 0 && r * r > S)
        --r;
    while ((r + 1) * (r + 1) <= S)
        ++r;
    return (S - r * r > r) ? r + 1 : r;
}

/* Exported for tests: -1 outside [0, 2^62), where (r + 1)^2 would leave int64. */
int64_t oracle_round_sqrt(int64_t S) { return (S < 0 || S >= ((int64_t)1 << 62)) ? -1 : round_sqrt_i64(S); }

/* Output size under a border rule. */
static int out_dims(int W, int H, int border, int *Wo, int *Ho)
{
    if (W <= 0 || H <= 0)
        return OR_EINVAL;
    if (border == OR_BORDER_REPLICATE || border == OR_BORDER_ZERO || border == OR_BORDER_REFLECT101) {
        *Wo = W;
        *Ho = H;
    } else if (border == OR_BORDER_VALID) {
        if (W < 5 || H < 5)
            return OR_EINVAL;
        *Wo = W - 4;
        *Ho = H - 4;
    } else {
        return OR_EINVAL;
    }
    return OR_OK;
}

/* The four responses at output pixel (yo, xo), in int64. */
static void responses_u8(const uint8_t *src, int W, int H, long pitch, int border,
                         const int32_t *K, long yo, long xo, int64_t G[4])
{
    long yc = yo, xc = xo;
    if (border == OR_BORDER_VALID) {
        yc += 2;
        xc += 2;
    }
    for (int k = 0; k < 4; ++k) {
        int64_t acc = 0;
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j)
                acc += (int64_t)K[(k * 5 + i) * 5 + j] * pixel_u8(src, W, H, pitch, border, yc + i - 2, xc + j - 2);
        G[k] = acc;
    }
}

/*
 * uint8 image -> uint8 magnitude and/or four int32 directional planes.
 *   src        : H rows of W bytes, row r starting at src + r*pitch.
 *   mag        : Ho rows of Wo bytes at mag + r*mag_pitch (may be NULL).
 *   dir        : four planes of Ho*Wo int32, plane k at dir + k*Ho*Wo, row-major
 *                (may be NULL).
 *   weights    : 4*25 int32 in plane order, or NULL for Eq. (sobel5_1).
 *   nthreads   : OpenMP threads (<= 0: runtime default).
 */
int oracle_u8(const uint8_t *src, int W, int H, long pitch, int border,
              uint8_t *mag, long mag_pitch, int32_t *dir,
              const int32_t *weights, int nthreads)
{
    int Wo, Ho;
    if (!src || pitch < W || out_dims(W, H, border, &Wo, &Ho) != OR_OK)
        return OR_EINVAL;
    if (mag && mag_pitch < Wo)
        return OR_EINVAL;
    const int32_t *K = pick_weights(weights);
    const long plane = (long)Wo * Ho;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_default_threads())
    for (long y = 0; y < Ho; ++y) {
        for (long x = 0; x < Wo; ++x) {
            int64_t G[4];
            responses_u8(src, W, H, pitch, border, K, y, x, G);
            if (dir)
                for (int k = 0; k < 4; ++k)
                    dir[k * plane + y * Wo + x] = (int32_t)G[k];
            if (mag) {
                int64_t S = G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + G[3] * G[3];
                int64_t r = round_sqrt_i64(S);
                mag[y * mag_pitch + x] = (uint8_t)(r > 255 ? 255 : r);
            }
        }
    }
    return OR_OK;
}

/* Same as oracle_u8, but only at n listed output pixels (ys[i], xs[i]).
 * mag: n bytes (may be NULL); dir: n*4 int32, pixel-major (may be NULL). */
int oracle_u8_points(const uint8_t *src, int W, int H, long pitch, int border,
                     const int32_t *ys, const int32_t *xs, long n,
                     uint8_t *mag, int32_t *dir, const int32_t *weights)
{
    int Wo, Ho;
    if (!src || pitch < W || out_dims(W, H, border, &Wo, &Ho) != OR_OK)
        return OR_EINVAL;
    const int32_t *K = pick_weights(weights);
    for (long i = 0; i < n; ++i) {
        if (ys[i] < 0 || ys[i] >= Ho || xs[i] < 0 || xs[i] >= Wo)
            return OR_EINVAL;
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        int64_t G[4];
        responses_u8(src, W, H, pitch, border, K, ys[i], xs[i], G);
        if (dir)
            for (int k = 0; k < 4; ++k)
                dir[i * 4 + k] = (int32_t)G[k];
        if (mag) {
            int64_t S = G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + G[3] * G[3];
            int64_t r = round_sqrt_i64(S);
            mag[i] = (uint8_t)(r > 255 ? 255 : r);
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Real-valued path (fp64): forward magnitude and its exact adjoint.       */
/* Images are B contiguous HxW planes; outputs are B contiguous HoxWo.     */
/* ---------------------------------------------------------------------- */

/*
 * The four responses at output pixel (yo, xo), in fp64.
 *
 * Sec. 3.1 notes that a Sobel filter whose two sides carry opposite weights
 * computes differences between the two sides.  All filters here satisfy
 * K[4-i][4-j] = -K[i][j], so each response is accumulated as
 * K[i][j] * (I(p + o) - I(p - o)) over the 12 taps before the centre, plus the
 * centre tap.  This is the same sum regrouped, and it makes a flat window give
 * exactly G = 0 for any real input (a direct sum of 0.3 * K[i][j] does not
 * cancel exactly in floating point, which would turn the rounding residue into
 * a spurious unit gradient direction G/M).  A weight table that is not
 * antisymmetric falls back to the direct sum term by term.
 */
/* Real-valued pixel at (y, x) under the border rule (0 where ZERO reads
 * outside the image). */
static inline double pixel_f64(const double *x, int W, int H, int border, long y, long xx)
{
    const long yy = border_index(y, H, border), xi = border_index(xx, W, border);
    return (yy < 0 || xi < 0) ? 0.0 : x[yy * W + xi];
}

static void responses_f64(const double *x, int W, int H, int border,
                          const int32_t *K, long yo, long xo, double G[4])
{
    long yc = yo, xc = xo;
    if (border == OR_BORDER_VALID) {
        yc += 2;
        xc += 2;
    }
    for (int k = 0; k < 4; ++k) {
        const int32_t *Kk = K + k * 25;
        double acc = 0.0;
        for (int t = 0; t < 12; ++t) {
            int i = t / 5, j = t % 5;
            int ii = 4 - i, jj = 4 - j;
            double a = pixel_f64(x, W, H, border, yc + i - 2, xc + j - 2);
            double b = pixel_f64(x, W, H, border, yc + ii - 2, xc + jj - 2);
            if (Kk[ii * 5 + jj] == -Kk[i * 5 + j])
                acc += (double)Kk[i * 5 + j] * (a - b);
            else
                acc += (double)Kk[i * 5 + j] * a + (double)Kk[ii * 5 + jj] * b;
        }
        acc += (double)Kk[12] * pixel_f64(x, W, H, border, yc, xc);
        G[k] = acc;
    }
}

/* mag: B*Ho*Wo (may be NULL); dir: B*4*Ho*Wo, plane k of image b at
 * dir + (b*4 + k)*Ho*Wo (may be NULL). */
int oracle_f64_fwd(const double *x, int B, int H, int W, int border,
                   double *mag, double *dir, const int32_t *weights, int nthreads)
{
    int Wo, Ho;
    if (!x || B < 0 || out_dims(W, H, border, &Wo, &Ho) != OR_OK)
        return OR_EINVAL;
    const int32_t *K = pick_weights(weights);
    const long plane_in = (long)W * H, plane_out = (long)Wo * Ho;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads > 0 ? nthreads : omp_default_threads())
    for (long b = 0; b < B; ++b) {
        for (long y = 0; y < Ho; ++y) {
            for (long xo = 0; xo < Wo; ++xo) {
                double G[4];
                responses_f64(x + b * plane_in, W, H, border, K, y, xo, G);
                if (dir)
                    for (int k = 0; k < 4; ++k)
                        dir[(b * 4 + k) * plane_out + y * Wo + xo] = G[k];
                if (mag)
                    mag[b * plane_out + y * Wo + xo] =
                        sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + G[3] * G[3]);
            }
        }
    }
    return OR_OK;
}

/*
 * Adjoint of the magnitude map: given dL/dM = g (B*Ho*Wo), writes
 * dL/dx (B*H*W, overwritten).  For every output pixel q with M(q) > 0 and
 * every direction k, u_k(q) = g(q) * G_k(q) / M(q); then every tap (i, j) of
 * filter k adds K_k[i][j] * u_k(q) to the input pixel it read in the forward
 * pass (the same clamped index).  Where M(q) = 0 nothing is added.
 *
 * With absmode set, it adds |K_k[i][j]| * |u_k(q)| instead: the magnitude of
 * the sum's terms at every input pixel, which scales the rounding error any
 * summation order can make (used for test tolerances).
 */
static int bwd_impl(const double *x, const double *g, int B, int H, int W, int border,
                    double *dx, const int32_t *weights, int nthreads, int absmode)
{
    int Wo, Ho;
    if (!x || !g || !dx || B < 0 || out_dims(W, H, border, &Wo, &Ho) != OR_OK)
        return OR_EINVAL;
    const int32_t *K = pick_weights(weights);
    const long plane_in = (long)W * H, plane_out = (long)Wo * Ho;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_default_threads())
    for (long b = 0; b < B; ++b) {
        const double *xb = x + b * plane_in;
        const double *gb = g + b * plane_out;
        double *db = dx + b * plane_in;
        for (long p = 0; p < plane_in; ++p)
            db[p] = 0.0;
        for (long y = 0; y < Ho; ++y) {
            for (long xo = 0; xo < Wo; ++xo) {
                double G[4];
                responses_f64(xb, W, H, border, K, y, xo, G);
                double M = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + G[3] * G[3]);
                if (!(M > 0.0))
                    continue;
                long yc = y, xc = xo;
                if (border == OR_BORDER_VALID) {
                    yc += 2;
                    xc += 2;
                }
                for (int k = 0; k < 4; ++k) {
                    double u = gb[y * Wo + xo] * G[k] / M;
                    if (absmode)
                        u = fabs(u);
                    for (int i = 0; i < 5; ++i) {
                        long yy = border_index(yc + i - 2, H, border);
                        for (int j = 0; j < 5; ++j) {
                            long xx = border_index(xc + j - 2, W, border);
                            if (yy < 0 || xx < 0)
                                continue;   /* ZERO: the tap read a constant */
                            double w = (double)K[(k * 5 + i) * 5 + j];
                            db[yy * W + xx] += (absmode ? fabs(w) : w) * u;
                        }
                    }
                }
            }
        }
    }
    return OR_OK;
}

int oracle_f64_bwd(const double *x, const double *g, int B, int H, int W, int border,
                   double *dx, const int32_t *weights, int nthreads)
{
    return bwd_impl(x, g, B, H, W, border, dx, weights, nthreads, 0);
}

int oracle_f64_bwd_scale(const double *x, const double *g, int B, int H, int W, int border,
                         double *A, const int32_t *weights, int nthreads)
{
    return bwd_impl(x, g, B, H, W, border, A, weights, nthreads, 1);
}

/*
 * Scale of the forward's rounding error at every output pixel:
 * max over the four filters of sum_t |K_k[t] * x(tap t)|.
 */
int oracle_f64_fwd_scale(const double *x, int B, int H, int W, int border, double *scale,
                         const int32_t *weights, int nthreads)
{
    int Wo, Ho;
    if (!x || !scale || B < 0 || out_dims(W, H, border, &Wo, &Ho) != OR_OK)
        return OR_EINVAL;
    const int32_t *K = pick_weights(weights);
    const long plane_in = (long)W * H, plane_out = (long)Wo * Ho;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads > 0 ? nthreads : omp_default_threads())
    for (long b = 0; b < B; ++b) {
        for (long y = 0; y < Ho; ++y) {
            for (long xo = 0; xo < Wo; ++xo) {
                long yc = y, xc = xo;
                if (border == OR_BORDER_VALID) {
                    yc += 2;
                    xc += 2;
                }
                double best = 0.0;
                for (int k = 0; k < 4; ++k) {
                    double acc = 0.0;
                    for (int i = 0; i < 5; ++i)
                        for (int j = 0; j < 5; ++j)
                            acc += fabs((double)K[(k * 5 + i) * 5 + j] *
                                        pixel_f64(x + b * plane_in, W, H, border, yc + i - 2, xc + j - 2));
                    if (acc > best)
                        best = acc;
                }
                scale[b * plane_out + y * Wo + xo] = best;
            }
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Two-directional operators: the paper's comparison point.                */
/* ---------------------------------------------------------------------- */

/* Eq. (sobel3_1), typed in from the printed matrices: 0 deg (Gx), 90 deg
 * (Gy).  Applied, like the 5x5 filters, as a correlation: tap (i, j)
 * multiplies the pixel at row offset i-1, column offset j-1. */
static const int32_t K3_PAPER[2][3][3] = {
    {{-1, 0, 1},
     {-2, 0, 2},
     {-1, 0, 1}},
    {{-1, -2, -1},
     {0, 0, 0},
     {1, 2, 1}},
};

/*
 * Two-directional operator on a uint8 image: G = sqrt(Gx^2 + Gy^2),
 * Eq. (sobel3_2).
 *   size 3 : Gx, Gy of Eq. (sobel3_1); radius 1, so VALID shrinks the image
 *            by 2: out(y, x) = full(y + 1, x + 1), W, H >= 3;
 *   size 5 : Gx, Gy of Eq. (sobel5_1) (the 0 and 90 deg filters of the
 *            four-directional operator); radius 2, VALID as for oracle_u8.
 *   REPLICATE clamps every tap's row and column to the image (output H x W).
 *   mag : Ho rows of Wo bytes at mag + r*mag_pitch, min(255, round(sqrt(S)))
 *         (may be NULL);
 *   dir : two int32 planes of Ho*Wo (Gx, then Gy), row-major (may be NULL).
 */
int oracle_u8_2dir(const uint8_t *src, int W, int H, long pitch, int border, int size,
                   uint8_t *mag, long mag_pitch, int32_t *dir, int nthreads)
{
    if (!src || W <= 0 || H <= 0 || pitch < W || (size != 3 && size != 5))
        return OR_EINVAL;
    const int r = size / 2;
    int Wo = W, Ho = H;
    if (border == OR_BORDER_VALID) {
        if (W < size || H < size)
            return OR_EINVAL;
        Wo = W - 2 * r;
        Ho = H - 2 * r;
    } else if (border != OR_BORDER_REPLICATE && border != OR_BORDER_ZERO && border != OR_BORDER_REFLECT101) {
        return OR_EINVAL;
    }
    if (mag && mag_pitch < Wo)
        return OR_EINVAL;
    const long plane = (long)Wo * Ho;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_default_threads())
    for (long y = 0; y < Ho; ++y) {
        for (long x = 0; x < Wo; ++x) {
            const long yc = border == OR_BORDER_VALID ? y + r : y;
            const long xc = border == OR_BORDER_VALID ? x + r : x;
            int64_t G[2];
            for (int k = 0; k < 2; ++k) {
                int64_t acc = 0;
                for (int i = 0; i < size; ++i) {
                    for (int j = 0; j < size; ++j) {
                        const int32_t w = size == 3 ? K3_PAPER[k][i][j] : K_PAPER[2 * k][i][j];
                        acc += (int64_t)w * pixel_u8(src, W, H, pitch, border, yc + i - r, xc + j - r);
                    }
                }
                G[k] = acc;
            }
            if (dir) {
                dir[y * Wo + x] = (int32_t)G[0];
                dir[plane + y * Wo + x] = (int32_t)G[1];
            }
            if (mag) {
                const int64_t rr = round_sqrt_i64(G[0] * G[0] + G[1] * G[1]);
                mag[y * mag_pitch + x] = (uint8_t)(rr > 255 ? 255 : rr);
            }
        }
    }
    return OR_OK;
}
