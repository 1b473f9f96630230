// fp32 forward and adjoint of the four-directional 5x5 Sobel magnitude.
//
// Not in the paper: an fp32 version of Eq. (sobel5_1) + Eq. (sobel5_2) for
// use as a differentiable edge loss.  The four responses are evaluated in
// the factored form of the uint8 path (rows first for Gx and Gd-, columns
// first for Gy and Gd+, with K_d+- = K_d +- K_dt as in Eq. (sobel5_kd+-)),
// and every first-stage term is a difference of two pixels, so a flat 5x5
// window yields exactly zero in all four responses and M = 0.
//
// With Gd+ and Gd-, S = Gx^2 + Gy^2 + (Gd+^2 + Gd-^2)/2 and
//   dM/dGx = Gx/M, dM/dGy = Gy/M, dM/dGd+ = Gd+/(2M), dM/dGd- = Gd-/(2M).
// The adjoint of a correlation with K is a correlation with rot180(K) = -K
// (every filter here is antisymmetric under a half turn), so the padded
// adjoint is P = -(Gx-structure(w_x) + Gy-structure(w_y) + Gd+-structure(w_p)
// + Gd--structure(w_m)) applied to the weighted planes w, zero outside the
// image.  The replicate border then folds P at the two virtual rows and
// columns beyond each edge onto that edge.

#include "internal.hpp"

namespace s4x5 {
namespace {

constexpr int TX = 32, TY = 32;   // output tile per workgroup
constexpr int NT = 256;           // threads per workgroup

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Row-first responses of a 5x5 window: Gx and Gd-.
__device__ __forceinline__ void rows_first(const float (&x)[5][5], float &Gx, float &Gm)
{
    float hr[5], hs[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        hs[r] = x[r][3] - x[r][1];
        hr[r] = (x[r][4] - x[r][0]) + 2.0f * hs[r];
    }
    const float x1 = hr[0] + hr[4], x2 = hr[1] + hr[3];
    Gx = x1 + 4.0f * x2 + 6.0f * hr[2];
    Gm = 6.0f * (x1 + x2) + 2.0f * hr[2] - 10.0f * (hs[0] + hs[4]) + 12.0f * hs[2];
}

// Column-first responses of a 5x5 window: Gy and Gd+.
__device__ __forceinline__ void cols_first(const float (&x)[5][5], float &Gy, float &Gp)
{
    float vr[5], vs[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        vs[c] = x[3][c] - x[1][c];
        vr[c] = (x[4][c] - x[0][c]) + 2.0f * vs[c];
    }
    const float y1 = vr[0] + vr[4], y2 = vr[1] + vr[3];
    Gy = y1 + 4.0f * y2 + 6.0f * vr[2];
    Gp = 6.0f * (y1 + y2) + 2.0f * vr[2] - 10.0f * (vs[0] + vs[4]) + 12.0f * vs[2];
}

template <int LD>
__device__ __forceinline__ void window(const float *lds, int r0, int c0, float (&x)[5][5])
{
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) x[i][j] = lds[(r0 + i) * LD + c0 + j];
}

__device__ __forceinline__ float mag_of(float Gx, float Gy, float Gp, float Gm)
{
    const float s = Gx * Gx + Gy * Gy + 0.5f * (Gp * Gp + Gm * Gm);
    return sqrtf(s);
}

// ---------------------------------------------------------------- forward
// Tile TY x TX outputs; LDS holds the (TY+4) x (TX+4) input window.
constexpr int FLD = TX + 4;

__global__ __launch_bounds__(NT) void k_f32_fwd(F32Args a)
{
    __shared__ float xs[(TY + 4) * FLD];
    const int b = blockIdx.z;
    const int ox0 = blockIdx.x * TX, oy0 = blockIdx.y * TY;
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride;
    // input window rows/cols: centre (oy + off) -2 .. +2
    const int iy0 = oy0 + a.off - 2, ix0 = ox0 + a.off - 2;
    for (int t = threadIdx.x; t < (TY + 4) * FLD; t += NT) {
        const int r = t / FLD, c = t % FLD;
        const int y = clampi(iy0 + r, 0, a.H - 1), x = clampi(ix0 + c, 0, a.W - 1);
        xs[t] = reinterpret_cast<const float *>(src + (int64_t)y * a.src_pitch)[x];
    }
    __syncthreads();
    const int tx = threadIdx.x % TX, tg = threadIdx.x / TX;   // 8 groups of 4 rows
    char *out = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride;
#pragma unroll
    for (int k = 0; k < TY / 8; ++k) {
        const int ty = tg * (TY / 8) + k;
        const int oy = oy0 + ty, ox = ox0 + tx;
        if (oy >= a.Ho || ox >= a.Wo) continue;
        float x[5][5];
        window<FLD>(xs, ty, tx, x);
        float Gx, Gy, Gp, Gm;
        rows_first(x, Gx, Gm);
        cols_first(x, Gy, Gp);
        reinterpret_cast<float *>(out + (int64_t)oy * a.out_pitch)[ox] = mag_of(Gx, Gy, Gp, Gm);
    }
}

// ---------------------------------------------------------------- adjoint
// Tile TY x TX of grad_src (input coordinates).  LDS: x on tile +- 6,
// the four weighted planes w on tile +- 4.
constexpr int XR = 6, WR = 4;
constexpr int XLD = TX + 2 * XR, XROWS = TY + 2 * XR;
constexpr int WLD = TX + 2 * WR, WROWS = TY + 2 * WR;

// P(p') at input-coordinate point (py, px) relative to the w planes' origin.
__device__ __forceinline__ float padded_adjoint(const float *wx, const float *wy, const float *wp,
                                                const float *wm, int r, int c)
{
    float win[5][5], g0, g1, acc;
    window<WLD>(wx, r - 2, c - 2, win);
    rows_first(win, g0, g1);
    acc = g0;
    window<WLD>(wm, r - 2, c - 2, win);
    rows_first(win, g0, g1);
    acc += g1;
    window<WLD>(wy, r - 2, c - 2, win);
    cols_first(win, g0, g1);
    acc += g0;
    window<WLD>(wp, r - 2, c - 2, win);
    cols_first(win, g0, g1);
    acc += g1;
    return -acc;
}

__global__ __launch_bounds__(NT) void k_f32_bwd(F32Args a)
{
    __shared__ float xs[XROWS * XLD];
    __shared__ float wpl[4][WROWS * WLD];
    const int b = blockIdx.z;
    const int tx0 = blockIdx.x * TX, ty0 = blockIdx.y * TY;   // input coordinates
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride;
    const char *gr = reinterpret_cast<const char *>(a.grad) + (int64_t)b * a.g_bstride;

    // 1. x on rows ty0-6 .. ty0+TY+5 (clamped: the forward's replicate read)
    for (int t = threadIdx.x; t < XROWS * XLD; t += NT) {
        const int r = t / XLD, c = t % XLD;
        const int y = clampi(ty0 - XR + r, 0, a.H - 1), x = clampi(tx0 - XR + c, 0, a.W - 1);
        xs[t] = reinterpret_cast<const float *>(src + (int64_t)y * a.src_pitch)[x];
    }
    __syncthreads();

    // 2. weighted planes at input-coordinate centres q on tile +- 4; zero where q
    //    is not the centre of an output pixel
    for (int t = threadIdx.x; t < WROWS * WLD; t += NT) {
        const int r = t / WLD, c = t % WLD;
        const int qy = ty0 - WR + r, qx = tx0 - WR + c;     // centre, input coords
        const int oy = qy - a.off, ox = qx - a.off;          // output pixel
        float vx = 0.f, vy = 0.f, vp = 0.f, vm = 0.f;
        if (oy >= 0 && oy < a.Ho && ox >= 0 && ox < a.Wo) {
            float x[5][5];
            window<XLD>(xs, r + (XR - WR) - 2, c + (XR - WR) - 2, x);
            float Gx, Gy, Gp, Gm;
            rows_first(x, Gx, Gm);
            cols_first(x, Gy, Gp);
            const float M = mag_of(Gx, Gy, Gp, Gm);
            if (M > 0.f) {
                const float g = reinterpret_cast<const float *>(gr + (int64_t)oy * a.g_pitch)[ox];
                const float s = g / M;
                vx = s * Gx;
                vy = s * Gy;
                vp = 0.5f * s * Gp;
                vm = 0.5f * s * Gm;
            }
        }
        wpl[0][t] = vx;
        wpl[1][t] = vy;
        wpl[2][t] = vp;
        wpl[3][t] = vm;
    }
    __syncthreads();

    // 3. dx(p) = sum of P(p') over the p' that the border clamps onto p
    char *dst = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride;
    const bool rep = a.off == 0;
    for (int t = threadIdx.x; t < TY * TX; t += NT) {
        const int ty = t / TX, tx = t % TX;
        const int y = ty0 + ty, x = tx0 + tx;
        if (y >= a.H || x >= a.W) continue;
        const int r = ty + WR, c = tx + WR;
        float acc = 0.f;
        const int ylo = (rep && y == 0) ? -2 : 0, yhi = (rep && y == a.H - 1) ? 2 : 0;
        const int xlo = (rep && x == 0) ? -2 : 0, xhi = (rep && x == a.W - 1) ? 2 : 0;
        for (int dy = ylo; dy <= yhi; ++dy)
            for (int dx = xlo; dx <= xhi; ++dx) {
                // virtual points beyond the edge only (plus p itself)
                if (dy != 0 && !((dy < 0 && y == 0) || (dy > 0 && y == a.H - 1))) continue;
                if (dx != 0 && !((dx < 0 && x == 0) || (dx > 0 && x == a.W - 1))) continue;
                acc += padded_adjoint(wpl[0], wpl[1], wpl[2], wpl[3], r + dy, c + dx);
            }
        reinterpret_cast<float *>(dst + (int64_t)y * a.out_pitch)[x] = acc;
    }
}

}  // namespace

hipError_t launch_f32_fwd(const F32Args &a, hipStream_t st)
{
    if (a.B <= 0) return hipSuccess;
    dim3 grid((a.Wo + TX - 1) / TX, (a.Ho + TY - 1) / TY, a.B);
    hipLaunchKernelGGL(k_f32_fwd, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_f32_bwd(const F32Args &a, hipStream_t st)
{
    if (a.B <= 0) return hipSuccess;
    dim3 grid((a.W + TX - 1) / TX, (a.H + TY - 1) / TY, a.B);
    hipLaunchKernelGGL(k_f32_bwd, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

}  // namespace s4x5
