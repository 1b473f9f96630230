// fp32 forward and adjoint of the four-directional 5x5 Sobel magnitude.
//
// Not in the paper: an fp32 version of Eq. (sobel5_1) + Eq. (sobel5_2) for
// use as a differentiable edge loss.  The four responses are evaluated in
// the factored form of the uint8 path (rows first for Gx and Gd-, columns
// first for Gy and Gd+, with K_d+- = K_d +- K_dt as in Eq. (sobel5_kd+-) and
// the two-term form of Eq. (sobel5_4)), and every first-stage term is a
// difference of two pixels, so a flat 5x5 window yields exactly zero in all
// four responses and M = 0.
//
// With Gd+ and Gd-, S = Gx^2 + Gy^2 + (Gd+^2 + Gd-^2)/2 and
//   dM/dGx = Gx/M, dM/dGy = Gy/M, dM/dGd+ = Gd+/(2M), dM/dGd- = Gd-/(2M).
// The adjoint of a correlation with K is a correlation with rot180(K) = -K
// (every filter here is antisymmetric under a half turn), so on the padded
// domain the adjoint is P = -(K_x * w_x + K_d- * w_m + K_y * w_y + K_d+ * w_p)
// (* = correlation) of the weighted planes w = g dM/dG, zero where no output
// pixel is centred.  The same factoring evaluates it.  The replicate border
// then folds P at the two virtual rows and columns beyond each edge onto
// that edge.
//
// Layout of the work: a wave owns a strip of columns and a range of rows of
// one image.  Each lane holds one column and walks down the rows, keeping
// five-row rings of every stage in registers; the horizontal taps (+-1, +-2
// columns) come from the neighbouring lanes by wave-wide DPP shifts.  A wave
// loads 64 columns and keeps the ones whose whole stencil chain lies inside
// its lanes (forward: 2 lanes of halo per side, adjoint: 6).

#include "internal.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

namespace s4x5 {
namespace {

constexpr int kWavesPerGroup = 4;
constexpr int kHaloF = 2, kOwnF = 64 - 2 * kHaloF;   // forward: 60 columns per wave
constexpr int kHaloB = 6, kOwnB = 64 - 2 * kHaloB;   // adjoint: 52 columns per wave

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// value held by lane + 1 / lane - 1 (wave-wide DPP shift; bound_ctrl gives
// the last / first lane 0, which no kept column uses, and lets the move
// write its destination without first clearing it)
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}

// Row filters of one row across the lanes (Eq. (Fx) and the D term of
// Eq. (Gd-_fast)): hs = v[+1] - v[-1], hr = (v[+2] - v[-2]) + 2 hs.
__device__ __forceinline__ void hfilters(float v, float &hr, float &hs)
{
    const float p1 = from_right(v), m1 = from_left(v);
    const float p2 = from_right(p1), m2 = from_left(m1);
    hs = p1 - m1;
    hr = (p2 - m2) + 2.0f * hs;
}

// c = [1,4,6,4,1] and c'/d combination over five values a0..a4, b0..b4:
//   C  = (a0 + a4) + 4 (a1 + a3) + 6 a2
//   C' = 6 (a0 + a1 + a3 + a4) + 2 a2 - 10 (b0 + b4) + 12 b2
__device__ __forceinline__ float comb_c(float a0, float a1, float a2, float a3, float a4)
{
    return (a0 + a4) + 4.0f * (a1 + a3) + 6.0f * a2;
}
__device__ __forceinline__ float comb_cd(float a0, float a1, float a2, float a3, float a4, float b0, float b2,
                                         float b4)
{
    return 6.0f * ((a0 + a4) + (a1 + a3)) + 2.0f * a2 - 10.0f * (b0 + b4) + 12.0f * b2;
}

// Columns-first pair (Gy, Gd+) at this lane's column from the lane's v_r and
// v_s of the centre row: horizontal combination across lanes.
__device__ __forceinline__ void hcombine(float vr, float vs, float &C, float &Cd)
{
    const float r1 = from_right(vr), l1 = from_left(vr);
    const float r2 = from_right(r1), l2 = from_left(l1);
    const float s1 = from_right(vs), t1 = from_left(vs);
    const float s2 = from_right(s1), t2 = from_left(t1);
    C = comb_c(l2, l1, vr, r1, r2);
    Cd = comb_cd(l2, l1, vr, r1, r2, t2, vs, s2);
}

__device__ __forceinline__ float sum_sq(float Gx, float Gy, float Gp, float Gm)
{
    return Gx * Gx + Gy * Gy + 0.5f * (Gp * Gp + Gm * Gm);
}

// M = sqrt(S) by the hardware square root (within 1 ulp; below S = 2^-100,
// i.e. M < 1e-15, its error is an absolute one far under the tolerance).
__device__ __forceinline__ float mag_of(float Gx, float Gy, float Gp, float Gm)
{
    return __builtin_amdgcn_sqrtf(sum_sq(Gx, Gy, Gp, Gm));
}

// g / M = g / sqrt(S) for S > 0, 0 for S = 0: the hardware reciprocal square
// root (within 1 ulp) for normal S, the exact library route below 2^-100.
__device__ __forceinline__ float scale_of(float g, float S)
{
    return S >= 0x1p-100f ? g * __builtin_amdgcn_rsqf(S) : (S > 0.f ? g / sqrtf(S) : 0.f);
}

template <int P>
using Ph = std::integral_constant<int, P>;

// ---------------------------------------------------------------- forward
// Wave (image b, strip s, chunk k): output columns [s*60, s*60+60), output
// rows [o0, o1).  Lane l holds output column s*60 - 2 + l (centre column
// + OFF).  Step t loads input row o0 + OFF - 2 + t and, from t = 4 on,
// finishes output row o0 + t - 4.
template <int OFF>
__global__ __launch_bounds__(64 * kWavesPerGroup) void k_f32_fwd(F32Args a, int nstrip, int nchunk)
{
    const int wave = blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per_img = nstrip * nchunk;
    if (wave >= a.B * per_img) return;
    const int b = wave / per_img, rem = wave % per_img;
    const int s = rem % nstrip, k = rem / nstrip;
    const int o0 = (int)((int64_t)k * a.Ho / nchunk), o1 = (int)((int64_t)(k + 1) * a.Ho / nchunk);
    if (o1 <= o0) return;
    const int lane = threadIdx.x & 63;
    const int ox = s * kOwnF - kHaloF + lane;
    const bool keep = lane >= kHaloF && lane < kHaloF + kOwnF && ox < a.Wo;
    const int xc = clampi(ox + OFF, 0, a.W - 1);
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride + (int64_t)xc * 4;
    char *dst = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride + (int64_t)(ox < 0 ? 0 : ox) * 4;
    const int r0 = o0 + OFF - 2;
    auto ld = [&](int t) {
        return *reinterpret_cast<const float *>(src + (int64_t)clampi(r0 + t, 0, a.H - 1) * a.src_pitch);
    };
    const int T = o1 - o0 + 4;

    float X[5], HR[5], HS[5];
    float pf[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) X[i] = HR[i] = HS[i] = pf[i] = 0.f;
    constexpr int PD = 3;   // rows loaded ahead
#pragma unroll
    for (int t = 0; t < PD; ++t) pf[t] = ld(t);

    auto step = [&](int t, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int s0 = (p + 1) % 5, s1 = (p + 2) % 5, s2 = (p + 3) % 5, s3 = (p + 4) % 5, s4 = p;
        pf[(p + PD) % 5] = ld(min(t + PD, T - 1));
        const float x = pf[p];
        X[s4] = x;
        hfilters(x, HR[s4], HS[s4]);
        if (t < 4) return;
        const float Gx = comb_c(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4]);
        const float Gm = comb_cd(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4]);
        const float vs = X[s3] - X[s1];
        const float vr = (X[s4] - X[s0]) + 2.0f * vs;
        float Gy, Gp;
        hcombine(vr, vs, Gy, Gp);
        if (keep) *reinterpret_cast<float *>(dst + (int64_t)(o0 + t - 4) * a.out_pitch) = mag_of(Gx, Gy, Gp, Gm);
    };
    for (int t = 0; t < T; t += 5) {
        step(t, Ph<0>{});
        if (t + 1 >= T) break;
        step(t + 1, Ph<1>{});
        if (t + 2 >= T) break;
        step(t + 2, Ph<2>{});
        if (t + 3 >= T) break;
        step(t + 3, Ph<3>{});
        if (t + 4 >= T) break;
        step(t + 4, Ph<4>{});
    }
}

// ---------------------------------------------------------------- adjoint
// Wave (image b, strip s, chunk k): grad_src columns [s*52, s*52+52), rows
// [X0, X1).  Lane l holds input column c = s*52 - 6 + l.  Step t loads input
// row r = X0 - 6 + t; the centre row q = r - 2 gets its weighted planes w;
// the padded adjoint row p = r - 4 is complete and is folded / stored.
template <int OFF>
__global__ __launch_bounds__(64 * kWavesPerGroup) void k_f32_bwd(F32Args a, int nstrip, int nchunk)
{
    const int wave = blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per_img = nstrip * nchunk;
    if (wave >= a.B * per_img) return;
    const int b = wave / per_img, rem = wave % per_img;
    const int s = rem % nstrip, k = rem / nstrip;
    const int X0 = (int)((int64_t)k * a.H / nchunk), X1 = (int)((int64_t)(k + 1) * a.H / nchunk);
    if (X1 <= X0) return;
    const int lane = threadIdx.x & 63;
    const int c = s * kOwnB - kHaloB + lane;                  // input column of the lane
    const bool keep = lane >= kHaloB && lane < kHaloB + kOwnB && c < a.W;
    const bool ocol = c - OFF >= 0 && c - OFF < a.Wo;          // an output pixel is centred here
    const int xc = clampi(c, 0, a.W - 1);
    const int gc = clampi(c - OFF, 0, a.Wo - 1);
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride + (int64_t)xc * 4;
    const char *gr = reinterpret_cast<const char *>(a.grad) + (int64_t)b * a.g_bstride + (int64_t)gc * 4;
    char *dst = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride + (int64_t)(c < 0 ? 0 : c) * 4;
    const int r0 = X0 - 6;
    const int T = X1 - X0 + 12;
    // replicate border: fold the virtual columns -2, -1 onto 0 and W, W+1
    // onto W-1 (wave-uniform: does this strip hold column 0 / W-1?)
    const bool rep = OFF == 0;
    const bool fold_l = rep && s == 0;
    const bool fold_r = rep && s * kOwnB + kOwnB >= a.W;

    auto ldx = [&](int t) {
        return *reinterpret_cast<const float *>(src + (int64_t)clampi(r0 + t, 0, a.H - 1) * a.src_pitch);
    };
    // grad of the output row whose centre is input row r0 + t - 2 (0 outside)
    auto ldg = [&](int t) {
        const int o = r0 + t - 2 - OFF;
        float v = 0.f;
        if (o >= 0 && o < a.Ho) v = *reinterpret_cast<const float *>(gr + (int64_t)o * a.g_pitch);
        return ocol ? v : 0.f;
    };

    // rings (slot = step mod 5): input rows, their row filters, centre-row
    // planes w_y, w_p, and the row filters of w_x, w_m
    float X[5], HR[5], HS[5], WY[5], WP[5], AX[5], AM[5], AS[5];
    float pfx[5], pfg[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) X[i] = HR[i] = HS[i] = WY[i] = WP[i] = AX[i] = AM[i] = AS[i] = pfx[i] = pfg[i] = 0.f;
    constexpr int PD = 3;
#pragma unroll
    for (int t = 0; t < PD; ++t) {
        pfx[t] = ldx(t);
        pfg[t] = ldg(t);
    }
    float acc_top = 0.f, acc_bot = 0.f;

    auto store = [&](int row, float v) {
        if (fold_l) {
            const float l1 = from_left(v), l2 = from_left(l1);
            if (c == 0) v += l1 + l2;
        }
        if (fold_r) {
            const float r1 = from_right(v), r2 = from_right(r1);
            if (c == a.W - 1) v += r1 + r2;
        }
        if (keep) *reinterpret_cast<float *>(dst + (int64_t)row * a.out_pitch) = v;
    };

    auto step = [&](int t, auto phase) {
        constexpr int p = decltype(phase)::value;
        // input rows t-4 .. t live in slots (p+1)%5 .. p
        constexpr int s0 = (p + 1) % 5, s1 = (p + 2) % 5, s2 = (p + 3) % 5, s3 = (p + 4) % 5, s4 = p;
        pfx[(p + PD) % 5] = ldx(min(t + PD, T - 1));
        pfg[(p + PD) % 5] = ldg(min(t + PD, T - 1));
        const float x = pfx[p];
        X[s4] = x;
        hfilters(x, HR[s4], HS[s4]);
        // centre row q = r - 2 (slot s2 of the input rings)
        const float Gx = comb_c(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4]);
        const float Gm = comb_cd(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4]);
        const float vs = X[s3] - X[s1];
        const float vr = (X[s4] - X[s0]) + 2.0f * vs;
        float Gy, Gp;
        hcombine(vr, vs, Gy, Gp);
        const float gq = pfg[p];                 // grad of the output row centred on q
        const float sc = scale_of(gq, sum_sq(Gx, Gy, Gp, Gm));
        const float wx = sc * Gx, wy = sc * Gy, wp = 0.5f * sc * Gp, wm = 0.5f * sc * Gm;
        // w rings hold centre rows q-4 .. q in slots (p+1)%5 .. p as well
        WY[s4] = wy;
        WP[s4] = wp;
        float hs_x;   // (only h_r of w_x enters K_x)
        hfilters(wx, AX[s4], hs_x);
        hfilters(wm, AM[s4], AS[s4]);
        // padded adjoint row p_ = q - 2 (slot s2 of the w rings)
        const float A = comb_c(AX[s0], AX[s1], AX[s2], AX[s3], AX[s4]) +
                        comb_cd(AM[s0], AM[s1], AM[s2], AM[s3], AM[s4], AS[s0], AS[s2], AS[s4]);
        const float vsy = WY[s3] - WY[s1];
        const float vry = (WY[s4] - WY[s0]) + 2.0f * vsy;
        const float vsp = WP[s3] - WP[s1];
        const float vrp = (WP[s4] - WP[s0]) + 2.0f * vsp;
        float By, By_d, Bp_c, Bp;   // K_y * w_y = c_h(v_r); K_d+ * w_p = c'_h(v_r) - d_h(v_s)
        hcombine(vry, vsy, By, By_d);
        hcombine(vrp, vsp, Bp_c, Bp);
        const float P = -(A + By + Bp);
        const int pr = r0 + t - 4;               // padded row of P
        if (pr < X0 - 2 || pr >= X1 + 2) return;  // warm-up and rows of other waves
        if (!rep) {
            if (pr >= X0 && pr < X1) store(pr, P);
            return;
        }
        if (pr < 0) {
            acc_top += P;
        } else if (pr >= a.H) {
            acc_bot += P;
            if (pr == a.H + 1) store(a.H - 1, acc_bot);
        } else if (pr >= X0 && pr < X1) {
            float v = P;
            if (pr == 0) v += acc_top;
            if (pr == a.H - 1)
                acc_bot = v;
            else
                store(pr, v);
        }
    };
    for (int t = 0; t < T; t += 5) {
        step(t, Ph<0>{});
        if (t + 1 >= T) break;
        step(t + 1, Ph<1>{});
        if (t + 2 >= T) break;
        step(t + 2, Ph<2>{});
        if (t + 3 >= T) break;
        step(t + 3, Ph<3>{});
        if (t + 4 >= T) break;
        step(t + 4, Ph<4>{});
    }
}

// Resident waves of a kernel (cached per kernel).
int resident_f32(const void *fn)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> cache;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : cache)
        if (e.first == fn) return e.second;
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kWavesPerGroup, 0) != hipSuccess)
        return 0;
    const int w = std::max(1, per_cu) * ncu * kWavesPerGroup;
    cache.emplace_back(fn, w);
    return w;
}

// Row chunks per strip so that the grid is about one round of resident waves
// (at least 32 rows per chunk: the pipeline costs 4 (forward) or 12 (adjoint)
// extra row steps per chunk).
int chunks_for(const void *fn, int64_t strips, int rows)
{
    int slots = resident_f32(fn);
    if (slots <= 0) slots = 4096;
    int64_t n = (slots + strips - 1) / strips;
    n = std::max<int64_t>(1, std::min<int64_t>(n, rows / 32));
    return (int)n;
}

}  // namespace

hipError_t launch_f32_fwd(const F32Args &a, hipStream_t st)
{
    if (a.B <= 0 || a.Ho <= 0 || a.Wo <= 0) return hipSuccess;
    const void *fn = a.off ? reinterpret_cast<const void *>(&k_f32_fwd<2>) : reinterpret_cast<const void *>(&k_f32_fwd<0>);
    int nstrip = (a.Wo + kOwnF - 1) / kOwnF;
    int nchunk = chunks_for(fn, (int64_t)a.B * nstrip, a.Ho);
    const int64_t waves = (int64_t)a.B * nstrip * nchunk;
    const int grid = (int)((waves + kWavesPerGroup - 1) / kWavesPerGroup);
    F32Args aa = a;
    void *args[] = {(void *)&aa, (void *)&nstrip, (void *)&nchunk};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWavesPerGroup), args, 0, st);
}

hipError_t launch_f32_bwd(const F32Args &a, hipStream_t st)
{
    if (a.B <= 0) return hipSuccess;
    const void *fn = a.off ? reinterpret_cast<const void *>(&k_f32_bwd<2>) : reinterpret_cast<const void *>(&k_f32_bwd<0>);
    int nstrip = (a.W + kOwnB - 1) / kOwnB;
    int nchunk = chunks_for(fn, (int64_t)a.B * nstrip, a.H);
    const int64_t waves = (int64_t)a.B * nstrip * nchunk;
    const int grid = (int)((waves + kWavesPerGroup - 1) / kWavesPerGroup);
    F32Args aa = a;
    void *args[] = {(void *)&aa, (void *)&nstrip, (void *)&nchunk};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWavesPerGroup), args, 0, st);
}

}  // namespace s4x5
