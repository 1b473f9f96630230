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
// pixel is centred.  Every factor pair is applied down the columns first;
// the five column results then meet in one correlation across the columns
// whose taps are the matching combinations of the five row filters, so the
// adjoint needs only four lane shifts per row.  P at the two virtual rows
// and columns beyond each edge then goes to the pixel the border rule read
// there: the edge pixel (replicate), the mirror pixel (reflect-101), or
// nowhere (zero: those taps read a constant).
//
// Layout of the work: a wave owns a strip of columns and a range of rows of
// one image.  Each lane holds two adjacent columns and walks down the rows,
// keeping five-row rings of every stage in registers; the horizontal taps
// (+-1, +-2 columns) are the lane's other column or come from the
// neighbouring lanes by wave-wide DPP shifts (four shifts give the whole
// +-2 neighbourhood of a column pair).  A wave loads 128 columns and keeps
// the ones whose whole stencil chain lies inside its lanes (forward: 2
// columns of halo per side, adjoint: 6).

#include "internal.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

namespace s4x5 {
namespace {

constexpr int kWavesPerGroup = 4;
constexpr int kHaloF = 2, kOwnF = 128 - 2 * kHaloF;   // forward: 124 columns per wave
constexpr int kHaloB = 6, kOwnB = 128 - 2 * kHaloB;   // adjoint: 116 columns per wave

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Border rules of the real-valued path (VALID reads like CLAMP: its taps
// never leave the image).
constexpr int kClamp = 0, kZero = 1, kRefl = 2;

// Index that stands in for position i of an axis of n pixels (0 <= i < n
// maps to itself): the nearest pixel, except under REFLECT101, which mirrors
// about the edge pixel without repeating it, again and again until the index
// lands inside (n = 1 gives 0).  ZERO takes the nearest pixel as a safe
// address and masks the value.
template <int BM>
__device__ __forceinline__ int edge_index(int i, int n)
{
    if constexpr (BM == kRefl) {
        if (n == 1) return 0;
        while (i < 0 || i >= n) i = i < 0 ? -i : 2 * (n - 1) - i;
        return i;
    } else {
        return clampi(i, 0, n - 1);
    }
}

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

// A lane's two adjacent columns (a = even offset, b = the next column).
struct F2 {
    float a, b;
};
__device__ __forceinline__ F2 operator+(F2 x, F2 y) { return {x.a + y.a, x.b + y.b}; }
__device__ __forceinline__ F2 operator-(F2 x, F2 y) { return {x.a - y.a, x.b - y.b}; }
__device__ __forceinline__ F2 operator*(float k, F2 x) { return {k * x.a, k * x.b}; }

// The +-1 and +-2 column neighbours of a pair.
struct Nb {
    F2 m2, m1, p1, p2;
};
__device__ __forceinline__ Nb neighbours(F2 v)
{
    const float la = from_left(v.a), lb = from_left(v.b), ra = from_right(v.a), rb = from_right(v.b);
    return {{la, lb}, {lb, v.a}, {v.b, ra}, {ra, rb}};
}

// Row filters across the columns (Eq. (Fx) and the D term of
// Eq. (Gd-_fast)): hs = v[+1] - v[-1], hr = (v[+2] - v[-2]) + 2 hs.
__device__ __forceinline__ void hfilters(F2 v, F2 &hr, F2 &hs)
{
    const Nb n = neighbours(v);
    hs = n.p1 - n.m1;
    hr = (n.p2 - n.m2) + 2.0f * hs;
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
__device__ __forceinline__ F2 comb_c(F2 a0, F2 a1, F2 a2, F2 a3, F2 a4)
{
    return {comb_c(a0.a, a1.a, a2.a, a3.a, a4.a), comb_c(a0.b, a1.b, a2.b, a3.b, a4.b)};
}
__device__ __forceinline__ F2 comb_cd(F2 a0, F2 a1, F2 a2, F2 a3, F2 a4, F2 b0, F2 b2, F2 b4)
{
    return {comb_cd(a0.a, a1.a, a2.a, a3.a, a4.a, b0.a, b2.a, b4.a),
            comb_cd(a0.b, a1.b, a2.b, a3.b, a4.b, b0.b, b2.b, b4.b)};
}

// Columns-first pair (Gy, Gd+) from the lane's v_r and v_s of the centre
// row: horizontal combination across the columns.
__device__ __forceinline__ void hcombine(F2 vr, F2 vs, F2 &C, F2 &Cd)
{
    const Nb r = neighbours(vr), t = neighbours(vs);
    C = comb_c(r.m2, r.m1, vr, r.p1, r.p2);
    Cd = comb_cd(r.m2, r.m1, vr, r.p1, r.p2, t.m2, vs, t.p2);
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
// root (within 1 ulp).  Below 2^-100 (down to the denormals, which the
// hardware operation does not take) S is first scaled by 2^100 and the
// result by 2^50; both scalings are exact, so the 1 ulp bound holds for
// every S > 0.
__device__ __forceinline__ float scale_of(float g, float S)
{
    const bool tiny = S < 0x1p-100f;
    const float r = __builtin_amdgcn_rsqf(S * (tiny ? 0x1p+100f : 1.0f)) * (tiny ? 0x1p+50f : 1.0f);
    return S > 0.f ? g * r : 0.f;
}

template <int P>
using Ph = std::integral_constant<int, P>;

// Steps 0 .. T-1 of a five-slot ring: whole blocks of five in a loop with a
// single exit, then the 0..4 remaining steps.  (Breaking out of the loop
// after any step makes flow blocks with edges back to the loop header; the
// memory-wait analysis merges their state into the header and waits there
// for every row in flight.)
template <class Step>
__device__ __forceinline__ void run_steps(int T, Step &step)
{
    const int nfull = T - T % 5;
    for (int t = 0; t < nfull; t += 5) {
        step(t, Ph<0>{});
        step(t + 1, Ph<1>{});
        step(t + 2, Ph<2>{});
        step(t + 3, Ph<3>{});
        step(t + 4, Ph<4>{});
    }
    if (nfull < T) {
        step(nfull, Ph<0>{});
        if (nfull + 1 < T) {
            step(nfull + 1, Ph<1>{});
            if (nfull + 2 < T) {
                step(nfull + 2, Ph<2>{});
                if (nfull + 3 < T) step(nfull + 3, Ph<3>{});
            }
        }
    }
}

// Steps t0 .. t1-1 (t0 a multiple of five, so the ring phase of step t is
// t % 5), in blocks of five with a single exit, then the rest.
template <class Step>
__device__ __forceinline__ void run_steps_from(int t0, int t1, Step &step)
{
    const int nfull = t0 + (t1 - t0) / 5 * 5;
    for (int t = t0; t < nfull; t += 5) {
        step(t, Ph<0>{});
        step(t + 1, Ph<1>{});
        step(t + 2, Ph<2>{});
        step(t + 3, Ph<3>{});
        step(t + 4, Ph<4>{});
    }
    if (nfull < t1) {
        step(nfull, Ph<0>{});
        if (nfull + 1 < t1) {
            step(nfull + 1, Ph<1>{});
            if (nfull + 2 < t1) {
                step(nfull + 2, Ph<2>{});
                if (nfull + 3 < t1) step(nfull + 3, Ph<3>{});
            }
        }
    }
}

// ---------------------------------------------------------------- forward
// Wave (image b, strip s, chunk k): output columns [s*124, s*124+124),
// output rows [o0, o1).  Lane l holds output columns s*124 - 2 + 2l + {0, 1}
// (centre columns + OFF).  Step t loads input row o0 + OFF - 2 + t and, from
// t = 4 on, finishes output row o0 + t - 4.  BM is the border rule.
template <int OFF, int BM>
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
    const int ox = s * kOwnF - kHaloF + 2 * lane;            // output column of element a
    const bool in_lane = lane >= kHaloF / 2 && lane < (kHaloF + kOwnF) / 2;
    const bool keep_a = in_lane && ox < a.Wo, keep_b = in_lane && ox + 1 < a.Wo;
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride;
    const int64_t xa = (int64_t)edge_index<BM>(ox + OFF, a.W) * 4, xb = (int64_t)edge_index<BM>(ox + 1 + OFF, a.W) * 4;
    // ZERO: does the lane's column lie inside the image?
    const bool ina = ox + OFF >= 0 && ox + OFF < a.W, inb = ox + 1 + OFF >= 0 && ox + 1 + OFF < a.W;
    char *dst = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride;
    const int64_t oa = (int64_t)(ox < 0 ? 0 : ox) * 4;
    const int r0 = o0 + OFF - 2;
    // both kept columns stored with one 8-byte store
    const bool vst = keep_a && keep_b && ((reinterpret_cast<uintptr_t>(dst) | (uintptr_t)a.out_pitch) & 7u) == 0;
    // a pair is two 4-byte loads at the lane's border-mapped columns (see
    // the adjoint's loads)
    auto ld = [&](int t) {
        const int r = r0 + t;
        const char *row = src + (int64_t)edge_index<BM>(r, a.H) * a.src_pitch;
        F2 v{*reinterpret_cast<const float *>(row + xa), *reinterpret_cast<const float *>(row + xb)};
        if constexpr (BM == kZero) {
            const bool rin = r >= 0 && r < a.H;
            v = F2{rin && ina ? v.a : 0.f, rin && inb ? v.b : 0.f};
        }
        return v;
    };
    const int T = o1 - o0 + 4;

    F2 X[5], HR[5], HS[5], pf[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) X[i] = HR[i] = HS[i] = pf[i] = F2{0.f, 0.f};
    constexpr int PD = 3;   // rows loaded ahead
    // prologue loads in row order (the loop's first steps consume them)
#pragma unroll
    for (int t = 0; t < PD; ++t) {
        pf[t] = ld(t);
        __builtin_amdgcn_sched_barrier(0);
    }

    auto step = [&](int t, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int s0 = (p + 1) % 5, s1 = (p + 2) % 5, s2 = (p + 3) % 5, s3 = (p + 4) % 5, s4 = p;
        pf[(p + PD) % 5] = ld(min(t + PD, T - 1));
        const F2 x = pf[p];
        X[s4] = x;
        hfilters(x, HR[s4], HS[s4]);
        if (t < 4) return;
        const F2 Gx = comb_c(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4]);
        const F2 Gm = comb_cd(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4]);
        const F2 vs = X[s3] - X[s1];
        const F2 vr = (X[s4] - X[s0]) + 2.0f * vs;
        F2 Gy, Gp;
        hcombine(vr, vs, Gy, Gp);
        float *row = reinterpret_cast<float *>(dst + (int64_t)(o0 + t - 4) * a.out_pitch + oa);
        const float ma = mag_of(Gx.a, Gy.a, Gp.a, Gm.a), mb = mag_of(Gx.b, Gy.b, Gp.b, Gm.b);
        if (vst) {
            *reinterpret_cast<float2 *>(row) = float2{ma, mb};
        } else {
            if (keep_a) row[0] = ma;
            if (keep_b) row[1] = mb;
        }
    };
    run_steps(T, step);
}

// ---------------------------------------------------------------- adjoint
// Wave (image b, strip s, chunk k): grad_src columns [s*116, s*116+116), rows
// [X0, X1).  Lane l holds input columns c = s*116 - 6 + 2l + {0, 1}.  Step t
// loads input row r = r0 + t; the centre row q = r - 2 gets its weighted
// planes w; the padded adjoint row p = r - 4 is complete and is folded /
// stored.  BM is the border rule: under REPLICATE and REFLECT101 the padded
// rows and columns -2, -1, H, H+1 (W, W+1) fold back onto the pixels that
// stood in for them; under ZERO and VALID they are dropped.
template <int OFF, int BM>
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
    const int c = s * kOwnB - kHaloB + 2 * lane;             // input column of element a
    // replicate: fold the padded columns -2, -1 onto 0 and W, W+1 onto W-1;
    // reflect-101: -1, -2 onto 1, 2 and W, W+1 onto W-2, W-3 (as the
    // index rule maps them for narrow images).  Wave-uniform: does this
    // strip hold column 0 / W-1?
    constexpr bool kFold = OFF == 0 && BM != kZero;
    const bool fold_l = kFold && s == 0;
    const bool fold_r = kFold && s * kOwnB + kOwnB >= a.W;
    // Columns this wave stores, [klo, khi): its own 116, except under
    // reflect-101, where the last strip (the only one whose lanes hold the
    // adjoint at the padded columns W and W+1) also takes W-3 and W-2, the
    // mirrors of those columns, and the strip before gives them up.  The
    // adjoint is complete on lanes 2..61 (columns s*116-2 .. s*116+117), and
    // W-3 >= s*116-2 holds for the last strip.
    int klo = s * kOwnB, khi = min(s * kOwnB + kOwnB, a.W);
    if constexpr (kFold && BM == kRefl) {
        if (fold_r)
            klo = max(0, min(klo, a.W - 3));
        else
            khi = min(khi, max(0, a.W - 3));
    }
    const bool keep_a = c >= klo && c < khi, keep_b = c + 1 >= klo && c + 1 < khi;
    // an output pixel is centred on the column
    const bool oc_a = c - OFF >= 0 && c - OFF < a.Wo, oc_b = c + 1 - OFF >= 0 && c + 1 - OFF < a.Wo;
    const int64_t xa = (int64_t)edge_index<BM>(c, a.W) * 4, xb = (int64_t)edge_index<BM>(c + 1, a.W) * 4;
    const bool ina = c >= 0 && c < a.W, inb = c + 1 >= 0 && c + 1 < a.W;   // (ZERO)
    const int64_t ga = (int64_t)clampi(c - OFF, 0, a.Wo - 1) * 4, gb = (int64_t)clampi(c + 1 - OFF, 0, a.Wo - 1) * 4;
    const char *src = reinterpret_cast<const char *>(a.src) + (int64_t)b * a.src_bstride;
    const char *gr = reinterpret_cast<const char *>(a.grad) + (int64_t)b * a.g_bstride;
    char *dst = reinterpret_cast<char *>(a.out) + (int64_t)b * a.out_bstride + (int64_t)(c < 0 ? 0 : c) * 4;
    const int c0 = s * kOwnB - kHaloB;                        // column of lane 0's element a
    // both kept columns stored with one 8-byte store (c is even)
    const bool vst = keep_a && keep_b && c >= 0 &&
                     ((reinterpret_cast<uintptr_t>(a.out) | (uintptr_t)a.out_pitch | (uintptr_t)a.out_bstride) & 7u) == 0;
    // input rows X0-4 .. X1+3 give the adjoint rows [X0, X1); at the top and
    // bottom of the image, where padded rows fold back, two more rows on
    // that side give the padded rows -2, -1 and H, H+1
    const int r0 = X0 - ((kFold && X0 == 0) ? 6 : 4);
    const int T = X1 + ((kFold && X1 == a.H) ? 6 : 4) - r0;

    auto ldx = [&](int t) {
        const int r = r0 + t;
        const char *row = src + (int64_t)edge_index<BM>(r, a.H) * a.src_pitch;
        // two 4-byte loads at the lane's border-mapped columns (inside the
        // image xb = xa + 4).  An 8-byte load for waves whose pairs all lie
        // inside took the same VALU count or more: behind the wave-uniform
        // choice the compiler computed both addresses and selected between
        // them on every row (adjoint interior loop: 1074 against 946 VALU
        // instructions per 5 rows).
        F2 v{*reinterpret_cast<const float *>(row + xa), *reinterpret_cast<const float *>(row + xb)};
        if constexpr (BM == kZero) {
            const bool rin = r >= 0 && r < a.H;
            v = F2{rin && ina ? v.a : 0.f, rin && inb ? v.b : 0.f};
        }
        return v;
    };
    // grad of the output row whose centre is input row r0 + t - 2 (0 outside;
    // ga, gb are clamped columns, masked where no output pixel is centred)
    auto ldg = [&](int t) {
        const int o = r0 + t - 2 - OFF;
        F2 v{0.f, 0.f};
        if (o >= 0 && o < a.Ho) {
            const char *row = gr + (int64_t)o * a.g_pitch;
            v = F2{*reinterpret_cast<const float *>(row + ga), *reinterpret_cast<const float *>(row + gb)};
        }
        return F2{oc_a ? v.a : 0.f, oc_b ? v.b : 0.f};
    };

    // rings (slot = step mod 5): input rows, their row filters, and the
    // centre-row planes -w_x, -w_m, -w_y, -w_p
    F2 X[5], HR[5], HS[5], WX[5], WM[5], WY[5], WP[5];
    F2 pfx[5], pfg[5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
        X[i] = HR[i] = HS[i] = WX[i] = WM[i] = WY[i] = WP[i] = pfx[i] = pfg[i] = F2{0.f, 0.f};
    constexpr int PD = 3;   // rows loaded ahead (measured: 2 is 9% slower, 4 no faster)
    // prologue loads in row order (the loop's first steps consume them)
#pragma unroll
    for (int t = 0; t < PD; ++t) {
        pfx[t] = ldx(t);
        pfg[t] = ldg(t);
        __builtin_amdgcn_sched_barrier(0);
    }
    // replicate: sums of the padded rows above row 0 / from row H-1 down;
    // reflect-101: padded rows -2, -1, and the last three rows, held until
    // the padded rows H, H+1 have been added
    F2 acc_top{0.f, 0.f}, acc_bot{0.f, 0.f};
    F2 top2{0.f, 0.f}, top1{0.f, 0.f}, hold0{0.f, 0.f}, hold1{0.f, 0.f}, hold2{0.f, 0.f};

    auto store = [&](int row, F2 v) __attribute__((always_inline)) {
        if constexpr (kFold && BM == kClamp) {
            if (fold_l || fold_r) {
                const Nb n = neighbours(v);   // from the row-folded values of every lane
                if (fold_l && c == 0) v.a += n.m2.a + n.m1.a;                  // columns -2, -1
                if (fold_r && c == a.W - 1) v.a += n.p1.a + n.p2.a;            // columns W, W+1
                if (fold_r && c + 1 == a.W - 1) v.b += n.p1.b + n.p2.b;
            }
        }
        if constexpr (kFold && BM == kRefl) {
            if (fold_l || fold_r) {
                // a padded column vc sits in lane (vc - c0) / 2 (lanes 2 .. 61),
                // element (vc - c0) & 1: read it there, add it at its mirror
                auto at = [&](int vc) __attribute__((always_inline)) {
                    const int d = vc - c0;
                    const int ea = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.a), d >> 1);
                    const int eb = __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.b), d >> 1);
                    return __builtin_bit_cast(float, (d & 1) ? eb : ea);
                };
                auto add_at = [&](int vc, float pv) __attribute__((always_inline)) {
                    const int tc = edge_index<kRefl>(vc, a.W);
                    if (c == tc) v.a += pv;
                    if (c + 1 == tc) v.b += pv;
                };
                // (targets lie inside the image, so no read sees an earlier add)
                if (fold_l) {
                    const float m2 = at(-2), m1 = at(-1);
                    add_at(-2, m2);
                    add_at(-1, m1);
                }
                if (fold_r) {
                    const float p0 = at(a.W), p1 = at(a.W + 1);
                    add_at(a.W, p0);
                    add_at(a.W + 1, p1);
                }
            }
        }
        float *p = reinterpret_cast<float *>(dst + (int64_t)row * a.out_pitch);
        if (vst) {
            *reinterpret_cast<float2 *>(p) = float2{v.a, v.b};
        } else {
            if (keep_a) p[0] = v.a;
            if (keep_b) p[1] = v.b;
        }
    };

    // INTERIOR: a row of P that is one of the wave's own rows and no padded
    // row folds onto (rows 3 .. H-4 under a folding rule): stored as is.
    auto step = [&](int t, auto phase, auto interior) __attribute__((always_inline)) {
        constexpr int p = decltype(phase)::value;
        constexpr bool INTERIOR = decltype(interior)::value;
        // input rows t-4 .. t live in slots (p+1)%5 .. p
        constexpr int s0 = (p + 1) % 5, s1 = (p + 2) % 5, s2 = (p + 3) % 5, s3 = (p + 4) % 5, s4 = p;
        pfx[(p + PD) % 5] = ldx(min(t + PD, T - 1));
        pfg[(p + PD) % 5] = ldg(min(t + PD, T - 1));
        const F2 x = pfx[p];
        X[s4] = x;
        hfilters(x, HR[s4], HS[s4]);
        // centre row q = r - 2 (slot s2 of the input rings)
        const F2 Gx = comb_c(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4]);
        const F2 Gm = comb_cd(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4]);
        const F2 vs = X[s3] - X[s1];
        const F2 vr = (X[s4] - X[s0]) + 2.0f * vs;
        F2 Gy, Gp;
        hcombine(vr, vs, Gy, Gp);
        const F2 gq = pfg[p];                    // grad of the output row centred on q
        // the planes enter negated, so the sums below are P itself
        const F2 sc{-scale_of(gq.a, sum_sq(Gx.a, Gy.a, Gp.a, Gm.a)), -scale_of(gq.b, sum_sq(Gx.b, Gy.b, Gp.b, Gm.b))};
        const F2 hsc = 0.5f * sc;
        // w rings hold centre rows q-4 .. q in slots (p+1)%5 .. p as well
        WX[s4] = F2{sc.a * Gx.a, sc.b * Gx.b};
        WY[s4] = F2{sc.a * Gy.a, sc.b * Gy.b};
        WP[s4] = F2{hsc.a * Gp.a, hsc.b * Gp.b};
        WM[s4] = F2{hsc.a * Gm.a, hsc.b * Gm.b};
        // padded adjoint row p_ = q - 2 (slot s2 of the w rings).  Each term
        // K = u_v (x) u_h is applied down the columns first:
        //   V1 = c_v(w_x) + c'_v(w_m)  (row filter r),   V2 = d_v(w_m)  (-s),
        //   V3 = r_v(w_y)              (row filter c),   V4 = r_v(w_p)  (c'),
        //   V5 = s_v(w_p)              (-d),
        // and then by one correlation across the columns whose tap dx takes
        // Q_dx = r[dx] V1 - s[dx] V2 + c[dx] V3 + c'[dx] V4 - d[dx] V5.
        const F2 e04m = WM[s0] + WM[s4];
        const F2 V1 = comb_c(WX[s0], WX[s1], WX[s2], WX[s3], WX[s4]) +
                      (6.0f * (e04m + (WM[s1] + WM[s3])) + 2.0f * WM[s2]);
        const F2 V2 = 10.0f * e04m - 12.0f * WM[s2];
        const F2 V3 = (WY[s4] - WY[s0]) + 2.0f * (WY[s3] - WY[s1]);
        const F2 V5 = WP[s3] - WP[s1];
        const F2 V4 = (WP[s4] - WP[s0]) + 2.0f * V5;
        // Q_+-2 = E +- V1, Q_+-1 = F +- O, Q_0
        const F2 E = V3 + 6.0f * V4 - 10.0f * V5;
        const F2 Fq = 4.0f * V3 + 6.0f * V4;
        const F2 O = 2.0f * V1 - V2;
        const F2 Qm2 = E - V1, Qp2 = E + V1, Qm1 = Fq - O, Qp1 = Fq + O;
        const F2 Q0 = 6.0f * V3 + 2.0f * V4 + 12.0f * V5;
        // column a takes Q_-2, Q_-1 from the left lane's a, b, Q_+1 from its
        // own b and Q_+2 from the right lane's a; column b likewise
        const F2 P{(Q0.a + Qp1.b) + from_left(Qm2.a + Qm1.b) + from_right(Qp2.a),
                   (Qm1.a + Q0.b) + from_left(Qm2.b) + from_right(Qp1.a + Qp2.b)};
        const int pr = r0 + t - 4;               // padded row of P
        if constexpr (INTERIOR) {
            store(pr, P);
            return;
        }
        if (pr < X0 - 2 || pr >= X1 + 2) return;  // warm-up and rows of other waves
        if constexpr (!kFold) {                   // VALID, ZERO: nothing folds back
            if (pr >= X0 && pr < X1) store(pr, P);
            return;
        }
        if constexpr (BM == kRefl) {
            // the last rows of the image, [H-3, H), are held: hold<k> is row
            // H-3+k (k is wave-uniform; selects, not an indexed array, keep
            // them in registers)
            if (pr < 0) {                          // padded rows -2, -1 (top chunk)
                if (pr == -2)
                    top2 = P;
                else
                    top1 = P;
                return;
            }
            if (pr >= a.H) {                       // padded rows H, H+1 (bottom chunk)
                const int k = edge_index<kRefl>(pr, a.H) - (a.H - 3);
                if (k == 0)
                    hold0 = hold0 + P;
                else if (k == 1)
                    hold1 = hold1 + P;
                else
                    hold2 = hold2 + P;
                return;                            // stored after the last step
            }
            if (pr < X0 || pr >= X1) return;
            F2 v = P;
            if (X0 == 0) {
                if (edge_index<kRefl>(-1, a.H) == pr) v = v + top1;
                if (edge_index<kRefl>(-2, a.H) == pr) v = v + top2;
            }
            if (X1 == a.H && pr >= a.H - 3) {
                const int k = pr - (a.H - 3);
                if (k == 0)
                    hold0 = v;
                else if (k == 1)
                    hold1 = v;
                else
                    hold2 = v;
            } else {
                store(pr, v);
            }
            return;
        }
        if (pr < 0) {
            acc_top = acc_top + P;
        } else if (pr >= a.H) {
            acc_bot = acc_bot + P;
            if (pr == a.H + 1) store(a.H - 1, acc_bot);
        } else if (pr >= X0 && pr < X1) {
            F2 v = P;
            if (pr == 0) v = v + acc_top;
            if (pr == a.H - 1)
                acc_bot = v;
            else
                store(pr, v);
        }
    };
    // steps whose P row is interior, [ta, tb) with ta a multiple of five
    // (the ring phase stays t % 5), run without the row checks; the others
    // take the general step
    const int plo = kFold ? max(X0, 3) : X0, phi = kFold ? min(X1, a.H - 3) : X1;
    int ta = min(T, (plo - r0 + 4 + 4) / 5 * 5);
    const int tb = max(ta, phi - r0 + 4);
    using Gen = std::false_type;
    using Int = std::true_type;
    auto gen = [&](int t, auto ph) __attribute__((always_inline)) { step(t, ph, Gen{}); };
    auto mid = [&](int t, auto ph) __attribute__((always_inline)) { step(t, ph, Int{}); };
    run_steps_from(0, ta, gen);
    const int tm = ta + (tb - ta) / 5 * 5;
    run_steps_from(ta, tm, mid);
    run_steps_from(tm, T, gen);
    if constexpr (kFold && BM == kRefl) {
        if (X1 == a.H) {                           // the held rows, with H and H+1 added
            if (a.H - 3 >= X0) store(a.H - 3, hold0);
            if (a.H - 2 >= X0) store(a.H - 2, hold1);
            store(a.H - 1, hold2);
        }
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

// Row chunks per strip so that the grid fills at most one round of resident
// waves (rounding up would leave a few waves to run as a second, nearly
// empty round), with at least 32 rows per chunk: the pipeline costs 4
// (forward) or 12 (adjoint) extra row steps per chunk.
int chunks_for(const void *fn, int64_t strips, int rows)
{
    int slots = resident_f32(fn);
    if (slots <= 0) slots = 4096;
    int64_t n = slots / strips;
    n = std::max<int64_t>(1, std::min<int64_t>(n, rows / 32));
    return (int)n;
}

}  // namespace

hipError_t launch_f32_fwd(const F32Args &a, hipStream_t st)
{
    if (a.B <= 0 || a.Ho <= 0 || a.Wo <= 0) return hipSuccess;
    const void *fn = a.off ? reinterpret_cast<const void *>(&k_f32_fwd<2, kClamp>)
                   : a.bmode == 1 ? reinterpret_cast<const void *>(&k_f32_fwd<0, kZero>)
                   : a.bmode == 2 ? reinterpret_cast<const void *>(&k_f32_fwd<0, kRefl>)
                                  : reinterpret_cast<const void *>(&k_f32_fwd<0, kClamp>);
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
    const void *fn = a.off ? reinterpret_cast<const void *>(&k_f32_bwd<2, kClamp>)
                   : a.bmode == 1 ? reinterpret_cast<const void *>(&k_f32_bwd<0, kZero>)
                   : a.bmode == 2 ? reinterpret_cast<const void *>(&k_f32_bwd<0, kRefl>)
                                  : reinterpret_cast<const void *>(&k_f32_bwd<0, kClamp>);
    int nstrip = (a.W + kOwnB - 1) / kOwnB;
    int nchunk = chunks_for(fn, (int64_t)a.B * nstrip, a.H);
    const int64_t waves = (int64_t)a.B * nstrip * nchunk;
    const int grid = (int)((waves + kWavesPerGroup - 1) / kWavesPerGroup);
    F32Args aa = a;
    void *args[] = {(void *)&aa, (void *)&nstrip, (void *)&nchunk};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWavesPerGroup), args, 0, st);
}

}  // namespace s4x5
