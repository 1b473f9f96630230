// uint8 four-directional 5x5 Sobel kernels for CDNA4 (gfx950).
//
// Operator: Eq. (sobel5_1) and Eq. (sobel5_2) of Chang et al. (Sec. 3.1),
// applied as a correlation.  The four responses are never formed tap by tap.
// They come from shared one-dimensional passes, in the spirit of the paper's
// separable row filters (Sec. 4.3, Eq. (Fx)/(Gx)) and its diagonal transform
// (K_d+- = K_d +- K_dt, Eq. (sobel5_kd+-); K_d- as a sum of two separable
// terms, Eq. (sobel5_4)):
//
//   Gx  = c_v(h_r)                     rows first:  h_r = [-1,-2,0,2,1] . row
//   Gd- = c'_v(h_r) - d_v(h_s)                       h_s = [0,-1,0,1,0] . row
//   Gy  = c_h(v_r)                     columns first: v_r = [-1,-2,0,2,1]^T . col
//   Gd+ = c'_h(v_r) - d_h(v_s)                         v_s = [0,-1,0,1,0]^T . col
//
// with c = [1,4,6,4,1], c' = [6,6,2,6,6], d = [10,0,-12,0,10].  K_d+ is the
// transpose of K_d-, so the transpose of Eq. (sobel5_4) gives the Gd+ line.
// Then Gd = (Gd+ + Gd-)/2 and Gdt = (Gd+ - Gd-)/2 (Eq. (sobel5_kd), exact)
// and 2S = 2(Gx^2 + Gy^2) + Gd+^2 + Gd-^2.
//
// Every intermediate fits in int16 (|G| <= 12240, |Gd+-| <= 17850, partial
// sums <= 28050), so the passes run on packed 16-bit lanes: one register
// holds pixels j and j + ppl/2 of a lane's ppl consecutive pixels.  The
// squares are summed with v_dot2_i32_i16 after a byte permute that pairs
// (Gx, Gy) and (Gd+, Gd-) of the same pixel.
//
// Memory side (replaces the paper's warp shuffles and one-row prefetch):
//   - a lane loads its ppl pixels of a row with one 128-/64-bit load;
//   - the two halo bytes on each side come from the neighbouring lanes by
//     DPP row_shr/row_shl inside a 16-lane row; the 16-lane group's outer
//     halo comes from one extra dword load by its first and last lane;
//   - a group sweeps its tile top to bottom, keeping a 5-row ring of the
//     unpacked rows and of the row filters in VGPRs (the ring index is the
//     loop phase, unrolled by 5), and loads PD rows ahead;
//   - the right image border (and widths that are not a multiple of 16) is
//     handled in registers: the lane's aligned 16-byte block is always a
//     block that holds a valid byte of the row, and bytes past the row end
//     are replaced by the last valid pixel (replicate).

#include "internal.hpp"

#include <type_traits>

namespace s4x5 {
namespace {

typedef short v2s __attribute__((ext_vector_type(2)));
typedef unsigned int u32;

__device__ __forceinline__ v2s S2(u32 v) { return __builtin_bit_cast(v2s, v); }
__device__ __forceinline__ u32 U2(v2s v) { return __builtin_bit_cast(u32, v); }
__device__ __forceinline__ u32 perm(u32 hi, u32 lo, u32 sel) { return __builtin_amdgcn_perm(hi, lo, sel); }

constexpr u32 kZeroByte = 0x0c;   // v_perm selector that yields 0x00
constexpr int kPD = 2;            // rows loaded ahead of use

// v_perm selector: byte0 <- byte `lob` of the low source, byte2 <- byte
// `hib` of the high source, bytes 1 and 3 <- 0: two zero-extended pixels.
constexpr u32 pair_sel(int lob, int hib)
{
    return (kZeroByte << 24) | ((4u + (u32)hib) << 16) | (kZeroByte << 8) | (u32)lob;
}

// Round-to-nearest of sqrt(s2 / 2), saturated to 255.  s2 = 2S is even, so
// s2 * 0.5f is S (exactly below 2^24; monotone above, where the result
// saturates anyway).  v_sqrt_f32 is within 1 ulp and an integer S is never
// closer than 4.9e-4 to a half-integer square root, so the rounding is exact.
__device__ __forceinline__ u32 round_mag(int s2)
{
    float f = (float)s2 * 0.5f;
    float r = __builtin_amdgcn_sqrtf(f);
    u32 m = (u32)(r + 0.5f);
    return m < 255u ? m : 255u;
}

// The 20-byte window of one lane for one row: the lane's own ppl bytes
// d[0..ppl/4) starting at column xo, L (bytes 2, 3 = columns xo-2, xo-1) and
// Rt (bytes 0..3 = columns xo+ppl .. xo+ppl+3).
template <int PPL>
struct Win {
    u32 L;
    u32 d[PPL / 4];
    u32 Rt;
};

// Window byte w covers column xo - 2 + w.
template <int PPL>
__device__ __forceinline__ u32 win_word(const Win<PPL> &w, int b)
{
    if (b < 2) return w.L;
    if (b < PPL + 2) return w.d[(b - 2) >> 2];
    return w.Rt;
}
template <int PPL>
constexpr int win_byte(int b)
{
    return b < 2 ? b + 2 : (b < PPL + 2 ? ((b - 2) & 3) : b - PPL - 2);
}

// Unpack a window into NP + 4 packed registers R[j + 2] = (p[j], p[j + NP]),
// j in [-2, NP + 2), where p[j] is the pixel at column (first centre + j) and
// the first centre is column xo + OFF.
template <int PPL, int OFF>
__device__ __forceinline__ void unpack(const Win<PPL> &w, v2s (&R)[PPL / 2 + 4])
{
    constexpr int NP = PPL / 2;
#pragma unroll
    for (int j = -2; j < NP + 2; ++j) {
        const int bl = OFF + j + 2, bh = OFF + j + NP + 2;
        R[j + 2] = S2(perm(win_word<PPL>(w, bh), win_word<PPL>(w, bl),
                           pair_sel(win_byte<PPL>(bl), win_byte<PPL>(bh))));
    }
}

// Row filters of one input row (Eq. (Fx) and the D term of Eq. (Gd-_fast)):
// h_s = p[+1] - p[-1], h_r = (p[+2] - p[-2]) + 2 h_s.
template <int NP>
__device__ __forceinline__ void row_filters(const v2s (&R)[NP + 4], v2s (&hr)[NP], v2s (&hs)[NP])
{
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        v2s s = R[j + 3] - R[j + 1];
        v2s e = R[j + 4] - R[j];
        hs[j] = s;
        hr[j] = e + s + s;
    }
}

// Gy and Gd+ at one output row (columns first).  vr = v_r and a2 = v_s of
// the output row's centre, both for NP + 4 columns.
template <int NP>
__device__ __forceinline__ void responses_y(const v2s (&vr)[NP + 4], const v2s (&a2)[NP + 4],
                                            v2s (&Gy)[NP], v2s (&Gp)[NP])
{
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int c = j + 2;
        v2s p4 = vr[c - 2] + vr[c + 2];
        v2s p2 = vr[c - 1] + vr[c + 1];
        Gy[j] = p4 + p2 * (short)4 + vr[c] * (short)6;
        Gp[j] = (p4 + p2) * (short)6 + vr[c] * (short)2 - (a2[c - 2] + a2[c + 2]) * (short)10 +
                a2[c] * (short)12;
    }
}

// Gx and Gd- at one output row (rows first) from the row filters of the
// five window rows.
template <int NP>
__device__ __forceinline__ void responses_x(const v2s (&hr0)[NP], const v2s (&hr1)[NP],
                                            const v2s (&hr2)[NP], const v2s (&hr3)[NP],
                                            const v2s (&hr4)[NP], const v2s (&hs0)[NP],
                                            const v2s (&hs2)[NP], const v2s (&hs4)[NP],
                                            v2s (&Gx)[NP], v2s (&Gm)[NP])
{
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        v2s x1 = hr0[j] + hr4[j];
        v2s x2 = hr1[j] + hr3[j];
        Gx[j] = x1 + x2 * (short)4 + hr2[j] * (short)6;
        Gm[j] = (x1 + x2) * (short)6 + hr2[j] * (short)2 - (hs0[j] + hs4[j]) * (short)10 +
                hs2[j] * (short)12;
    }
}

// Replace the bytes of `v` at positions >= keep (0..4) by `fill` (a byte
// replicated four times).
__device__ __forceinline__ u32 keep_bytes(u32 v, int keep, u32 fill)
{
    u32 mask = keep >= 4 ? 0xffffffffu : ((1u << (8 * (keep > 0 ? keep : 0))) - 1u);
    return (v & mask) | (fill & ~mask);
}

// Byte b (runtime, 0..PPL-1) of the lane's own block, by v_perm with a
// runtime selector (keeps the block in registers).
template <int PPL>
__device__ __forceinline__ u32 byte_of(const u32 (&d)[PPL / 4], int b)
{
    u32 lo = d[0], hi = d[1];
    if constexpr (PPL == 16) {
        const bool up = (b & 8) != 0;
        lo = up ? d[2] : d[0];
        hi = up ? d[3] : d[1];
    }
    return perm(hi, lo, (kZeroByte << 24) | (kZeroByte << 16) | (kZeroByte << 8) | (u32)(b & 7));
}

template <int PPL>
struct RawRow {
    u32 d[PPL / 4];
    u32 hw;   // lane 0 of a group: left halo dword; lane 15: right halo dword
};

// Issue the loads of one row (fast path: 16-byte aligned rows).
template <int PPL>
__device__ __forceinline__ void load_row(RawRow<PPL> &r, const uint8_t *rowp, int ldx, int hx)
{
    if constexpr (PPL == 16) {
        uint4 v = *reinterpret_cast<const uint4 *>(rowp + ldx);
        r.d[0] = v.x; r.d[1] = v.y; r.d[2] = v.z; r.d[3] = v.w;
    } else {
        uint2 v = *reinterpret_cast<const uint2 *>(rowp + ldx);
        r.d[0] = v.x; r.d[1] = v.y;
    }
    r.hw = *reinterpret_cast<const u32 *>(rowp + hx);
}

// Turn a loaded row into the lane's window: border fix-ups, then DPP halo.
template <int PPL, int OFF>
__device__ __forceinline__ Win<PPL> finish_row(RawRow<PPL> r, int lane16, int xo, int W,
                                               bool fix_right, bool fix_left)
{
    constexpr int ND = PPL / 4;
    if (fix_right) {
        // own block: bytes at columns >= W take the value of column W-1
        const int nv = W - xo;
        if (nv < PPL) {
            const int lb = nv >= 1 ? nv - 1 : ((W - 1) & (PPL - 1));
            const u32 fill = byte_of<PPL>(r.d, lb) * 0x01010101u;
#pragma unroll
            for (int m = 0; m < ND; ++m) r.d[m] = keep_bytes(r.d[m], nv - 4 * m, fill);
        }
        // right halo dword of lane 15 (nominal columns xo+PPL .. xo+PPL+3)
        const int nh = W - (xo + PPL);
        if (lane16 == 15 && nh < 4) {
            const int lb = nh >= 1 ? nh - 1 : ((W - 1) & 3);
            const u32 fill = ((r.hw >> (8 * lb)) & 0xffu) * 0x01010101u;
            r.hw = keep_bytes(r.hw, nh, fill);
        }
    }
    if (OFF == 0 && fix_left && lane16 == 0 && xo == 0) r.hw = (r.d[0] & 0xffu) * 0x01010101u;
    Win<PPL> w;
#pragma unroll
    for (int m = 0; m < ND; ++m) w.d[m] = r.d[m];
    // row_shr:1 -> value of lane-1 within the 16-lane row; lane 0 keeps `old`
    w.L = (u32)__builtin_amdgcn_update_dpp((int)r.hw, (int)r.d[ND - 1], 0x111, 0xf, 0xf, false);
    // row_shl:1 -> value of lane+1; lane 15 keeps `old`
    w.Rt = (u32)__builtin_amdgcn_update_dpp((int)r.hw, (int)r.d[0], 0x101, 0xf, 0xf, false);
    return w;
}

// Slow path for rows that are not 16-byte aligned: every window byte is read
// on its own at its clamped column.
template <int PPL>
__device__ __forceinline__ Win<PPL> load_row_bytes(const uint8_t *rowp, int xo, int W)
{
    Win<PPL> w;
    auto px = [&](int x) -> u32 { return rowp[x < 0 ? 0 : (x >= W ? W - 1 : x)]; };
    w.L = (px(xo - 2) << 16) | (px(xo - 1) << 24);
#pragma unroll
    for (int m = 0; m < PPL / 4; ++m) {
        const int x = xo + 4 * m;
        w.d[m] = px(x) | (px(x + 1) << 8) | (px(x + 2) << 16) | (px(x + 3) << 24);
    }
    const int x = xo + PPL;
    w.Rt = px(x) | (px(x + 1) << 8) | (px(x + 2) << 16) | (px(x + 3) << 24);
    return w;
}

// Stores of one output row for one lane.
template <int NP, bool DIR>
__device__ __forceinline__ void store_row(const U8Job &J, int yo, int xo, bool row_ok,
                                          const v2s (&Gx)[NP], const v2s (&Gp)[NP],
                                          const v2s (&Gy)[NP], const v2s (&Gm)[NP])
{
    constexpr int PPL = 2 * NP;
    if (!row_ok) return;
    const int nvalid = J.Wo - xo;          // pixels of this lane inside the image
    if (nvalid <= 0) return;
    const bool full = nvalid >= PPL;
    if (J.mag) {
        u32 out[PPL / 4];
#pragma unroll
        for (int m = 0; m < PPL / 4; ++m) out[m] = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const u32 xyl = perm(U2(Gy[j]), U2(Gx[j]), 0x05040100u);
            const u32 xyh = perm(U2(Gy[j]), U2(Gx[j]), 0x07060302u);
            const u32 ddl = perm(U2(Gm[j]), U2(Gp[j]), 0x05040100u);
            const u32 ddh = perm(U2(Gm[j]), U2(Gp[j]), 0x07060302u);
            const int tl = __builtin_amdgcn_sdot2(S2(xyl), S2(xyl), 0, false);
            const int th = __builtin_amdgcn_sdot2(S2(xyh), S2(xyh), 0, false);
            const int sl = __builtin_amdgcn_sdot2(S2(ddl), S2(ddl), tl * 2, false);
            const int sh = __builtin_amdgcn_sdot2(S2(ddh), S2(ddh), th * 2, false);
            const int ql = j, qh = j + NP;   // pixel indices inside the lane
            out[ql >> 2] |= round_mag(sl) << (8 * (ql & 3));
            out[qh >> 2] |= round_mag(sh) << (8 * (qh & 3));
        }
        uint8_t *p = J.mag + (int64_t)yo * J.mag_pitch + xo;
        if (full && J.mag_vec) {
            if constexpr (PPL == 16)
                *reinterpret_cast<uint4 *>(p) = make_uint4(out[0], out[1], out[2], out[3]);
            else
                *reinterpret_cast<uint2 *>(p) = make_uint2(out[0], out[1]);
        } else {
#pragma unroll
            for (int q = 0; q < PPL; ++q)
                if (q < nvalid) p[q] = (uint8_t)(out[q >> 2] >> (8 * (q & 3)));
        }
    }
    if (DIR && J.dir_type != 0) {
        // plane order: 0 deg Gx, 45 deg Gd, 90 deg Gy, 135 deg Gdt
        v2s P[4][NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            P[0][j] = Gx[j];
            P[2][j] = Gy[j];
            v2s sum = Gp[j] + Gm[j];
            v2s dif = Gp[j] - Gm[j];
            P[1][j] = sum >> (short)1;            // exact: Gd+ + Gd- = 2 Gd
            P[3][j] = dif >> (short)1;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            char *base = static_cast<char *>(J.dir[k]) + (int64_t)yo * J.dir_pitch;
            if (J.dir_type == 1) {
                u32 o[NP];   // int16 pixels (2m, 2m+1)
#pragma unroll
                for (int m = 0; m < NP; ++m) {
                    const int a = 2 * m;
                    o[m] = a < NP ? perm(U2(P[k][a + 1]), U2(P[k][a]), 0x05040100u)
                                  : perm(U2(P[k][a - NP + 1]), U2(P[k][a - NP]), 0x07060302u);
                }
                int16_t *p = reinterpret_cast<int16_t *>(base) + xo;
                if (full && J.dir_vec) {
#pragma unroll
                    for (int m = 0; m < NP; m += 4)
                        *reinterpret_cast<uint4 *>(p + 2 * m) = make_uint4(o[m], o[m + 1], o[m + 2], o[m + 3]);
                } else {
#pragma unroll
                    for (int q = 0; q < PPL; ++q)
                        if (q < nvalid) p[q] = (int16_t)(o[q >> 1] >> (16 * (q & 1)));
                }
            } else {
                int o[PPL];
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    o[j] = P[k][j].x;
                    o[j + NP] = P[k][j].y;
                }
                int32_t *p = reinterpret_cast<int32_t *>(base) + xo;
                if (full && J.dir_vec) {
#pragma unroll
                    for (int q = 0; q < PPL; q += 4)
                        *reinterpret_cast<int4 *>(p + q) = make_int4(o[q], o[q + 1], o[q + 2], o[q + 3]);
                } else {
#pragma unroll
                    for (int q = 0; q < PPL; ++q)
                        if (q < nvalid) p[q] = o[q];
                }
            }
        }
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// One wave-tile: 4 tiles stacked vertically in one tile column, one per
// 16-lane group.  `wt` is the wave-tile index inside image J.
template <int PPL, int OFF, bool ALIGNED, bool DIR>
__device__ void wave_tile(const U8Job &J, int wt, int TH)
{
    constexpr int NP = PPL / 2;
    constexpr int TW = 16 * PPL;
    const int lane = threadIdx.x & 63;
    const int lane16 = lane & 15;
    const int grp = lane >> 4;
    const int tx = wt % J.ntx;                       // wave-uniform
    const int ty = (wt / J.ntx) * 4 + grp;           // per group
    const int xo = tx * TW + lane16 * PPL;
    const int yo0 = ty * TH;
    const int nrow = ty < J.nty ? min(TH, J.Ho - yo0) : 0;
    int niter = max(max(__builtin_amdgcn_readlane(nrow, 0), __builtin_amdgcn_readlane(nrow, 16)),
                    max(__builtin_amdgcn_readlane(nrow, 32), __builtin_amdgcn_readlane(nrow, 48)));
    if (niter <= 0) return;
    const int W = J.W;
    const int ymax = J.H - 1;
    const int yin0 = yo0 + OFF - 2;                  // input row of window slot 0

    // fast path: load columns and halo columns (fixed for the whole tile)
    const int ldx = xo < W ? xo : ((W - 1) & ~(PPL - 1));
    const int hxr = xo + PPL;
    const int hx = lane16 == 0 ? (xo >= 4 ? xo - 4 : 0)
                 : (lane16 == 15 ? (hxr < W ? hxr : ((W - 1) & ~3)) : ldx);
    const bool fix_right = (tx + 1) * TW + 4 > W;    // wave-uniform
    const bool fix_left = tx == 0;

    const uint8_t *src = J.src;
    const int64_t pitch = J.src_pitch;
    auto rowp = [&](int t) { return src + (int64_t)clampi(yin0 + t, 0, ymax) * pitch; };

    // Rings indexed by input row mod 5.  Live ranges are short: an unpacked
    // row lives 3 steps, v_s (A2, indexed by its centre row) 3 steps, the row
    // filters 5 steps.
    v2s Rr[5][NP + 4];
    v2s A2r[5][NP + 4];
    v2s HR[5][NP], HS[5][NP];
    RawRow<PPL> raw[5];

    auto fetch = [&](int t, RawRow<PPL> &r) {
        if constexpr (ALIGNED) load_row<PPL>(r, rowp(t), ldx, hx);
    };
    auto process = [&](int t, RawRow<PPL> &r, v2s (&R)[NP + 4], v2s (&hr)[NP], v2s (&hs)[NP]) {
        Win<PPL> w;
        if constexpr (ALIGNED)
            w = finish_row<PPL, OFF>(r, lane16, xo, W, fix_right, fix_left);
        else
            w = load_row_bytes<PPL>(rowp(t), xo, W);
        unpack<PPL, OFF>(w, R);
        row_filters<NP>(R, hr, hs);
    };

    // prologue: rows t = 0..4 in flight, rows 0..3 processed (which frees
    // their slots), then rows 5 .. 3 + kPD.  Row t always lives in raw[t % 5].
    static_assert(kPD >= 1 && kPD <= 4, "prefetch distance must fit the 5-slot ring");
#pragma unroll
    for (int t = 0; t < 5; ++t)
        if (t <= niter + 3) fetch(t, raw[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) process(t, raw[t], Rr[t], HR[t], HS[t]);
#pragma unroll
    for (int t = 5; t < 4 + kPD; ++t)
        if (t <= niter + 3) fetch(t, raw[t % 5]);
#pragma unroll
    for (int c = 0; c < NP + 4; ++c) {
        A2r[1][c] = Rr[2][c] - Rr[0][c];
        A2r[2][c] = Rr[3][c] - Rr[1][c];
    }

    // step i: input row t = i + 4 enters; output row i has its centre at t - 2
    auto step = [&](int i, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int s0 = p, s1 = (p + 1) % 5, s2 = (p + 2) % 5, s3 = (p + 3) % 5, s4 = (p + 4) % 5;
        constexpr int sp = (p + 4 + kPD) % 5;
        if (i + 4 + kPD <= niter + 3) fetch(i + 4 + kPD, raw[sp]);
        process(i + 4, raw[s4], Rr[s4], HR[s4], HS[s4]);
        v2s vr[NP + 4];
#pragma unroll
        for (int c = 0; c < NP + 4; ++c) {
            A2r[s3][c] = Rr[s4][c] - Rr[s2][c];                          // v_s at t - 1
            vr[c] = A2r[s1][c] + A2r[s2][c] + A2r[s2][c] + A2r[s3][c];   // v_r at t - 2
        }
        v2s Gx[NP], Gp[NP], Gy[NP], Gm[NP];
        responses_y<NP>(vr, A2r[s2], Gy, Gp);
        responses_x<NP>(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4], Gx, Gm);
        store_row<NP, DIR>(J, yo0 + i, xo, i < nrow, Gx, Gp, Gy, Gm);
    };

    for (int i = 0; i < niter; i += 5) {
        step(i, std::integral_constant<int, 0>{});
        if (i + 1 >= niter) break;
        step(i + 1, std::integral_constant<int, 1>{});
        if (i + 2 >= niter) break;
        step(i + 2, std::integral_constant<int, 2>{});
        if (i + 3 >= niter) break;
        step(i + 3, std::integral_constant<int, 3>{});
        if (i + 4 >= niter) break;
        step(i + 4, std::integral_constant<int, 4>{});
    }
}

constexpr int kWaves = 4;   // waves per workgroup

template <int PPL, int OFF, bool ALIGNED, bool DIR>
__global__ __launch_bounds__(64 * kWaves) void k_u8_single(U8Job J, int TH)
{
    const int w = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (w >= J.nwt) return;
    wave_tile<PPL, OFF, ALIGNED, DIR>(J, w, TH);
}

// Persistent work-queue kernel: every wave takes the next wave-tile of the
// whole batch from queue[0] until none are left, then counts itself out in
// queue[1]; the last wave out resets both words for the next launch.
template <int PPL, int OFF, bool ALIGNED>
__global__ __launch_bounds__(64 * kWaves) void k_u8_batched(const U8Job *__restrict__ jobs,
                                                            const int32_t *__restrict__ prefix,
                                                            int32_t count, uint32_t *queue, int TH)
{
    const int lane = threadIdx.x & 63;
    const int total = prefix[count];
    for (;;) {
        u32 t = 0;
        if (lane == 0) t = atomicAdd(&queue[0], 1u);
        t = (u32)__builtin_amdgcn_readfirstlane((int)t);
        if ((int)t >= total) break;
        // image i with prefix[i] <= t < prefix[i+1] (wave-uniform search)
        int lo = 0, hi = count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= (int)t) lo = mid; else hi = mid;
        }
        const U8Job J = jobs[lo];
        wave_tile<PPL, OFF, ALIGNED, false>(J, (int)t - prefix[lo], TH);
    }
    if (lane == 0) {
        __threadfence();
        const u32 nwaves = gridDim.x * kWaves;
        if (atomicAdd(&queue[1], 1u) == nwaves - 1) {
            queue[0] = 0;
            queue[1] = 0;
            __threadfence();
        }
    }
}

__global__ void k_round_mag(const int32_t *s2, uint8_t *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint8_t)round_mag(s2[i]);
}

template <int PPL, int OFF, bool DIR>
hipError_t launch_single_t(const U8Job &j, const U8Shape &s, hipStream_t st)
{
    const int grid = (j.nwt + kWaves - 1) / kWaves;
    if (u8_rows_aligned(j))
        hipLaunchKernelGGL((k_u8_single<PPL, OFF, true, DIR>), dim3(grid), dim3(64 * kWaves), 0, st, j, s.th);
    else
        hipLaunchKernelGGL((k_u8_single<PPL, OFF, false, DIR>), dim3(grid), dim3(64 * kWaves), 0, st, j, s.th);
    return hipGetLastError();
}

template <int PPL, int OFF>
hipError_t launch_single_d(const U8Job &j, const U8Shape &s, hipStream_t st)
{
    return j.dir_type ? launch_single_t<PPL, OFF, true>(j, s, st) : launch_single_t<PPL, OFF, false>(j, s, st);
}

template <int PPL, int OFF>
const void *batched_fn(bool aligned)
{
    return aligned ? reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, true>)
                   : reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, false>);
}

const void *pick_batched(int ppl, int valid, bool aligned)
{
    if (ppl == 16) return valid ? batched_fn<16, 2>(aligned) : batched_fn<16, 0>(aligned);
    return valid ? batched_fn<8, 2>(aligned) : batched_fn<8, 0>(aligned);
}

}  // namespace

bool u8_rows_aligned(const U8Job &j)
{
    return ((reinterpret_cast<uintptr_t>(j.src) | (uintptr_t)j.src_pitch) & 15u) == 0;
}

void u8_tile(U8Job &j, const U8Shape &s)
{
    const int tw = 16 * s.ppl;
    j.ntx = (j.Wo + tw - 1) / tw;
    j.nty = (j.Ho + s.th - 1) / s.th;
    j.nty4 = (j.nty + 3) / 4;
    j.nwt = j.ntx * j.nty4;
    j.mag_vec = ((reinterpret_cast<uintptr_t>(j.mag) | (uintptr_t)j.mag_pitch) & 15u) == 0;
    uintptr_t da = (uintptr_t)j.dir_pitch;
    for (int k = 0; k < 4; ++k) da |= reinterpret_cast<uintptr_t>(j.dir[k]);
    j.dir_vec = (da & 15u) == 0;
}

hipError_t launch_u8_single(const U8Job &j, int border_valid, const U8Shape &s, hipStream_t st)
{
    if (j.nwt <= 0) return hipSuccess;
    if (s.ppl == 16)
        return border_valid ? launch_single_d<16, 2>(j, s, st) : launch_single_d<16, 0>(j, s, st);
    return border_valid ? launch_single_d<8, 2>(j, s, st) : launch_single_d<8, 0>(j, s, st);
}

hipError_t launch_u8_batched(const U8Job *jobs, const int32_t *prefix, int32_t count, uint32_t *queue,
                             int border_valid, bool aligned, const U8Shape &s, int grid, hipStream_t st)
{
    const void *fn = pick_batched(s.ppl, border_valid, aligned);
    int th = s.th;
    void *args[] = {(void *)&jobs, (void *)&prefix, (void *)&count, (void *)&queue, (void *)&th};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

int u8_persistent_grid(const U8Shape &s, int border_valid, bool aligned)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick_batched(s.ppl, border_valid, aligned),
                                                     64 * kWaves, 0) != hipSuccess)
        return 0;
    if (per_cu < 1) per_cu = 1;
    return ncu * per_cu;
}

hipError_t launch_round_mag(const int32_t *s2, uint8_t *out, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_round_mag, dim3((unsigned)blocks), dim3(256), 0, st, s2, out, n);
    return hipGetLastError();
}

}  // namespace s4x5
