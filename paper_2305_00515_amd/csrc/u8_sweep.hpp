// uint8 Sobel sweep for CDNA4 (gfx950), shared by the kernels of the
// four-directional 5x5 operator and of the two-directional operators.
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
//
// The same sweep serves the two-directional operators the paper compares
// with (Sec. 3.1, Sec. 5): the 0 and 90 deg filters of Eq. (sobel5_1) alone,
// and the 3x3 pair of Eq. (sobel3_1), whose filters are [1, 2, 1]
// smoothings of the central differences h_s and v_s the 5x5 passes already
// form.  Their magnitude is Eq. (sobel3_2), S = Gx^2 + Gy^2.

#pragma once

#include "internal.hpp"
#include "load_columns.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

namespace s4x5 {
namespace {

typedef short v2s __attribute__((ext_vector_type(2)));

// Image and output accesses go through global-address-space pointers.  A
// pointer read from memory (the batched job table) is otherwise a generic
// pointer, accessed with FLAT instructions, which count in both vmcnt and
// lgkmcnt and may complete out of order: every wait for one becomes a full
// drain of the row prefetch.
#define GMEM __attribute__((address_space(1)))
typedef unsigned int gv4u __attribute__((ext_vector_type(4)));
typedef unsigned int gv2u __attribute__((ext_vector_type(2)));
// Output rows need no alignment: the HSA runtime runs the GPU in unaligned
// access mode, so a 16-byte store at any byte address is one
// global_store_dwordx4 that writes exactly those 16 bytes.
typedef gv4u gv4u_u __attribute__((aligned(1)));
typedef gv2u gv2u_u __attribute__((aligned(1)));
typedef unsigned int u32;

__device__ __forceinline__ v2s S2(u32 v) { return __builtin_bit_cast(v2s, v); }
__device__ __forceinline__ u32 U2(v2s v) { return __builtin_bit_cast(u32, v); }
__device__ __forceinline__ u32 perm(u32 hi, u32 lo, u32 sel) { return __builtin_amdgcn_perm(hi, lo, sel); }

constexpr u32 kZeroByte = 0x0c;   // v_perm selector that yields 0x00
constexpr int kPD = 4;            // rows loaded ahead of use

// How pixels outside the image read (VALID uses kBmRep: its outputs never
// reach outside).
constexpr int kBmRep = 0;    // the nearest edge pixel
constexpr int kBmZero = 1;   // 0
constexpr int kBmRefl = 2;   // reflect-101: mirrored about the edge pixel

// Operators the sweep computes (the values of the public SOBEL4X5_OP_*).
constexpr int kOp4x5 = 0;   // Eq. (sobel5_1) + Eq. (sobel5_2): four directions, 5x5
constexpr int kOp2x5 = 1;   // the 0 and 90 deg filters of Eq. (sobel5_1) alone
constexpr int kOp2x3 = 2;   // Eq. (sobel3_1) + Eq. (sobel3_2): the 3x3 pair

// Kernels in the binomial form (sweep4): the four-directional operator and
// its 0 / 90 deg pair, without directional planes (see sweep).
constexpr bool binomial_form(int opr, bool dir) { return (opr == kOp4x5 || opr == kOp2x5) && !dir; }

// v_perm selector: byte0 <- byte `lob` of the low source, byte2 <- byte
// `hib` of the high source, bytes 1 and 3 <- 0: two zero-extended pixels.
constexpr u32 pair_sel(int lob, int hib)
{
    return (kZeroByte << 24) | ((4u + (u32)hib) << 16) | (kZeroByte << 8) | (u32)lob;
}

// Round-to-nearest of sqrt(S), saturated to 255.  (float)S is exact below
// 2^24 and monotone above, where the result saturates anyway; v_sqrt_f32 is
// within 1 ulp, and an integer S is never closer than 4.9e-4 to a
// half-integer square root, so rounding the float result is exact.
__device__ __forceinline__ float mag_f(int S) { return __builtin_amdgcn_sqrtf((float)S); }

__device__ __forceinline__ u32 round_mag(int S)
{
    // v_cvt_pk_u8_f32: round to nearest, saturate to [0, 255] (no ties occur)
    return __builtin_amdgcn_cvt_pk_u8_f32(mag_f(S), 0, 0u);
}

// Rounded uint8 magnitude of every S below 2^16, the same function as
// round_mag: k for k^2 - k < S <= k^2 + k (the S whose square root rounds to
// k; ties cannot occur), 0 for S = 0, 255 from 255^2 + 256 = 65281 on.  It
// is built at compile time into device memory; a kernel that rounds through
// it copies it into LDS once per workgroup and then rounds a pixel with one
// clamp (min(S, 65535)) and one LDS byte read instead of a conversion, a
// half-rate square root and a pack.
constexpr int kLutSize = 1 << 16;
struct MagLut {
    uint8_t v[kLutSize];
};
constexpr MagLut make_mag_lut()
{
    MagLut t{};
    int S = 1;
    for (int k = 1; k <= 255; ++k)
        for (const int hi = k * k + k; S <= hi && S < kLutSize; ++S) t.v[S] = (uint8_t)k;
    for (; S < kLutSize; ++S) t.v[S] = 255;
    return t;
}
constexpr MagLut kMagLut = make_mag_lut();
static_assert(kMagLut.v[0] == 0 && kMagLut.v[1] == 1 && kMagLut.v[2] == 1 && kMagLut.v[3] == 2 &&
                  kMagLut.v[1088] == 33 && kMagLut.v[64770] == 254 && kMagLut.v[64771] == 255 &&
                  kMagLut.v[kLutSize - 1] == 255,
              "rounding table");

typedef const uint8_t __attribute__((address_space(3))) lds_u8;

// Copy the table into LDS (`threads` threads of the workgroup, 16 bytes per
// load; every load is issued before the first store).  The caller
// synchronises the workgroup before the first read.
template <int THREADS>
__device__ __forceinline__ void lut_fill(uint8_t *lut)
{
    static_assert(kLutSize % (16 * THREADS) == 0, "table split");
    constexpr int kPer = kLutSize / (16 * THREADS);
    uint4 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = reinterpret_cast<const uint4 *>(kMagLut.v)[threadIdx.x + k * THREADS];
#pragma unroll
    for (int k = 0; k < kPer; ++k) reinterpret_cast<uint4 *>(lut)[threadIdx.x + k * THREADS] = v[k];
}

__device__ __forceinline__ u32 lut_mag(lds_u8 *lut, int S) { return lut[min((u32)S, (u32)kLutSize - 1u)]; }

// The four-directional sweep forms T = S / 2 (below) saturated to 2^15 - 1
// and rounds through a table of min(255, round(sqrt(2 T))) for T < 2^15:
// k for 2T in (k^2 - k, k^2 + k], 255 from 2T >= 255^2 + 256 (T >= 32386),
// so the saturated value rounds like the exact one.
constexpr int kLutTSize = 1 << 15;
struct alignas(16) MagLutT {
    uint8_t v[kLutTSize];
};
constexpr MagLutT make_mag_lut_t()
{
    MagLutT t{};
    int T = 1;
    for (int k = 1; k <= 255; ++k)
        for (const int hi = k * k + k; 2 * T <= hi && T < kLutTSize; ++T) t.v[T] = (uint8_t)k;
    for (; T < kLutTSize; ++T) t.v[T] = 255;
    return t;
}
constexpr MagLutT kMagLutT = make_mag_lut_t();
static_assert(kMagLutT.v[0] == 0 && kMagLutT.v[1] == 1 && kMagLutT.v[2] == 2 && kMagLutT.v[544] == 33 &&
                  kMagLutT.v[32385] == 254 && kMagLutT.v[32386] == 255 && kMagLutT.v[kLutTSize - 1] == 255,
              "rounding table of T = S/2");

// The T table's copy into LDS in two halves: the loads (into registers of
// the calling thread), then the LDS stores.  A kernel issues its first image
// row loads together with the table loads, so that the table's trip through
// L2 overlaps their HBM latency instead of preceding it; the caller
// synchronises the workgroup after fill().
template <int THREADS>
struct LutTFill {
    static_assert(kLutTSize % (16 * THREADS) == 0, "table split");
    static constexpr int kPer = kLutTSize / (16 * THREADS);
    uint4 v[kPer];
    __device__ __forceinline__ void issue()
    {
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = reinterpret_cast<const uint4 *>(kMagLutT.v)[threadIdx.x + k * THREADS];
    }
    __device__ __forceinline__ void fill(uint8_t *lut) const
    {
#pragma unroll
        for (int k = 0; k < kPer; ++k) reinterpret_cast<uint4 *>(lut)[threadIdx.x + k * THREADS] = v[k];
    }
};

template <int THREADS>
__device__ __forceinline__ void lut_fill_t(uint8_t *lut)
{
    LutTFill<THREADS> f;
    f.issue();
    f.fill(lut);
}

// What a sweep runs around its first row loads: nothing, or the table copy
// (issue() before the loads, finish() after them).
struct NoPrelude {
    __device__ __forceinline__ void issue() {}
    __device__ __forceinline__ void finish() {}
};
template <int THREADS>
struct LutPrelude {
    LutTFill<THREADS> f;
    uint8_t *lut;
    __device__ __forceinline__ void issue() { f.issue(); }
    __device__ __forceinline__ void finish()
    {
        f.fill(lut);
        __syncthreads();
    }
};

// Per 16-bit half: min(32767, a^2 + acc) for acc >= 0.  The clamp bit of
// v_pk_mad_i16 saturates the exact a * b + c of each half to the int16
// range, so a sum of squares that overflows int16 reads 32767.
__device__ __forceinline__ u32 sq_sat(u32 a)
{
    u32 r;
    asm("v_pk_mad_i16 %0, %1, %1, 0 clamp" : "=v"(r) : "v"(a));
    return r;
}
__device__ __forceinline__ u32 sq_sat_acc(u32 a, u32 acc)
{
    u32 r;
    asm("v_pk_mad_i16 %0, %1, %1, %2 clamp" : "=v"(r) : "v"(a), "v"(acc));
    return r;
}

// (a << s) | b in one v_lshl_or_b32
__device__ __forceinline__ u32 lshl_or(u32 a, int s, u32 b)
{
    u32 r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(s), "v"(b));
    return r;
}

// a.lo^2 + a.hi^2 of two int16 halves (VOP3P dot with a zero accumulator)
__device__ __forceinline__ int dot2_sq(u32 a)
{
    int r;
    asm("v_dot2_i32_i16 %0, %1, %1, 0" : "=v"(r) : "v"(a));
    return r;
}

// A packed (c, c) constant the optimiser cannot see through, so that
// products with it stay single v_pk_mad_u16 instructions instead of being
// strength-reduced into shift + add pairs.
template <int C>
__device__ __forceinline__ v2s kconst()
{
    u32 r;
    asm("s_mov_b32 %0, %1" : "=s"(r) : "i"((int)(((unsigned)C & 0xffffu) | ((unsigned)C << 16))));
    return S2(r);
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
        hr[j] = s * kconst<2>() + e;
    }
}

// Gy and Hp = Gd+/2 at one output row (columns first).  vr = v_r and a2 =
// v_s of the output row's centre, both for NP + 4 columns.  Every entry of
// K_d+ and K_d- is even, so Gd+/2 and Gd-/2 are integers and take one
// multiply-add less than Gd+- itself.
template <int NP>
__device__ __forceinline__ void responses_y(const v2s (&vr)[NP + 4], const v2s (&a2)[NP + 4],
                                            v2s (&Gy)[NP], v2s (&Hp)[NP])
{
    const v2s k3 = kconst<3>(), k4 = kconst<4>(), k6 = kconst<6>(), km5 = kconst<-5>();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int c = j + 2;
        v2s p4 = vr[c - 2] + vr[c + 2];
        v2s p2 = vr[c - 1] + vr[c + 1];
        Gy[j] = vr[c] * k6 + (p2 * k4 + p4);
        v2s t = (p4 + p2) * k3 + vr[c];
        t = (a2[c - 2] + a2[c + 2]) * km5 + t;
        Hp[j] = a2[c] * k6 + t;
    }
}

// Gx and Hm = Gd-/2 at one output row (rows first) from the row filters of
// the five window rows.
template <int NP>
__device__ __forceinline__ void responses_x(const v2s (&hr0)[NP], const v2s (&hr1)[NP],
                                            const v2s (&hr2)[NP], const v2s (&hr3)[NP],
                                            const v2s (&hr4)[NP], const v2s (&hs0)[NP],
                                            const v2s (&hs2)[NP], const v2s (&hs4)[NP],
                                            v2s (&Gx)[NP], v2s (&Hm)[NP])
{
    const v2s k3 = kconst<3>(), k4 = kconst<4>(), k6 = kconst<6>(), km5 = kconst<-5>();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        v2s x1 = hr0[j] + hr4[j];
        v2s x2 = hr1[j] + hr3[j];
        Gx[j] = hr2[j] * k6 + (x2 * k4 + x1);
        v2s t = (x1 + x2) * k3 + hr2[j];
        t = (hs0[j] + hs4[j]) * km5 + t;
        Hm[j] = hs2[j] * k6 + t;
    }
}

// Gx and Gy of Eq. (sobel3_1) at one output row.  Both filters are a
// [1, 2, 1] smoothing of a central difference: Gx smooths the row
// differences h_s of the rows above, at and below the centre; Gy smooths
// the column differences v_s (row below minus row above, a2 = v_s of the
// centre row for NP + 4 columns) over the three columns around the centre.
template <int NP>
__device__ __forceinline__ void responses_3x3(const v2s (&hs0)[NP], const v2s (&hs1)[NP],
                                              const v2s (&hs2)[NP], const v2s (&a2)[NP + 4],
                                              v2s (&Gx)[NP], v2s (&Gy)[NP])
{
    const v2s k2 = kconst<2>();
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        Gx[j] = hs1[j] * k2 + (hs0[j] + hs2[j]);
        Gy[j] = a2[j + 2] * k2 + (a2[j + 1] + a2[j + 3]);
    }
}

// Row filters of one input row for the four-directional operator in the
// binomial form (see sweep4).  R[k] holds the pixels at column k - 2 (relative
// to the lane's first centre), k in [0, NP + 4).  With the running sums
// b1 = (1 + v) p, b2 = (1 + v)^2 p, b3 = (1 + v)^3 p (anchored at their
// first tap), every filter of the row is a few adds of them:
//   b3[c]               [1, 3, 3, 1] at columns c .. c+3, for the smoothed
//                       image P (columns -2 .. NP-2);
//   hs = p[+1] - p[-1]  = b1[x] - b1[x-1];
//   hr = [-1,-2,0,2,1]  = b3[x-1] - b3[x-2];
//   ch = [3,3,1,3,3]    = 3 (b1[x-2] + b1[x+1]) + p[x];
//   mh = [1,6,8,6,1]    = (b3[x-2] + b3[x-1]) + 2 (b1[x-1] + p[x+1]).
template <int NP>
__device__ __forceinline__ void row_filters_bin(const v2s (&R)[NP + 4], v2s (&b3)[NP + 1], v2s (&hs)[NP],
                                                v2s (&hr)[NP], v2s (&ch)[NP], v2s (&mh)[NP])
{
    const v2s k2 = kconst<2>(), k3 = kconst<3>();
    v2s b1[NP + 3], b2[NP + 2];
#pragma unroll
    for (int k = 0; k < NP + 3; ++k) b1[k] = R[k] + R[k + 1];
#pragma unroll
    for (int k = 0; k < NP + 2; ++k) b2[k] = b1[k] + b1[k + 1];
#pragma unroll
    for (int k = 0; k < NP + 1; ++k) b3[k] = b2[k] + b2[k + 1];
#pragma unroll
    for (int x = 0; x < NP; ++x) {
        hs[x] = b1[x + 2] - b1[x + 1];
        hr[x] = b3[x + 1] - b3[x];
        ch[x] = (b1[x] + b1[x + 3]) * k3 + R[x + 2];
        mh[x] = (b1[x + 1] + R[x + 3]) * k2 + (b3[x] + b3[x + 1]);
    }
}

// The binomial row sums alone (b3 = (1 + v)^3 p), for the operator without
// the diagonal pair.
template <int NP>
__device__ __forceinline__ void row_sums_bin(const v2s (&R)[NP + 4], v2s (&b3)[NP + 1])
{
    v2s b1[NP + 3], b2[NP + 2];
#pragma unroll
    for (int k = 0; k < NP + 3; ++k) b1[k] = R[k] + R[k + 1];
#pragma unroll
    for (int k = 0; k < NP + 2; ++k) b2[k] = b1[k] + b1[k + 1];
#pragma unroll
    for (int k = 0; k < NP + 1; ++k) b3[k] = b2[k] + b2[k + 1];
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
__device__ __forceinline__ void load_row(RawRow<PPL> &r, const GMEM uint8_t *rowp, unsigned ldx, unsigned hx)
{
    // Re-defining the 32-bit column offsets here (an empty asm) keeps their
    // zero extension next to the load, so the load takes the row base from
    // SGPRs and the offset from one VGPR (global_load ... vN, s[..]) instead
    // of a 64-bit VGPR address built by two 64-bit adds a row.
    asm volatile("" : "+v"(ldx), "+v"(hx));
    if constexpr (PPL == 16) {
        const gv4u v = *reinterpret_cast<const GMEM gv4u *>(rowp + ldx);
        r.d[0] = v.x; r.d[1] = v.y; r.d[2] = v.z; r.d[3] = v.w;
    } else {
        const gv2u v = *reinterpret_cast<const GMEM gv2u *>(rowp + ldx);
        r.d[0] = v.x; r.d[1] = v.y;
    }
    r.hw = *reinterpret_cast<const GMEM u32 *>(rowp + hx);
}

// Window byte b (runtime, 0 .. PPL+5; column xo - 2 + b) and its update.
template <int PPL>
__device__ __forceinline__ u32 win_get(const Win<PPL> &w, int b)
{
    u32 word = w.Rt;
    int sh = 8 * (b - PPL - 2);
    if (b < 2) {
        word = w.L;
        sh = 8 * (b + 2);
    } else if (b < PPL + 2) {
#pragma unroll
        for (int m = 0; m < PPL / 4; ++m)
            if (((b - 2) >> 2) == m) word = w.d[m];
        sh = 8 * ((b - 2) & 3);
    }
    return (word >> sh) & 0xffu;
}

template <int PPL>
__device__ __forceinline__ void win_set(Win<PPL> &w, int b, u32 v)
{
    auto put = [&](u32 &word, int pos) {
        const u32 m = 0xffu << (8 * pos);
        word = (word & ~m) | ((v << (8 * pos)) & m);
    };
    if (b < 2) {
        put(w.L, b + 2);
    } else if (b < PPL + 2) {
#pragma unroll
        for (int m = 0; m < PPL / 4; ++m)
            if (((b - 2) >> 2) == m) put(w.d[m], (b - 2) & 3);
    } else {
        put(w.Rt, b - PPL - 2);
    }
}

// Reflect-101 at the right edge, on a lane's window after the halo
// exchange: columns W and W+1 (the only ones past the edge that an output
// inside the image reads) take columns W-2 and W-3.  A lane with an output
// inside the image (xo <= W-1) holds both sources in its window.  Needs
// W >= 3 (narrower images take the byte path).
template <int PPL>
__device__ __forceinline__ void reflect_right(Win<PPL> &w, int xo, int W)
{
    const int nv = W - xo;
    if (nv >= 1 && nv <= PPL + 3) {
        win_set<PPL>(w, nv + 2, win_get<PPL>(w, nv));
        if (nv + 3 <= PPL + 5) win_set<PPL>(w, nv + 3, win_get<PPL>(w, nv - 1));
    }
}

// v_perm selector that fills the left-halo dword of the lane at column 0
// (bytes 2, 3 = columns -2, -1) from its first own dword: replicate puts
// column 0 everywhere, zero puts 0, reflect-101 puts columns 2 and 1.
template <int BM>
constexpr u32 left_sel()
{
    return BM == kBmRep ? 0u : (BM == kBmZero ? 0x0c0c0c0cu : 0x01020c0cu);
}

// Turn a loaded row into the lane's window: border fix-ups, then DPP halo.
template <int PPL, int OFF, int BM>
__device__ __forceinline__ Win<PPL> finish_row(RawRow<PPL> &r, int lane16, int xo, int W,
                                               bool fix_right, bool fix_left)
{
    constexpr int ND = PPL / 4;
    if (fix_right) {
        // own block: bytes at columns >= W take the value of column W-1
        // (zero border: 0; reflect-101 corrects columns W, W+1 below)
        const int nv = W - xo;
        if (nv < PPL) {
            const int lb = nv >= 1 ? nv - 1 : ((W - 1) & (PPL - 1));
            const u32 fill = BM == kBmZero ? 0u : byte_of<PPL>(r.d, lb) * 0x01010101u;
#pragma unroll
            for (int m = 0; m < ND; ++m) r.d[m] = keep_bytes(r.d[m], nv - 4 * m, fill);
        }
        // right halo dword of lane 15 (nominal columns xo+PPL .. xo+PPL+3)
        const int nh = W - (xo + PPL);
        if (lane16 == 15 && nh < 4) {
            const int lb = nh >= 1 ? nh - 1 : ((W - 1) & 3);
            const u32 fill = BM == kBmZero ? 0u : ((r.hw >> (8 * lb)) & 0xffu) * 0x01010101u;
            r.hw = keep_bytes(r.hw, nh, fill);
        }
    }
    if (OFF == 0 && fix_left && lane16 == 0 && xo == 0) {
        if constexpr (BM == kBmRep)
            r.hw = (r.d[0] & 0xffu) * 0x01010101u;
        else
            r.hw = perm(r.d[0], r.d[0], left_sel<BM>());
    }
    Win<PPL> w;
#pragma unroll
    for (int m = 0; m < ND; ++m) w.d[m] = r.d[m];
    // row_shr:1 -> value of lane-1 within the 16-lane row; lane 0 keeps `old`
    w.L = (u32)__builtin_amdgcn_update_dpp((int)r.hw, (int)r.d[ND - 1], 0x111, 0xf, 0xf, false);
    // row_shl:1 -> value of lane+1; lane 15 keeps `old`
    w.Rt = (u32)__builtin_amdgcn_update_dpp((int)r.hw, (int)r.d[0], 0x101, 0xf, 0xf, false);
    if constexpr (BM == kBmRefl)
        if (fix_right) reflect_right<PPL>(w, xo, W);
    return w;
}

// Border fix-ups of the group halo dwords for a fast wave at the image's
// left / right edge (its lanes' own blocks all lie inside the row): loop-
// invariant per-lane masks and selectors, so the fix-up is two v_perm + two
// v_bfi per row and no branch.  mask bits set = keep the loaded byte.
struct EdgeFix {
    u32 keep_l;   // lane 0 at column 0 (OFF == 0): 0, else all ones
    u32 keep_r;   // lane 15 whose halo reaches column W: bytes < W - (xo + ppl), else all ones
    u32 sel_r;    // v_perm selector of the replacement bytes from (hw, last own dword)
};

// sel_r by border rule, for nh = W - (xo + ppl) valid halo bytes (0..3):
//   replicate: the byte of column W-1 everywhere;
//   zero:      0;
//   reflect-101: halo byte k (column W + k - nh, k < 2 are the only ones
//   read) takes column W - 2 - (k - nh), which is byte 2 + 2nh - k of the
//   pair (last own dword = bytes 0..3, hw = bytes 4..7).
template <int PPL, int OFF, int BM>
__device__ __forceinline__ EdgeFix edge_fix(int lane16, int xo, int W, bool at_left, bool at_right)
{
    EdgeFix e;
    e.keep_l = (OFF == 0 && at_left && lane16 == 0 && xo == 0) ? 0u : ~0u;
    const int nh = W - (xo + PPL);   // valid bytes of the right halo dword (>= 0 here)
    const bool r = at_right && lane16 == 15 && nh < 4;
    e.keep_r = r ? ((1u << (8 * nh)) - 1u) : ~0u;
    if constexpr (BM == kBmRep) {
        e.sel_r = (nh >= 1 ? (u32)(4 + nh - 1) : 3u) * 0x01010101u;
    } else if constexpr (BM == kBmZero) {
        e.sel_r = 0x0c0c0c0cu;
    } else {
        u32 sel = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32 b = (k >= nh && k <= 1 && nh >= 0) ? (u32)(2 + 2 * nh - k) : kZeroByte;
            sel |= b << (8 * k);
        }
        e.sel_r = sel;
    }
    return e;
}

template <int PPL, int BM>
__device__ __forceinline__ void apply_edge(RawRow<PPL> &r, const EdgeFix &e)
{
    constexpr int ND = PPL / 4;
    const u32 fr = perm(r.hw, r.d[ND - 1], e.sel_r);          // right replacement bytes
    const u32 fl = perm(r.d[0], r.d[0], left_sel<BM>());       // left replacement bytes
    r.hw = (r.hw & e.keep_r) | (fr & ~e.keep_r);
    r.hw = (r.hw & e.keep_l) | (fl & ~e.keep_l);
}

// Slow path for rows that are not 16-byte aligned (and for reflect-101 on
// images narrower than 3): every window byte is read on its own at the
// column the border rule maps it to.  row_in: the row lies inside the image
// (zero border: otherwise every byte reads 0).
template <int PPL, int BM>
__device__ __forceinline__ Win<PPL> load_row_bytes(const GMEM uint8_t *rowp, int xo, int W, bool row_in)
{
    Win<PPL> w;
    auto px = [&](int x) -> u32 {
        if constexpr (BM == kBmRefl) {
            return rowp[reflect101(x, W)];
        } else {
            const u32 v = rowp[x < 0 ? 0 : (x >= W ? W - 1 : x)];
            if constexpr (BM == kBmZero) return (row_in && x >= 0 && x < W) ? v : 0u;
            return v;
        }
    };
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

// Directional planes of one output row for one lane (int16 or int32, as the
// job asks), from Gx, Gy, Hp = Gd+/2 and Hm = Gd-/2 (two-directional
// operators: Gx and Gy only).
template <int NP, bool FAST, int OPR>
__device__ __forceinline__ void store_dir(const U8Job &J, int yo, int xo, bool row_ok, const v2s (&Gx)[NP],
                                          const v2s (&Hp)[NP], const v2s (&Gy)[NP], const v2s (&Hm)[NP])
{
    constexpr int PPL = 2 * NP;
    if (!FAST && !row_ok) return;
    const int nvalid = J.Wo - xo;          // pixels of this lane inside the image
    if (!FAST && nvalid <= 0) return;
    const bool full = FAST || nvalid >= PPL;
    if (J.dir_type != 0) {
        // plane order: 0 deg Gx, 45 deg Gd, 90 deg Gy, 135 deg Gdt (the
        // two-directional operators write planes 0 and 2)
        v2s P[4][NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            P[0][j] = Gx[j];
            P[2][j] = Gy[j];
            if constexpr (OPR == kOp4x5) {
                P[1][j] = Hp[j] + Hm[j];          // Gd  = (Gd+ + Gd-)/2 = Hp + Hm
                P[3][j] = Hp[j] - Hm[j];          // Gdt = (Gd+ - Gd-)/2 = Hp - Hm
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (OPR != kOp4x5 && (k & 1)) continue;
            GMEM char *base = (GMEM char *)J.dir[k] + (int64_t)yo * J.dir_pitch;
            if (J.dir_type == 1) {
                u32 o[NP];   // int16 pixels (2m, 2m+1)
#pragma unroll
                for (int m = 0; m < NP; ++m) {
                    const int a = 2 * m;
                    o[m] = a < NP ? perm(U2(P[k][a + 1]), U2(P[k][a]), 0x05040100u)
                                  : perm(U2(P[k][a - NP + 1]), U2(P[k][a - NP]), 0x07060302u);
                }
                GMEM int16_t *p = reinterpret_cast<GMEM int16_t *>(base) + xo;
                if (FAST || full) {
#pragma unroll
                    for (int m = 0; m < NP; m += 4)
                        *reinterpret_cast<GMEM gv4u_u *>(p + 2 * m) = gv4u{o[m], o[m + 1], o[m + 2], o[m + 3]};
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
                GMEM int32_t *p = reinterpret_cast<GMEM int32_t *>(base) + xo;
                if (FAST || full) {
#pragma unroll
                    for (int q = 0; q < PPL; q += 4)
                        *reinterpret_cast<GMEM gv4u_u *>(p + q) = gv4u{(u32)o[q], (u32)o[q + 1], (u32)o[q + 2], (u32)o[q + 3]};
                } else {
#pragma unroll
                    for (int q = 0; q < PPL; ++q)
                        if (q < nvalid) p[q] = o[q];
                }
            }
        }
    }
}

// Stores of one output row for one lane, from Gx, Gy, Hp = Gd+/2 and
// Hm = Gd-/2 (two-directional operators: Gx and Gy only; Hp, Hm unread).
template <int NP, bool DIR, bool FAST, int OPR, bool LUT>
__device__ __forceinline__ void store_row(const U8Job &J, int yo, int xo, bool row_ok,
                                          const v2s (&Gx)[NP], const v2s (&Hp)[NP],
                                          const v2s (&Gy)[NP], const v2s (&Hm)[NP], lds_u8 *lut)
{
    constexpr int PPL = 2 * NP;
    if (!FAST && !row_ok) return;
    const int nvalid = J.Wo - xo;          // pixels of this lane inside the image
    if (!FAST && nvalid <= 0) return;
    const bool full = FAST || nvalid >= PPL;
    if (DIR ? J.mag != nullptr : true) {
        u32 out[PPL / 4];
        u32 mb[LUT ? PPL : 1];   // LUT: the rounded byte of every pixel
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            // S = Gx^2 + Gy^2 + Gd^2 + Gdt^2 = Gx^2 + Gy^2 + 2 (Hp^2 + Hm^2):
            // byte permutes pair (Gx, Gy) and (Hp, Hm) of one pixel, v_dot2
            // squares and sums each pair.
            const u32 xyl = perm(U2(Gy[j]), U2(Gx[j]), 0x05040100u);
            const u32 xyh = perm(U2(Gy[j]), U2(Gx[j]), 0x07060302u);
            int sl, sh;
            if constexpr (OPR == kOp4x5) {
                const u32 hhl = perm(U2(Hm[j]), U2(Hp[j]), 0x05040100u);
                const u32 hhh = perm(U2(Hm[j]), U2(Hp[j]), 0x07060302u);
                sl = 2 * dot2_sq(hhl) + dot2_sq(xyl);
                sh = 2 * dot2_sq(hhh) + dot2_sq(xyh);
            } else {
                sl = dot2_sq(xyl);
                sh = dot2_sq(xyh);
            }
            const int ql = j, qh = j + NP;   // pixel indices inside the lane
            if constexpr (LUT) {
                mb[ql] = lut_mag(lut, sl);
                mb[qh] = lut_mag(lut, sh);
            } else {
                const float fl = mag_f(sl), fh = mag_f(sh);
                // the first byte written into a word starts from any value: all
                // four bytes of every word are overwritten
                out[ql >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(fl, ql & 3, (ql & 3) ? out[ql >> 2] : __builtin_bit_cast(u32, fl));
                out[qh >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(fh, qh & 3, (qh & 3) ? out[qh >> 2] : __builtin_bit_cast(u32, fh));
            }
        }
        if constexpr (LUT) {
            // three shift-ors a word (each byte is zero-extended)
#pragma unroll
            for (int w = 0; w < PPL / 4; ++w)
                out[w] = lshl_or(lshl_or(mb[4 * w + 3], 8, mb[4 * w + 2]), 16, lshl_or(mb[4 * w + 1], 8, mb[4 * w]));
        }
        GMEM uint8_t *p = ((GMEM uint8_t *)J.mag + (int64_t)yo * J.mag_pitch) + (unsigned)xo;
        if (FAST || full) {
            if constexpr (PPL == 16)
                *reinterpret_cast<GMEM gv4u_u *>(p) = gv4u{out[0], out[1], out[2], out[3]};
            else
                *reinterpret_cast<GMEM gv2u_u *>(p) = gv2u{out[0], out[1]};
        } else {
#pragma unroll
            for (int q = 0; q < PPL; ++q)
                if (q < nvalid) p[q] = (uint8_t)(out[q >> 2] >> (8 * (q & 3)));
        }
    }
    if (DIR) store_dir<NP, FAST, OPR>(J, yo, xo, row_ok, Gx, Hp, Gy, Hm);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }


// What one wave sweeps: per lane the output column xo of its first pixel,
// per 16-lane group the first output row yo0 and its row count nrow (0 for
// an idle group); the wave walks niter rows (the largest nrow).  fix_right /
// fix_left: the wave touches the right / left image border (replicate).
struct Sweep {
    int xo, yo0, nrow, niter;
    bool fix_right, fix_left;
};

// Sweep the wave's tiles top to bottom.  FAST: every group active for all
// niter rows, every lane's block and outputs inside the image, 16-byte
// aligned input rows (EDGE: with the group-halo fix-ups of an image edge):
// the loop body has no branches, so the compiler can schedule across steps.
// BLOCKS: whole 5-step blocks in a single-exit loop plus a tail (long row
// ranges); otherwise one loop that leaves after any step (short row ranges
// of the batched kernel, where the tail's extra code costs more than the
// waits it saves).
template <int PPL, int OFF, bool ALIGNED, bool DIR, bool FAST, bool EDGE, int OPR, int BM, bool LUT, bool BLOCKS>
__device__ __forceinline__ void sweep_sep(const U8Job &J, const Sweep &g, lds_u8 *lut)
{
    static_assert(!EDGE || FAST, "edge fix-ups by mask exist for fast waves only");
    constexpr int NP = PPL / 2;
    const int lane16 = threadIdx.x & 15;
    const int xo = g.xo, yo0 = g.yo0, nrow = g.nrow, niter = g.niter;
    const int W = J.W;
    const int ymax = J.H - 1;
    const int yin0 = yo0 + OFF - 2;                  // input row of window slot 0
    const int tlast = niter + 3;                     // last input row slot needed

    // load columns: the lane's aligned block and the group's outer halo dwords
    const LoadCols lc = load_columns(xo, lane16, W, PPL);
    const unsigned ldx = lc.ldx, hx = lc.hx;
    const bool fix_right = FAST ? false : g.fix_right;
    const bool fix_left = FAST ? false : g.fix_left;
    const EdgeFix efix = edge_fix<PPL, OFF, BM>(lane16, xo, W, EDGE && g.fix_left, EDGE && g.fix_right);

    const GMEM uint8_t *src = (const GMEM uint8_t *)J.src;
    const int64_t pitch = J.src_pitch;
    // input row of slot t under the border rule (zero border: the nearest
    // row, whose bytes row_in() then discards)
    auto row_of = [&](int t) {
        if constexpr (BM == kBmRefl) return reflect101(yin0 + t, J.H);
        else return clampi(yin0 + t, 0, ymax);
    };
    auto row_in = [&](int t) { return (unsigned)(yin0 + t) <= (unsigned)ymax; };
    auto rowp = [&](int t) { return src + (int64_t)row_of(t) * pitch; };

    // Rings indexed by input row mod 5 (A2 and B by the row they are centred
    // on).  Live ranges are short: an unpacked row lives 3 steps, v_s (A2) and
    // the pair sums B 2-3 steps, the row filters 5 steps.
    v2s Rr[5][NP + 4];
    v2s A2r[5][NP + 4], Br[5][NP + 4];
    v2s HR[5][NP], HS[5][NP];
    RawRow<PPL> raw[5];

    // FAST waves load a row past the end as a repeat of the last needed row
    // (a cache hit) instead of branching around the load.
    auto fetch = [&](int t, RawRow<PPL> &r) {
        if constexpr (ALIGNED) load_row<PPL>(r, rowp(FAST ? min(t, tlast) : t), ldx, hx);
    };
    auto fetch_if = [&](int t, RawRow<PPL> &r) {
        if (FAST || t <= tlast) fetch(t, r);
    };
    auto process = [&](int t, RawRow<PPL> &r, v2s (&R)[NP + 4], v2s (&hr)[NP], v2s (&hs)[NP]) {
        Win<PPL> w;
        if constexpr (ALIGNED && BM == kBmZero) {
            if (!row_in(t)) {
#pragma unroll
                for (int m = 0; m < PPL / 4; ++m) r.d[m] = 0;
                r.hw = 0;
            }
        }
        if constexpr (EDGE) apply_edge<PPL, BM>(r, efix);
        if constexpr (ALIGNED)
            w = finish_row<PPL, OFF, BM>(r, lane16, xo, W, fix_right, fix_left);
        else
            w = load_row_bytes<PPL, BM>(rowp(t), xo, W, row_in(t));
        unpack<PPL, OFF>(w, R);
        row_filters<NP>(R, hr, hs);
    };

    // prologue: rows t = 0..4 in flight, rows 0..3 processed (which frees
    // their slots), then rows 5 .. 3 + kPD.  Row t always lives in raw[t % 5].
    static_assert(kPD >= 1 && kPD <= 4, "prefetch distance must fit the 5-slot ring");
    // The loads stay in row order (scheduling barriers): the loop's first
    // step consumes row 4 and its wait is merged with the steady state at
    // the loop header, so row 4 has to be older than rows 5 .. 3 + kPD.  Left
    // free, the scheduler sinks row 4's load below the processing of rows
    // 0..3 and after the later rows, and the merged wait drains every row in
    // flight once per five rows.
#pragma unroll
    for (int t = 0; t < 5; ++t) fetch_if(t, raw[t]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) process(t, raw[t], Rr[t], HR[t], HS[t]);
#pragma unroll
    for (int t = 5; t < 4 + kPD; ++t) {
        __builtin_amdgcn_sched_barrier(0);
        fetch_if(t, raw[t % 5]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NP + 4; ++c) {
        A2r[1][c] = Rr[2][c] - Rr[0][c];        // v_s centred on row 1
        A2r[2][c] = Rr[3][c] - Rr[1][c];        // v_s centred on row 2
        Br[2][c] = A2r[1][c] + A2r[2][c];       // B(2) = v_s(1) + v_s(2)
    }

    // step i: input row t = i + 4 enters; output row i has its centre at t - 2.
    // v_r(y) = v_s(y-1) + 2 v_s(y) + v_s(y+1) = B(y) + B(y+1).
    auto step = [&](int i, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int s0 = p, s1 = (p + 1) % 5, s2 = (p + 2) % 5, s3 = (p + 3) % 5, s4 = (p + 4) % 5;
        constexpr int sp = (p + 4 + kPD) % 5;
        fetch_if(i + 4 + kPD, raw[sp]);
        process(i + 4, raw[s4], Rr[s4], HR[s4], HS[s4]);
        v2s vr[NP + 4];
#pragma unroll
        for (int c = 0; c < NP + 4; ++c) {
            A2r[s3][c] = Rr[s4][c] - Rr[s2][c];     // v_s(t-1)
            Br[s3][c] = A2r[s2][c] + A2r[s3][c];    // B(t-1)
            vr[c] = Br[s2][c] + Br[s3][c];          // v_r(t-2)
        }
        v2s Gx[NP], Hp[NP], Gy[NP], Hm[NP];
        if constexpr (OPR == kOp2x3) {
            // window rows 1..3 around the centre row; the unused row filters,
            // pair sums and v_r are dropped by the compiler
            responses_3x3<NP>(HS[s1], HS[s2], HS[s3], A2r[s2], Gx, Gy);
        } else {
            responses_y<NP>(vr, A2r[s2], Gy, Hp);
            responses_x<NP>(HR[s0], HR[s1], HR[s2], HR[s3], HR[s4], HS[s0], HS[s2], HS[s4], Gx, Hm);
        }
        store_row<NP, DIR, FAST, OPR, LUT>(J, yo0 + i, xo, FAST || i < nrow, Gx, Hp, Gy, Hm, lut);
        // keep each row's work in its own scheduling region: interleaving
        // rows buys little ILP and costs the registers of a second row
        __builtin_amdgcn_sched_barrier(0);
    };

    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    using P3 = std::integral_constant<int, 3>;
    using P4 = std::integral_constant<int, 4>;
    // Whole 5-step blocks in a loop with one exit, then the 0..4 remaining
    // steps after it.  Exits from inside the loop become flow blocks with an
    // edge back to the loop header; the memory-wait analysis merges their
    // state (a row loaded one step earlier) into the header and waits for
    // every row in flight there, once per five rows.
    if constexpr (!BLOCKS) {
        for (int i = 0; i < niter; i += 5) {
            step(i, P0{});
            if (i + 1 >= niter) break;
            step(i + 1, P1{});
            if (i + 2 >= niter) break;
            step(i + 2, P2{});
            if (i + 3 >= niter) break;
            step(i + 3, P3{});
            if (i + 4 >= niter) break;
            step(i + 4, P4{});
        }
        return;
    }
    const int nfull = niter - niter % 5;
    for (int i = 0; i < nfull; i += 5) {
        step(i, P0{});
        step(i + 1, P1{});
        step(i + 2, P2{});
        step(i + 3, P3{});
        step(i + 4, P4{});
    }
    if (nfull < niter) {
        step(nfull, P0{});
        if (nfull + 1 < niter) {
            step(nfull + 1, P1{});
            if (nfull + 2 < niter) {
                step(nfull + 2, P2{});
                if (nfull + 3 < niter) step(nfull + 3, P3{});
            }
        }
    }
}

// Magnitude bytes of one output row for one lane (mb[q]: pixel q of the
// lane, zero-extended), packed with three shift-ors a word.
template <int PPL, bool FAST>
__device__ __forceinline__ void store_mag_bytes(const U8Job &J, int yo, int xo, bool row_ok, const u32 (&mb)[PPL])
{
    if (!FAST && !row_ok) return;
    const int nvalid = J.Wo - xo;
    if (!FAST && nvalid <= 0) return;
    u32 out[PPL / 4];
#pragma unroll
    for (int w = 0; w < PPL / 4; ++w)
        out[w] = lshl_or(lshl_or(mb[4 * w + 3], 8, mb[4 * w + 2]), 16, lshl_or(mb[4 * w + 1], 8, mb[4 * w]));
    GMEM uint8_t *p = ((GMEM uint8_t *)J.mag + (int64_t)yo * J.mag_pitch) + (unsigned)xo;
    if (FAST || nvalid >= PPL) {
        if constexpr (PPL == 16)
            *reinterpret_cast<GMEM gv4u_u *>(p) = gv4u{out[0], out[1], out[2], out[3]};
        else
            *reinterpret_cast<GMEM gv2u_u *>(p) = gv2u{out[0], out[1]};
    } else {
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            if (q < nvalid) p[q] = (uint8_t)(out[q >> 2] >> (8 * (q & 3)));
    }
}

// 5x5 sweep in the binomial form, magnitude only: the four-directional
// operator, or (OPR == kOp2x5) its 0 and 90 deg filters alone, for which
// S = Gx^2 + Gy^2 = 2 (E1^2 + E2^2) and the diagonal terms below are
// skipped.  With u one row down and v one column right, the 0 and 90 deg filters of
// Eq. (sobel5_1) share the factor (1 + u)^3 (1 + v)^3:
//   K_x + K_y = 2 (1 + u)^3 (1 + v)^3 (uv - 1),
//   K_x - K_y = 2 (1 + u)^3 (1 + v)^3 (v - u),
// so with P the [1,3,3,1] x [1,3,3,1] smoothing of the image, anchored at
// its top-left tap,
//   E1 = (Gx + Gy) / 2 = P(y-1, x-1) - P(y-2, x-2),
//   E2 = (Gx - Gy) / 2 = P(y-2, x-1) - P(y-1, x-2),
// and Gx = E1 + E2, Gy = E1 - E2.  The diagonal pair is Hp = Gd+/2 and
// Hm = Gd-/2 (K_d+- = K_d +- K_dt, Eq. (sobel5_kd+-); Gd = Hp + Hm and
// Gdt = Hp - Hm, Eq. (sobel5_kd)), both from row filters:
//   Hp = ch(y+2) - ch(y-2) + mh(y+1) - mh(y-1)       (the rows of K_d+ / 2)
//   Hm = [3,3,1,3,3]_v hr + [-5,0,6,0,-5]_v hs       (Eq. (sobel5_4) / 2)
// Then S = Gx^2 + Gy^2 + Gd^2 + Gdt^2 = 2 (E1^2 + E2^2 + Hp^2 + Hm^2) = 2 T.
// |E| <= 16320 and |H| <= 8925, so T is summed on the packed int16 halves,
// saturating at 2^15 - 1, and rounded through the table of round(sqrt(2 T)):
// four multiply-adds and one LDS byte read a pixel pair.
//
// Vertical passes on a ring of five input rows (ring slot = input slot mod
// 5, a compile-time index in the unrolled loop): the P smoothing as three
// running pair sums, Hp and Hm as partial sums of the outputs still open
// that each new row adds its terms to (Hp kept negated until its last row).
// The LDS reads of one row's magnitudes are issued at the end of its step
// and consumed by the next step's store, so their latency hides behind a
// whole row of arithmetic.
template <int PPL, int OFF, bool ALIGNED, bool FAST, bool EDGE, int BM, bool BLOCKS, int OPR, class Prelude>
__device__ __forceinline__ void sweep4(const U8Job &J, const Sweep &g, lds_u8 *lut, Prelude &pre)
{
    static_assert(!EDGE || FAST, "edge fix-ups by mask exist for fast waves only");
    static_assert(OPR == kOp4x5 || OPR == kOp2x5, "binomial form of the 5x5 operators");
    constexpr int NP = PPL / 2;
    constexpr bool DIAG = OPR == kOp4x5;   // the diagonal pair Hp, Hm too
    const int lane16 = threadIdx.x & 15;
    const int xo = g.xo, yo0 = g.yo0, nrow = g.nrow, niter = g.niter;
    const int W = J.W;
    const int ymax = J.H - 1;
    const int yin0 = yo0 + OFF - 2;                  // input row of window slot 0
    const int tlast = niter + 3;                     // last input row slot needed

    const LoadCols lc = load_columns(xo, lane16, W, PPL);
    const unsigned ldx = lc.ldx, hx = lc.hx;
    const bool fix_right = FAST ? false : g.fix_right;
    const bool fix_left = FAST ? false : g.fix_left;
    const EdgeFix efix = edge_fix<PPL, OFF, BM>(lane16, xo, W, EDGE && g.fix_left, EDGE && g.fix_right);

    const GMEM uint8_t *src = (const GMEM uint8_t *)J.src;
    const int64_t pitch = J.src_pitch;
    auto row_of = [&](int t) {
        if constexpr (BM == kBmRefl) return reflect101(yin0 + t, J.H);
        else return clampi(yin0 + t, 0, ymax);
    };
    auto row_in = [&](int t) { return (unsigned)(yin0 + t) <= (unsigned)ymax; };
    auto rowp = [&](int t) { return src + (int64_t)row_of(t) * pitch; };

    RawRow<PPL> raw[5];
    v2s b3r[5][NP + 1], v1r[5][NP + 1], v2r[5][NP + 1], Pr[5][NP + 1];
    v2s nacc[5][NP], hacc[5][NP];
    u32 mb[PPL];   // rounded magnitudes of the last output row (LDS reads in flight)

    auto fetch = [&](int t, RawRow<PPL> &r) {
        if constexpr (ALIGNED) load_row<PPL>(r, rowp(FAST ? min(t, tlast) : t), ldx, hx);
    };
    auto fetch_if = [&](int t, RawRow<PPL> &r) {
        if (FAST || t <= tlast) fetch(t, r);
    };
    auto window = [&](int t, RawRow<PPL> &r, v2s (&R)[NP + 4]) {
        Win<PPL> w;
        if constexpr (ALIGNED && BM == kBmZero) {
            if (!row_in(t)) {
#pragma unroll
                for (int m = 0; m < PPL / 4; ++m) r.d[m] = 0;
                r.hw = 0;
            }
        }
        if constexpr (EDGE) apply_edge<PPL, BM>(r, efix);
        if constexpr (ALIGNED)
            w = finish_row<PPL, OFF, BM>(r, lane16, xo, W, fix_right, fix_left);
        else
            w = load_row_bytes<PPL, BM>(rowp(t), xo, W, row_in(t));
        unpack<PPL, OFF>(w, R);
    };

    // Input slot t (ring slot S = t % 5; H = min(t, 4) earlier slots exist).
    // With H == 4 it completes output row t - 4: E1, E2, Hp, Hm.
    auto ingest = [&](int t, auto sc, auto hc, v2s (&E1)[NP], v2s (&E2)[NP], v2s (&Hp)[NP], v2s (&Hm)[NP]) {
        constexpr int S = decltype(sc)::value, H = decltype(hc)::value;
        constexpr int S1 = (S + 4) % 5, S2 = (S + 3) % 5, S3 = (S + 2) % 5, S4 = (S + 1) % 5;   // t-1 .. t-4
        v2s R[NP + 4];
        window(t, raw[S], R);
        v2s hs[NP], hr[NP], ch[NP], mh[NP];
        if constexpr (DIAG)
            row_filters_bin<NP>(R, b3r[S], hs, hr, ch, mh);
        else
            row_sums_bin<NP>(R, b3r[S]);
#pragma unroll
        for (int k = 0; k < NP + 1; ++k) {
            if constexpr (H >= 1) v1r[S1][k] = b3r[S1][k] + b3r[S][k];   // rows t-1, t
            if constexpr (H >= 2) v2r[S2][k] = v1r[S2][k] + v1r[S1][k];  // rows t-2 .. t
            if constexpr (H >= 3) Pr[S3][k] = v2r[S3][k] + v2r[S2][k];   // P at row t-3
        }
        const v2s k3 = kconst<3>(), km5 = kconst<-5>(), k6 = kconst<6>();
#pragma unroll
        for (int x = 0; x < NP; ++x) {
            if constexpr (DIAG) {
                // Hm of output r - 2 + d takes, from row r: 3 hr - 5 hs at d = -2
                // and +2, 3 hr at d = -1 and +1, hr + 6 hs at d = 0
                const v2s B = hr[x] * k3;
                const v2s A = hs[x] * km5 + B;
                const v2s C = hs[x] * k6 + hr[x];
                nacc[S][x] = ch[x];
                hacc[S][x] = A;
                if constexpr (H >= 1) {
                    nacc[S1][x] = nacc[S1][x] + mh[x];
                    hacc[S1][x] = hacc[S1][x] + B;
                }
                if constexpr (H >= 2) hacc[S2][x] = hacc[S2][x] + C;
                if constexpr (H >= 3) {
                    nacc[S3][x] = nacc[S3][x] - mh[x];
                    hacc[S3][x] = hacc[S3][x] + B;
                }
                if constexpr (H >= 4) {
                    Hp[x] = ch[x] - nacc[S4][x];
                    Hm[x] = hacc[S4][x] + A;
                }
            }
            if constexpr (H >= 4) {
                E1[x] = Pr[S3][x + 1] - Pr[S4][x];
                E2[x] = Pr[S4][x + 1] - Pr[S3][x];
            }
        }
    };

    // T of one output row and its table reads (into mb)
    auto mag_issue = [&](const v2s (&E1)[NP], const v2s (&E2)[NP], const v2s (&Hp)[NP], const v2s (&Hm)[NP]) {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            u32 T = sq_sat(U2(E1[j]));
            T = sq_sat_acc(U2(E2[j]), T);
            if constexpr (DIAG) {
                T = sq_sat_acc(U2(Hp[j]), T);
                T = sq_sat_acc(U2(Hm[j]), T);
            }
            mb[j] = lut[T & 0xffffu];
            mb[j + NP] = lut[T >> 16];
        }
    };

    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    using P3 = std::integral_constant<int, 3>;
    using P4 = std::integral_constant<int, 4>;

    // step i: input slot i + 4 enters and completes output row i; the
    // magnitudes of row i - 1 are stored (FIRST: there is none).
    auto step = [&](int i, auto phase, auto first) {
        constexpr int p = decltype(phase)::value;   // i % 5
        constexpr bool FIRST = decltype(first)::value;
        fetch_if(i + 4 + kPD, raw[(p + 4 + kPD) % 5]);
        v2s E1[NP], E2[NP], Hp[NP], Hm[NP];
        ingest(i + 4, std::integral_constant<int, (p + 4) % 5>{}, P4{}, E1, E2, Hp, Hm);
        if constexpr (!FIRST) store_mag_bytes<PPL, FAST>(J, yo0 + i - 1, xo, FAST || i - 1 < nrow, mb);
        mag_issue(E1, E2, Hp, Hm);
        __builtin_amdgcn_sched_barrier(0);
    };

    // prologue: rows 0..4 in flight, slots 0..3 ingested, rows 5 .. 3 + kPD
    // loaded (row t always lives in raw[t % 5]; the loads stay in row order,
    // as in the separable sweep)
    static_assert(kPD >= 1 && kPD <= 4, "prefetch distance must fit the 5-slot ring");
    pre.issue();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 5; ++t) fetch_if(t, raw[t]);
    __builtin_amdgcn_sched_barrier(0);
    pre.finish();
    __builtin_amdgcn_sched_barrier(0);
    {
        v2s d0[NP], d1[NP], d2[NP], d3[NP];   // no output yet
        ingest(0, P0{}, P0{}, d0, d1, d2, d3);
        __builtin_amdgcn_sched_barrier(0);
        ingest(1, P1{}, P1{}, d0, d1, d2, d3);
        __builtin_amdgcn_sched_barrier(0);
        ingest(2, P2{}, P2{}, d0, d1, d2, d3);
        __builtin_amdgcn_sched_barrier(0);
        ingest(3, P3{}, P3{}, d0, d1, d2, d3);
    }
#pragma unroll
    for (int t = 5; t < 4 + kPD; ++t) {
        __builtin_amdgcn_sched_barrier(0);
        fetch_if(t, raw[t % 5]);
    }
    __builtin_amdgcn_sched_barrier(0);
    using Yes = std::true_type;
    using No = std::false_type;
    step(0, P0{}, Yes{});

    if constexpr (!BLOCKS) {
        for (int i = 1; i < niter; i += 5) {
            step(i, P1{}, No{});
            if (i + 1 >= niter) break;
            step(i + 1, P2{}, No{});
            if (i + 2 >= niter) break;
            step(i + 2, P3{}, No{});
            if (i + 3 >= niter) break;
            step(i + 3, P4{}, No{});
            if (i + 4 >= niter) break;
            step(i + 4, P0{}, No{});
        }
    } else {
        // whole 5-step blocks in a loop with one exit, then the 0..4 left
        const int nfull = 1 + (niter - 1) / 5 * 5;
        for (int i = 1; i < nfull; i += 5) {
            step(i, P1{}, No{});
            step(i + 1, P2{}, No{});
            step(i + 2, P3{}, No{});
            step(i + 3, P4{}, No{});
            step(i + 4, P0{}, No{});
        }
        if (nfull < niter) {
            step(nfull, P1{}, No{});
            if (nfull + 1 < niter) {
                step(nfull + 1, P2{}, No{});
                if (nfull + 2 < niter) {
                    step(nfull + 2, P3{}, No{});
                    if (nfull + 3 < niter) step(nfull + 3, P4{}, No{});
                }
            }
        }
    }
    store_mag_bytes<PPL, FAST>(J, yo0 + niter - 1, xo, FAST || niter - 1 < nrow, mb);
}

// The 5x5 operators' magnitude-only kernels (four directions, or the 0 and
// 90 deg pair alone) take the binomial form: its passes run once per input
// row, and it rounds on int16.  Kernels that may write directional planes
// are bound by those stores (9 or 17 bytes a pixel) and keep the separable
// form, whose per-input-row work is lighter (their row ranges are short),
// as does the 3x3 pair.
template <int PPL, int OFF, bool ALIGNED, bool DIR, bool FAST, bool EDGE, int OPR, int BM, bool LUT, bool BLOCKS = true,
          class Prelude = NoPrelude>
__device__ __forceinline__ void sweep(const U8Job &J, const Sweep &g, lds_u8 *lut, Prelude &&pre = Prelude{})
{
    if constexpr (binomial_form(OPR, DIR)) {
        sweep4<PPL, OFF, ALIGNED, FAST, EDGE, BM, BLOCKS, OPR>(J, g, lut, pre);
    } else {
        pre.issue();
        pre.finish();
        sweep_sep<PPL, OFF, ALIGNED, DIR, FAST, EDGE, OPR, BM, LUT, BLOCKS>(J, g, lut);
    }
}

constexpr int kWaves = 4;   // waves per workgroup

// Kernels that run two waves per SIMD (8 per CU, two 4-wave workgroups) round
// through the table in LDS: two 64 KiB copies fit in a CU's 160 KiB.  The
// others (three waves per SIMD) keep the square-root rounding.
constexpr bool use_lut(int waves_per_simd) { return waves_per_simd == 2; }

// LDS table bytes of a kernel: the binomial sweep rounds through the table
// of T = S / 2, the separable one through the S table when use_lut, else
// by square root.
constexpr int lut_bytes(int opr, bool dir, int waves_per_simd)
{
    return binomial_form(opr, dir) ? kLutTSize : (use_lut(waves_per_simd) ? kLutSize : 16);
}

// Fill the kernel's table (all THREADS threads of the workgroup) and
// synchronise the workgroup before any wave leaves.
template <int OPR, bool DIR, int WAVES_PER_SIMD, int THREADS>
__device__ __forceinline__ void lut_setup(uint8_t *lut)
{
    if constexpr (binomial_form(OPR, DIR)) {
        lut_fill_t<THREADS>(lut);
        __syncthreads();
    } else if constexpr (use_lut(WAVES_PER_SIMD)) {
        lut_fill<THREADS>(lut);
        __syncthreads();
    }
}

// Waves per SIMD the single-image kernel is compiled for (register budget
// 512 / waves): 16 pixels per lane needs ~220 VGPRs (2 waves), 8 pixels per
// lane ~134 (3 waves), or 128 with a few spilled values (4 waves).  The
// two-directional operators keep fewer rings live.
#ifndef SOBEL4X5_WAVES_PPL16
#define SOBEL4X5_WAVES_PPL16 2
#endif
#ifndef SOBEL4X5_WAVES_PPL8
#define SOBEL4X5_WAVES_PPL8 3
#endif
#ifndef SOBEL4X5_WAVES_2DIR_PPL16
#define SOBEL4X5_WAVES_2DIR_PPL16 3
#endif
#ifndef SOBEL4X5_WAVES_2DIR_PPL8
#define SOBEL4X5_WAVES_2DIR_PPL8 4
#endif
// (the byte-wise loads of unaligned rows and the directional stores need
// more registers: one wave less for them)
constexpr int single_waves(int ppl, int opr, bool aligned, bool dir)
{
    if (opr == kOp4x5) return ppl == 8 ? SOBEL4X5_WAVES_PPL8 : SOBEL4X5_WAVES_PPL16;
    if (ppl == 8) return aligned ? SOBEL4X5_WAVES_2DIR_PPL8 : SOBEL4X5_WAVES_2DIR_PPL8 - 1;
    return aligned && !dir ? SOBEL4X5_WAVES_2DIR_PPL16 : SOBEL4X5_WAVES_2DIR_PPL16 - 1;
}

// Single image.  Wave w takes tile strip w / nchunk (four tiles side by
// side, so all groups walk the same rows and row addresses stay scalar) and
// the (w % nchunk)-th of nchunk equal row ranges of it: every resident wave
// gets the same amount of work and there is no tail of a second round.
template <int PPL, int OFF, bool ALIGNED, bool DIR, int OPR, int BM>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(
    single_waves(PPL, OPR, ALIGNED, DIR), single_waves(PPL, OPR, ALIGNED, DIR)))) void k_u8_single(U8Job J, int nchunk)
{
    constexpr int TW = 16 * PPL;
    constexpr int WV = single_waves(PPL, OPR, ALIGNED, DIR);
    constexpr bool LUT = use_lut(WV);
    constexpr bool BIN = binomial_form(OPR, DIR);
    __shared__ __attribute__((aligned(16))) uint8_t lut[lut_bytes(OPR, DIR, WV)];
    // the binomial kernels copy their table between the first row loads and
    // the first row (every wave of the workgroup reaches that one barrier)
    if constexpr (!BIN) lut_setup<OPR, DIR, WV, 64 * kWaves>(lut);
    lds_u8 *lutp = (lds_u8 *)lut;
    const int w = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntxw = (J.ntx + 3) >> 2;
    const int strip = w / nchunk, k = w % nchunk;
    const int y0 = (int)(((int64_t)k * J.Ho) / nchunk);
    const int y1 = (int)(((int64_t)(k + 1) * J.Ho) / nchunk);
    if (w >= ntxw * nchunk || y1 <= y0) {
        if constexpr (BIN) lut_setup<OPR, DIR, WV, 64 * kWaves>(lut);
        return;
    }
    const int grp = (threadIdx.x >> 4) & 3;
    const int tx = strip * 4 + grp;
    Sweep g;
    g.xo = tx * TW + (threadIdx.x & 15) * PPL;
    g.yo0 = y0;
    g.niter = y1 - y0;
    g.nrow = tx < J.ntx ? g.niter : 0;
    g.fix_right = (strip * 4 + 4) * TW + 4 > J.W;
    g.fix_left = OFF == 0 && strip == 0;
    // fast: all four tiles complete (every lane's block and output inside
    // the image); the strips at the image edges take the fast path with mask
    // fix-ups of their group halos
    const bool fast = ALIGNED && (strip * 4 + 4) * TW <= J.Wo;
    auto run = [&](auto pre) {
        if (fast && !g.fix_right && !g.fix_left)
            sweep<PPL, OFF, ALIGNED, DIR, true, false, OPR, BM, LUT>(J, g, lutp, pre);
        else if (fast)
            sweep<PPL, OFF, ALIGNED, DIR, true, true, OPR, BM, LUT>(J, g, lutp, pre);
        else
            sweep<PPL, OFF, ALIGNED, DIR, false, false, OPR, BM, LUT>(J, g, lutp, pre);
    };
    if constexpr (BIN)
        run(LutPrelude<64 * kWaves>{{}, lut});
    else
        run(NoPrelude{});
}


}  // namespace
}  // namespace s4x5
