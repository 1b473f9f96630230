// Four-directional 5x5 magnitudes (uint8 in, uint8 out) on the matrix cores.
//
// Each of the four responses is a 5x5 correlation, so for one output row
// segment it is a banded (Toeplitz) product of the input rows around it
// with a constant weight matrix.  One v_mfma_i32_32x32x32_i8 multiplies a
// 32 x 32 int8 weight block A by a 32 x 32 int8 image block B:
//   B[k][n]: n = output row of the tile (32 rows), k = (input row dy of a
//            pair of the 5, byte b of a 16-byte window of that row);
//   A[m][k]: m = (output column s of 8, response f of 4), holding the
//            weight of response f at (dy, b - s - 2), zero off the band;
//   D[m][n]: response f of output (row n, column s), int32.
// Three such products (input rows 0-1, 2-3, 4) cover the 5 rows of 8 output
// columns x 32 output rows; a tile of 16 column groups is 32 x 128 outputs.
//
// uint8 pixels enter as int8 via x ^ 0x80 = x - 128: every filter of
// Eq. (sobel5_1) sums to zero, so subtracting 128 from every pixel leaves
// every response unchanged.
//
// The responses carried are E1 = (Gx + Gy)/2, E2 = (Gx - Gy)/2,
// Hp = (Gd + Gdt)/2 and Hm = (Gd - Gdt)/2 (all integer: every entry of
// Gx +- Gy and Gd +- Gdt is even), so S = Gx^2 + Gy^2 + Gd^2 + Gdt^2
// (Eq. (sobel5_2) squared) is 2 T with T = E1^2 + E2^2 + Hp^2 + Hm^2.
// |E| <= 16320 and |H| <= 8925, so T < 2^31 and each square is one 24-bit
// multiply(-add).  The magnitude round(sqrt(S)), capped at 255, is read from
// the table of T (kMagLutT, T >= 32386 reads 255) at min(T, 32767).
//
// The same products serve run-time kernels whose weights fit int8 (the
// family of Eq. (sobel5_param) with small weights), with S = sum G^2 and a
// square root for the rounding (MagS).
//
// A lane of D holds, for its output row n = lane % 32 and half
// h = lane / 32, the four responses of columns 4h .. 4h + 3 of the group:
// its four magnitude bytes are one contiguous dword of the output row.
// Requires gfx950 (the 32x32x32 int8 products).
#pragma once

#include "load_columns.hpp"
#include "u8_sweep.hpp"

namespace s4x5 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned long long u64;
typedef u32 u32_u __attribute__((aligned(1)));
typedef v4i v4i_a8 __attribute__((aligned(8)));
typedef gv4u gv4u_a8 __attribute__((aligned(8)));
#define LDS __attribute__((address_space(3)))

// The four filters of Eq. (sobel5_1), row dy top to bottom, column dx left
// to right (response at (y, x) = sum K[dy][dx] I(y + dy - 2, x + dx - 2)).
constexpr int kG5[4][5][5] = {
    {{-1, -2, 0, 2, 1}, {-4, -8, 0, 8, 4}, {-6, -12, 0, 12, 6}, {-4, -8, 0, 8, 4}, {-1, -2, 0, 2, 1}},   // Gx
    {{-1, -4, -6, -4, -1}, {-2, -8, -12, -8, -2}, {0, 0, 0, 0, 0}, {2, 8, 12, 8, 2}, {1, 4, 6, 4, 1}},   // Gy
    {{-6, -4, -1, -2, 0}, {-4, -12, -8, 0, 2}, {-1, -8, 0, 8, 1}, {-2, 0, 8, 12, 4}, {0, 2, 1, 4, 6}},   // Gd
    {{0, -2, -1, -4, -6}, {2, 0, -8, -12, -4}, {1, 8, 0, -8, -1}, {4, 12, 8, 0, -2}, {6, 4, 1, 2, 0}},   // Gdt
};

struct Resp5 {
    int k[4][5][5];   // E1, E2, Hp, Hm
};
constexpr Resp5 make_resp5()
{
    Resp5 r{};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            r.k[0][i][j] = (kG5[0][i][j] + kG5[1][i][j]) / 2;
            r.k[1][i][j] = (kG5[0][i][j] - kG5[1][i][j]) / 2;
            r.k[2][i][j] = (kG5[2][i][j] + kG5[3][i][j]) / 2;
            r.k[3][i][j] = (kG5[2][i][j] - kG5[3][i][j]) / 2;
        }
    return r;
}
constexpr Resp5 kResp5 = make_resp5();

constexpr bool resp5_ok()
{
    for (int f = 0; f < 4; ++f) {
        int sum = 0;
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) {
                const int a = kG5[f / 2 * 2][i][j], b = kG5[f / 2 * 2 + 1][i][j];
                if ((a + b) % 2 != 0) return false;   // halving is exact
                if (kResp5.k[f][i][j] < -128 || kResp5.k[f][i][j] > 127) return false;
                sum += kG5[f][i][j];
            }
        if (sum != 0) return false;   // the x - 128 shift leaves the response unchanged
    }
    return true;
}
static_assert(resp5_ok(), "filters of Eq. (sobel5_1): even sums and differences, zero sum, int8 weights");

// Tile geometry.
constexpr int kMRows = 32;             // output rows of a tile (the product's n)
constexpr int kMGroups = 16;           // 8-column groups of a tile
constexpr int kMCols = 8 * kMGroups;   // output columns of a tile
constexpr int kMInRows = kMRows + 4;   // input rows a tile reads
constexpr int kMInLead = 12;           // input columns before the tile's first output column
constexpr int kMPieces = 9;            // 16-byte pieces of an input row: columns [X - 12, X + 132)
constexpr int kMPitch = 152;           // LDS row pitch: 38 dwords, 8-byte reads of 32 rows hit distinct banks
constexpr int kMOutPitch = 136;        // staged output rows of their own: 34 dwords
constexpr int kMOutBytes = kMRows * kMOutPitch;
// Where a tile's outputs wait for their full-line stores (see mfma_tile).
constexpr int kStageOwn = 1, kStageInPlace = 2;
constexpr int kMTileBytes = kMInRows * kMPitch;
constexpr int kMWaves = 8;             // waves per workgroup (one table copy for eight tiles)
static_assert(16 * kMPieces == kMInLead + kMCols + 4, "input row = lead + outputs + right halo");
static_assert(kMPitch % 8 == 0 && kMPitch >= 16 * kMPieces, "row pitch");
static_assert(kLutTSize + kMWaves * kMTileBytes <= 81920, "two workgroups per CU (with the T table)");
static_assert(kMWaves * (kMTileBytes + kMOutBytes) <= 81920, "two workgroups per CU (staged outputs)");

// Weight operands of the three products for every lane: 16 bytes each,
// k = 16 (lane / 32) + byte, from four 5x5 kernels k[f][dy][dx] whose
// weights fit int8 (used at compile time for the operator of Eq. (sobel5_1)
// and on the host for run-time kernels).
struct MfmaWeights {
    u32 w[3][64][4];
};
template <class K>
constexpr MfmaWeights mfma_weights(const K &k)
{
    MfmaWeights a{};
    for (int t = 0; t < 3; ++t)
        for (int lane = 0; lane < 64; ++lane) {
            const int m = lane & 31, g = lane >> 5;
            const int f = m & 3, s = 4 * ((m >> 2) & 1) + (m >> 3);
            const int dy = 2 * t + g;
            for (int b = 0; b < 16; ++b) {
                const int dx = b - 2 - s;
                const int v = (dy <= 4 && dx >= 0 && dx <= 4) ? k(f, dy, dx) : 0;
                a.w[t][lane][b >> 2] |= (u32)(uint8_t)(int8_t)v << (8 * (b & 3));
            }
        }
    return a;
}
struct Resp5Taps {
    constexpr int operator()(int f, int dy, int dx) const { return kResp5.k[f][dy][dx]; }
};
constexpr MfmaWeights kAWords = mfma_weights(Resp5Taps{});

// The lane's three weight operands: of the operator of Eq. (sobel5_1) from
// the table above, or run-time ones (built on the host by mfma_weights).
__device__ __forceinline__ void mfma_a_default(v4i (&A)[3])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        A[t] = v4i{(int)kAWords.w[t][lane][0], (int)kAWords.w[t][lane][1], (int)kAWords.w[t][lane][2],
                   (int)kAWords.w[t][lane][3]};
}

__device__ __forceinline__ void mfma_a_runtime(const MfmaWeights &W, v4i (&A)[3])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        A[t] = v4i{(int)W.w[t][lane][0], (int)W.w[t][lane][1], (int)W.w[t][lane][2], (int)W.w[t][lane][3]};
}

// Index of input position i of an axis of n pixels under border rule BM
// (kBmZero: -1 for a position outside).
template <int BM>
__device__ __forceinline__ int border_map(int i, int n)
{
    if (i >= 0 && i < n) return i;
    if constexpr (BM == kBmZero) return -1;
    if constexpr (BM == kBmRefl) return reflect101(i, n);
    return i < 0 ? 0 : n - 1;
}

// One 16-byte piece of the LDS tile: image row yi (or -1: a row of zeros),
// columns cs .. cs + 15, as int8 (x ^ 0x80).
__device__ __forceinline__ void mfma_put_piece(LDS uint8_t *dst, u32 w0, u32 w1, u32 w2, u32 w3)
{
    LDS u64 *d = reinterpret_cast<LDS u64 *>(dst);
    d[0] = (u64)(w0 ^ 0x80808080u) | ((u64)(w1 ^ 0x80808080u) << 32);
    d[1] = (u64)(w2 ^ 0x80808080u) | ((u64)(w3 ^ 0x80808080u) << 32);
}

// Input rows of the tile at output (y0, X) into the wave's LDS tile.  Tile
// byte (r, c) is image pixel (y0 - 2 + OFF + r, X - 12 + OFF + c) under the
// border rule.  A piece whose 16 columns lie inside the image is one 16-byte
// load.  In the tiles at the left and right edge the pieces that cross an
// edge (usually one a row) are gathered in a second pass, byte by byte
// through the column map, with all sixteen loads of a piece in flight.
template <int OFF, int BM>
__device__ __forceinline__ void mfma_load_tile(const U8Job &J, int y0, int X, LDS uint8_t *tile)
{
    // recomputed per tile rather than held in registers across the tile loop
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const GMEM uint8_t *src = (const GMEM uint8_t *)J.src;
    const int c0 = X - kMInLead + OFF;
    constexpr int kN = kMInRows * kMPieces;
    const bool all_inside = c0 >= 0 && c0 + 16 * kMPieces <= J.W;
#pragma unroll
    for (int k = 0; k < (kN + 63) / 64; ++k) {
        const int p = lane + 64 * k;
        if (p < kN) {
            const int r = p / kMPieces, q = p - kMPieces * r;
            const int cs = c0 + 16 * q;
            if (all_inside || (cs >= 0 && cs + 16 <= J.W)) {
                const int yi = border_map<BM>(y0 - 2 + OFF + r, J.H);
                gv4u v = {0u, 0u, 0u, 0u};
                if (BM != kBmZero || yi >= 0)
                    v = *reinterpret_cast<const GMEM gv4u_u *>(src + (int64_t)yi * J.src_pitch + cs);
                mfma_put_piece(tile + r * kMPitch + 16 * q, v.x, v.y, v.z, v.w);
            }
        }
    }
    if (all_inside) return;
    // the pieces that cross an edge (the same in every row): their indices,
    // four bits each
    u64 list = 0;
    int nc = 0;
    for (int q = 0; q < kMPieces; ++q) {
        const int cs = c0 + 16 * q;
        if (!(cs >= 0 && cs + 16 <= J.W)) {
            list |= (u64)q << (4 * nc);
            ++nc;
        }
    }
#pragma unroll 1
    for (int i = lane; i < kMInRows * nc; i += 64) {
        const int r = i / nc, q = (int)((list >> (4 * (i - r * nc))) & 15u);
        const int yi = border_map<BM>(y0 - 2 + OFF + r, J.H);
        const int cs = c0 + 16 * q;
        u32 b[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int xi = border_map<BM>(cs + e, J.W);
            b[e] = (yi >= 0 && xi >= 0) ? (u32)src[(int64_t)yi * J.src_pitch + xi] : 0u;
        }
        u32 w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = lshl_or(lshl_or(b[4 * k + 3], 8, b[4 * k + 2]), 16, lshl_or(b[4 * k + 1], 8, b[4 * k]));
        mfma_put_piece(tile + r * kMPitch + 16 * q, w[0], w[1], w[2], w[3]);
    }
}

// The three image operands of column group j: 16 bytes of input rows
// (n + h, n + 2 + h, n + 4) from the window start of the group.
struct MfmaRows {
    const LDS uint8_t *r0, *r1, *r2;
};
__device__ __forceinline__ void mfma_load_b(const MfmaRows &rb, int j, v4i (&B)[3])
{
    B[0] = *reinterpret_cast<const LDS v4i_a8 *>(rb.r0 + 8 * j);
    B[1] = *reinterpret_cast<const LDS v4i_a8 *>(rb.r1 + 8 * j);
    B[2] = *reinterpret_cast<const LDS v4i_a8 *>(rb.r2 + 8 * j);
}

__device__ __forceinline__ v16i mfma_products(const v4i (&A)[3], const v4i (&B)[3])
{
    v16i D = {};
    D = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[0], B[0], D, 0, 0, 0);
    D = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[1], B[1], D, 0, 0, 0);
    D = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[2], B[2], D, 0, 0, 0);
    return D;
}

// a * a + acc on the 24-bit multiplier (|a| < 2^23), one instruction; the
// compiler would otherwise pair the squares and add them with add3.
__device__ __forceinline__ int sq24_acc(int a, int acc)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %1, %2" : "=v"(r) : "v"(a), "v"(acc));
    return r;
}


// Interior tiles (every input row and column inside the image: no border
// rule applies) load in six instructions per lane.  Lane (r0, q) =
// (lane / 9, lane % 9), lanes 0..62, holds piece q of tile rows r0 + 7k,
// k = 0..5 (k = 5 only for r0 = 0): each load takes its row base from
// SGPRs and the lane's offset r0 * pitch + 16 q from one VGPR, and each LDS
// write an immediate offset of 7k rows.
constexpr int kMFetch = 6;
struct MfmaFetch {
    gv4u v[kMFetch];
};

template <int OFF>
__device__ __forceinline__ bool mfma_interior(const U8Job &J, int y0, int X)
{
    const int c0 = X - kMInLead + OFF, r0 = y0 - 2 + OFF;
    return c0 >= 0 && c0 + 16 * kMPieces <= J.W && r0 >= 0 && r0 + kMInRows <= J.H && J.src_pitch <= (1 << 28);
}

template <int OFF>
__device__ __forceinline__ void mfma_fetch(const U8Job &J, int y0, int X, MfmaFetch &f)
{
    const int lane = threadIdx.x & 63;
    const int r0 = (lane * 57) >> 9, q = lane - 9 * r0;   // lane / 9 for lane < 64
    const u32 voff = (u32)r0 * (u32)J.src_pitch + 16u * (u32)q;
    const GMEM uint8_t *base = (const GMEM uint8_t *)J.src + (int64_t)(y0 - 2 + OFF) * J.src_pitch + (X - kMInLead + OFF);
#pragma unroll
    for (int k = 0; k < kMFetch; ++k) {
        const bool on = k < kMFetch - 1 ? lane < 63 : lane < 9;
        if (on) f.v[k] = *reinterpret_cast<const GMEM gv4u_u *>(base + (int64_t)(7 * k) * J.src_pitch + voff);
    }
}

__device__ __forceinline__ void mfma_commit(const MfmaFetch &f, u32 tile)
{
    const int lane = threadIdx.x & 63;
    const int r0 = (lane * 57) >> 9, q = lane - 9 * r0;
    LDS uint8_t *dst = (LDS uint8_t *)(size_t)(tile + (u32)(r0 * kMPitch + 16 * q));
#pragma unroll
    for (int k = 0; k < kMFetch; ++k) {
        const bool on = k < kMFetch - 1 ? lane < 63 : lane < 9;
        if (on) mfma_put_piece(dst + 7 * k * kMPitch, f.v[k].x, f.v[k].y, f.v[k].z, f.v[k].w);
    }
}

// Magnitude policies: lookup() turns a group's responses (D: four pixels of
// the lane, four responses each) into what pack() makes the lane's output
// dword of, one pipeline step later.
//
// MagT, the operator of Eq. (sobel5_1): the responses are E1, E2, Hp, Hm;
// T = E1^2 + E2^2 + Hp^2 + Hm^2 indexes the T table in LDS (reads issued
// in lookup, consumed in pack).
struct MagT {
    const LDS uint8_t *lut;
    __device__ __forceinline__ void lookup(const v16i &D, u32 (&mb)[4]) const
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int T = __mul24(D[4 * i], D[4 * i]);
            T = sq24_acc(D[4 * i + 1], T);
            T = sq24_acc(D[4 * i + 2], T);
            T = sq24_acc(D[4 * i + 3], T);
            mb[i] = lut[min((u32)T, (u32)kLutTSize - 1u)];
        }
    }
    __device__ __forceinline__ u32 pack(const u32 (&mb)[4]) const
    {
        return lshl_or(lshl_or(mb[3], 8, mb[2]), 16, lshl_or(mb[1], 8, mb[0]));
    }
};

// MagS, four run-time kernels G_f (Eq. (sobel5_param) or any half-turn
// antisymmetric ones): S = sum G_f^2, min(255, round(sqrt(S))).  CLAMP:
// each G is first clamped to [-256, 256] (one G of 256 or more already
// makes S >= 65536, which rounds to 255, and the clamped S stays below
// 2^19); without it the kernels' absolute sums must keep 4 G^2 < 2^31.
// (float)S is exact below 2^24 and monotone above, where the result
// saturates; v_sqrt_f32 is within 1 ulp and round(sqrt(S)) is never a tie,
// with a margin that 1 ulp does not cross; v_cvt_pk_u8_f32 rounds to
// nearest and saturates to [0, 255].
template <bool CLAMP>
struct MagS {
    __device__ __forceinline__ static int g(int v) { return CLAMP ? min(max(v, -256), 256) : v; }
    __device__ __forceinline__ void lookup(const v16i &D, u32 (&mb)[4]) const
    {
        u32 out = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int S = __mul24(g(D[4 * i]), g(D[4 * i]));
            S = sq24_acc(g(D[4 * i + 1]), S);
            S = sq24_acc(g(D[4 * i + 2]), S);
            S = sq24_acc(g(D[4 * i + 3]), S);
            out = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_amdgcn_sqrtf((float)S), i, out);
        }
        mb[0] = out;
    }
    __device__ __forceinline__ u32 pack(const u32 (&mb)[4]) const { return mb[0]; }
};

// The 32 x 128 output tile at (y0, X) from the wave's LDS tile (byte address
// `tile`).  FULL: every output of the tile lies inside the image.  Pipeline
// over the 16 column groups: in step j the products of group j + 1 run, the
// operands of group j + 2 load, group j's table reads are issued and group
// j - 1's bytes (read in step j - 1) are packed.
//
// Stores: after group j, lane (n, h) holds the magnitude bytes of columns
// 8j + 4h .. 8j + 4h + 3 of row n.  They wait in an output tile in LDS (row
// n, bytes 8j + 4h), and after the 16 groups every row leaves as eight
// 16-byte stores by eight lanes, one full 128-byte line.  Stored straight
// from the lanes (even four groups at a time, 16 bytes a lane after two
// v_permlane32_swap), each line leaves in 32-byte pieces from several
// instructions, and those partial lines cost about 1.4x the output bytes in
// HBM writes.  Rows 16..31 keep each group's two dwords swapped, so that a
// half-wave of writes (rows 0..31, one h) covers 32 distinct banks.
//   kStageOwn: an output tile of its own (pitch kMOutPitch);
//   kStageInPlace: the input tile itself (pitch kMPitch).  Group j's
//   outputs land in bytes [8j, 8j + 8) of rows 0..31, written after group
//   j's products: the operand reads of group j and later groups start at
//   byte 8j + 8 of a row, and those of earlier groups were consumed by
//   their products already.
template <bool FULL, class Mag, int STAGE>
__device__ __forceinline__ void mfma_tile(const U8Job &J, int y0, int X, u32 tile, u32 otile, const v4i (&A)[3],
                                          const Mag &mag)
{
    static_assert(STAGE == kStageOwn || STAGE == kStageInPlace, "output staging");
    // a fresh base each tile, so that the 48 operand addresses of the tile
    // are the three row bases plus immediate offsets, not registers held
    // across tiles
    asm volatile("" : "+v"(tile));
    const int lane = threadIdx.x & 63;
    const int n = lane & 31, h = lane >> 5;
    const MfmaRows rb{(const LDS uint8_t *)(size_t)(tile + (u32)((n + h) * kMPitch + 8)),
                      (const LDS uint8_t *)(size_t)(tile + (u32)((n + 2 + h) * kMPitch + 8)),
                      (const LDS uint8_t *)(size_t)(tile + (u32)((n + 4) * kMPitch + 8))};
    constexpr int OP = STAGE == kStageInPlace ? kMPitch : kMOutPitch;
    LDS u32 *orow_lds = (LDS u32 *)(size_t)(otile + (u32)(n * OP + 4 * (h ^ (n >> 4))));
    v4i B[3];
    mfma_load_b(rb, 0, B);
    v16i Dn = mfma_products(A, B);
    mfma_load_b(rb, 1, B);
    u32 mbp[4];
#pragma unroll
    for (int j = 0; j < kMGroups; ++j) {
        const v16i D = Dn;
        if (j + 1 < kMGroups) Dn = mfma_products(A, B);
        if (j + 2 < kMGroups) mfma_load_b(rb, j + 2, B);
        u32 mb[4];
        mag.lookup(D, mb);
        if (j > 0) orow_lds[2 * (j - 1)] = mag.pack(mbp);
#pragma unroll
        for (int i = 0; i < 4; ++i) mbp[i] = mb[i];
        __builtin_amdgcn_sched_barrier(0);
    }
    orow_lds[2 * (kMGroups - 1)] = mag.pack(mbp);
    // the rows were written by the two lanes that hold them
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const int col = 16 * (lane & 7);
#pragma unroll
    for (int k = 0; k < kMRows / 8; ++k) {
        const int r = (lane >> 3) + 8 * k;
        gv4u v = *(const LDS gv4u_a8 *)(size_t)(otile + (u32)(r * OP + col));
        if (k >= 2) v = gv4u{v.y, v.x, v.w, v.z};   // rows 16..31
        const int y = y0 + r;
        GMEM uint8_t *p = (GMEM uint8_t *)J.mag + (int64_t)(FULL || y < J.Ho ? y : 0) * J.mag_pitch + X + col;
        if (FULL) {
            *reinterpret_cast<GMEM gv4u_u *>(p) = v;
        } else if (y < J.Ho) {
            const int nvalid = J.Wo - X - col;
            if (nvalid >= 16) {
                *reinterpret_cast<GMEM gv4u_u *>(p) = v;
            } else {
                const u32 w[4] = {v.x, v.y, v.z, v.w};
                for (int q = 0; q < nvalid; ++q) p[q] = (uint8_t)(w[q >> 2] >> (8 * (q & 3)));
            }
        }
    }
    // the next tile's writes to this LDS come after these reads
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// One wave: tiles [b0, b1) of column strip sx, top to bottom, in the LDS
// tile at byte address `tile`, with weight operands A.  An interior tile's
// rows are fetched into registers while the tile before it is computed,
// then written to LDS; the tiles at the image edges load through the border
// rule in between.
template <int OFF, int BM, class Mag, int STAGE>
__device__ __forceinline__ void mfma_strip(const U8Job &J, int sx, int b0, int b1, u32 tile, const v4i (&A)[3],
                                           const Mag &mag, u32 otile)
{
    const int X = sx * kMCols;
    const bool cols_full = X + kMCols <= J.Wo;
    LDS uint8_t *tp = (LDS uint8_t *)(size_t)tile;
    if (b0 >= b1) return;
    if (mfma_interior<OFF>(J, b0 * kMRows, X)) {
        MfmaFetch f;
        mfma_fetch<OFF>(J, b0 * kMRows, X, f);
        mfma_commit(f, tile);
    } else {
        mfma_load_tile<OFF, BM>(J, b0 * kMRows, X, tp);
    }
    for (int b = b0; b < b1; ++b) {
        const int y0 = b * kMRows;
        const bool next = b + 1 < b1;
        const bool fetch_next = next && mfma_interior<OFF>(J, y0 + kMRows, X);
        MfmaFetch f;
        if (fetch_next) mfma_fetch<OFF>(J, y0 + kMRows, X, f);
        // the tile's rows were written by other lanes of this wave
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (cols_full && y0 + kMRows <= J.Ho)
            mfma_tile<true, Mag, STAGE>(J, y0, X, tile, otile, A, mag);
        else
            mfma_tile<false, Mag, STAGE>(J, y0, X, tile, otile, A, mag);
        // every operand read of this tile has returned (the products and
        // stores consumed them) before its rows are overwritten
        if (fetch_next)
            mfma_commit(f, tile);
        else if (next)
            mfma_load_tile<OFF, BM>(J, y0 + kMRows, X, tp);
    }
}

}  // namespace
}  // namespace s4x5
