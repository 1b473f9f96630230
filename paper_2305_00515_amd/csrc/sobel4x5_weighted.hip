// uint8 four-directional 5x5 operator with run-time integer weights.
//
// Sec. 3.2 generalises the filters of Eq. (sobel5_1) to the family
// K(a, b, n, m) of Eq. (sobel5_param): integer 5x5 kernels K_x, K_d, K_y,
// K_dt built from a, a*b, a*n, a*m, a*n*b, a*m*b.  Every kernel of that
// family is antisymmetric under a half turn (k[4-i][4-j] = -k[i][j]), and
// this path serves any four integer kernels with that property:
//
//   G_k(p) = sum over the 12 taps (i, j) of the upper half
//            k[i][j] * (I(p + (i-2, j-2)) - I(p + (2-i, 2-j)))
//
// The 12 pair differences are shared by the four responses.  They are
// formed two at a time as int16 pairs (|difference| <= 255), and each
// response is six v_dot2_i32_i16 against int16 pairs of coefficients:
// antisymmetry puts every weight twice into sum |k| <= 32768, so |k| <=
// 16384 fits int16, and |G| <= 255 * 16384 stays far inside int32.  The
// pairs: taps (i, j), (i, j+1) of one row meet the partner row's bytes in
// reverse order, so each input row is packed once, as it enters the ring,
// into adjacent-byte pairs in both orders; the two taps left over, (0, 4)
// and (1, 4), form the sixth pair.  The magnitude rounds min(255,
// round(sqrt(S))) exactly: every G_k is clamped to [-256, 256] first, which
// changes S only where S >= 65536 and the result saturates anyway, so S
// stays below 2^24 and its float square root rounds correctly (no integer S
// is within 4.9e-4 of a half-integer root); the clamped responses are
// squared and summed with v_dot2 as well.  The paper's own factoring
// (Eq. (sobel5_kd+-), (sobel5_4)) serves the default weights on the packed
// fast path.
//
// Work layout: a lane owns 4 consecutive output pixels of a row and walks a
// range of rows with a 5-row register ring of the int16 pairs packed from
// the 8 input bytes it needs; a wave covers 256 columns.

#include "internal.hpp"
#include "load_columns.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

namespace s4x5 {
namespace {

#define GMEM __attribute__((address_space(1)))

constexpr int kWavesW = 4;
constexpr int kPplW = 4;                 // output pixels per lane
constexpr int kColsW = 64 * kPplW;       // output columns per wave

typedef unsigned int u32;
typedef short v2s __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ v2s V2(u32 v) { return __builtin_bit_cast(v2s, v); }
__device__ __forceinline__ u32 U2(v2s v) { return __builtin_bit_cast(u32, v); }
// low 16 bits of lo, then low 16 bits of hi
__device__ __forceinline__ u32 pair16(u32 lo, u32 hi) { return __builtin_amdgcn_perm(hi, lo, 0x05040100u); }
__device__ __forceinline__ int dot2(v2s a, v2s b, int c) { return __builtin_amdgcn_sdot2(a, b, c, false); }
// a.lo*b.lo + a.hi*b.hi with no accumulator: the three-operand form with an
// inline 0 (the compiler otherwise clears a register for the two-operand
// accumulate-in-place form)
__device__ __forceinline__ int dot2_0(v2s a, v2s b)
{
    int r;
    asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(U2(a)), "v"(U2(b)));
    return r;
}
__device__ __forceinline__ int dot2_0s(v2s a, u32 b_uniform)
{
    int r;
    asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(U2(a)), "s"(b_uniform));
    return r;
}

template <int P>
using PhW = std::integral_constant<int, P>;

// Upper-half taps u in the order of the coefficient table: (0, 0..4) are
// u = 0..4, (1, 0..4) are 5..9, (2, 0), (2, 1) are 10, 11; the partner of
// tap (i, j) is (4 - i, 4 - j).  The six pairs of taps whose differences
// share one v_dot2:
//   (0,0)(0,1)  (0,2)(0,3)  (1,0)(1,1)  (1,2)(1,3)  (2,0)(2,1)  (0,4)(1,4)
__device__ constexpr int kPairLo[6] = {0, 2, 5, 7, 10, 4};
__device__ constexpr int kPairHi[6] = {1, 3, 6, 8, 11, 9};

// BM: how pixels outside the image read (0 nearest, 1 zero, 2 reflect-101).
template <int OFF, int DT, int BM>
__global__ __launch_bounds__(64 * kWavesW) void k_u8_weighted(WJob J, int nstrip, int nchunk)
{
    const int wave = blockIdx.x * kWavesW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nstrip * nchunk) return;
    const int s = wave % nstrip, k = wave / nstrip;
    const int y0 = (int)((int64_t)k * J.Ho / nchunk), y1 = (int)((int64_t)(k + 1) * J.Ho / nchunk);
    if (y1 <= y0) return;
    const int lane = threadIdx.x & 63;
    const int xo = s * kColsW + lane * kPplW;          // first output column of the lane
    int col[kPplW + 4];                                 // input columns of the window, mapped inside
    u32 colin = 0;                                      // zero border: bit j = column j lies inside
#pragma unroll
    for (int j = 0; j < kPplW + 4; ++j) {
        const int x = xo + OFF - 2 + j;
        col[j] = BM == 2 ? reflect101(x, J.W) : clampi(x, 0, J.W - 1);
        colin |= (x >= 0 && x < J.W) ? (1u << j) : 0u;
    }
    const GMEM uint8_t *src = (const GMEM uint8_t *)J.src;
    const int r0 = y0 + OFF - 2;                       // input row of step 0
    const int T = y1 - y0 + 4;
    auto ldrow = [&](int t, uint8_t (&v)[kPplW + 4]) {
        const int r = r0 + min(t, T - 1);
        const int rr = BM == 2 ? reflect101(r, J.H) : clampi(r, 0, J.H - 1);
        const GMEM uint8_t *row = src + (int64_t)rr * J.src_pitch;
#pragma unroll
        for (int j = 0; j < kPplW + 4; ++j) v[j] = row[col[j]];
    };
    // zero border: which bytes of step t's row lie inside the image (applied
    // when the row enters the ring, so that the loads stay in flight)
    auto inside = [&](int t) -> u32 {
        const int r = r0 + min(t, T - 1);
        return (unsigned)r <= (unsigned)(J.H - 1) ? colin : 0u;
    };

    // coefficient pairs (k[lo], k[hi]) as int16 halves, wave-uniform
    u32 cp[4][6];
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
#pragma unroll
        for (int q = 0; q < 6; ++q)
            cp[pl][q] = (u32)(uint16_t)J.coef[pl][kPairLo[q]] | ((u32)(uint16_t)J.coef[pl][kPairHi[q]] << 16);

    // Ring of packed input rows, R the row's 8 window bytes (low half
    // first): F[c] = (R[c], R[c+1]) for c = 0..5, and B[c] = (R[c+2], R[c+1])
    // for c = 0..5, the reversed pair that starts at c + 1.  R[c] is the low
    // half of F[c] (c <= 5) or of B[c-2] (c = 6, 7).
    u32 F[5][6], B[5][6];
    uint8_t pf[5][kPplW + 4];
    constexpr int PD = 2;   // rows loaded ahead
#pragma unroll
    for (int t = 0; t < PD; ++t) {
        ldrow(t, pf[t]);
        __builtin_amdgcn_sched_barrier(0);   // prologue rows in row order
    }

    auto step = [&](int t, auto phase) {
        constexpr int p = decltype(phase)::value;
        ldrow(t + PD, pf[(p + PD) % 5]);
        {
            u32 b[kPplW + 4];
            if constexpr (BM == 1) {
                const u32 in = inside(t);
#pragma unroll
                for (int j = 0; j < kPplW + 4; ++j) b[j] = ((in >> j) & 1u) ? (u32)pf[p][j] : 0u;
            } else {
#pragma unroll
                for (int j = 0; j < kPplW + 4; ++j) b[j] = pf[p][j];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                F[p][c] = b[c] | (b[c + 1] << 16);
                B[p][c] = b[c + 2] | (b[c + 1] << 16);
            }
        }
        if (t < 4) return;
        // window row i (0..4) = input row t - 4 + i, in slot (p + 1 + i) % 5
        constexpr int w0 = (p + 1) % 5, w1 = (p + 2) % 5, w2 = (p + 3) % 5, w3 = (p + 4) % 5, w4 = p;
        auto lo16 = [&](const u32 (&f)[6], const u32 (&r)[6], int c) -> u32 { return c <= 5 ? f[c] : r[c - 2]; };
        const int yo = y0 + t - 4;
        int G[kPplW][4];
#pragma unroll
        for (int q = 0; q < kPplW; ++q) {
            // pair (j, j+1) of row i: F[q + j] of row i minus the reversed
            // pair of row 4 - i that starts at q + 3 - j, B[q + 2 - j]
            v2s d[6];
            d[0] = V2(F[w0][q]) - V2(B[w4][q + 2]);
            d[1] = V2(F[w0][q + 2]) - V2(B[w4][q]);
            d[2] = V2(F[w1][q]) - V2(B[w3][q + 2]);
            d[3] = V2(F[w1][q + 2]) - V2(B[w3][q]);
            d[4] = V2(F[w2][q]) - V2(B[w2][q + 2]);
            d[5] = V2(pair16(lo16(F[w0], B[w0], q + 4), lo16(F[w1], B[w1], q + 4))) -
                   V2(pair16(F[w4][q], F[w3][q]));
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
                int acc = dot2_0s(d[0], cp[pl][0]);
#pragma unroll
                for (int u = 1; u < 6; ++u) acc = dot2(d[u], V2(cp[pl][u]), acc);
                G[q][pl] = acc;
            }
        }
        if (J.mag) {
            u32 out = 0;
            const int nvalid = J.Wo - xo;
#pragma unroll
            for (int q = 0; q < kPplW; ++q) {
                int g[4];
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) g[pl] = min(max(G[q][pl], -256), 256);
                const v2s g01 = V2(pair16((u32)g[0], (u32)g[1])), g23 = V2(pair16((u32)g[2], (u32)g[3]));
                const int S = dot2(g01, g01, dot2_0(g23, g23));
                // v_cvt_pk_u8_f32 rounds to nearest and saturates at 255
                const u32 m = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_amdgcn_sqrtf((float)S), 0, 0u);
                out |= m << (8 * q);
            }
            GMEM uint8_t *mp = (GMEM uint8_t *)J.mag + (int64_t)yo * J.mag_pitch + (xo < 0 ? 0 : xo);
            if (nvalid >= kPplW) {
                typedef u32 u32u __attribute__((aligned(1)));
                *reinterpret_cast<GMEM u32u *>(mp) = out;
            } else {
#pragma unroll
                for (int q = 0; q < kPplW; ++q)
                    if (q < nvalid) mp[q] = (uint8_t)(out >> (8 * q));
            }
        }
        if constexpr (DT != 0) {
            const int nvalid = J.Wo - xo;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
                GMEM char *base = (GMEM char *)J.dir[pl] + (int64_t)yo * J.dir_pitch;
#pragma unroll
                for (int q = 0; q < kPplW; ++q) {
                    if (q >= nvalid) continue;
                    if constexpr (DT == 1)
                        reinterpret_cast<GMEM int16_t *>(base)[xo + q] = (int16_t)G[q][pl];
                    else
                        reinterpret_cast<GMEM int32_t *>(base)[xo + q] = G[q][pl];
                }
            }
        }
    };
    // whole blocks of five steps in a loop with a single exit, then the
    // 0..4 remaining steps (breaking out after any step makes flow blocks
    // whose state the memory-wait analysis merges into the loop header)
    const int nfull = T - T % 5;
    for (int t = 0; t < nfull; t += 5) {
        step(t, PhW<0>{});
        step(t + 1, PhW<1>{});
        step(t + 2, PhW<2>{});
        step(t + 3, PhW<3>{});
        step(t + 4, PhW<4>{});
    }
    if (nfull < T) {
        step(nfull, PhW<0>{});
        if (nfull + 1 < T) {
            step(nfull + 1, PhW<1>{});
            if (nfull + 2 < T) {
                step(nfull + 2, PhW<2>{});
                if (nfull + 3 < T) step(nfull + 3, PhW<3>{});
            }
        }
    }
}

int resident_w(const void *fn)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> cache;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : cache)
        if (e.first == fn) return e.second;
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kWavesW, 0) != hipSuccess)
        return 0;
    const int w = std::max(1, per_cu) * ncu * kWavesW;
    cache.emplace_back(fn, w);
    return w;
}

template <int OFF, int BM>
const void *weighted_fn(int dir_type)
{
    return dir_type == 2 ? reinterpret_cast<const void *>(&k_u8_weighted<OFF, 2, BM>)
                         : dir_type == 1 ? reinterpret_cast<const void *>(&k_u8_weighted<OFF, 1, BM>)
                                         : reinterpret_cast<const void *>(&k_u8_weighted<OFF, 0, BM>);
}

}  // namespace

hipError_t launch_u8_weighted(const WJob &j, hipStream_t st)
{
    if (j.Wo <= 0 || j.Ho <= 0) return hipSuccess;
    const void *fn = j.off ? weighted_fn<2, 0>(j.dir_type)
                           : j.bmode == 1 ? weighted_fn<0, 1>(j.dir_type)
                                          : j.bmode == 2 ? weighted_fn<0, 2>(j.dir_type) : weighted_fn<0, 0>(j.dir_type);
    int nstrip = (j.Wo + kColsW - 1) / kColsW;
    int slots = resident_w(fn);
    if (slots <= 0) slots = 4096;
    // at most one round of resident waves (rounding up would leave a few
    // waves for a second, nearly empty round), at least 16 rows per chunk
    int nchunk = std::max(1, std::min(slots / nstrip, std::max(1, j.Ho / 16)));
    const int64_t waves = (int64_t)nstrip * nchunk;
    const int grid = (int)((waves + kWavesW - 1) / kWavesW);
    WJob jj = j;
    void *args[] = {(void *)&jj, (void *)&nstrip, (void *)&nchunk};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWavesW), args, 0, st);
}

}  // namespace s4x5
