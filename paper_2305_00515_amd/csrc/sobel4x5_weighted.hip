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
// The 12 pair differences are shared by the four responses, so a pixel
// costs 12 subtractions and 48 multiply-adds (v_mad_i32_i24: |k| < 2^23,
// |difference| <= 255), all exact in int32 for the weight bounds the host
// checks.  The magnitude rounds min(255, round(sqrt(S))) exactly: every
// |G_k| is clamped at 256 first, which changes S only where S >= 65536 and
// the result saturates anyway, so S stays below 2^24 and its float square
// root rounds correctly (no integer S is within 4.9e-4 of a half-integer
// root).  The paper's own factoring (Eq. (sobel5_kd+-), (sobel5_4)) serves
// the default weights on the packed fast path.
//
// Work layout: a lane owns 4 consecutive output pixels of a row and walks a
// range of rows with a 5-row register ring of the 8 input bytes it needs;
// a wave covers 256 columns.

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

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Sign-extend from 24 bits: a no-op for the coefficients (the host checks
// |k| < 2^23) that lets the products use the full-rate 24-bit multiplier.
__device__ __forceinline__ int s24(int v) { return (v << 8) >> 8; }

template <int P>
using PhW = std::integral_constant<int, P>;

// Upper-half taps (i, j) in the order of the coefficient table: row 0, row 1,
// then (2, 0), (2, 1); the partner tap is (4 - i, 4 - j).
__device__ __forceinline__ constexpr int tap_i(int t) { return t < 5 ? 0 : (t < 10 ? 1 : 2); }
__device__ __forceinline__ constexpr int tap_j(int t) { return t < 10 ? t % 5 : t - 10; }

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

    // bytes, so that every pair difference is known to fit 24 bits
    uint8_t ring[5][kPplW + 4], pf[5][kPplW + 4];
    constexpr int PD = 2;   // rows loaded ahead
#pragma unroll
    for (int t = 0; t < PD; ++t) {
        ldrow(t, pf[t]);
        __builtin_amdgcn_sched_barrier(0);   // prologue rows in row order
    }

    auto step = [&](int t, auto phase) {
        constexpr int p = decltype(phase)::value;
        ldrow(t + PD, pf[(p + PD) % 5]);
        if constexpr (BM == 1) {
            const u32 in = inside(t);
#pragma unroll
            for (int j = 0; j < kPplW + 4; ++j) ring[p][j] = ((in >> j) & 1u) ? pf[p][j] : (uint8_t)0;
        } else {
#pragma unroll
            for (int j = 0; j < kPplW + 4; ++j) ring[p][j] = pf[p][j];
        }
        if (t < 4) return;
        // window row i (0..4) = input row t - 4 + i, in slot (p + 1 + i) % 5
        const int yo = y0 + t - 4;
        int G[kPplW][4];
#pragma unroll
        for (int q = 0; q < kPplW; ++q) {
            int d[12];
#pragma unroll
            for (int u = 0; u < 12; ++u) {
                const int i = tap_i(u), jj = tap_j(u);
                d[u] = (int)ring[(p + 1 + i) % 5][q + jj] - (int)ring[(p + 1 + 4 - i) % 5][q + 4 - jj];
            }
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
                int acc = 0;
#pragma unroll
                for (int u = 0; u < 12; ++u) acc += s24(J.coef[pl][u]) * d[u];
                G[q][pl] = acc;
            }
        }
        if (J.mag) {
            u32 out = 0;
            const int nvalid = J.Wo - xo;
#pragma unroll
            for (int q = 0; q < kPplW; ++q) {
                int S = 0;
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) {
                    const int g = min(abs(G[q][pl]), 256);
                    S += g * g;
                }
                const u32 m = S >= 65281 ? 255u
                                         : __builtin_amdgcn_cvt_pk_u8_f32(__builtin_amdgcn_sqrtf((float)S), 0, 0u);
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
