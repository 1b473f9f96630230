// Single-image four-directional 5x5 magnitudes on the matrix cores
// (u8_mfma.hpp), every border rule.

#include "u8_mfma.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace s4x5 {
namespace {

// Workgroup of kMWaves waves: one copy of the T table, then each wave sweeps
// its own tiles through its own LDS tile.  Wave w takes column strip
// w % ntx and the w / ntx-th of nchunk equal runs of 32-row tiles, so the
// waves of a workgroup hold neighbouring strips of the same rows and the
// workgroups that share an XCD (every eighth) hold vertically neighbouring
// runs: the rows a run re-reads above and below come from the same L2.
template <int OFF, int BM>
__global__ __launch_bounds__(64 * kMWaves) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_u8_mfma(U8Job J, int nchunk)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLutTSize + kMWaves * kMTileBytes];
    lut_fill_t<64 * kMWaves>(lds);
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ntx = (J.Wo + kMCols - 1) / kMCols, nty = (J.Ho + kMRows - 1) / kMRows;
    const int w = (int)blockIdx.x * kMWaves + wv;
    if (w >= ntx * nchunk) return;
    const int sx = w % ntx, ch = w / ntx;
    const int b0 = (int)((int64_t)ch * nty / nchunk), b1 = (int)((int64_t)(ch + 1) * nty / nchunk);
    const u32 tile = (u32)(size_t)(LDS uint8_t *)lds + (u32)(kLutTSize + (wv & (kMWaves - 1)) * kMTileBytes);
    v4i A[3];
    mfma_a_default(A);
    mfma_strip<OFF, BM, MagT, kStageInPlace>(J, sx, b0, b1, tile, A, MagT{(const LDS uint8_t *)lds}, tile);
}

// Run-time kernels (weights fitting int8): the same sweep, weight operands
// from the launch's arguments, no table (square-root rounding), so each
// wave also stages its output tile in LDS for full-line stores.
template <int OFF, int BM, bool CLAMP>
__global__ __launch_bounds__(64 * kMWaves) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_u8_mfma_w(U8Job J, int nchunk,
                                                                                                     MfmaWeights W)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[kMWaves * (kMTileBytes + kMOutBytes)];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ntx = (J.Wo + kMCols - 1) / kMCols, nty = (J.Ho + kMRows - 1) / kMRows;
    const int w = (int)blockIdx.x * kMWaves + wv;
    if (w >= ntx * nchunk) return;
    const int sx = w % ntx, ch = w / ntx;
    const int b0 = (int)((int64_t)ch * nty / nchunk), b1 = (int)((int64_t)(ch + 1) * nty / nchunk);
    const u32 base = (u32)(size_t)(LDS uint8_t *)lds + (u32)((wv & (kMWaves - 1)) * (kMTileBytes + kMOutBytes));
    v4i A[3];
    mfma_a_runtime(W, A);
    mfma_strip<OFF, BM, MagS<CLAMP>, kStageOwn>(J, sx, b0, b1, base, A, MagS<CLAMP>{}, base + kMTileBytes);
}

const void *mfma_fn(int border)
{
    switch (border) {
    case 1: return reinterpret_cast<const void *>(&k_u8_mfma<2, kBmRep>);
    case 2: return reinterpret_cast<const void *>(&k_u8_mfma<0, kBmZero>);
    case 3: return reinterpret_cast<const void *>(&k_u8_mfma<0, kBmRefl>);
    default: return reinterpret_cast<const void *>(&k_u8_mfma<0, kBmRep>);
    }
}

template <bool CLAMP>
const void *mfma_w_fn(int border)
{
    switch (border) {
    case 1: return reinterpret_cast<const void *>(&k_u8_mfma_w<2, kBmRep, CLAMP>);
    case 2: return reinterpret_cast<const void *>(&k_u8_mfma_w<0, kBmZero, CLAMP>);
    case 3: return reinterpret_cast<const void *>(&k_u8_mfma_w<0, kBmRefl, CLAMP>);
    default: return reinterpret_cast<const void *>(&k_u8_mfma_w<0, kBmRep, CLAMP>);
    }
}

// Resident waves of the kernel on the current device.
int mfma_slots(const void *fn)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kMWaves, 0) != hipSuccess)
        return 0;
    return std::max(1, per_cu) * ncu * kMWaves;
}

}  // namespace

namespace {

// Waves of a launch over the image's 32 x 128 tiles: `waves` (> 0) or four
// rounds of resident waves, as runs of whole tiles per strip.
hipError_t mfma_launch(const void *fn, const U8Job &j, int waves, void *extra, hipStream_t st)
{
    const int64_t ntx = (j.Wo + kMCols - 1) / kMCols, nty = (j.Ho + kMRows - 1) / kMRows;
    // default: four rounds of resident waves, about one tile each (8192^2:
    // 56.1 us against 62.5 for one round of four tiles per wave)
    int64_t slots = waves > 0 ? waves : 4 * (int64_t)mfma_slots(fn);
    if (slots <= 0) slots = 16384;
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(nty, slots / ntx));
    nchunk = std::min<int64_t>(nchunk, std::max<int64_t>(1, ((int64_t)1 << 30) / ntx));
    const int64_t total = ntx * nchunk;
    const int grid = (int)((total + kMWaves - 1) / kMWaves);
    U8Job jj = j;
    int nc = (int)nchunk;
    void *args[] = {(void *)&jj, (void *)&nc, extra};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kMWaves), args, 0, st);
}

}  // namespace

hipError_t launch_u8_mfma(const U8Job &j, int border, int waves, hipStream_t st)
{
    if (j.Wo <= 0 || j.Ho <= 0) return hipSuccess;
    return mfma_launch(mfma_fn(border), j, waves, nullptr, st);
}

bool mfma_weights_fit(const int32_t *weights)
{
    for (int i = 0; i < 100; ++i)
        if (weights[i] < -128 || weights[i] > 127) return false;
    return true;
}

hipError_t launch_u8_mfma_weighted(const U8Job &j, int border, const int32_t *weights, int waves, hipStream_t st)
{
    if (j.Wo <= 0 || j.Ho <= 0) return hipSuccess;
    struct Taps {
        const int32_t *w;
        int operator()(int f, int dy, int dx) const { return w[25 * f + 5 * dy + dx]; }
    };
    // the operands of the last weights this thread launched with (a run of
    // calls with the same kernels builds them once)
    thread_local int32_t last[100];
    thread_local MfmaWeights W;
    thread_local bool have = false;
    if (!have || std::memcmp(last, weights, sizeof(last)) != 0) {
        W = mfma_weights(Taps{weights});
        std::memcpy(last, weights, sizeof(last));
        have = true;
    }
    // without the clamp, 4 G^2 must stay below 2^31: |G| <= 128 sum|k| <= 23168
    int64_t most = 0;
    for (int f = 0; f < 4; ++f) {
        int64_t a = 0;
        for (int t = 0; t < 25; ++t) a += weights[25 * f + t] < 0 ? -(int64_t)weights[25 * f + t] : weights[25 * f + t];
        most = std::max(most, a);
    }
    const void *fn = most <= 181 ? mfma_w_fn<false>(border) : mfma_w_fn<true>(border);
    return mfma_launch(fn, j, waves, (void *)&W, st);
}

}  // namespace s4x5
