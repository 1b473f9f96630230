// Single-image four-directional 5x5 magnitudes on the matrix cores
// (u8_mfma.hpp), every border rule.

#include "u8_mfma.hpp"

#include <algorithm>
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
    mfma_strip<OFF, BM>(J, sx, b0, b1, tile, (const LDS uint8_t *)lds);
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

hipError_t launch_u8_mfma(const U8Job &j, int border, int waves, hipStream_t st)
{
    if (j.Wo <= 0 || j.Ho <= 0) return hipSuccess;
    const void *fn = mfma_fn(border);
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
    void *args[] = {(void *)&jj, (void *)&nc};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kMWaves), args, 0, st);
}

}  // namespace s4x5
