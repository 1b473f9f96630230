// Host side of the uint8 single-image launches: kernel selection, the
// resident-wave query and the row-range split.  Separate from u8_sweep.hpp,
// which holds only what the kernels are compiled from.
#pragma once

#include "u8_sweep.hpp"

namespace s4x5 {
namespace {

template <int PPL, int OFF, bool ALIGNED, bool DIR, int OPR, int BM>
const void *single_fn()
{
    return reinterpret_cast<const void *>(&k_u8_single<PPL, OFF, ALIGNED, DIR, OPR, BM>);
}

// Resident waves of a kernel on this device and the device's CU count
// (cached per kernel; zeros if the queries fail).
struct Residency {
    int waves, cus;
};
Residency residency(const void *fn)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, Residency>> cache;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : cache)
        if (e.first == fn) return e.second;
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kWaves, 0) != hipSuccess)
        return Residency{0, 0};
    const Residency r{std::max(1, per_cu) * ncu * kWaves, ncu};
    cache.emplace_back(fn, r);
    return r;
}

// Reflect-101 on an image narrower than 3 columns folds more than once:
// such images take the byte path, whose column map is the general fold.
template <int BM>
bool vector_path_ok(const U8Job &j)
{
    return u8_rows_aligned(j) && !(BM == kBmRefl && j.W < 3);
}

template <int PPL, int OFF, bool DIR, int OPR, int BM>
hipError_t launch_single_t(const U8Job &j, const U8Shape &s, hipStream_t st)
{
    const bool aligned = vector_path_ok<BM>(j);
    const void *fn = aligned ? single_fn<PPL, OFF, true, DIR, OPR, BM>() : single_fn<PPL, OFF, false, DIR, OPR, BM>();
    const int ntxw = (j.ntx + 3) / 4;
    const Residency res = residency(fn);
    int slots = s.waves > 0 ? s.waves : res.waves;
    if (slots <= 0) slots = 2048;
    // equal row ranges per strip, at least s.min_rows rows each, and at most
    // 2^28 waves in all (the kernel numbers waves in 32 bits)
    int nchunk = std::max(1, slots / std::max(1, ntxw));
    nchunk = std::min(nchunk, std::max(1, j.Ho / std::max(1, s.min_rows)));
    nchunk = std::min(nchunk, std::max(1, (1 << 28) / std::max(1, ntxw)));
    // Workgroups spread evenly over the CUs: in a launch of one round with
    // more workgroups than CUs and a remainder, the CUs that hold one more
    // set the time (1920x1080: 540 workgroups 6.81 us, 512 6.22 us), so
    // their number is rounded down to a multiple of the CU count.
    const int64_t wgs = ((int64_t)ntxw * nchunk + kWaves - 1) / kWaves;
    if (res.cus > 0 && wgs > res.cus && wgs % res.cus != 0 && wgs * kWaves <= res.waves) {
        const int64_t n2 = wgs / res.cus * res.cus * kWaves / ntxw;
        if (n2 >= 1) nchunk = (int)n2;
    }
    const int64_t waves = (int64_t)ntxw * nchunk;
    const int grid = (int)((waves + kWaves - 1) / kWaves);
    U8Job jj = j;
    void *args[] = {(void *)&jj, (void *)&nchunk};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

template <int PPL, int OFF, int OPR, int BM>
hipError_t launch_single_d(const U8Job &j, const U8Shape &s, hipStream_t st)
{
    // the kernels compiled with planes also write magnitudes alone (dir_type 0),
    // in the separable form
    return (j.dir_type || s.sep) ? launch_single_t<PPL, OFF, true, OPR, BM>(j, s, st)
                                 : launch_single_t<PPL, OFF, false, OPR, BM>(j, s, st);
}

// Single-image launch of operator OPR under border rule BM; with kBmRep,
// `valid` selects the VALID border (output centred at offset VOFF, the
// operator's radius).  A translation unit compiles the kernels of the rules
// it calls this with.
template <int OPR, int VOFF, int BM>
hipError_t launch_single_border(const U8Job &j, bool valid, const U8Shape &s, hipStream_t st)
{
    if (j.ntx <= 0 || j.Ho <= 0) return hipSuccess;
    if constexpr (BM == kBmRep) {
        if (valid)
            return s.ppl == 16 ? launch_single_d<16, VOFF, OPR, BM>(j, s, st) : launch_single_d<8, VOFF, OPR, BM>(j, s, st);
    }
    return s.ppl == 16 ? launch_single_d<16, 0, OPR, BM>(j, s, st) : launch_single_d<8, 0, OPR, BM>(j, s, st);
}

}  // namespace
}  // namespace s4x5
