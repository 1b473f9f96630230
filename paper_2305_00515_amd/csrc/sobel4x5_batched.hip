// Batched uint8 four-directional kernel: many images of uneven sizes in one
// persistent launch of the sweep in u8_sweep.hpp, for every border rule,
// with or without directional planes.

#include "u8_sweep.hpp"

#include <algorithm>
#include <cstdlib>
#include <mutex>

namespace s4x5 {
namespace {

// Geometry of one wave-tile of the batched kernel, ti = {image, kind | rows << 1,
// tx, y0} (built on the host by batched_tiles):
//   kind 0: four tiles side by side, tile columns tx .. tx+3 (a complete
//           strip), output rows [y0, y0 + rows): every group walks the same
//           rows and each load instruction covers one contiguous row segment;
//   kind 1: four tiles of th rows stacked in tile column tx, starting at
//           row y0, for the columns an image has beyond its last complete
//           strip.
// The two kinds run the sweep from separate call sites: a kind-0 tile's rows
// are the same in every lane, so its row addresses stay in scalar registers
// (with one call site for both, the stacked rows of kind 1 made them
// per-lane, about 17 more vector instructions per row).
__device__ __forceinline__ Sweep strip_geometry(const U8Job &J, const int4 &ti, int ppl)
{
    const int tw = 16 * ppl;
    const int grp = (threadIdx.x >> 4) & 3;
    const int lane16 = threadIdx.x & 15;
    Sweep g;
    const int tx = ti.z + grp;
    g.xo = tx * tw + lane16 * ppl;
    g.yo0 = ti.w;
    g.nrow = min(ti.y >> 1, J.Ho - g.yo0);
    g.niter = g.nrow;
    g.fix_right = (ti.z + 4) * tw + 4 > J.W;
    g.fix_left = ti.z == 0;
    return g;
}
__device__ __forceinline__ Sweep stack_geometry(const U8Job &J, const int4 &ti, int ppl, int th)
{
    const int tw = 16 * ppl;
    const int grp = (threadIdx.x >> 4) & 3;
    const int lane16 = threadIdx.x & 15;
    Sweep g;
    g.xo = ti.z * tw + lane16 * ppl;
    g.yo0 = ti.w + grp * th;
    g.nrow = g.yo0 < J.Ho ? min(th, J.Ho - g.yo0) : 0;
    g.niter = max(max(__builtin_amdgcn_readlane(g.nrow, 0), __builtin_amdgcn_readlane(g.nrow, 16)),
                  max(__builtin_amdgcn_readlane(g.nrow, 32), __builtin_amdgcn_readlane(g.nrow, 48)));
    g.fix_right = (ti.z + 1) * tw + 4 > J.W;
    g.fix_left = ti.z == 0;
    return g;
}

// Persistent work-queue kernel: every wave takes the next wave-tile of the
// whole batch from queue[0] until none are left, then counts itself out in
// queue[1]; the last wave out resets both words for the next launch.  With
// queue == nullptr the grid holds one wave per tile instead (static form).  A
// ticket indexes the host-built tile table, so finding a tile is one load.
// claims (debug launches only, else nullptr): one counter per tile, plus one
// for every time a wave takes that tile, so a launch that leaves any counter
// other than 1 has skipped or repeated a tile.
// DIR: images whose job asks for them also get their directional planes.
// The sweeps run whole blocks of five row steps plus a tail, as in the
// single-image kernel: with the tall chunks of 128 rows this measured 2.7%
// faster than the loop that leaves after any step (0.8005 against 0.8227
// ms on the 256-image batch, 1.7% fewer vector instructions).
template <int PPL, int OFF, bool ALIGNED, bool DIR, int BM>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(
    single_waves(PPL, kOp4x5, ALIGNED, DIR), single_waves(PPL, kOp4x5, ALIGNED, DIR)))) void k_u8_batched(const U8Job *__restrict__ jobs,
                                                            const int4 *__restrict__ tiles, int32_t total,
                                                            uint32_t *queue, int TH, uint32_t *claims)
{
    constexpr int TW = 16 * PPL;
    constexpr int WV = single_waves(PPL, kOp4x5, ALIGNED, DIR);
    constexpr bool LUT = use_lut(WV);
    constexpr bool BIN = binomial_form(kOp4x5, DIR);
    __shared__ __attribute__((aligned(16))) uint8_t lut[lut_bytes(kOp4x5, DIR, WV)];
    lds_u8 *lutp = (lds_u8 *)lut;
    const int lane = threadIdx.x & 63;
    // one tile of the table; `pre` runs around its first row loads
    auto run_tile = [&](int t, auto pre) __attribute__((always_inline)) {
        const int4 ti = tiles[t];
        const U8Job J = jobs[ti.x];
        // fast: every group has its full rows, every lane's block and output
        // inside the image
        auto run = [&](Sweep g, bool fast) __attribute__((always_inline)) {
            g.fix_left = g.fix_left && OFF == 0;
            if (g.niter <= 0) {
                pre.issue();
                pre.finish();
                return;
            }
            if (fast && !g.fix_right && !g.fix_left)
                sweep<PPL, OFF, ALIGNED, DIR, true, false, kOp4x5, BM, LUT, true>(J, g, lutp, pre);
            else if (fast)
                sweep<PPL, OFF, ALIGNED, DIR, true, true, kOp4x5, BM, LUT, true>(J, g, lutp, pre);
            else
                sweep<PPL, OFF, ALIGNED, DIR, false, false, kOp4x5, BM, LUT, true>(J, g, lutp, pre);
        };
        if ((ti.y & 1) == 0) {
            run(strip_geometry(J, ti, PPL), ALIGNED && (ti.z + 4) * TW <= J.Wo);
        } else {
            const Sweep g = stack_geometry(J, ti, PPL, TH);
            const bool full = __builtin_amdgcn_readlane(g.nrow, 0) == TH && __builtin_amdgcn_readlane(g.nrow, 16) == TH &&
                              __builtin_amdgcn_readlane(g.nrow, 32) == TH && __builtin_amdgcn_readlane(g.nrow, 48) == TH;
            run(g, ALIGNED && full && (ti.z + 1) * TW <= J.Wo);
        }
    };
    if (queue == nullptr) {
        // static form: wave w of the grid takes tile w, no queue; the
        // binomial kernel copies its table while the tile's first rows load
        // (every wave of the workgroup reaches that one barrier)
        const int t = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (claims != nullptr && lane == 0 && t < total) atomicAdd(&claims[t], 1u);
        if constexpr (BIN) {
            if (t < total)
                run_tile(t, LutPrelude<64 * kWaves>{{}, lut});
            else
                lut_setup<kOp4x5, DIR, WV, 64 * kWaves>(lut);
        } else {
            lut_setup<kOp4x5, DIR, WV, 64 * kWaves>(lut);
            if (t < total) run_tile(t, NoPrelude{});
        }
        return;
    }
    lut_setup<kOp4x5, DIR, WV, 64 * kWaves>(lut);
    for (;;) {
        u32 tv = 0;
        if (lane == 0) tv = atomicAdd(&queue[0], 1u);
        const int t = __builtin_amdgcn_readfirstlane((int)tv);
        if (t >= total) break;
        if (claims != nullptr && lane == 0) atomicAdd(&claims[t], 1u);
        run_tile(t, NoPrelude{});
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

template <int PPL, int OFF, int BM>
const void *batched_fn(bool aligned, bool dir)
{
    if (dir)
        return aligned ? reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, true, true, BM>)
                       : reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, false, true, BM>);
    return aligned ? reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, true, false, BM>)
                   : reinterpret_cast<const void *>(&k_u8_batched<PPL, OFF, false, false, BM>);
}

template <int PPL>
const void *pick_ppl(int border, bool aligned, bool dir)
{
    switch (border) {
    case 1: return batched_fn<PPL, 2, kBmRep>(aligned, dir);
    case 2: return batched_fn<PPL, 0, kBmZero>(aligned, dir);
    case 3: return batched_fn<PPL, 0, kBmRefl>(aligned, dir);
    default: return batched_fn<PPL, 0, kBmRep>(aligned, dir);
    }
}

// border: the public SOBEL4X5_BORDER_* code
const void *pick_batched(int ppl, int border, bool aligned, bool dir)
{
    return ppl == 16 ? pick_ppl<16>(border, aligned, dir) : pick_ppl<8>(border, aligned, dir);
}

}  // namespace

// The split of an image's strips into tall and short row chunks (see
// batched_tiles_each): tall chunks of `tallx` tile heights, the last
// 1/`shortq` of the rows in chunks of one.  Tall chunks of 2 tile heights
// measured best with the autotuned tile height (256 mixed images: 0.817 ms
// against 0.836 for 4 and 0.876 for 8); SOBEL4X5_BATCH_TALLX and
// SOBEL4X5_BATCH_SHORTQ override them (read once per process).
BatchSplit batched_split()
{
    static const BatchSplit s = [] {
        auto get = [](const char *name, int dflt) {
            const char *v = std::getenv(name);
            const int x = v ? std::atoi(v) : 0;
            return x >= 1 && x <= 64 ? x : dflt;
        };
        return BatchSplit{get("SOBEL4X5_BATCH_TALLX", 2), get("SOBEL4X5_BATCH_SHORTQ", 4)};
    }();
    return s;
}

void batched_tiles(const U8Job &j, int32_t img, int th, int tallx, std::vector<int4> &first,
                   std::vector<int4> &last)
{
    batched_tiles_each(j, img, th, tallx, [&](int4 t) { first.push_back(t); }, [&](int4 t) { last.push_back(t); });
}

// Static grid: workgroup g (four wave-tiles, in dispatch order) runs on XCD
// g mod 8, so in the table order the workgroups that share an XCD's L2 are
// eight apart, and a row band's neighbours above and to the side (whose
// halo rows and columns it reads again) sit on other XCDs.  Reordered,
// each XCD takes one of eight contiguous stretches of [b, e) (whole
// workgroups of the table order, the ones left over stay at the end), and
// the rows those neighbours read come from its own L2.  b is a multiple of
// four, so the workgroups of [b, e) start at a workgroup boundary and each
// residue of their index mod 8 is one XCD.  SOBEL4X5_BATCH_XCD=0 keeps the
// table order (read once per process).
void xcd_order(std::vector<int4> &v, size_t b, size_t e)
{
    static const bool on = [] {
        const char *s = std::getenv("SOBEL4X5_BATCH_XCD");
        return !(s && std::atoi(s) == 0);
    }();
    constexpr size_t kX = 8, kG = kWaves;
    const size_t ng = (e - b) / kG;
    if (!on || ng < 2 * kX) return;
    std::vector<int4> src(v.begin() + b, v.begin() + b + ng * kG);
    size_t start[kX + 1] = {0};
    for (size_t x = 0; x < kX; ++x) start[x + 1] = start[x] + (ng - x + kX - 1) / kX;   // groups g = x mod 8
    for (size_t g = 0; g < ng; ++g) {
        const size_t from = start[g % kX] + g / kX;
        std::copy(src.begin() + from * kG, src.begin() + (from + 1) * kG, v.begin() + b + g * kG);
    }
}

hipError_t launch_u8_batched(const U8Job *jobs, const int4 *tiles, int32_t total, uint32_t *queue, int border,
                             bool aligned, bool dir, const U8Shape &s, int grid, hipStream_t st, uint32_t *claims)
{
    const void *fn = pick_batched(s.ppl, border, aligned, dir);
    int th = s.th;
    void *args[] = {(void *)&jobs, (void *)&tiles, (void *)&total, (void *)&queue, (void *)&th, (void *)&claims};
    return hipLaunchKernel(fn, dim3(grid), dim3(64 * kWaves), args, 0, st);
}

// The fixed buffer of the allocation-free batched call.  In host code this
// name is only a handle for hipGetSymbolAddress; kernels get the device
// address that call returns.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

hipError_t noalloc_scratch(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

int u8_persistent_grid(const U8Shape &s, int border, bool aligned, bool dir)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick_batched(s.ppl, border, aligned, dir),
                                                     64 * kWaves, 0) != hipSuccess)
        return 0;
    if (per_cu < 1) per_cu = 1;
    return ncu * per_cu;
}

}  // namespace s4x5
