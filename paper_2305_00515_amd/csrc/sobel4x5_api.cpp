// C-ABI layer of the four-directional 5x5 Sobel library: argument checks,
// tile-shape choice, launches, batched plans (hipGraph), autotuning.
#include "../../include/sobel4x5.h"

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include <sys/stat.h>

#include "internal.hpp"

using namespace s4x5;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    return SOBEL4X5_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SOBEL4X5_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Test hook (sobel4x5_debug_inject_failure): while armed with n > 0, the
// n-th HIP call that passes through guard() reports hipErrorUnknown in place
// of its own result, which exercises the error paths without a real runtime
// failure.  The call itself still ran (an enqueued copy is still queued).
std::atomic<int> g_inject{0};

hipError_t guard(hipError_t e)
{
    int n = g_inject.load(std::memory_order_relaxed);
    while (n > 0) {
        if (g_inject.compare_exchange_weak(n, n - 1, std::memory_order_relaxed)) return n == 1 ? hipErrorUnknown : e;
    }
    return e;
}

constexpr int64_t kMaxDim = 1 << 30;

// Output size of an operator of radius r (2 for the 5x5 filters, 1 for 3x3).
int out_dims_r(int32_t W, int32_t H, int32_t border, int r, int32_t *Wo, int32_t *Ho)
{
    if (border != SOBEL4X5_BORDER_REPLICATE && border != SOBEL4X5_BORDER_VALID && border != SOBEL4X5_BORDER_ZERO &&
        border != SOBEL4X5_BORDER_REFLECT101)
        return fail(SOBEL4X5_EINVAL, "border must be REPLICATE (0), VALID (1), ZERO (2) or REFLECT101 (3), got %d",
                    border);
    if (W < 1 || H < 1) return fail(SOBEL4X5_EINVAL, "width and height must be >= 1 (got %d x %d)", W, H);
    if (W > kMaxDim || H > kMaxDim) return fail(SOBEL4X5_EINVAL, "image too large");
    if (border == SOBEL4X5_BORDER_VALID) {
        if (W < 2 * r + 1 || H < 2 * r + 1)
            return fail(SOBEL4X5_EINVAL, "VALID border needs width and height >= %d (got %d x %d)", 2 * r + 1, W, H);
        *Wo = W - 2 * r;
        *Ho = H - 2 * r;
    } else {
        *Wo = W;
        *Ho = H;
    }
    return ok();
}

int out_dims(int32_t W, int32_t H, int32_t border, int32_t *Wo, int32_t *Ho)
{
    return out_dims_r(W, H, border, 2, Wo, Ho);
}

struct Range {
    uintptr_t lo, hi;   // [lo, hi)
};

Range span(const void *p, int64_t rows, int64_t pitch, int64_t row_bytes)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    return {a, a + (uintptr_t)((rows - 1) * pitch + row_bytes)};
}

bool overlap(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

int check_pitch(const char *name, int64_t pitch, int64_t row_bytes, int64_t rows)
{
    if (pitch < row_bytes)
        return fail(SOBEL4X5_EINVAL, "%s pitch %lld is smaller than a row (%lld bytes)", name,
                    (long long)pitch, (long long)row_bytes);
    if (rows > 0 && pitch > (INT64_MAX / 2) / rows) return fail(SOBEL4X5_EINVAL, "%s pitch overflows", name);
    return ok();
}

// Arguments of one uint8 image for operator `op` (SOBEL4X5_OP_*): the
// two-directional operators write directional planes 0 and 2 only.
int validate_u8(const uint8_t *src, int32_t W, int32_t H, int64_t pitch, int32_t border,
                const sobel4x5_outputs *out, int32_t *pWo, int32_t *pHo, int32_t op = SOBEL4X5_OP_4DIR_5X5)
{
    int32_t Wo, Ho;
    if (op != SOBEL4X5_OP_4DIR_5X5 && op != SOBEL4X5_OP_2DIR_5X5 && op != SOBEL4X5_OP_2DIR_3X3)
        return fail(SOBEL4X5_EINVAL, "op must be 0, 1 or 2, got %d", op);
    if (int rc = out_dims_r(W, H, border, op == SOBEL4X5_OP_2DIR_3X3 ? 1 : 2, &Wo, &Ho)) return rc;
    if (!src) return fail(SOBEL4X5_EINVAL, "src is NULL");
    if (!out) return fail(SOBEL4X5_EINVAL, "out is NULL");
    if (int rc = check_pitch("src", pitch, W, H)) return rc;
    if (out->dir_type != SOBEL4X5_DIR_NONE && out->dir_type != SOBEL4X5_DIR_S16 &&
        out->dir_type != SOBEL4X5_DIR_S32)
        return fail(SOBEL4X5_EINVAL, "dir_type must be 0, 1 or 2, got %d", out->dir_type);
    if (!out->mag && out->dir_type == SOBEL4X5_DIR_NONE)
        return fail(SOBEL4X5_EINVAL, "no output requested (mag is NULL and dir_type is NONE)");
    const Range rs = span(src, H, pitch, W);
    std::vector<Range> outs;
    if (out->mag) {
        if (int rc = check_pitch("mag", out->mag_pitch, Wo, Ho)) return rc;
        outs.push_back(span(out->mag, Ho, out->mag_pitch, Wo));
    }
    if (out->dir_type != SOBEL4X5_DIR_NONE) {
        const int64_t es = out->dir_type == SOBEL4X5_DIR_S16 ? 2 : 4;
        if (int rc = check_pitch("dir", out->dir_pitch, (int64_t)Wo * es, Ho)) return rc;
        if (out->dir_pitch % es) return fail(SOBEL4X5_EINVAL, "dir pitch must be a multiple of the element size");
        for (int k = 0; k < 4; ++k) {
            if (op != SOBEL4X5_OP_4DIR_5X5 && (k & 1)) continue;
            if (!out->dir[k]) return fail(SOBEL4X5_EINVAL, "dir[%d] is NULL", k);
            if (reinterpret_cast<uintptr_t>(out->dir[k]) % es)
                return fail(SOBEL4X5_EINVAL, "dir[%d] is not aligned to its element size", k);
            outs.push_back(span(out->dir[k], Ho, out->dir_pitch, (int64_t)Wo * es));
        }
    }
    for (size_t i = 0; i < outs.size(); ++i) {
        if (overlap(outs[i], rs)) return fail(SOBEL4X5_EINVAL, "an output overlaps src");
        for (size_t k = i + 1; k < outs.size(); ++k)
            if (overlap(outs[i], outs[k])) return fail(SOBEL4X5_EINVAL, "two outputs overlap");
    }
    *pWo = Wo;
    *pHo = Ho;
    return ok();
}

U8Job make_job(const uint8_t *src, int32_t W, int32_t H, int64_t pitch, int32_t Wo, int32_t Ho,
               uint8_t *mag, int64_t mag_pitch, const void *const dir[4], int64_t dir_pitch, int32_t dir_type)
{
    U8Job j;
    std::memset(&j, 0, sizeof j);
    j.src = src;
    j.mag = mag;
    for (int k = 0; k < 4; ++k) j.dir[k] = dir ? const_cast<void *>(dir[k]) : nullptr;
    j.src_pitch = pitch;
    j.mag_pitch = mag_pitch;
    j.dir_pitch = dir_pitch;
    j.W = W;
    j.H = H;
    j.Wo = Wo;
    j.Ho = Ho;
    j.dir_type = dir_type;
    return j;
}

int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    const long x = std::strtol(v, &end, 10);
    return (end && *end == 0 && x >= 0 && x < (1 << 30)) ? (int)x : dflt;
}

// Shape for one image: 16 pixels per lane when a strip of four 256-column
// tiles is mostly inside the image, else 8; directional outputs use 8 (their
// kernel keeps more values live).  SOBEL4X5_U8_PPL (8 or 16),
// SOBEL4X5_U8_WAVES (waves to launch) and SOBEL4X5_U8_MIN_ROWS (fewest rows
// per wave) override the choice for tuning runs.
// U8Shape::waves of a batched plan that launches one wave per tile (static
// form, no work queue) instead of a persistent grid.
constexpr int kStaticGrid = 1 << 30;

// Compute units of the current device (cached per device; 256 if unknown).
int device_cus()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

U8Shape default_shape(int32_t Wo, int32_t Ho, int32_t dir_type, int32_t op = SOBEL4X5_OP_4DIR_5X5)
{
    U8Shape s;
    // The four-directional magnitude kernel (binomial form) runs 8 pixels
    // per lane at three waves per SIMD at every size: at 16 it needs more
    // than the 256 registers of two waves per SIMD (8192^2: 46.2 against
    // 60.4 us; 16384^2: 162 against 180 us).  The two-directional operators
    // take 16 pixels per lane (1024-column strips) only where that shape
    // alone fills one round of resident waves (2 per SIMD, 8 per CU) with
    // its 2-row minimum ranges; smaller images have too few waves.
    const int64_t strips16 = (Wo + 1023) / 1024;
    const bool fills = strips16 * (Ho / 2) >= 8 * (int64_t)device_cus();
    s.ppl = (fills && dir_type == SOBEL4X5_DIR_NONE && op != SOBEL4X5_OP_4DIR_5X5) ? 16 : 8;
    // The binomial form does most of its work once per input row, so a
    // wave that gets few rows pays heavily for the 4 rows above its range:
    // below 8 rows per wave (one round of 12 waves per CU over 512-column
    // strips) the four-directional magnitude takes the separable form
    // (graph replay: 512^2 3.48 against 4.32 us, 1920x1080 6.92 against
    // 9.33, 3840x2160 12.6 against 13.9; from 4096^2 on the binomial form
    // wins: 17.4 against 18.1), with 4-row minimum ranges from 2048 rows on.
    // The same holds for the 0 / 90 deg pair of the 5x5 operator at 8 pixels
    // per lane (graph replay: 1024^2 4.00 against 4.34 us; 8192^2 binomial
    // 31.2 against 37.2); at 16 (from 2048^2 on) its separable kernel that
    // can also write planes runs one wave per SIMD fewer, and the binomial
    // form stays (2048^2: 6.96 against 7.39 us).
    if ((op == SOBEL4X5_OP_4DIR_5X5 || (op == SOBEL4X5_OP_2DIR_5X5 && s.ppl == 8)) &&
        dir_type == SOBEL4X5_DIR_NONE) {
        const int64_t strips8 = (Wo + 511) / 512;
        const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(12 * (int64_t)device_cus() / strips8, Ho / 2));
        if (Ho < 8 * nchunk) {
            s.sep = true;
            if (op == SOBEL4X5_OP_4DIR_5X5 && Ho >= 2048) s.min_rows = 4;
        }
    }
    const int ppl = env_int("SOBEL4X5_U8_PPL", 0);
    if (ppl == 8 || ppl == 16) s.ppl = ppl;
    s.th = 32;
    s.wpg = 4;
    // Directional planes (up to 17 B/px) are bound by the stores: many short
    // row ranges, 4 rows each, beat one round of resident waves (8192^2 int16
    // planes: 487 against 432 Gpx/s).
    if (dir_type != SOBEL4X5_DIR_NONE) {
        s.waves = 1 << 30;
        s.min_rows = 4;
    }
    const int waves = env_int("SOBEL4X5_U8_WAVES", 0);
    if (waves > 0) s.waves = waves;
    const int mr = env_int("SOBEL4X5_U8_MIN_ROWS", 0);
    if (mr >= 1 && mr <= 64) s.min_rows = mr;
    const int sep = env_int("SOBEL4X5_U8_SEP", -1);
    if (sep == 0 || sep == 1) s.sep = sep == 1;
    return s;
}

// Border rule of the fp32 kernels: 0 reads the nearest pixel (REPLICATE,
// and VALID, whose taps stay inside), 1 ZERO, 2 REFLECT101.
int f32_bmode(int32_t border)
{
    return border == SOBEL4X5_BORDER_ZERO ? 1 : border == SOBEL4X5_BORDER_REFLECT101 ? 2 : 0;
}

// A batch of `batch` fp32 images of rows x cols, image b at p + b*bstride.
int check_f32_buf(const char *name, const float *p, int32_t batch, int32_t cols, int32_t rows, int64_t pitch,
                  int64_t bstride, Range *r)
{
    if (!p) return fail(SOBEL4X5_EINVAL, "%s is NULL", name);
    if ((reinterpret_cast<uintptr_t>(p) & 3u) || (pitch & 3) || (bstride & 3))
        return fail(SOBEL4X5_EINVAL, "%s: pointer, pitch and batch stride must be multiples of 4 bytes", name);
    if (int rc = check_pitch(name, pitch, (int64_t)cols * 4, rows)) return rc;
    const int64_t img = (int64_t)(rows - 1) * pitch + (int64_t)cols * 4;
    if (batch > 1 && bstride < img) return fail(SOBEL4X5_EINVAL, "%s batch stride is smaller than an image", name);
    if (batch > 1 && bstride > (INT64_MAX / 2) / batch) return fail(SOBEL4X5_EINVAL, "%s batch stride overflows", name);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    *r = {a, a + (uintptr_t)((batch > 0 ? batch - 1 : 0) * bstride + img)};
    return ok();
}

// Outputs of batch image i: outs[i] when given, else the image's own mag.
sobel4x5_outputs batch_outputs(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t i)
{
    if (outs) return outs[i];
    sobel4x5_outputs o;
    std::memset(&o, 0, sizeof o);
    o.mag = imgs[i].mag;
    o.mag_pitch = imgs[i].mag_pitch;
    return o;
}

// Memory ranges every output of one image writes.
void output_ranges(const sobel4x5_outputs &o, int32_t Wo, int32_t Ho, std::vector<Range> &v)
{
    if (o.mag) v.push_back(span(o.mag, Ho, o.mag_pitch, Wo));
    if (o.dir_type != SOBEL4X5_DIR_NONE) {
        const int64_t es = o.dir_type == SOBEL4X5_DIR_S16 ? 2 : 4;
        for (int k = 0; k < 4; ++k) v.push_back(span(o.dir[k], Ho, o.dir_pitch, (int64_t)Wo * es));
    }
}

int validate_batch(const sobel4x5_image *imgs, const sobel4x5_outputs *outs_in, int32_t count, int32_t border)
{
    if (!imgs) return fail(SOBEL4X5_EINVAL, "imgs is NULL");
    if (count < 1) return fail(SOBEL4X5_EINVAL, "count must be >= 1 (got %d)", count);
    std::vector<Range> outs;
    for (int32_t i = 0; i < count; ++i) {
        const sobel4x5_image &m = imgs[i];
        const sobel4x5_outputs o = batch_outputs(imgs, outs_in, i);
        if (!outs_in && !m.mag) return fail(SOBEL4X5_EINVAL, "image %d: mag is NULL", i);
        int32_t Wo, Ho;
        if (validate_u8(m.src, m.width, m.height, m.src_pitch, border, &o, &Wo, &Ho))
            return fail(SOBEL4X5_EINVAL, "image %d: %s", i, g_last_error.c_str());
        output_ranges(o, Wo, Ho, outs);
    }
    // outputs of different images must not overlap each other (sorted sweep)
    std::sort(outs.begin(), outs.end(), [](const Range &a, const Range &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].lo < outs[i - 1].hi) return fail(SOBEL4X5_EINVAL, "outputs of two images overlap");
    // no output may overlap any input
    std::vector<Range> ins(count);
    for (int32_t i = 0; i < count; ++i) ins[i] = span(imgs[i].src, imgs[i].height, imgs[i].src_pitch, imgs[i].width);
    std::sort(ins.begin(), ins.end(), [](const Range &a, const Range &b) { return a.lo < b.lo; });
    for (const Range &o : outs) {
        auto it = std::upper_bound(ins.begin(), ins.end(), o.hi,
                                   [](uintptr_t v, const Range &r) { return v <= r.lo; });
        for (auto k = ins.begin(); k != it; ++k)
            if (overlap(*k, o)) return fail(SOBEL4X5_EINVAL, "an output overlaps an input");
    }
    return ok();
}

// ------------------------------------------------------------------ plans

constexpr uint32_t kPlanMagic = 0x534f4234u;   // "SOB4"

}  // namespace

struct sobel4x5_plan_s {
    uint32_t magic = kPlanMagic;
    int device = 0;
    int32_t count = 0;
    int32_t border = 0;
    U8Shape shape{};
    int grid = 0;
    bool use_graph = true;
    bool aligned = true;
    std::vector<sobel4x5_image> imgs;
    std::vector<sobel4x5_outputs> outs;   // per image: mag and/or directional planes
    bool dir = false;                     // some image asks for directional planes
    U8Job *d_jobs = nullptr;
    int4 *d_tiles = nullptr;      // {image, kind | rows << 1, tx, y0} per queue ticket
    int32_t total = 0;            // wave-tiles of the batch
    uint32_t *d_queue = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free_device(sobel4x5_plan_s *p)
{
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->d_jobs) hipFree(p->d_jobs);
    if (p->d_tiles) hipFree(p->d_tiles);
    if (p->d_queue) hipFree(p->d_queue);
    p->exec = nullptr;
    p->graph = nullptr;
    p->d_jobs = nullptr;
    p->d_tiles = nullptr;
    p->d_queue = nullptr;
}

// Build device tables for `shape` (no graph).
int plan_setup(sobel4x5_plan_s *p, const U8Shape &shape)
{
    plan_free_device(p);
    p->shape = shape;
    std::vector<U8Job> jobs(p->count);
    bool aligned = true;
    for (int32_t i = 0; i < p->count; ++i) {
        const sobel4x5_image &m = p->imgs[i];
        const sobel4x5_outputs &o = p->outs[i];
        int32_t Wo, Ho;
        out_dims(m.width, m.height, p->border, &Wo, &Ho);
        jobs[i] = make_job(m.src, m.width, m.height, m.src_pitch, Wo, Ho, o.mag, o.mag_pitch,
                           o.dir_type ? o.dir : nullptr, o.dir_pitch, o.dir_type);
        u8_tile(jobs[i], shape);
        // reflect-101 on an image narrower than 3 columns needs the byte path
        aligned = aligned && u8_rows_aligned(jobs[i]) &&
                  !(p->border == SOBEL4X5_BORDER_REFLECT101 && m.width < 3);
    }
    p->aligned = aligned;
    std::vector<int4> tiles, tail;
    for (int32_t i = 0; i < p->count; ++i) {
        batched_tiles(jobs[i], i, shape.th, shape.tallx, tiles, tail);
        if (tiles.size() + tail.size() > (size_t)INT32_MAX) return fail(SOBEL4X5_EINVAL, "batch too large for one plan");
    }
    const size_t nfirst = tiles.size();
    tiles.insert(tiles.end(), tail.begin(), tail.end());
    if (shape.waves == kStaticGrid) {   // each part from a workgroup boundary (4 tiles)
        xcd_order(tiles, 0, nfirst);
        xcd_order(tiles, std::min(tiles.size(), (nfirst + 3) / 4 * 4), tiles.size());
    }
    p->total = (int32_t)tiles.size();
    hipError_t e;
    if ((e = hipMalloc(&p->d_jobs, sizeof(U8Job) * p->count)) != hipSuccess ||
        (e = hipMalloc(&p->d_tiles, sizeof(int4) * std::max<size_t>(1, tiles.size()))) != hipSuccess ||
        (e = hipMalloc(&p->d_queue, 2 * sizeof(uint32_t))) != hipSuccess) {
        plan_free_device(p);
        return fail(SOBEL4X5_ENOMEM, "hipMalloc for plan tables: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(p->d_jobs, jobs.data(), sizeof(U8Job) * p->count, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemset(p->d_queue, 0, 2 * sizeof(uint32_t))) != hipSuccess) {
        plan_free_device(p);
        return hip_fail(e, "uploading plan tables");
    }
    const int need = (p->total + 3) / 4;   // never more workgroups than work (4 waves each)
    if (shape.waves == kStaticGrid) {       // one wave per tile, no queue
        p->grid = std::max(1, need);
        return ok();
    }
    p->grid = u8_persistent_grid(shape, p->border, p->aligned, p->dir);
    if (p->grid <= 0) {
        plan_free_device(p);
        return fail(SOBEL4X5_EHIP, "could not query occupancy");
    }
    p->grid = std::max(1, std::min(p->grid, need));
    return ok();
}

int plan_direct_launch(sobel4x5_plan_s *p, hipStream_t st, uint32_t *claims = nullptr)
{
    uint32_t *queue = p->shape.waves == kStaticGrid ? nullptr : p->d_queue;
    hipError_t e = launch_u8_batched(p->d_jobs, p->d_tiles, p->total, queue, p->border, p->aligned, p->dir,
                                     p->shape, p->grid, st, claims);
    return e == hipSuccess ? ok() : hip_fail(e, "batched launch");
}

int plan_capture(sobel4x5_plan_s *p)
{
    hipStream_t st;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    int rc = ok();
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        rc = hip_fail(e, "hipStreamBeginCapture");
    } else {
        const int lrc = plan_direct_launch(p, st);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (lrc != SOBEL4X5_OK) {
            rc = lrc;
            if (g) hipGraphDestroy(g);
        } else if (e != hipSuccess) {
            rc = hip_fail(e, "hipStreamEndCapture");
        } else {
            p->graph = g;
            if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess)
                rc = hip_fail(e, "hipGraphInstantiate");
        }
    }
    hipStreamDestroy(st);
    return rc;
}

// Every output plane of image i: (device pointer, pitch, row bytes, rows).
struct Plane {
    void *p;
    int64_t pitch, row_bytes, rows;
};

std::vector<Plane> image_planes(const sobel4x5_plan_s *p, int32_t i)
{
    const sobel4x5_image &m = p->imgs[i];
    const sobel4x5_outputs &o = p->outs[i];
    int32_t Wo, Ho;
    out_dims(m.width, m.height, p->border, &Wo, &Ho);
    std::vector<Plane> v;
    if (o.mag) v.push_back({o.mag, o.mag_pitch, Wo, Ho});
    if (o.dir_type != SOBEL4X5_DIR_NONE) {
        const int64_t es = o.dir_type == SOBEL4X5_DIR_S16 ? 2 : 4;
        for (int k = 0; k < 4; ++k) v.push_back({o.dir[k], o.dir_pitch, Wo * es, Ho});
    }
    return v;
}

// 64-bit fingerprint of every output plane, used by the autotuner to check
// that a candidate shape reproduces the reference bytes: a device kernel sums
// a mix of (row, column, byte) per 16-row block, and the host folds the block
// sums of each plane in order.
int batch_fingerprint(const sobel4x5_plan_s *p, std::vector<uint64_t> &out)
{
    out.clear();
    int64_t most = 1;
    for (int32_t i = 0; i < p->count; ++i)
        for (const Plane &pl : image_planes(p, i)) most = std::max(most, fingerprint_blocks(pl.rows));
    uint64_t *d_part = nullptr;
    hipError_t e = hipMalloc(&d_part, sizeof(uint64_t) * most);
    if (e != hipSuccess) return fail(SOBEL4X5_ENOMEM, "hipMalloc for the autotuner's check: %s", hipGetErrorString(e));
    std::vector<uint64_t> part;
    int rc = ok();
    for (int32_t i = 0; i < p->count && rc == SOBEL4X5_OK; ++i)
        for (const Plane &pl : image_planes(p, i)) {
            const int64_t nb = fingerprint_blocks(pl.rows);
            part.assign(nb, 0);
            if ((e = launch_fingerprint(pl.p, pl.pitch, pl.row_bytes, pl.rows, d_part, nullptr)) != hipSuccess ||
                (e = hipMemcpy(part.data(), d_part, sizeof(uint64_t) * nb, hipMemcpyDeviceToHost)) != hipSuccess) {
                rc = hip_fail(e, "reading outputs for verification");
                break;
            }
            uint64_t h = 1469598103934665603ull;
            for (uint64_t v : part) h = (h ^ v) * 1099511628211ull;
            out.push_back(h);
        }
    hipFree(d_part);
    return rc;
}

double time_plan(sobel4x5_plan_s *p, int reps)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
        hipEventDestroy(a);
        return -1;
    }
    // the best of `reps` rounds of four back-to-back launches (per launch):
    // candidates a few percent apart need more than single launches
    constexpr int kPerRound = 4;
    double best = 1e30;
    for (int r = 0; r < reps && best >= 0; ++r) {
        hipEventRecord(a, nullptr);
        for (int k = 0; k < kPerRound; ++k)
            if (plan_direct_launch(p, nullptr) != SOBEL4X5_OK) {
                best = -1;
                break;
            }
        hipEventRecord(b, nullptr);
        hipEventSynchronize(b);
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        if (best >= 0) best = std::min(best, (double)ms / kPerRound);
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return best;
}

std::string tune_cache_path()
{
    if (const char *e = std::getenv("SOBEL4X5_TUNE_CACHE")) return e;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/sobel4x5_tune.txt";
}

// Hash of the kernel sources the library was built from (set by the build):
// a tuned shape is only as good as the code it was timed and checked with.
#ifndef SOBEL4X5_KERNEL_HASH
#define SOBEL4X5_KERNEL_HASH 0ull
#endif

std::string tune_key(const sobel4x5_plan_s *p)
{
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof prop);
    hipGetDeviceProperties(&prop, p->device);
    // the key describes the workload shape, not the pointers
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    int64_t px = 0;
    for (const auto &m : p->imgs) {
        mix((uint64_t)m.width);
        mix((uint64_t)m.height);
        px += (int64_t)m.width * m.height;
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "v%d|k%016llx|%s|b%d|d%d|n%d|px%lld|h%016llx", SOBEL4X5_VERSION,
                  (unsigned long long)(SOBEL4X5_KERNEL_HASH), prop.gcnArchName, p->border, (int)p->dir, p->count,
                  (long long)px, (unsigned long long)h);
    std::string key = buf;
    for (char &c : key)
        if (c == ' ' || c == '\n') c = '_';
    return key;
}

bool tune_lookup(const std::string &key, U8Shape &s)
{
    FILE *f = std::fopen(tune_cache_path().c_str(), "r");
    if (!f) return false;
    // one entry a line: key ppl th wpg [static [tallx]]; a line without
    // the static field is a persistent grid, one without tallx takes the
    // default split
    char line[1024], k[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int ppl = 0, th = 0, wpg = 0, st = 0, tx = 0;
        const int n = std::sscanf(line, "%511s %d %d %d %d %d", k, &ppl, &th, &wpg, &st, &tx);
        if (n >= 4 && key == k && (ppl == 8 || ppl == 16) && th >= 4 && th <= 256 && wpg == 4 &&
            (st == 0 || st == 1) && tx >= 0 && tx <= 64) {
            s = U8Shape{ppl, th, wpg};
            if (n >= 5 && st == 1) s.waves = kStaticGrid;
            if (n == 6) s.tallx = tx;
            found = true;   // last entry wins
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const std::string &key, const U8Shape &s)
{
    const std::string path = tune_cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) mkdir(path.substr(0, slash).c_str(), 0755);   // best effort
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), s.ppl, s.th, s.wpg, s.waves == kStaticGrid ? 1 : 0, s.tallx);
    std::fclose(f);
}

// Shape of a batched plan without autotuning.
// - Magnitudes only: 8 pixels per lane (the binomial kernel runs three
//   waves per SIMD there; at 16 it needs more registers than two waves per
//   SIMD have), 32-row tiles and the static grid: on 256 mixed images 0.848
//   against 0.970 ms for the persistent grid, whose per-tile ticket, table
//   and job loads run in series before each tile's first row.
// - With directional planes, which are bound by their stores: 8 pixels per
//   lane (the plane stores keep more values live), 4-row tiles and the
//   static grid, one wave per tile, so that many short-lived waves keep the
//   stores in flight: 352 Gpx/s against 299 for the persistent grid with
//   8-row tiles.
// SOBEL4X5_BATCH_PPL (8 or 16), SOBEL4X5_BATCH_TH (4..256) and
// SOBEL4X5_BATCH_STATIC (0 or 1) override it.
U8Shape batch_default_shape(const std::vector<sobel4x5_image> &imgs, bool dir)
{
    (void)imgs;
    U8Shape s{8, dir ? 4 : 32, 4};
    s.waves = kStaticGrid;
    const int ppl = env_int("SOBEL4X5_BATCH_PPL", 0);
    if (ppl == 8 || ppl == 16) s.ppl = ppl;
    const int th = env_int("SOBEL4X5_BATCH_TH", 0);
    if (th >= 4 && th <= 256) s.th = th;
    const int st = env_int("SOBEL4X5_BATCH_STATIC", -1);
    if (st == 0) s.waves = 0;
    if (st == 1) s.waves = kStaticGrid;
    return s;
}

// Clear every output plane, so that a candidate that skips pixels cannot
// reproduce the reference bytes.
void clear_outputs(const sobel4x5_plan_s *p)
{
    for (int32_t i = 0; i < p->count; ++i)
        for (const Plane &pl : image_planes(p, i)) hipMemset2D(pl.p, pl.pitch, 0xA5, pl.row_bytes, pl.rows);
}

// Run shape c once on cleared outputs; true when its bytes equal `want`.
bool candidate_matches(sobel4x5_plan_s *p, const U8Shape &c, const std::vector<uint64_t> &want, int *rc)
{
    *rc = SOBEL4X5_OK;
    if (plan_setup(p, c) != SOBEL4X5_OK) return false;
    clear_outputs(p);
    if (plan_direct_launch(p, nullptr) != SOBEL4X5_OK) return false;
    if (hipDeviceSynchronize() != hipSuccess) {
        *rc = fail(SOBEL4X5_EHIP, "autotune candidate run failed");
        return false;
    }
    std::vector<uint64_t> got;
    return batch_fingerprint(p, got) == SOBEL4X5_OK && got == want;   // never trust a mismatch
}

int plan_autotune(sobel4x5_plan_s *p)
{
    const std::string key = tune_key(p);

    // reference bytes with the default shape
    const U8Shape ref = batch_default_shape(p->imgs, p->dir);
    if (int rc = plan_setup(p, ref)) return rc;
    if (int rc = plan_direct_launch(p, nullptr)) return rc;
    if (hipError_t e = hipDeviceSynchronize(); e != hipSuccess) return hip_fail(e, "autotune reference run");
    std::vector<uint64_t> want;
    if (int rc = batch_fingerprint(p, want)) return rc;

    // a cached shape is used only after it has reproduced the reference
    // bytes once on these images
    U8Shape cached;
    if (tune_lookup(key, cached)) {
        int rc;
        if (candidate_matches(p, cached, want, &rc)) return ok();
        if (rc != SOBEL4X5_OK) return rc;
        if (int rc2 = plan_setup(p, ref)) return rc2;
    }

    U8Shape best = ref;
    double best_ms = time_plan(p, 10);
    const int ppls[] = {8, 16};
    const int ths[] = {8, 16, 32, 64, 128};
    for (int grid_form = 0; grid_form < 2; ++grid_form)   // persistent, static
        for (int ppl : ppls)
            for (int th : ths) {
                U8Shape c{ppl, th, 4};
                if (grid_form == 1) c.waves = kStaticGrid;
                if (c.ppl == ref.ppl && c.th == ref.th && c.waves == ref.waves) continue;
                int rc;
                if (!candidate_matches(p, c, want, &rc)) {
                    if (rc != SOBEL4X5_OK) return rc;
                    continue;
                }
                const double ms = time_plan(p, 10);
                if (ms > 0 && ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    // then the height of the tall chunks around the best shape (the default
    // split takes 2 tile heights)
    for (int tx : {1, 4}) {
        U8Shape c = best;
        c.tallx = tx;
        int rc;
        if (!candidate_matches(p, c, want, &rc)) {
            if (rc != SOBEL4X5_OK) return rc;
            continue;
        }
        const double ms = time_plan(p, 10);
        if (ms > 0 && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    tune_store(key, best);
    return plan_setup(p, best);
}

// --------------------------------------------------------- one-shot cache

struct CachedPlan {
    std::string key;
    sobel4x5_plan plan;
    hipStream_t stream;   // the only stream this plan is launched on
};

struct PlanCache {
    std::mutex mu;
    std::vector<CachedPlan> lru;   // most recent last
};

PlanCache &plan_cache()
{
    static PlanCache *c = new PlanCache();   // intentionally leaked: plans live to process end
    return *c;
}

// Key of a one-shot batched call, from the descriptor fields one by one (not
// the structs' raw bytes, whose padding a C caller may leave uninitialised),
// the border, the device and the stream.  A plan's work queue admits one
// launch at a time, so every stream gets plans of its own; launches of one
// plan on one stream run in order.
std::string batch_key(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count, int32_t border,
                      int device, hipStream_t stream)
{
    std::string k;
    auto put = [&](uint64_t v) { k.append(reinterpret_cast<const char *>(&v), sizeof v); };
    put((uint64_t)(uint32_t)count);
    put((uint64_t)(uint32_t)border);
    put((uint64_t)(uint32_t)device);
    put((uint64_t)reinterpret_cast<uintptr_t>(stream));
    put(outs ? 1u : 0u);
    for (int32_t i = 0; i < count; ++i) {
        const sobel4x5_image &m = imgs[i];
        put((uint64_t)reinterpret_cast<uintptr_t>(m.src));
        put(((uint64_t)(uint32_t)m.width << 32) | (uint32_t)m.height);
        put((uint64_t)m.src_pitch);
        if (outs) {
            const sobel4x5_outputs &o = outs[i];
            put((uint64_t)reinterpret_cast<uintptr_t>(o.mag));
            put((uint64_t)o.mag_pitch);
            put((uint64_t)(uint32_t)o.dir_type);
            if (o.dir_type != SOBEL4X5_DIR_NONE) {
                for (int d = 0; d < 4; ++d) put((uint64_t)reinterpret_cast<uintptr_t>(o.dir[d]));
                put((uint64_t)o.dir_pitch);
            }
        } else {
            put((uint64_t)reinterpret_cast<uintptr_t>(m.mag));
            put((uint64_t)m.mag_pitch);
        }
    }
    return k;
}


// ------------------------------------------------------- host pipeline

// One in-flight image of a pipeline: device buffers (sized for the largest
// image), pinned staging buffers for callers whose host memory is pageable,
// and a stream of its own (default priority).
struct PipeSlot {
    hipStream_t st = nullptr;
    uint8_t *d_src = nullptr, *d_mag = nullptr;
    uint8_t *h_src = nullptr, *h_mag = nullptr;   // pinned staging
    int64_t pitch = 0;                            // device and staging row pitch
    int pending = -1;                             // image whose magnitudes are in flight
    bool staged_out = false;                      // D2H went to h_mag (copy on finish)
};

// true when p points to pinned (page-locked) host memory
bool is_pinned(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // pageable memory is not an error here
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

}  // namespace

struct sobel4x5_pipe_s {
    int32_t max_w = 0, max_h = 0;
    std::vector<PipeSlot> slots;
};

namespace {

void pipe_free(sobel4x5_pipe_s *p)
{
    for (auto &s : p->slots) {
        if (s.st) hipStreamSynchronize(s.st);
        if (s.d_src) hipFree(s.d_src);
        if (s.d_mag) hipFree(s.d_mag);
        if (s.h_src) hipHostFree(s.h_src);
        if (s.h_mag) hipHostFree(s.h_mag);
        if (s.st) hipStreamDestroy(s.st);
        s = PipeSlot{};
    }
}

// Copy the magnitudes of the slot's finished image out of pinned staging.
void pipe_finish(PipeSlot &s, const sobel4x5_image *imgs, int32_t border)
{
    if (s.pending < 0) return;
    if (s.staged_out) {
        const sobel4x5_image &m = imgs[s.pending];
        int32_t Wo, Ho;
        out_dims(m.width, m.height, border, &Wo, &Ho);
        for (int32_t r = 0; r < Ho; ++r) std::memcpy(m.mag + r * m.mag_pitch, s.h_mag + r * s.pitch, (size_t)Wo);
    }
    s.pending = -1;
    s.staged_out = false;
}

}  // namespace

extern "C" {

const char *sobel4x5_status_string(int status)
{
    switch (status) {
    case SOBEL4X5_OK: return "ok";
    case SOBEL4X5_EINVAL: return "invalid argument";
    case SOBEL4X5_EUNSUPPORTED: return "unsupported request";
    case SOBEL4X5_EHIP: return "HIP runtime error";
    case SOBEL4X5_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char *sobel4x5_last_error(void) { return g_last_error.c_str(); }

int sobel4x5_version(void) { return SOBEL4X5_VERSION; }

int sobel4x5_validate_u8(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t border,
                         const sobel4x5_outputs *out)
{
    int32_t Wo, Ho;
    return validate_u8(src, width, height, src_pitch, border, out, &Wo, &Ho);
}

int sobel4x5_u8(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t border,
                const sobel4x5_outputs *out, void *stream)
{
    int32_t Wo, Ho;
    if (int rc = validate_u8(src, width, height, src_pitch, border, out, &Wo, &Ho)) return rc;
    U8Job j = make_job(src, width, height, src_pitch, Wo, Ho, out->mag, out->mag_pitch,
                       out->dir_type ? out->dir : nullptr, out->dir_pitch, out->dir_type);
    const U8Shape s = default_shape(Wo, Ho, out->dir_type);
    u8_tile(j, s);
    if (out->dir_type == SOBEL4X5_DIR_NONE && out->mag && env_int("SOBEL4X5_U8_MFMA", 0) == 1) {
        hipError_t e = guard(launch_u8_mfma(j, border, env_int("SOBEL4X5_U8_WAVES", 0), static_cast<hipStream_t>(stream)));
        return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_u8 launch");
    }
    hipError_t e = guard(launch_u8_single(j, border, s, static_cast<hipStream_t>(stream)));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_u8 launch");
}

int sobel4x5_validate_u8_op(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t op,
                            int32_t border, const sobel4x5_outputs *out)
{
    int32_t Wo, Ho;
    return validate_u8(src, width, height, src_pitch, border, out, &Wo, &Ho, op);
}

int sobel4x5_u8_op(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t op,
                   int32_t border, const sobel4x5_outputs *out, void *stream)
{
    int32_t Wo, Ho;
    if (int rc = validate_u8(src, width, height, src_pitch, border, out, &Wo, &Ho, op)) return rc;
    if (op == SOBEL4X5_OP_4DIR_5X5) return sobel4x5_u8(src, width, height, src_pitch, border, out, stream);
    void *dirs[4] = {nullptr, nullptr, nullptr, nullptr};
    if (out->dir_type) {
        dirs[0] = out->dir[0];
        dirs[2] = out->dir[2];
    }
    U8Job j = make_job(src, width, height, src_pitch, Wo, Ho, out->mag, out->mag_pitch,
                       out->dir_type ? dirs : nullptr, out->dir_pitch, out->dir_type);
    U8Shape s = default_shape(Wo, Ho, out->dir_type, op);
    u8_tile(j, s);
    // The two-directional operators are lighter on arithmetic, so the 4-row
    // prologue each wave re-reads weighs more: on large images they take
    // 32-row ranges as long as one round of resident waves (8 per CU)
    // remains (8192^2 3x3: 2128 -> 2232 Gpx/s).
    if (out->dir_type == SOBEL4X5_DIR_NONE && env_int("SOBEL4X5_U8_MIN_ROWS", 0) == 0 &&
        (int64_t)((j.ntx + 3) / 4) * (Ho / 32) >= 8 * (int64_t)device_cus())
        s.min_rows = 32;
    hipError_t e = launch_u8_2dir(j, op, border, s, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_u8_op launch");
}

int sobel4x5_validate_batch(const sobel4x5_image *imgs, int32_t count, int32_t border)
{
    return validate_batch(imgs, nullptr, count, border);
}

int sobel4x5_validate_batch_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count,
                               int32_t border)
{
    return validate_batch(imgs, outs, count, border);
}

int sobel4x5_plan_create_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count, int32_t border,
                            uint32_t flags, sobel4x5_plan *out)
{
    if (!out) return fail(SOBEL4X5_EINVAL, "out is NULL");
    *out = nullptr;
    if (int rc = validate_batch(imgs, outs, count, border)) return rc;
    if (flags & ~(SOBEL4X5_PLAN_AUTOTUNE | SOBEL4X5_PLAN_NO_GRAPH))
        return fail(SOBEL4X5_EINVAL, "unknown plan flags 0x%x", flags);
    auto *p = new (std::nothrow) sobel4x5_plan_s();
    if (!p) return fail(SOBEL4X5_ENOMEM, "plan allocation");
    p->count = count;
    p->border = border;
    p->use_graph = !(flags & SOBEL4X5_PLAN_NO_GRAPH);
    p->imgs.assign(imgs, imgs + count);
    p->outs.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        p->outs[i] = batch_outputs(imgs, outs, i);
        p->dir = p->dir || p->outs[i].dir_type != SOBEL4X5_DIR_NONE;
    }
    hipGetDevice(&p->device);
    int rc = (flags & SOBEL4X5_PLAN_AUTOTUNE) ? plan_autotune(p) : plan_setup(p, batch_default_shape(p->imgs, p->dir));
    if (rc == SOBEL4X5_OK && p->use_graph) rc = plan_capture(p);
    if (rc != SOBEL4X5_OK) {
        plan_free_device(p);
        p->magic = 0;
        delete p;
        return rc;
    }
    *out = p;
    return ok();
}

int sobel4x5_plan_create(const sobel4x5_image *imgs, int32_t count, int32_t border, uint32_t flags,
                         sobel4x5_plan *out)
{
    return sobel4x5_plan_create_ex(imgs, nullptr, count, border, flags, out);
}

int sobel4x5_plan_launch(sobel4x5_plan plan, void *stream)
{
    if (!plan || plan->magic != kPlanMagic) return fail(SOBEL4X5_EINVAL, "invalid plan handle");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->use_graph) {
        hipError_t e = guard(hipGraphLaunch(plan->exec, st));
        return e == hipSuccess ? ok() : hip_fail(e, "hipGraphLaunch");
    }
    return plan_direct_launch(plan, st);
}

int sobel4x5_debug_plan_claims(sobel4x5_plan plan, uint32_t *claims, int64_t capacity, int64_t *ntiles, void *stream)
{
    if (!plan || plan->magic != kPlanMagic) return fail(SOBEL4X5_EINVAL, "invalid plan handle");
    if (!ntiles) return fail(SOBEL4X5_EINVAL, "ntiles is NULL");
    *ntiles = plan->total;
    if (!claims) return ok();
    if (capacity < plan->total)
        return fail(SOBEL4X5_EINVAL, "claims holds %lld counters, the plan has %d tiles", (long long)capacity,
                    plan->total);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = guard(hipMemsetAsync(claims, 0, sizeof(uint32_t) * (size_t)std::max<int32_t>(plan->total, 1), st));
    if (e != hipSuccess) return hip_fail(e, "clearing the claim counters");
    return plan_direct_launch(plan, st, claims);
}

int sobel4x5_plan_info(sobel4x5_plan plan, int32_t *px_per_lane, int32_t *rows_per_tile, int32_t *waves_per_group,
                       int32_t *grid)
{
    if (!plan || plan->magic != kPlanMagic) return fail(SOBEL4X5_EINVAL, "invalid plan handle");
    if (px_per_lane) *px_per_lane = plan->shape.ppl;
    if (rows_per_tile) *rows_per_tile = plan->shape.th;
    if (waves_per_group) *waves_per_group = plan->shape.wpg;
    if (grid) *grid = plan->grid;
    return ok();
}

int sobel4x5_plan_destroy(sobel4x5_plan plan)
{
    if (!plan || plan->magic != kPlanMagic) return fail(SOBEL4X5_EINVAL, "invalid plan handle");
    plan_free_device(plan);
    plan->magic = 0;
    delete plan;
    return ok();
}

int sobel4x5_batched_ex(const sobel4x5_image *imgs, const sobel4x5_outputs *outs, int32_t count, int32_t border,
                        void *stream)
{
    if (int rc = validate_batch(imgs, outs, count, border)) return rc;
    int dev = 0;
    hipGetDevice(&dev);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const std::string key = batch_key(imgs, outs, count, border, dev, st);
    // Lookups, launches and evictions all hold the cache lock, so a plan is
    // never destroyed between another thread's lookup and its launch.
    PlanCache &c = plan_cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (size_t i = 0; i < c.lru.size(); ++i)
            if (c.lru[i].key == key) {
                CachedPlan e = c.lru[i];
                c.lru.erase(c.lru.begin() + i);
                c.lru.push_back(e);
                return sobel4x5_plan_launch(e.plan, stream);
            }
    }
    sobel4x5_plan plan = nullptr;
    if (int rc = sobel4x5_plan_create_ex(imgs, outs, count, border, 0, &plan)) return rc;
    std::lock_guard<std::mutex> lk(c.mu);
    c.lru.push_back(CachedPlan{key, plan, st});
    if (c.lru.size() > 8) {
        const CachedPlan evicted = c.lru.front();
        c.lru.erase(c.lru.begin());
        (void)hipStreamSynchronize(evicted.stream);   // it may still be running there
        sobel4x5_plan_destroy(evicted.plan);
    }
    return sobel4x5_plan_launch(plan, stream);
}

int sobel4x5_batched(const sobel4x5_image *imgs, int32_t count, int32_t border, void *stream)
{
    return sobel4x5_batched_ex(imgs, nullptr, count, border, stream);
}

static_assert(SOBEL4X5_NOALLOC_MAX_IMAGES == kNoallocMaxImages && SOBEL4X5_NOALLOC_MAX_TILES == kNoallocMaxTiles,
              "public limits of the allocation-free batched call");

int sobel4x5_batched_noalloc(const sobel4x5_image *imgs, int32_t count, int32_t border, void *stream)
{
    if (int rc = validate_batch(imgs, nullptr, count, border)) return rc;
    if (count > kNoallocMaxImages)
        return fail(SOBEL4X5_EINVAL, "%d images: the allocation-free call takes at most %d", count,
                    kNoallocMaxImages);
    // Tables built on the host in fixed static buffers (no allocation, host
    // or device), then copied into the fixed device buffer on `stream`.  The
    // lock covers the building and both copies: a copy from pageable memory
    // has read its source when hipMemcpyAsync returns.
    static std::mutex mu;
    static unsigned char stage[kNoallocBytes];     // queue words, jobs, tiles: the device layout
    static int4 tail[kNoallocMaxTiles];            // short chunks, queued after every other tile
    std::lock_guard<std::mutex> lk(mu);
    const std::vector<sobel4x5_image> none;
    const U8Shape shape = batch_default_shape(none, false);
    std::memset(stage, 0, kNoallocJobsOff);   // queue words start at zero
    int4 *first = reinterpret_cast<int4 *>(stage + kNoallocTilesOff);
    int32_t nfirst = 0, ntail = 0;
    bool over = false;
    bool aligned = true;
    for (int32_t i = 0; i < count && !over; ++i) {
        const sobel4x5_image &m = imgs[i];
        int32_t Wo, Ho;
        out_dims(m.width, m.height, border, &Wo, &Ho);
        U8Job j = make_job(m.src, m.width, m.height, m.src_pitch, Wo, Ho, m.mag, m.mag_pitch, nullptr, 0, 0);
        u8_tile(j, shape);
        aligned = aligned && u8_rows_aligned(j) && !(border == SOBEL4X5_BORDER_REFLECT101 && m.width < 3);
        std::memcpy(stage + kNoallocJobsOff + sizeof(U8Job) * i, &j, sizeof(U8Job));
        batched_tiles_each(
            j, i, shape.th, shape.tallx,
            [&](int4 t) {
                if (nfirst + ntail < kNoallocMaxTiles) first[nfirst++] = t; else over = true;
            },
            [&](int4 t) {
                if (nfirst + ntail < kNoallocMaxTiles) tail[ntail++] = t; else over = true;
            });
    }
    if (over)
        return fail(SOBEL4X5_EINVAL, "the batch needs more than %d wave-tiles, the allocation-free call's limit",
                    kNoallocMaxTiles);
    const int32_t total = nfirst + ntail;
    std::memcpy(first + nfirst, tail, sizeof(int4) * ntail);
    void *scr = nullptr;
    hipError_t e = guard(noalloc_scratch(&scr));
    if (e != hipSuccess) return hip_fail(e, "looking up the fixed device buffer");
    unsigned char *base = static_cast<unsigned char *>(scr);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // queue words and the count jobs, then the total tiles
    if ((e = guard(hipMemcpyAsync(base, stage, kNoallocJobsOff + sizeof(U8Job) * count, hipMemcpyHostToDevice,
                                  st))) != hipSuccess ||
        (e = guard(hipMemcpyAsync(base + kNoallocTilesOff, stage + kNoallocTilesOff, sizeof(int4) * total,
                                  hipMemcpyHostToDevice, st))) != hipSuccess)
        return hip_fail(e, "copying the batch tables");
    // the default shape's grid form: one wave per tile, or a persistent grid
    // on the queue words
    const int need = (total + 3) / 4;
    int grid = std::max(1, need);
    uint32_t *queue = nullptr;
    if (shape.waves != kStaticGrid) {
        grid = u8_persistent_grid(shape, border, aligned, false);
        if (grid <= 0) return fail(SOBEL4X5_EHIP, "could not query occupancy");
        grid = std::max(1, std::min(grid, need));
        queue = reinterpret_cast<uint32_t *>(base);
    }
    e = guard(launch_u8_batched(reinterpret_cast<const U8Job *>(base + kNoallocJobsOff),
                                reinterpret_cast<const int4 *>(base + kNoallocTilesOff), total, queue, border,
                                aligned, false, shape, grid, st));
    return e == hipSuccess ? ok() : hip_fail(e, "batched launch");
}

int sobel4x5_validate_f32(const float *src, int32_t batch, int32_t width, int32_t height, int64_t src_pitch,
                          int64_t src_bstride, int32_t border, const float *out, int64_t out_pitch,
                          int64_t out_bstride)
{
    int32_t Wo, Ho;
    if (int rc = out_dims(width, height, border, &Wo, &Ho)) return rc;
    if (batch < 0) return fail(SOBEL4X5_EINVAL, "batch must be >= 0");
    Range rs, ro;
    if (int rc = check_f32_buf("src", src, batch, width, height, src_pitch, src_bstride, &rs)) return rc;
    if (int rc = check_f32_buf("output", out, batch, Wo, Ho, out_pitch, out_bstride, &ro)) return rc;
    if (batch > 0 && overlap(rs, ro)) return fail(SOBEL4X5_EINVAL, "output overlaps src");
    return ok();
}

int sobel4x5_f32_fwd(const float *src, int32_t batch, int32_t width, int32_t height, int64_t src_pitch,
                     int64_t src_bstride, int32_t border, float *mag, int64_t mag_pitch, int64_t mag_bstride,
                     void *stream)
{
    if (int rc = sobel4x5_validate_f32(src, batch, width, height, src_pitch, src_bstride, border, mag, mag_pitch,
                                       mag_bstride))
        return rc;
    F32Args a{};
    a.src = src;
    a.src_pitch = src_pitch;
    a.src_bstride = src_bstride;
    a.out = mag;
    a.out_pitch = mag_pitch;
    a.out_bstride = mag_bstride;
    a.B = batch;
    a.W = width;
    a.H = height;
    out_dims(width, height, border, &a.Wo, &a.Ho);
    a.off = border == SOBEL4X5_BORDER_VALID ? 2 : 0;
    a.bmode = f32_bmode(border);
    hipError_t e = launch_f32_fwd(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_f32_fwd launch");
}

int sobel4x5_f32_bwd(const float *src, int64_t src_pitch, int64_t src_bstride, const float *grad_mag,
                     int64_t g_pitch, int64_t g_bstride, int32_t batch, int32_t width, int32_t height,
                     int32_t border, float *grad_src, int64_t gs_pitch, int64_t gs_bstride, void *stream)
{
    int32_t Wo, Ho;
    if (int rc = out_dims(width, height, border, &Wo, &Ho)) return rc;
    if (batch < 0) return fail(SOBEL4X5_EINVAL, "batch must be >= 0");
    Range rs, rg, rd;
    if (int rc = check_f32_buf("src", src, batch, width, height, src_pitch, src_bstride, &rs)) return rc;
    if (int rc = check_f32_buf("grad_mag", grad_mag, batch, Wo, Ho, g_pitch, g_bstride, &rg)) return rc;
    if (int rc = check_f32_buf("grad_src", grad_src, batch, width, height, gs_pitch, gs_bstride, &rd)) return rc;
    if (batch > 0 && (overlap(rd, rs) || overlap(rd, rg)))
        return fail(SOBEL4X5_EINVAL, "grad_src overlaps src or grad_mag");
    F32Args a{};
    a.src = src;
    a.src_pitch = src_pitch;
    a.src_bstride = src_bstride;
    a.grad = grad_mag;
    a.g_pitch = g_pitch;
    a.g_bstride = g_bstride;
    a.out = grad_src;
    a.out_pitch = gs_pitch;
    a.out_bstride = gs_bstride;
    a.B = batch;
    a.W = width;
    a.H = height;
    a.Wo = Wo;
    a.Ho = Ho;
    a.off = border == SOBEL4X5_BORDER_VALID ? 2 : 0;
    a.bmode = f32_bmode(border);
    hipError_t e = launch_f32_bwd(a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_f32_bwd launch");
}

int sobel4x5_validate_weights(const int32_t *w, int32_t dir_type)
{
    if (!w) return fail(SOBEL4X5_EINVAL, "weights is NULL");
    const int64_t limit = dir_type == SOBEL4X5_DIR_S16 ? 128 : 32768;
    for (int k = 0; k < 4; ++k) {
        const int32_t *K = w + 25 * k;
        int64_t sum = 0;
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) {
                if ((int64_t)K[5 * i + j] != -(int64_t)K[5 * (4 - i) + (4 - j)])
                    return fail(SOBEL4X5_EINVAL,
                                "kernel %d is not antisymmetric under a half turn at tap (%d, %d)", k, i, j);
                sum += K[5 * i + j] < 0 ? -(int64_t)K[5 * i + j] : K[5 * i + j];
            }
        if (sum > limit)
            return fail(SOBEL4X5_EINVAL, "kernel %d: sum of |weights| = %lld exceeds %lld%s", k, (long long)sum,
                        (long long)limit, dir_type == SOBEL4X5_DIR_S16 ? " (int16 planes)" : "");
    }
    return ok();
}

int sobel4x5_family_weights(int32_t a, int32_t ab, int32_t an, int32_t am, int32_t anb, int32_t amb,
                            int32_t *out)
{
    if (!out) return fail(SOBEL4X5_EINVAL, "weights_out is NULL");
    if (a <= 0 || ab <= 0 || an <= 0 || am <= 0 || anb <= 0 || amb <= 0)
        return fail(SOBEL4X5_EINVAL, "the six family weights must be positive");
    if ((int64_t)an * ab != (int64_t)a * anb || (int64_t)am * ab != (int64_t)a * amb)
        return fail(SOBEL4X5_EINVAL, "inconsistent family weights: need (a*n)(a*b) = a(a*n*b), (a*m)(a*b) = a(a*m*b)");
    // K_x = a [1 n m n 1]^T x [-1 -b 0 b 1]; K_y its transpose
    const int32_t col[5] = {a, an, am, an, a};          // a * [1 n m n 1]
    const int32_t colb[5] = {ab, anb, amb, anb, ab};    // a * b * [1 n m n 1]
    int32_t Kx[5][5], Kd[5][5];
    for (int i = 0; i < 5; ++i) {
        Kx[i][0] = -col[i];
        Kx[i][1] = -colb[i];
        Kx[i][2] = 0;
        Kx[i][3] = colb[i];
        Kx[i][4] = col[i];
    }
    // K_d as printed in Eq. (sobel5_param)
    const int32_t d[5][5] = {{-am, -an, -a, -ab, 0},
                             {-an, -amb, -anb, 0, ab},
                             {-a, -anb, 0, anb, a},
                             {-ab, 0, anb, amb, an},
                             {0, ab, a, an, am}};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Kd[i][j] = d[i][j];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            out[0 * 25 + 5 * i + j] = Kx[i][j];           // 0 deg
            out[1 * 25 + 5 * i + j] = Kd[i][j];           // 45 deg
            out[2 * 25 + 5 * i + j] = Kx[j][i];           // 90 deg: transpose
            out[3 * 25 + 5 * i + j] = Kd[i][4 - j];       // 135 deg: left-right mirror
        }
    return ok();
}

int sobel4x5_u8_weighted(const uint8_t *src, int32_t width, int32_t height, int64_t src_pitch, int32_t border,
                         const int32_t *weights, const sobel4x5_outputs *out, void *stream)
{
    int32_t Wo, Ho;
    if (int rc = validate_u8(src, width, height, src_pitch, border, out, &Wo, &Ho)) return rc;
    if (int rc = sobel4x5_validate_weights(weights, out->dir_type)) return rc;
    // magnitudes alone with weights that fit int8 (the family K(a, b, n, m)
    // with small weights, Eq. (sobel5_1) among them): the matrix-core form
    if (out->dir_type == SOBEL4X5_DIR_NONE && out->mag && env_int("SOBEL4X5_W_MFMA", 1) == 1 &&
        mfma_weights_fit(weights)) {
        const U8Job mj = make_job(src, width, height, src_pitch, Wo, Ho, out->mag, out->mag_pitch, nullptr, 0,
                                  SOBEL4X5_DIR_NONE);
        hipError_t e = guard(launch_u8_mfma_weighted(mj, border, weights, env_int("SOBEL4X5_U8_WAVES", 0),
                                                     static_cast<hipStream_t>(stream)));
        return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_u8_weighted launch");
    }
    WJob j{};
    j.src = src;
    j.mag = out->mag;
    for (int k = 0; k < 4; ++k) j.dir[k] = out->dir_type ? out->dir[k] : nullptr;
    j.src_pitch = src_pitch;
    j.mag_pitch = out->mag_pitch;
    j.dir_pitch = out->dir_pitch;
    j.W = width;
    j.H = height;
    j.Wo = Wo;
    j.Ho = Ho;
    j.off = border == SOBEL4X5_BORDER_VALID ? 2 : 0;
    j.bmode = border == SOBEL4X5_BORDER_ZERO ? 1 : (border == SOBEL4X5_BORDER_REFLECT101 ? 2 : 0);
    j.dir_type = out->dir_type;
    // upper-half taps (0, 0..4), (1, 0..4), (2, 0), (2, 1)
    for (int k = 0; k < 4; ++k)
        for (int t = 0; t < 12; ++t) {
            const int i = t < 5 ? 0 : (t < 10 ? 1 : 2), jj = t < 10 ? t % 5 : t - 10;
            j.coef[k][t] = weights[25 * k + 5 * i + jj];
        }
    hipError_t e = launch_u8_weighted(j, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_u8_weighted launch");
}

int sobel4x5_debug_inject_failure(int32_t nth_call)
{
    if (nth_call < 0) return fail(SOBEL4X5_EINVAL, "nth_call must be >= 0");
    g_inject.store(nth_call, std::memory_order_relaxed);
    return ok();
}

int sobel4x5_debug_copy(const void *src, void *dst, int64_t nbytes, void *stream)
{
    if (nbytes < 0 || (nbytes % 16) || (nbytes > 0 && (!src || !dst)) ||
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u))
        return fail(SOBEL4X5_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    hipError_t e = launch_copy16(src, dst, nbytes / 16, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_debug_copy launch");
}

int sobel4x5_debug_round_mag_ex(const int32_t *S, uint8_t *out, int64_t n, int32_t method, void *stream)
{
    if (n < 0 || (n > 0 && (!S || !out))) return fail(SOBEL4X5_EINVAL, "bad arguments");
    if (method != 0 && method != 1) return fail(SOBEL4X5_EINVAL, "method must be 0 or 1, got %d", method);
    hipError_t e = launch_round_mag(S, out, n, method, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_debug_round_mag launch");
}

int sobel4x5_debug_round_mag(const int32_t *S, uint8_t *out, int64_t n, void *stream)
{
    return sobel4x5_debug_round_mag_ex(S, out, n, 0, stream);
}

int sobel4x5_debug_round_quad(const int16_t *q, uint8_t *out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!q || !out))) return fail(SOBEL4X5_EINVAL, "bad arguments");
    if (n > (INT64_MAX / 8)) return fail(SOBEL4X5_EINVAL, "n too large");
    hipError_t e = launch_round_quad(q, out, n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "sobel4x5_debug_round_quad launch");
}

int sobel4x5_pipe_create(int32_t max_width, int32_t max_height, int32_t depth, sobel4x5_pipe *out)
{
    if (!out) return fail(SOBEL4X5_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_width < 1 || max_height < 1) return fail(SOBEL4X5_EINVAL, "max sizes must be >= 1");
    if (depth < 1 || depth > 16) return fail(SOBEL4X5_EINVAL, "depth must be in [1, 16], got %d", depth);
    auto *p = new (std::nothrow) sobel4x5_pipe_s;
    if (!p) return fail(SOBEL4X5_ENOMEM, "host allocation failed");
    p->max_w = max_width;
    p->max_h = max_height;
    p->slots.resize(depth);
    const int64_t pitch = (max_width + 255) / 256 * 256;
    const size_t bytes = (size_t)pitch * (size_t)max_height;
    for (auto &sl : p->slots) {
        sl.pitch = pitch;
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipMalloc(&sl.d_src, bytes)) != hipSuccess || (e = hipMalloc(&sl.d_mag, bytes)) != hipSuccess ||
            (e = hipHostMalloc(&sl.h_src, bytes, hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(&sl.h_mag, bytes, hipHostMallocDefault)) != hipSuccess) {
            pipe_free(p);
            delete p;
            return fail(SOBEL4X5_ENOMEM, "pipeline allocation failed: %s", hipGetErrorString(e));
        }
    }
    *out = p;
    return ok();
}

int sobel4x5_pipe_run(sobel4x5_pipe p, const sobel4x5_image *imgs, int32_t count, int32_t border)
{
    if (!p) return fail(SOBEL4X5_EINVAL, "pipe is NULL");
    if (count < 0 || (count > 0 && !imgs)) return fail(SOBEL4X5_EINVAL, "bad image array");
    for (int32_t i = 0; i < count; ++i) {
        const sobel4x5_image &m = imgs[i];
        int32_t Wo, Ho;
        if (int rc = out_dims(m.width, m.height, border, &Wo, &Ho)) return rc;
        if (!m.src || !m.mag) return fail(SOBEL4X5_EINVAL, "image %d: NULL pointer", i);
        if (m.width > p->max_w || m.height > p->max_h)
            return fail(SOBEL4X5_EINVAL, "image %d (%d x %d) exceeds the pipeline's %d x %d", i, m.width, m.height,
                        p->max_w, p->max_h);
        if (int rc = check_pitch("src", m.src_pitch, m.width, m.height)) return rc;
        if (int rc = check_pitch("mag", m.mag_pitch, Wo, Ho)) return rc;
    }
    const int depth = (int)p->slots.size();
    // A slot's `pending` indexes THIS call's image array.  Every return path
    // leaves every slot idle: on an error, wait for whatever the slots still
    // have queued (a copy into a caller's pinned buffer must not land after
    // the return) and drop the pending images without copying them out, so
    // that a later call, with another array, never finishes an image of
    // this one.
    auto abandon = [&](int rc) {
        for (auto &sl : p->slots) {
            if (sl.st) (void)hipStreamSynchronize(sl.st);
            sl.pending = -1;
            sl.staged_out = false;
        }
        return rc;
    };
    for (auto &sl : p->slots)   // idle after every earlier call; keep it so
        if (sl.pending >= 0) abandon(SOBEL4X5_OK);
    auto drain = [&](PipeSlot &sl) -> hipError_t {
        if (sl.pending < 0) return hipSuccess;
        hipError_t e = guard(hipStreamSynchronize(sl.st));
        if (e == hipSuccess) pipe_finish(sl, imgs, border);
        return e;
    };
    for (int32_t i = 0; i < count; ++i) {
        PipeSlot &sl = p->slots[i % depth];
        if (hipError_t e = drain(sl); e != hipSuccess) return abandon(hip_fail(e, "pipeline wait"));
        const sobel4x5_image &m = imgs[i];
        int32_t Wo, Ho;
        out_dims(m.width, m.height, border, &Wo, &Ho);
        // host to device (pageable sources go through the slot's pinned
        // staging buffer, so that the copy itself is asynchronous)
        const uint8_t *hs = m.src;
        int64_t hp = m.src_pitch;
        if (!is_pinned(m.src)) {
            for (int32_t r = 0; r < m.height; ++r)
                std::memcpy(sl.h_src + r * sl.pitch, m.src + r * m.src_pitch, (size_t)m.width);
            hs = sl.h_src;
            hp = sl.pitch;
        }
        // the slot owns image i from its first enqueued operation on
        sl.pending = i;
        sl.staged_out = false;
        hipError_t e = guard(
            hipMemcpy2DAsync(sl.d_src, sl.pitch, hs, hp, m.width, m.height, hipMemcpyHostToDevice, sl.st));
        if (e != hipSuccess) return abandon(hip_fail(e, "pipeline host-to-device copy"));
        U8Job j = make_job(sl.d_src, m.width, m.height, sl.pitch, Wo, Ho, sl.d_mag, sl.pitch, nullptr, 0, 0);
        const U8Shape shape = default_shape(Wo, Ho, SOBEL4X5_DIR_NONE);
        u8_tile(j, shape);
        if ((e = guard(launch_u8_single(j, border, shape, sl.st))) != hipSuccess)
            return abandon(hip_fail(e, "pipeline launch"));
        sl.staged_out = !is_pinned(m.mag);
        e = guard(hipMemcpy2DAsync(sl.staged_out ? sl.h_mag : m.mag, sl.staged_out ? sl.pitch : m.mag_pitch,
                                   sl.d_mag, sl.pitch, Wo, Ho, hipMemcpyDeviceToHost, sl.st));
        if (e != hipSuccess) return abandon(hip_fail(e, "pipeline device-to-host copy"));
    }
    for (auto &sl : p->slots)
        if (hipError_t e = drain(sl); e != hipSuccess) return abandon(hip_fail(e, "pipeline wait"));
    return ok();
}

int sobel4x5_pipe_destroy(sobel4x5_pipe p)
{
    if (!p) return fail(SOBEL4X5_EINVAL, "pipe is NULL");
    pipe_free(p);
    delete p;
    return ok();
}

}  // extern "C"
