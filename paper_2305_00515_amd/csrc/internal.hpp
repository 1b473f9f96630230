// Internal declarations shared by the C-ABI layer (sobel4x5_api.cpp) and the
// HIP kernel translation units.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace s4x5 {

// One uint8 image as the kernels see it.  Output pixel (yo, xo) is the
// operator centred on input pixel (yo + off, xo + off): off = 0 for the
// replicate border, the operator's radius (2, or 1 for the 3x3 pair) for the
// valid border.
struct U8Job {
    const uint8_t *src;
    uint8_t *mag;          // may be null
    void *dir[4];          // used iff dir_type != 0
    int64_t src_pitch;
    int64_t mag_pitch;
    int64_t dir_pitch;
    int32_t W, H;          // input size
    int32_t Wo, Ho;        // output size
    int32_t dir_type;      // 0 none, 1 int16, 2 int32
    int32_t ntx;           // tile columns (tile width = 16 lanes * px_per_lane)
    int32_t nty4;          // ceil(tile rows / 4): a wave takes 4 stacked tiles
    int32_t nty;           // tile rows
    int32_t nwt;           // wave tiles, 4 tiles stacked per wave = ntx * nty4
    int32_t nwt_h;         // wave tiles, 4 tiles side by side = ceil(ntx / 4) * nty
};

// Tile shape.  A 16-lane group owns a tile of (16 * ppl) columns x th rows;
// a wave owns 4 vertically stacked tiles.
struct U8Shape {
    int ppl;        // pixels per lane: 8 or 16
    int th;         // rows per tile (batched kernel)
    int wpg;        // waves per workgroup (4)
    int waves = 0;  // single-image kernel: waves to launch (0 = all resident waves)
    int min_rows = 2;   // single-image kernel: fewest output rows per wave (small images are latency-bound)
    bool sep = false;   // four-directional magnitudes in the separable form (the kernel that also serves planes)
    int tallx = 0;      // batched kernel: tall chunks of tallx tile heights (0: batched_split())
};

// True when the fast (vector-load) kernel may read this image: 16-byte
// aligned base and pitch.
bool u8_rows_aligned(const U8Job &j);

// Fills the tiling fields of `j` for shape `s`.
void u8_tile(U8Job &j, const U8Shape &s);

// Single image: one launch; every resident wave takes an equal row range of
// one strip of four tiles.  `border` is the public SOBEL4X5_BORDER_* code
// (replicate 0, valid 1, zero 2, reflect-101 3); the zero and reflect-101
// kernels live in their own translation unit (launch_u8_single_zr).
hipError_t launch_u8_single(const U8Job &j, int border, const U8Shape &s, hipStream_t stream);
hipError_t launch_u8_single_zr(const U8Job &j, int border, const U8Shape &s, hipStream_t stream);

// Magnitudes alone of the four-directional operator on the matrix cores
// (u8_mfma.hpp): 32 x 128 output tiles, `waves` waves in all (0 = four
// rounds of resident waves).  `border`: the public code.
hipError_t launch_u8_mfma(const U8Job &j, int border, int waves, hipStream_t stream);

// Magnitudes of four run-time kernels (HOST array of 4*25 int32, the layout
// of sobel4x5_u8_weighted, already validated) on the matrix cores, when
// every weight fits int8 (mfma_weights_fit).
bool mfma_weights_fit(const int32_t *weights);
hipError_t launch_u8_mfma_weighted(const U8Job &j, int border, const int32_t *weights, int waves, hipStream_t stream);

// Two-directional operators on the single-image sweep: op 1 = the 0 / 90 deg
// filters of the 5x5 operator, op 2 = the 3x3 pair (VALID: off = 1).  The
// job's Wo, Ho and tiling are those of the operator's own border rule.
hipError_t launch_u8_2dir(const U8Job &j, int op, int border, const U8Shape &s, hipStream_t stream);
hipError_t launch_u8_2dir_zr(const U8Job &j, int op, int border, const U8Shape &s, hipStream_t stream);

// Batched persistent launch (`aligned`: every image may take the vector
// path: 16-byte aligned src rows, and at least 3 columns under reflect-101).
// `jobs` (device) holds the images; `tiles` (device, `total` entries) lists
// every wave-tile of the batch as {image, kind | rows << 1, tx, y0}
// (batched_tiles); `queue` (device, 2 words, zero before the first launch)
// is the work counter and the exit counter, reset by the last wave to
// finish.  `border`: the public code; `dir`: some job asks for directional
// planes.  `claims` (device, `total` counters, or null): each tile's counter
// gains one for every wave that takes the tile.
hipError_t launch_u8_batched(const U8Job *jobs, const int4 *tiles, int32_t total, uint32_t *queue, int border,
                             bool aligned, bool dir, const U8Shape &s, int grid, hipStream_t stream,
                             uint32_t *claims = nullptr);

// Wave-tiles of image `img` (tiled by u8_tile with th rows per tile): the
// complete four-tile strips side by side (kind 0) in tall row chunks
// (passed to `first`) and short ones (passed to `last`, queued after every
// tall chunk of the batch), then the remaining tile columns with four row
// blocks stacked (kind 1, passed to `first`).
struct BatchSplit {
    int tallx;    // tall chunks: tallx tile heights
    int shortq;   // the last 1/shortq of the rows in chunks of one tile height
};
BatchSplit batched_split();

template <class First, class Last>
void batched_tiles_each(const U8Job &j, int32_t img, int th, int tallx, First &&first, Last &&last)
{
    const BatchSplit sp = batched_split();
    const int strips = j.ntx / 4, tall = (tallx > 0 ? tallx : sp.tallx) * th;
    const int htall = (j.Ho - j.Ho / sp.shortq) / tall * tall;
    for (int y = 0; y < htall; y += tall)
        for (int s = 0; s < strips; ++s) first(make_int4(img, tall << 1, 4 * s, y));
    for (int y = htall; y < j.Ho; y += th)
        for (int s = 0; s < strips; ++s) last(make_int4(img, th << 1, 4 * s, y));
    for (int tx = 4 * strips; tx < j.ntx; ++tx)
        for (int y = 0; y < j.Ho; y += 4 * th) first(make_int4(img, 1, tx, y));
}

// The same into two vectors.
void batched_tiles(const U8Job &j, int32_t img, int th, int tallx, std::vector<int4> &first,
                   std::vector<int4> &last);

// Reorders tiles [b, e) of a static-grid table so that each XCD's
// workgroups take a contiguous stretch of it (sobel4x5_batched.hip).
void xcd_order(std::vector<int4> &v, size_t b, size_t e);

// Allocation-free batched call (sobel4x5_batched_noalloc): the queue
// words, the job table and the tile table of one batch live in a fixed
// device buffer of kNoallocBytes per device, laid out as below.  The limits
// are the public SOBEL4X5_NOALLOC_MAX_*.
constexpr int32_t kNoallocMaxImages = 1024;
constexpr int32_t kNoallocMaxTiles = 65536;
constexpr size_t kNoallocJobsOff = 256;   // bytes [0, 8): queue[0], queue[1]
constexpr size_t kNoallocTilesOff = (kNoallocJobsOff + sizeof(U8Job) * kNoallocMaxImages + 255) / 256 * 256;
constexpr size_t kNoallocBytes = kNoallocTilesOff + sizeof(int4) * kNoallocMaxTiles;

// Device address of this device's buffer (looked up once per device, with
// that device current).
hipError_t noalloc_scratch(void **out);

// Number of workgroups of the persistent kernel that fit on the device at
// once for shape `s` (occupancy x CUs), or 0 on error.
int u8_persistent_grid(const U8Shape &s, int border, bool aligned, bool dir);

// uint8 operator with run-time weights (four integer kernels that are
// antisymmetric under a half turn), as coefficients of the 12 upper-half
// pair differences: coef[plane][t] = k_plane[i_t][j_t] with taps (0,0..4),
// (1,0..4), (2,0), (2,1).
struct WJob {
    const uint8_t *src;
    uint8_t *mag;          // may be null
    void *dir[4];          // used iff dir_type != 0
    int64_t src_pitch, mag_pitch, dir_pitch;
    int32_t W, H, Wo, Ho;
    int32_t off;           // 0 replicate / zero / reflect-101, 2 valid
    int32_t bmode;         // pixels outside the image: 0 nearest, 1 zero, 2 reflect-101
    int32_t dir_type;      // 0 none, 1 int16, 2 int32
    int32_t coef[4][12];
};
hipError_t launch_u8_weighted(const WJob &j, hipStream_t stream);

hipError_t launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t stream);

// Fingerprint of one plane of `rows` rows of `row_bytes` bytes (device):
// fingerprint_blocks(rows) workgroup sums written to `partials` (device).
int64_t fingerprint_blocks(int64_t rows);
hipError_t launch_fingerprint(const void *base, int64_t pitch, int64_t row_bytes, int64_t rows, uint64_t *partials,
                              hipStream_t stream);
// method 0: the square-root rounding; 1: the LDS table (u8_sweep.hpp)
hipError_t launch_round_mag(const int32_t *S, uint8_t *out, int64_t n, int method, hipStream_t stream);
// The four-directional sweep's rounding of n int16 quadruples (E1, E2, Hp, Hm)
hipError_t launch_round_quad(const int16_t *q, uint8_t *out, int64_t n, hipStream_t stream);

// fp32 path (pointers and strides as in the public header).
struct F32Args {
    const float *src;
    int64_t src_pitch, src_bstride;       // bytes
    float *out;
    int64_t out_pitch, out_bstride;       // bytes
    const float *grad;                    // bwd only
    int64_t g_pitch, g_bstride;           // bytes
    int32_t B, W, H, Wo, Ho;
    int32_t off;                          // 0 replicate / zero / reflect-101, 2 valid
    int32_t bmode;                        // 0 clamp (replicate, valid), 1 zero, 2 reflect-101
};

hipError_t launch_f32_fwd(const F32Args &a, hipStream_t stream);
hipError_t launch_f32_bwd(const F32Args &a, hipStream_t stream);

}  // namespace s4x5
