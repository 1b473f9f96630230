// uint8 four-directional 5x5 kernel for CDNA4 (gfx950): the single-image
// launch of the sweep in u8_sweep.hpp for the replicate and valid borders
// (zero and reflect-101: sobel4x5_u8_border.hip), and a plain copy kernel
// that serves as the bandwidth reference.

#include "u8_launch.hpp"

namespace s4x5 {
namespace {

// Plain streaming copy: the reference point for the achievable HBM
// bandwidth and for calibrating the memory-traffic counters.  Each
// workgroup copies one contiguous 16 KiB block, four 16-byte loads per lane
// in flight before the stores (measured 5.7 TB/s on 1 GiB, against 4.6 TB/s
// for a grid-stride loop).
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n16) v[k] = src[base + 256 * k];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n16) dst[base + 256 * k] = v[k];
}

// Order-independent fingerprint of one output plane (the autotuner's check
// that a candidate tile shape reproduces the reference bytes): the byte at
// (row r, column c) contributes mix(r, c, byte), with the splitmix64
// finaliser as the mix; each workgroup sums (mod 2^64) the contributions of
// kFpRows rows into out[blockIdx.x].
constexpr int kFpRows = 16;

__global__ __launch_bounds__(256) void k_fingerprint(const uint8_t *__restrict__ base, int64_t pitch,
                                                     int64_t row_bytes, int64_t rows, uint64_t *__restrict__ out)
{
    const int64_t r0 = (int64_t)blockIdx.x * kFpRows;
    const int64_t r1 = r0 + kFpRows < rows ? r0 + kFpRows : rows;
    uint64_t acc = 0;
    for (int64_t r = r0; r < r1; ++r) {
        const uint8_t *row = base + r * pitch;
        for (int64_t c = threadIdx.x; c < row_bytes; c += 256) {
            uint64_t v = ((uint64_t)r << 40) ^ ((uint64_t)c << 8) ^ (uint64_t)row[c];
            v = (v ^ (v >> 30)) * 0xbf58476d1ce4e5b9ull;
            v = (v ^ (v >> 27)) * 0x94d049bb133111ebull;
            acc += v ^ (v >> 31);
        }
    }
    __shared__ uint64_t red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_round_mag(const int32_t *S, uint8_t *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint8_t)round_mag(S[i]);
}

// The same rounding through the LDS table, filled and read exactly as the
// sweep does.
__global__ __launch_bounds__(256) void k_round_mag_lut(const int32_t *S, uint8_t *out, int64_t n)
{
    __shared__ __attribute__((aligned(16))) uint8_t lut[kLutSize];
    lut_fill<256>(lut);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint8_t)lut_mag((lds_u8 *)lut, S[i]);
}

// The four-directional sweep's rounding, step for step: quadruples
// (E1, E2, Hp, Hm) of int16 in pairs on the packed halves of a register,
// T = E1^2 + E2^2 + Hp^2 + Hm^2 saturated at 2^15 - 1 by the clamped
// multiply-adds, then the table of round(sqrt(2 T)) in LDS.
__global__ __launch_bounds__(256) void k_round_quad(const int16_t *q, uint8_t *out, int64_t n)
{
    __shared__ __attribute__((aligned(16))) uint8_t lut[kLutTSize];
    lut_fill_t<256>(lut);
    __syncthreads();
    const int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    u32 c[4];
    for (int k = 0; k < 4; ++k) {
        const u32 lo = (uint16_t)q[4 * i + k];
        const u32 hi = i + 1 < n ? (uint16_t)q[4 * (i + 1) + k] : 0u;
        c[k] = lo | (hi << 16);
    }
    u32 T = sq_sat(c[0]);
    T = sq_sat_acc(c[1], T);
    T = sq_sat_acc(c[2], T);
    T = sq_sat_acc(c[3], T);
    const lds_u8 *lp = (lds_u8 *)lut;
    out[i] = (uint8_t)lp[T & 0xffffu];
    if (i + 1 < n) out[i + 1] = (uint8_t)lp[T >> 16];
}

}  // namespace

bool u8_rows_aligned(const U8Job &j)
{
    return ((reinterpret_cast<uintptr_t>(j.src) | (uintptr_t)j.src_pitch) & 15u) == 0;
}

void u8_tile(U8Job &j, const U8Shape &s)
{
    const int tw = 16 * s.ppl;
    j.ntx = (j.Wo + tw - 1) / tw;
    j.nty = (j.Ho + s.th - 1) / s.th;
    j.nty4 = (j.nty + 3) / 4;
    j.nwt = j.ntx * j.nty4;
    j.nwt_h = ((j.ntx + 3) / 4) * j.nty;
}

hipError_t launch_u8_single(const U8Job &j, int border, const U8Shape &s, hipStream_t st)
{
    if (border == 2 || border == 3) return launch_u8_single_zr(j, border, s, st);
    return launch_single_border<kOp4x5, 2, kBmRep>(j, border == 1, s, st);
}

hipError_t launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t st)
{
    if (n16 <= 0) return hipSuccess;
    const int64_t blocks = (n16 + 1023) / 1024;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n16);
    return hipGetLastError();
}

int64_t fingerprint_blocks(int64_t rows) { return (rows + kFpRows - 1) / kFpRows; }

hipError_t launch_fingerprint(const void *base, int64_t pitch, int64_t row_bytes, int64_t rows, uint64_t *partials,
                              hipStream_t st)
{
    const int64_t blocks = fingerprint_blocks(rows);
    if (blocks <= 0 || row_bytes <= 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fingerprint, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const uint8_t *>(base),
                       pitch, row_bytes, rows, partials);
    return hipGetLastError();
}

hipError_t launch_round_quad(const int16_t *q, uint8_t *out, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 511) / 512;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_round_quad, dim3((unsigned)blocks), dim3(256), 0, st, q, out, n);
    return hipGetLastError();
}

hipError_t launch_round_mag(const int32_t *S, uint8_t *out, int64_t n, int method, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (method == 1)
        hipLaunchKernelGGL(k_round_mag_lut, dim3((unsigned)blocks), dim3(256), 0, st, S, out, n);
    else
        hipLaunchKernelGGL(k_round_mag, dim3((unsigned)blocks), dim3(256), 0, st, S, out, n);
    return hipGetLastError();
}

}  // namespace s4x5
