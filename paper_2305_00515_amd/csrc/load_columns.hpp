// Byte columns a lane of the uint8 kernels loads from every row it reads
// (aligned-row path), and the reflect-101 index map.  Plain integer code,
// shared by the kernels and by host-side checks that enumerate every lane of
// every launch geometry and every index the map can be asked for.
//
// A lane owns ppl (8 or 16) consecutive pixels starting at column xo (a
// multiple of ppl); it loads the aligned ppl-byte block at `ldx`, and the
// first / last lane of its 16-lane group also loads one aligned dword at
// `hx` for the group's outer halo (columns xo-4..xo-1 / xo+ppl..xo+ppl+3).
//
// Invariant: every block loaded holds at least one byte of the row
// (column < W).  With a 16-byte aligned row start, such an aligned block
// never reaches into another page than that byte, so over-reading it can
// never touch unmapped memory; the bytes past the row end are replaced in
// registers.  Lanes past the right edge (xo >= W, e.g. idle groups of a
// wave whose tiles end inside the image) load the block of the row's last
// byte instead.
#pragma once

#if defined(__HIPCC__)
#define S4X5_HD __host__ __device__
#else
#define S4X5_HD
#endif

namespace s4x5 {

struct LoadCols {
    unsigned ldx;   // start of the lane's own ppl-byte block
    unsigned hx;    // start of the halo dword (lanes 0 and 15 of a group; == ldx otherwise)
};

S4X5_HD inline LoadCols load_columns(int xo, int lane16, int W, int ppl)
{
    const unsigned last_block = (unsigned)((W - 1) & ~(ppl - 1));   // block of column W-1
    const unsigned last_dword = (unsigned)((W - 1) & ~3);           // dword of column W-1
    LoadCols c;
    c.ldx = xo < W ? (unsigned)xo : last_block;
    if (lane16 == 0)
        c.hx = xo < 4 ? 0u : (xo - 4 < W ? (unsigned)(xo - 4) : last_dword);
    else if (lane16 == 15)
        c.hx = xo + ppl < W ? (unsigned)(xo + ppl) : last_dword;
    else
        c.hx = c.ldx;
    return c;
}

// Reflect-101 border: the index that stands in for position i of an axis of
// n >= 1 pixels, mirroring about the edge pixel without repeating it
// (..., 2, 1 | 0, 1, ..., n-1 | n-2, ...).  The extended axis is periodic
// with period 2(n-1); n = 1 maps everything to 0.  One reflection suffices
// for the 5x5 operator's reach (|i - edge| <= 2) once n >= 3; the general
// fold serves narrower axes.  The result always lies in [0, n-1].
S4X5_HD inline int reflect101(int i, int n)
{
    if (i >= 0 && i < n) return i;
    if (n == 1) return 0;
    const int p = 2 * (n - 1);
    if (i < 0 && -i < n) return -i;
    if (i >= n && p - i >= 0) return p - i;
    int m = i % p;
    if (m < 0) m += p;
    return m < n ? m : p - m;
}

}  // namespace s4x5
