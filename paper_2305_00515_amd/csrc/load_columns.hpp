// Byte columns a lane of the uint8 kernels loads from every row it reads
// (aligned-row path).  Plain integer code, shared by the kernels and by a
// host-side check that enumerates every lane of every launch geometry.
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

}  // namespace s4x5
