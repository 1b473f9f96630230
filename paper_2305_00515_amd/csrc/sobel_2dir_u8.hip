// uint8 two-directional Sobel operators for CDNA4 (gfx950): the 3x3 pair of
// Eq. (sobel3_1) and the 0 / 90 deg pair of Eq. (sobel5_1), each with the
// magnitude of Eq. (sobel3_2), on the row sweep of u8_sweep.hpp.  The
// paper compares its four-directional 5x5 kernels with the 3x3 operator
// (Sec. 5, Table 1); these kernels make that comparison on the same sweep.
//
// Offsets: the 3x3 pair has radius 1, so its VALID output is centred on
// input pixel (y + 1, x + 1); the 5x5 pair, like the four-directional
// operator, on (y + 2, x + 2).  This file holds the replicate and valid
// borders; sobel_2dir_u8_border.hip the zero and reflect-101 ones.

#include "u8_launch.hpp"

namespace s4x5 {

hipError_t launch_u8_2dir(const U8Job &j, int op, int border, const U8Shape &s, hipStream_t st)
{
    if (border == 2 || border == 3) return launch_u8_2dir_zr(j, op, border, s, st);
    if (op == kOp2x3) return launch_single_border<kOp2x3, 1, kBmRep>(j, border == 1, s, st);
    if (op == kOp2x5) return launch_single_border<kOp2x5, 2, kBmRep>(j, border == 1, s, st);
    return hipErrorInvalidValue;
}

}  // namespace s4x5
