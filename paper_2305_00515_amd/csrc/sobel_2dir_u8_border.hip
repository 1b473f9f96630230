// uint8 two-directional Sobel operators (the 3x3 pair of Eq. (sobel3_1) and
// the 0 / 90 deg pair of Eq. (sobel5_1)) for the zero and reflect-101
// borders: the single-image launch of the sweep in u8_sweep.hpp.

#include "u8_launch.hpp"

namespace s4x5 {

hipError_t launch_u8_2dir_zr(const U8Job &j, int op, int border, const U8Shape &s, hipStream_t st)
{
    if (op == kOp2x3) {
        if (border == 2) return launch_single_border<kOp2x3, 1, kBmZero>(j, false, s, st);
        if (border == 3) return launch_single_border<kOp2x3, 1, kBmRefl>(j, false, s, st);
    } else if (op == kOp2x5) {
        if (border == 2) return launch_single_border<kOp2x5, 2, kBmZero>(j, false, s, st);
        if (border == 3) return launch_single_border<kOp2x5, 2, kBmRefl>(j, false, s, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace s4x5
