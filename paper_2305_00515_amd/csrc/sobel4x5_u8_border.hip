// uint8 four-directional 5x5 kernel for the zero and reflect-101 borders:
// the single-image launch of the sweep in u8_sweep.hpp.

#include "u8_launch.hpp"

namespace s4x5 {

hipError_t launch_u8_single_zr(const U8Job &j, int border, const U8Shape &s, hipStream_t st)
{
    if (border == 2) return launch_single_border<kOp4x5, 0, kBmZero>(j, false, s, st);
    if (border == 3) return launch_single_border<kOp4x5, 0, kBmRefl>(j, false, s, st);
    return hipErrorInvalidValue;
}

}  // namespace s4x5
