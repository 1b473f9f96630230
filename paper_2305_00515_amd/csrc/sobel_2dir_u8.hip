// uint8 two-directional Sobel operators for CDNA4 (gfx950): the 3x3 pair of
// Eq. (sobel3_1) and the 0 / 90 deg pair of Eq. (sobel5_1), each with the
// magnitude of Eq. (sobel3_2), on the row sweep of u8_sweep.hpp.  The
// paper compares its four-directional 5x5 kernels with the 3x3 operator
// (Sec. 5, Table 1); these kernels make that comparison on the same sweep.
//
// Offsets: the 3x3 pair has radius 1, so its VALID output is centred on
// input pixel (y + 1, x + 1); the 5x5 pair, like the four-directional
// operator, on (y + 2, x + 2).

#include "u8_sweep.hpp"

namespace s4x5 {
namespace {

template <int PPL, int OFF, int OPR>
hipError_t launch_2dir_d(const U8Job &j, const U8Shape &s, hipStream_t st)
{
    return j.dir_type ? launch_single_t<PPL, OFF, true, OPR>(j, s, st)
                      : launch_single_t<PPL, OFF, false, OPR>(j, s, st);
}

template <int OPR, int VOFF>
hipError_t launch_2dir_o(const U8Job &j, int border_valid, const U8Shape &s, hipStream_t st)
{
    if (s.ppl == 16)
        return border_valid ? launch_2dir_d<16, VOFF, OPR>(j, s, st) : launch_2dir_d<16, 0, OPR>(j, s, st);
    return border_valid ? launch_2dir_d<8, VOFF, OPR>(j, s, st) : launch_2dir_d<8, 0, OPR>(j, s, st);
}

}  // namespace

hipError_t launch_u8_2dir(const U8Job &j, int op, int border_valid, const U8Shape &s, hipStream_t st)
{
    if (j.ntx <= 0 || j.Ho <= 0) return hipSuccess;
    if (op == kOp2x3) return launch_2dir_o<kOp2x3, 1>(j, border_valid, s, st);
    if (op == kOp2x5) return launch_2dir_o<kOp2x5, 2>(j, border_valid, s, st);
    return hipErrorInvalidValue;
}

}  // namespace s4x5
