// Host-only stand-ins for the kernel translation units, so that the C-ABI
// layer (sobel4x5_api.cpp) can be built with the host sanitizers and linked
// into a test driver without any device code.  The driver only exercises
// the argument checks, which never reach these functions; any call that
// does reports that no device is present.
#include "../../paper_2305_00515_amd/csrc/internal.hpp"

namespace s4x5 {

bool u8_rows_aligned(const U8Job &) { return false; }
void u8_tile(U8Job &, const U8Shape &) {}
hipError_t launch_u8_single(const U8Job &, int, const U8Shape &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_u8_single_zr(const U8Job &, int, const U8Shape &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_u8_mfma(const U8Job &, int, int, hipStream_t) { return hipErrorNoDevice; }
bool mfma_weights_fit(const int32_t *) { return false; }
hipError_t launch_u8_mfma_weighted(const U8Job &, int, const int32_t *, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_u8_2dir(const U8Job &, int, int, const U8Shape &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_u8_2dir_zr(const U8Job &, int, int, const U8Shape &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_u8_batched(const U8Job *, const int4 *, int32_t, uint32_t *, int, bool, bool, const U8Shape &, int,
                             hipStream_t, uint32_t *)
{
    return hipErrorNoDevice;
}
void batched_tiles(const U8Job &, int32_t, int, int, std::vector<int4> &, std::vector<int4> &) {}
BatchSplit batched_split() { return BatchSplit{2, 4}; }
void xcd_order(std::vector<int4> &, size_t, size_t) {}
int u8_persistent_grid(const U8Shape &, int, bool, bool) { return 0; }
hipError_t launch_u8_weighted(const WJob &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_copy16(const void *, void *, int64_t, hipStream_t) { return hipErrorNoDevice; }
int64_t fingerprint_blocks(int64_t rows) { return rows; }
hipError_t launch_fingerprint(const void *, int64_t, int64_t, int64_t, uint64_t *, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_round_mag(const int32_t *, uint8_t *, int64_t, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_round_quad(const int16_t *, uint8_t *, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t noalloc_scratch(void **) { return hipErrorNoDevice; }
hipError_t launch_f32_fwd(const F32Args &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_f32_bwd(const F32Args &, hipStream_t) { return hipErrorNoDevice; }

}  // namespace s4x5
