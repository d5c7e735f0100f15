// Encoder instantiations for the fp8 compute type.
#include "hdc_encode_impl.h"

namespace hdc {
hipError_t launch_encode_fp8(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    return launch_encode_ct<C_FP8>(a, mode, tile, st);
}
}  // namespace hdc
