// Encoder instantiations for the f32 compute type.
#include "hdc_encode_impl.h"

namespace hdc {
hipError_t launch_encode_f32(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    return launch_encode_ct<C_F32>(a, mode, tile, st);
}
}  // namespace hdc
