// Encoder instantiations for the i8 compute type.
#include "hdc_encode_impl.h"

namespace hdc {
hipError_t launch_encode_i8(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    return launch_encode_ct<C_I8>(a, mode, tile, st);
}
}  // namespace hdc
