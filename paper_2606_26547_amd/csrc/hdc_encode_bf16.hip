// Encoder instantiations for the bf16 compute type.
#include "hdc_encode_impl.h"

namespace hdc {
hipError_t launch_encode_bf16(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    return launch_encode_ct<C_BF16>(a, mode, tile, st);
}
}  // namespace hdc
