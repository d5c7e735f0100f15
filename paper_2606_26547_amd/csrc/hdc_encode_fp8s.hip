// Encoder instantiations for the split E4M3 compute type.
#include "hdc_encode_impl.h"

namespace hdc {
hipError_t launch_encode_fp8s(const EncodeArgs &a, int mode, Tile tile, hipStream_t st)
{
    return launch_encode_ct<C_FP8S>(a, mode, tile, st);
}
}  // namespace hdc
