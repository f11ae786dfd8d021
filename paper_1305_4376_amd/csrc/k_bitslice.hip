// k_bitslice.hip -- placeholder until the bitsliced variant lands.
#include "internal.h"

namespace tdes {
hipError_t launch_bitslice(const uint32_t *, const uint8_t *, uint8_t *, uint64_t, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace tdes
