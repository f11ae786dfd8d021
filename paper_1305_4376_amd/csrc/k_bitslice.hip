// k_bitslice.hip -- Triple-DES ECB over one message, bitsliced variant (plain launch).
//
// The paper maps one 64-bit block to one GPU thread and notes that the cipher
// is almost entirely bit operations on integers (Abstract; Section IV).  Here a
// lane instead holds 32 blocks as bit planes (bitslice_core.h): no lookup
// tables and no LDS, a fixed data-independent cost per block, and the three
// DES stages of EDE fused in one pass over the data.
//
// Launch: one wave per 2048-block tile (16 KiB of the message), four waves
// per workgroup; tiles beyond 2^22 loop grid-stride.  The key is the same for
// the whole launch, so its masks come from scalar registers.
#include <hip/hip_runtime.h>

#include "bitslice_core.h"
#include "internal.h"

namespace {

using namespace tdes_bs;

constexpr int kThreads = 256;  // 4 waves per workgroup
constexpr KeyMode kWaveKeys = kScalarMasks;

__global__ __launch_bounds__(kThreads) void tdes_bitslice_kernel(const uint32_t *__restrict__ ks, const uint8_t *in,
                                                                 uint8_t *out, uint64_t n_blocks, int vec16) {
    const uint32_t lane = threadIdx.x % kLanes;
    const uint64_t tiles = (n_blocks + kTileBlocks - 1) / kTileBlocks;
    const uint64_t stride = (uint64_t)gridDim.x * (kThreads / kLanes);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    for (uint64_t tile = (uint64_t)blockIdx.x * (kThreads / kLanes) + wave; tile < tiles; tile += stride) {
        const uint64_t first = tile * kTileBlocks;
        const uint64_t left = n_blocks - first;
        const uint32_t n_valid = left < kTileBlocks ? (uint32_t)left : kTileBlocks;
        if (vec16 && n_valid == kTileBlocks)
            wave_tile<true, kWaveKeys>(ks, in + 8 * first, out + 8 * first, n_valid, lane);
        else
            wave_tile<false, kWaveKeys>(ks, in + 8 * first, out + 8 * first, n_valid, lane);
    }
}

}  // namespace

namespace tdes {

hipError_t launch_bitslice(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                           hipStream_t stream) {
    const uint64_t tiles = (n_blocks + kTileBlocks - 1) / kTileBlocks;
    uint64_t grid = (tiles + kThreads / kLanes - 1) / (kThreads / kLanes);
    if (grid > (1u << 20)) grid = 1u << 20;  // larger messages loop over tiles
    const int vec16 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    hipLaunchKernelGGL(tdes_bitslice_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, ks, in, out, n_blocks,
                       vec16);
    return hipGetLastError();
}

}  // namespace tdes
