// k_bitslice.hip -- Triple-DES over one message, bitsliced: ECB, and the CTR and
// CBC-decrypt modes on the same core (plain launches).
//
// The paper maps one 64-bit block to one GPU thread and notes that the cipher
// is almost entirely bit operations on integers (Abstract; Section IV).  Here a
// lane instead holds 32 blocks as bit planes (bitslice_core.h): no lookup
// tables and no LDS, a fixed data-independent cost per block, and the three
// DES stages of EDE fused in one pass over the data.
//
// Two kernels.  The main one takes every whole 2048-block tile (16 KiB of the
// message, one wave each) of a message whose buffers are 16-byte aligned; its
// code has only that path, so it fits 128 VGPRs and runs four waves per SIMD.
// The tail kernel takes the last partial tile, or every tile when a buffer is
// only 8-byte aligned, with per-block loads and stores.  Tiles beyond 2^22
// per launch loop grid-stride.  The key is the same for the whole launch, so
// its masks come from scalar registers.
#include <hip/hip_runtime.h>

#include "bitslice_core.h"
#include "internal.h"

namespace {

using namespace tdes_bs;

constexpr int kDefaultThreads = 256;     // 4 waves per workgroup
constexpr int kWavesPerSimd = 4;         // at most 128 VGPRs per lane
constexpr uint64_t kMaxGrid = 1u << 20;

// Workgroups of kThreads threads (one wave per 64); the main kernel is built for
// four waves per SIMD whatever the workgroup size (launch_bounds' second
// argument is the minimum number of waves per execution unit).
template <TileMode kMode, int kThreads = kDefaultThreads>
__global__ __launch_bounds__(kThreads, kWavesPerSimd) void tdes_bitslice_kernel(const uint32_t *__restrict__ ks,
                                                                                   const uint8_t *in, uint8_t *out,
                                                                                   uint64_t n_tiles, uint64_t iv) {
    constexpr int kWaves = kThreads / kLanes;
    const uint32_t lane = threadIdx.x % kLanes;
    const uint64_t stride = (uint64_t)gridDim.x * kWaves;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    for (uint64_t tile = (uint64_t)blockIdx.x * kWaves + wave; tile < n_tiles; tile += stride) {
        const uint64_t first = tile * kTileBlocks;
        mode_tile<kMode, true>(ks, in + 8 * first, out + 8 * first, kTileBlocks, lane, first, iv);
    }
}

// Tiles first_tile.. of the message, any of them partial; 8-byte alignment suffices.
template <TileMode kMode, int kThreads = kDefaultThreads>
__global__ __launch_bounds__(kThreads) void tdes_bitslice_tail_kernel(const uint32_t *__restrict__ ks,
                                                                      const uint8_t *in, uint8_t *out,
                                                                      uint64_t first_tile, uint64_t n_blocks,
                                                                      uint64_t iv) {
    constexpr int kWaves = kThreads / kLanes;
    const uint32_t lane = threadIdx.x % kLanes;
    const uint64_t tiles = (n_blocks + kTileBlocks - 1) / kTileBlocks;
    const uint64_t stride = (uint64_t)gridDim.x * kWaves;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    for (uint64_t tile = first_tile + (uint64_t)blockIdx.x * kWaves + wave; tile < tiles; tile += stride) {
        const uint64_t first = tile * kTileBlocks;
        const uint64_t left = n_blocks - first;
        const uint32_t n_valid = left < kTileBlocks ? (uint32_t)left : kTileBlocks;
        mode_tile<kMode, false>(ks, in + 8 * first, out + 8 * first, n_valid, lane, first, iv);
    }
}

uint32_t grid_for(uint64_t tiles, int waves_per_group) {
    const uint64_t g = (tiles + waves_per_group - 1) / waves_per_group;
    return (uint32_t)(g < kMaxGrid ? g : kMaxGrid);
}

template <TileMode kMode, int kThreads = kDefaultThreads>
hipError_t launch(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, uint64_t iv,
                  hipStream_t stream) {
    constexpr int kWaves = kThreads / kLanes;
    const bool vec16 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    const uint64_t whole = vec16 ? n_blocks / kTileBlocks : 0;
    if (whole) {
        hipLaunchKernelGGL((tdes_bitslice_kernel<kMode, kThreads>), dim3(grid_for(whole, kWaves)), dim3(kThreads), 0,
                           stream, ks, in, out, whole, iv);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (whole * kTileBlocks < n_blocks) {
        const uint64_t rest = (n_blocks - whole * kTileBlocks + kTileBlocks - 1) / kTileBlocks;
        hipLaunchKernelGGL((tdes_bitslice_tail_kernel<kMode, kThreads>), dim3(grid_for(rest, kWaves)), dim3(kThreads),
                           0, stream, ks, in, out, whole, n_blocks, iv);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

namespace tdes {

hipError_t launch_bitslice(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                           hipStream_t stream, uint32_t threads) {
    switch (threads) {
        case 0:
        case kDefaultThreads: return launch<TileMode::kEcb>(ks, in, out, n_blocks, 0, stream);
        case 64: return launch<TileMode::kEcb, 64>(ks, in, out, n_blocks, 0, stream);
        case 128: return launch<TileMode::kEcb, 128>(ks, in, out, n_blocks, 0, stream);
        case 512: return launch<TileMode::kEcb, 512>(ks, in, out, n_blocks, 0, stream);
        case 1024: return launch<TileMode::kEcb, 1024>(ks, in, out, n_blocks, 0, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ctr(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, uint64_t iv,
                      hipStream_t stream) {
    return launch<TileMode::kCtr>(ks, in, out, n_blocks, iv, stream);
}

hipError_t launch_cbc_decrypt(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, uint64_t iv,
                              hipStream_t stream) {
    return launch<TileMode::kCbcDecrypt>(ks, in, out, n_blocks, iv, stream);
}

}  // namespace tdes
