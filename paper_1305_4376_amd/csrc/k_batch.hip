// k_batch.hip -- persistent kernel for a batch of messages, each with its own key and direction.
//
// The paper's host loop launches one kernel per 1 MiB chunk and finds the
// launch granularity matters (Section II.B and Table II).  Here a whole batch
// of messages of any lengths is one launch: the host cuts the work into tiles
// (batch.cpp) and a fixed grid of waves draws tiles from an atomic counter
// until none are left.
//
// Two tile kinds, both running the bitsliced core (bitslice_core.h):
//   wave tile  -- up to 2048 consecutive blocks of one message: one key for the
//                 whole wave, its masks in scalar registers;
//   lane tile  -- 64 lane slots of up to 32 blocks each, packed from the short
//                 remainders of many messages: every lane reads its own slot,
//                 key and direction (key masks then come from vector registers).
//
// Work counter.  Each wave takes tickets until it draws one at or past the
// tile count, so exactly n_tiles + (number of waves) tickets are drawn per
// launch; the wave that draws the last one resets the counter to zero for the
// next launch.  The kernel therefore needs no reset node and can be replayed
// from a captured graph.  Every wave exits once the tiles run out.
#include <hip/hip_runtime.h>

#include "batch_plan.h"
#include "bitslice_core.h"
#include "internal.h"

namespace {

using namespace tdes_bs;

constexpr int kMaxThreads = 256;

__global__ __launch_bounds__(kMaxThreads) void tdes_batch_kernel(const uint32_t *__restrict__ sched,
                                                                 const tdes::PlanHeader *__restrict__ hdr,
                                                                 const uint32_t *__restrict__ tiles,
                                                                 const tdes::Slot *__restrict__ slots,
                                                                 uint32_t *counter, uint8_t *base) {
    const uint32_t lane = threadIdx.x % kLanes;
    const uint32_t n_tiles = hdr->n_tiles;
    const uint32_t n_slots = hdr->n_slots;
    const uint32_t n_waves = gridDim.x * (blockDim.x / kLanes);
    for (;;) {
        uint32_t ticket = 0;
        if (lane == 0) ticket = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        if (ticket >= n_tiles) {
            if (ticket == n_tiles + n_waves - 1 && lane == 0)
                __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        const uint32_t t = tiles[ticket];
        const uint32_t first_slot = t & ~tdes::kLaneTileBit;
        if (t & tdes::kLaneTileBit) {
            // Lane tile: 64 slots, one per lane.
            if (first_slot + kLanes > n_slots) continue;
            const tdes::Slot s = slots[first_slot + lane];
            lane_slot(sched + s.ks_off, base + s.in_off, base + s.out_off, s.count);
        } else {
            if (first_slot >= n_slots) continue;
            const tdes::Slot s = slots[first_slot];
            const uint32_t *ks = sched + s.ks_off;
            const uint8_t *tin = base + s.in_off;
            uint8_t *tout = base + s.out_off;
            const bool full = s.count == kTileBlocks &&
                              ((reinterpret_cast<uintptr_t>(tin) | reinterpret_cast<uintptr_t>(tout)) & 15) == 0;
            if (full)
                wave_tile<true, kScalarMasks>(ks, tin, tout, kTileBlocks, lane);
            else
                wave_tile<false, kScalarMasks>(ks, tin, tout, s.count, lane);
        }
    }
}

}  // namespace

namespace tdes {

hipError_t launch_batch(const uint32_t *sched, const PlanHeader *hdr, const uint32_t *tiles, const Slot *slots,
                        uint32_t *counter, uint8_t *base, uint32_t grid, uint32_t threads, hipStream_t stream) {
    if (threads == 0 || threads > kMaxThreads || threads % kLanes != 0 || grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tdes_batch_kernel, dim3(grid), dim3(threads), 0, stream, sched, hdr, tiles, slots, counter,
                       base);
    return hipGetLastError();
}

}  // namespace tdes
