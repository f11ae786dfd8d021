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
// Work assignment.  Wave w of the grid takes tile w first, with no atomic;
// afterwards it draws from a counter, and draw d gives it the k tiles from
// n_waves + k d on (k = tiles per draw, a tuning parameter); it stops at the
// first draw that starts at or past the tile count.  (All waves drawing their
// first tile from the counter at the same moment made them queue on one
// atomic address at launch: 8% slower on whole-tile batches.)  Every wave
// that had a first tile makes exactly one failing draw, so a launch makes
// W + S draws (W = min(n_waves, n_tiles) waves with a first tile, S =
// ceil((n_tiles - n_waves) / k) successful draws, 0 if n_tiles <= n_waves)
// and the draw that returns W + S - 1 is the last: that wave resets the
// counter to zero for the next launch.  The kernel therefore needs no reset
// node and can be replayed from a captured graph.  Every wave exits once the
// tiles run out.
#include <hip/hip_runtime.h>

#include "batch_plan.h"
#include "bitslice_core.h"
#include "internal.h"

namespace {

using namespace tdes_bs;

constexpr int kMaxThreads = 256;
// Register budget of four 256-thread workgroups per CU (4 waves per SIMD, at
// most 128 VGPRs): the rounds of every tile kind fit it without spills; the
// lane tiles' per-lane load and store phases spill a few values to scratch.
constexpr int kMinGroupsPerCU = 4;

// One counter draw (the old value), wave-uniform; the draw numbered `last` resets the counter.
__device__ __forceinline__ uint32_t draw(uint32_t *counter, uint32_t last, uint32_t lane) {
    uint32_t d = 0;
    if (lane == 0) d = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d = __builtin_amdgcn_readfirstlane(d);
    if (d == last && lane == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return d;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The server's steps launch the same kernel held to 120 VGPRs instead of 128
// (k_batch_capped.hip builds this file with TDES_BATCH_CAPPED defined; on this
// target the attribute counts the unified VGPR/AGPR budget in pairs: 60 -> 120
// registers, no AGPR is used).  Four such waves per SIMD leave 32 registers
// free, room for two waves of a small kernel on another stream (the server's
// payload fill) to run beside the persistent cipher instead of waiting for its
// workgroups to retire; a few more values spill in the tile load and store
// phases.  Each variant is built in a translation unit of its own: with both in
// one, the uncapped kernel's code moved and ran the C4 batch 2% slower.
#ifdef TDES_BATCH_CAPPED
#define TDES_BATCH_KERNEL \
    __global__ __launch_bounds__(kMaxThreads, kMinGroupsPerCU) __attribute__((amdgpu_num_vgpr(60))) void tdes_batch_kernel_capped
#else
#define TDES_BATCH_KERNEL __global__ __launch_bounds__(kMaxThreads, kMinGroupsPerCU) void tdes_batch_kernel
#endif

TDES_BATCH_KERNEL(const uint32_t *__restrict__ sched, const tdes::PlanHeader *__restrict__ hdr,
                  const uint32_t *__restrict__ tiles, const tdes::Slot *__restrict__ slots, uint32_t *counter,
                  uint8_t *base, uint32_t per_draw) {
    const uint32_t lane = threadIdx.x % kLanes;
    const uint32_t n_tiles = hdr->n_tiles;
    const uint32_t n_slots = hdr->n_slots;
    const uint32_t n_waves = gridDim.x * (blockDim.x / kLanes);
    const uint32_t wave_id = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kLanes) + threadIdx.x / kLanes);
    if (wave_id >= n_tiles) return;
    const uint32_t with_first = min(n_waves, n_tiles);
    const uint32_t good_draws = n_tiles > n_waves ? (n_tiles - n_waves + per_draw - 1) / per_draw : 0;
    const uint32_t last = with_first + good_draws - 1;
    uint64_t first = wave_id, count = 1;  // the wave's current run of tiles
    while (first < n_tiles) {
        const uint32_t end = (uint32_t)min((uint64_t)n_tiles, first + count);
        for (uint32_t ticket = (uint32_t)first; ticket < end; ticket++) {
            const uint32_t t = __builtin_amdgcn_readfirstlane(tiles[ticket]);
            const uint32_t first_slot = t & ~tdes::kLaneTileBit;
            if (t & tdes::kLaneTileBit) {
                // Lane tile: 64 slots, one per lane.
                if (first_slot + kLanes > n_slots) continue;
                const tdes::Slot s = slots[first_slot + lane];
                lane_slot(sched + s.ks_off, base + s.in_off, base + s.out_off, s.count);
            } else {
                if (first_slot >= n_slots) continue;
                // The slot is the same for the whole wave: keep its fields in scalar registers.
                const tdes::Slot &sl = slots[first_slot];
                const uint64_t in_off = uniform64(sl.in_off), out_off = uniform64(sl.out_off);
                const uint32_t cnt = __builtin_amdgcn_readfirstlane(sl.count);
                const uint32_t *ks = sched + __builtin_amdgcn_readfirstlane(sl.ks_off);
                const uint8_t *tin = base + in_off;
                uint8_t *tout = base + out_off;
                const bool full = cnt == kTileBlocks &&
                                  ((reinterpret_cast<uintptr_t>(tin) | reinterpret_cast<uintptr_t>(tout)) & 15) == 0;
                if (full)
                    wave_tile<true>(ks, tin, tout, kTileBlocks, lane);
                else
                    wave_tile<false>(ks, tin, tout, cnt, lane);
            }
        }
        const uint32_t d = draw(counter, last, lane);
        first = n_waves + (uint64_t)d * per_draw;
        count = per_draw;
    }
}

}  // namespace

namespace tdes {

#ifdef TDES_BATCH_CAPPED
hipError_t launch_batch_capped(const uint32_t *sched, const PlanHeader *hdr, const uint32_t *tiles, const Slot *slots,
                               uint32_t *counter, uint8_t *base, uint32_t grid, uint32_t threads,
                               uint32_t tiles_per_draw, hipStream_t stream) {
    hipLaunchKernelGGL(tdes_batch_kernel_capped, dim3(grid), dim3(threads), 0, stream, sched, hdr, tiles, slots,
                       counter, base, tiles_per_draw);
    return hipGetLastError();
}
#else
hipError_t launch_batch(const uint32_t *sched, const PlanHeader *hdr, const uint32_t *tiles, const Slot *slots,
                        uint32_t *counter, uint8_t *base, uint32_t grid, uint32_t threads, uint32_t tiles_per_draw,
                        bool capped, hipStream_t stream) {
    if (threads == 0 || threads > kMaxThreads || threads % kLanes != 0 || grid == 0 || tiles_per_draw == 0)
        return hipErrorInvalidValue;
    if (capped) return launch_batch_capped(sched, hdr, tiles, slots, counter, base, grid, threads, tiles_per_draw, stream);
    hipLaunchKernelGGL(tdes_batch_kernel, dim3(grid), dim3(threads), 0, stream, sched, hdr, tiles, slots, counter,
                       base, tiles_per_draw);
    return hipGetLastError();
}
#endif

}  // namespace tdes
