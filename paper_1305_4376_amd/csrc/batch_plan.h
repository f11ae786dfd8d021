// batch_plan.h -- the device-side plan of a batch, shared by the planner (batch.cpp) and the kernel.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace tdes {

// Plan buffer: [PlanHeader][tile words][slots], each part 256-byte aligned.
struct PlanHeader {
    uint32_t n_tiles;
    uint32_t n_slots;
    uint32_t pad[62];
};
static_assert(sizeof(PlanHeader) == 256, "header is one 256-byte line");

// A run of consecutive blocks of one message: byte offsets from the batch base,
// the number of blocks (a wave tile: up to 2048; a lane slot: up to 32; 0 for
// an idle lane) and the word offset of its 96 subkey words in the schedule table.
struct Slot {
    uint64_t in_off;
    uint64_t out_off;
    uint32_t count;
    uint32_t ks_off;
    uint64_t pad;
};
static_assert(sizeof(Slot) == 32, "slot is 32 bytes");

// Tile word: index of its first slot; the top bit marks a lane tile (64 slots).
constexpr uint32_t kLaneTileBit = 0x80000000u;

// capped: the variant held to 120 VGPRs (room for another kernel's waves beside it).
hipError_t launch_batch(const uint32_t *sched, const PlanHeader *hdr, const uint32_t *tiles, const Slot *slots,
                        uint32_t *counter, uint8_t *base, uint32_t grid, uint32_t threads, uint32_t tiles_per_draw,
                        bool capped, hipStream_t stream);
// The capped variant alone (k_batch_capped.hip); arguments checked by launch_batch.
hipError_t launch_batch_capped(const uint32_t *sched, const PlanHeader *hdr, const uint32_t *tiles, const Slot *slots,
                               uint32_t *counter, uint8_t *base, uint32_t grid, uint32_t threads,
                               uint32_t tiles_per_draw, hipStream_t stream);

}  // namespace tdes
