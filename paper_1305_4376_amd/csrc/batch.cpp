// batch.cpp -- batched ECB: validation, tile planning, plan upload, graph capture, tuning.
//
// A batch is many messages, each with its own key triple (an index into a
// device table of schedules) and direction.  The paper runs one message and
// launches one kernel per 1 MiB chunk (Listing 1.1, Section II.B); with
// thousands of short messages, per-launch cost would dominate, so the whole
// batch becomes one launch of the persistent kernel in k_batch.hip.
//
// Planning.  Each message is cut into wave tiles of 2048 blocks (one key per
// wave, scalar key masks).  Its remainder, if shorter than the context's
// wave_remainder (1800 unless tuned), is cut into lane slots of 32 blocks
// instead; lane slots from all messages are packed 64 to a lane tile, where
// each lane has its own key.  A 2048-block
// tile then never runs mostly empty for short messages.  Lane tiles go first
// so that the cheaper wave tiles fill the tail of the launch.
//
// Graphs.  The kernel reads the tile count from the uploaded plan, so one
// captured graph (a single kernel node) serves every batch with the same
// base pointer, schedule table and launch shape; it is captured on a private
// stream and replayed on the caller's.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "batch_plan.h"
#include "internal.h"

namespace {

constexpr uint32_t kWaveBlocks = 2048;
constexpr uint32_t kLaneBlocks = 32;
constexpr uint32_t kLanesPerTile = 64;
// Default cut-over: a remainder this long still takes a wave tile.  A lane
// tile costs about 14% more per block (per-lane key masks), so a wave tile
// wins above ~1800 blocks; the autotuner may choose another value.
constexpr uint32_t kDefaultWaveRemainder = 1800;
constexpr uint32_t kMaxTilesPerDraw = 16;
constexpr uint64_t kMaxJobBlocks = 1ull << 40;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct tdes_ctx {
    int device = 0;
    int cu_count = 0;
    hipStream_t capture_stream = nullptr;
    uint32_t *d_counter = nullptr;
    // Plan buffers: device and pinned host staging with the same layout.
    uint8_t *d_plan = nullptr;
    uint8_t *h_plan = nullptr;
    size_t cap_tiles = 0, cap_slots = 0;
    hipEvent_t staging_free = nullptr;  // the last upload has read the staging buffer
    hipEvent_t plan_done = nullptr;     // the last kernel has finished with the device plan
    bool have_plan = false;
    // Last planned batch (for replay).
    const void *last_sched = nullptr;
    uint8_t *last_base = nullptr;
    uint32_t last_tiles = 0;
    // Launch shape and tiling.
    uint32_t threads = 256;
    uint32_t groups_per_cu = 4;
    uint32_t wave_remainder = kDefaultWaveRemainder;  // remainders this long take a wave tile
    uint32_t tiles_per_draw = 1;                      // tiles a wave takes per counter draw
    bool capped = false;                              // launch the 120-VGPR kernel variant
    // Captured graph and what it was captured for.
    hipGraphExec_t exec = nullptr;
    const void *g_sched = nullptr;
    const void *g_base = nullptr;
    const void *g_tiles = nullptr;  // every pointer the kernel node was captured with
    const void *g_slots = nullptr;
    uint32_t g_grid = 0, g_threads = 0, g_draw = 0;
    bool g_capped = false;
    tdes_batch_info info{};
};

namespace {

size_t slots_offset(size_t cap_tiles) { return 256 + align256(cap_tiles * 4); }
size_t plan_bytes(size_t cap_tiles, size_t cap_slots) { return slots_offset(cap_tiles) + cap_slots * sizeof(tdes::Slot); }

int ensure_capacity(tdes_ctx *c, size_t tiles, size_t slots) {
    if (tiles <= c->cap_tiles && slots <= c->cap_slots && c->d_plan) return TDES_OK;
    size_t nt = std::max<size_t>(tiles, std::max<size_t>(1024, c->cap_tiles * 2));
    size_t ns = std::max<size_t>(slots, std::max<size_t>(8192, c->cap_slots * 2));
    // The old buffers may still be in use by an upload or a kernel.
    if (c->d_plan) {
        if (hipEventSynchronize(c->plan_done) != hipSuccess) return TDES_ERR_HIP;
        if (hipEventSynchronize(c->staging_free) != hipSuccess) return TDES_ERR_HIP;
        // The captured graph points into the old buffer (and at the old slot offset, which
        // moves with the capacity even if the allocator returns the same address): drop it.
        if (c->exec) {
            (void)hipGraphExecDestroy(c->exec);
            c->exec = nullptr;
        }
        (void)hipFree(c->d_plan);
        (void)hipHostFree(c->h_plan);
        c->d_plan = c->h_plan = nullptr;
        c->have_plan = false;
    }
    const size_t bytes = plan_bytes(nt, ns);
    if (hipMalloc(&c->d_plan, bytes) != hipSuccess) { c->d_plan = nullptr; return TDES_ERR_NOMEM; }
    if (hipHostMalloc(&c->h_plan, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(c->d_plan);
        c->d_plan = c->h_plan = nullptr;
        return TDES_ERR_NOMEM;
    }
    c->cap_tiles = nt;
    c->cap_slots = ns;
    return TDES_OK;
}

struct Interval {
    uint64_t lo, hi;
    uint32_t job;
};

int validate_jobs(const tdes_job *jobs, uint32_t n_jobs, uint64_t n_scheds, uintptr_t base) {
    std::vector<Interval> outs;
    outs.reserve(n_jobs);
    for (uint32_t j = 0; j < n_jobs; j++) {
        const tdes_job &x = jobs[j];
        if (x.direction != TDES_ENCRYPT && x.direction != TDES_DECRYPT) return TDES_ERR_ARG;
        if (x.sched_idx >= n_scheds) return TDES_ERR_SIZE;
        if (x.n_blocks > kMaxJobBlocks) return TDES_ERR_SIZE;
        if (((base + x.in_off) | (base + x.out_off)) & 7) return TDES_ERR_ALIGN;
        if (x.n_blocks == 0) continue;
        const uint64_t bytes = x.n_blocks * 8;
        if (x.in_off + bytes < x.in_off || x.out_off + bytes < x.out_off) return TDES_ERR_SIZE;
        if (x.in_off != x.out_off && x.in_off < x.out_off + bytes && x.out_off < x.in_off + bytes)
            return TDES_ERR_OVERLAP;
        outs.push_back({x.out_off, x.out_off + bytes, j});
    }
    std::sort(outs.begin(), outs.end(), [](const Interval &a, const Interval &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); i++)
        if (outs[i].lo < outs[i - 1].hi) return TDES_ERR_OVERLAP;  // two outputs share bytes
    // No message may read bytes that another message writes.
    for (uint32_t j = 0; j < n_jobs; j++) {
        const tdes_job &x = jobs[j];
        if (x.n_blocks == 0) continue;
        const uint64_t lo = x.in_off, hi = x.in_off + x.n_blocks * 8;
        size_t k = std::upper_bound(outs.begin(), outs.end(), hi,
                                    [](uint64_t v, const Interval &iv) { return v <= iv.lo; }) -
                   outs.begin();
        while (k > 0) {
            const Interval &iv = outs[--k];
            if (iv.hi <= lo) break;
            if (iv.job != j) return TDES_ERR_OVERLAP;
        }
    }
    return TDES_OK;
}

// Fills the staging buffer; returns the tile and slot counts.
void plan_jobs(tdes_ctx *c, const tdes_job *jobs, uint32_t n_jobs, uint32_t *n_tiles_out, uint32_t *n_slots_out,
               tdes_batch_info *info) {
    std::vector<tdes::Slot> lane, wave;
    uint64_t blocks = 0;
    for (uint32_t j = 0; j < n_jobs; j++) {
        const tdes_job &x = jobs[j];
        const uint32_t ks_off = x.sched_idx * (TDES_SCHED_BYTES / 4) + x.direction * tdes::kDirWords;
        blocks += x.n_blocks;
        const uint64_t full = x.n_blocks / kWaveBlocks;
        const uint32_t rem = (uint32_t)(x.n_blocks % kWaveBlocks);
        for (uint64_t t = 0; t < full; t++)
            wave.push_back({x.in_off + t * kWaveBlocks * 8, x.out_off + t * kWaveBlocks * 8, kWaveBlocks, ks_off, 0});
        if (rem == 0) continue;
        const uint64_t at = full * kWaveBlocks * 8;
        if (rem >= c->wave_remainder) {
            wave.push_back({x.in_off + at, x.out_off + at, rem, ks_off, 0});
            continue;
        }
        for (uint32_t s = 0; s < rem; s += kLaneBlocks)
            lane.push_back({x.in_off + at + 8ull * s, x.out_off + at + 8ull * s, std::min(kLaneBlocks, rem - s),
                            ks_off, 0});
    }
    const uint32_t lane_tiles = (uint32_t)((lane.size() + kLanesPerTile - 1) / kLanesPerTile);
    lane.resize((size_t)lane_tiles * kLanesPerTile, tdes::Slot{0, 0, 0, 0, 0});  // idle lanes
    const uint32_t n_slots = (uint32_t)(lane.size() + wave.size());
    const uint32_t n_tiles = lane_tiles + (uint32_t)wave.size();
    // Callers have made room: ensure_capacity ran with upper bounds.
    tdes::PlanHeader *hdr = reinterpret_cast<tdes::PlanHeader *>(c->h_plan);
    uint32_t *tiles = reinterpret_cast<uint32_t *>(c->h_plan + 256);
    tdes::Slot *slots = reinterpret_cast<tdes::Slot *>(c->h_plan + slots_offset(c->cap_tiles));
    memset(hdr, 0, sizeof *hdr);
    hdr->n_tiles = n_tiles;
    hdr->n_slots = n_slots;
    for (uint32_t t = 0; t < lane_tiles; t++) tiles[t] = (t * kLanesPerTile) | tdes::kLaneTileBit;
    for (size_t w = 0; w < wave.size(); w++) tiles[lane_tiles + w] = (uint32_t)(lane.size() + w);
    if (!lane.empty()) memcpy(slots, lane.data(), lane.size() * sizeof(tdes::Slot));
    if (!wave.empty()) memcpy(slots + lane.size(), wave.data(), wave.size() * sizeof(tdes::Slot));
    *n_tiles_out = n_tiles;
    *n_slots_out = n_slots;
    info->tiles = n_tiles;
    info->wave_tiles = wave.size();
    info->lane_tiles = lane_tiles;
    info->slots = n_slots;
    info->blocks = blocks;
    info->padded_blocks = (uint64_t)n_tiles * kWaveBlocks;
}

// Upper bounds of tiles and slots for capacity, before planning.
void count_bounds(const tdes_job *jobs, uint32_t n_jobs, uint32_t wave_remainder, size_t *tiles, size_t *slots) {
    size_t wave = 0, lane = 0;
    for (uint32_t j = 0; j < n_jobs; j++) {
        const uint64_t n = jobs[j].n_blocks;
        const uint32_t rem = (uint32_t)(n % kWaveBlocks);
        wave += n / kWaveBlocks + (rem >= wave_remainder ? 1 : 0);
        if (rem && rem < wave_remainder) lane += (rem + kLaneBlocks - 1) / kLaneBlocks;
    }
    const size_t lane_tiles = (lane + kLanesPerTile - 1) / kLanesPerTile;
    *tiles = wave + lane_tiles;
    *slots = wave + lane_tiles * kLanesPerTile;
}

int launch_plan(tdes_ctx *c, const void *sched, uint8_t *base, bool use_graph, hipStream_t stream) {
    const uint32_t grid = (uint32_t)c->cu_count * c->groups_per_cu;
    const tdes::PlanHeader *hdr = reinterpret_cast<const tdes::PlanHeader *>(c->d_plan);
    const uint32_t *tiles = reinterpret_cast<const uint32_t *>(c->d_plan + 256);
    const tdes::Slot *slots = reinterpret_cast<const tdes::Slot *>(c->d_plan + slots_offset(c->cap_tiles));
    const uint32_t *ks = static_cast<const uint32_t *>(sched);
    if (!use_graph) {
        if (tdes::launch_batch(ks, hdr, tiles, slots, c->d_counter, base, grid, c->threads, c->tiles_per_draw,
                               c->capped, stream) != hipSuccess)
            return TDES_ERR_HIP;
    } else {
        if (!c->exec || c->g_sched != sched || c->g_base != base || c->g_tiles != tiles || c->g_slots != slots ||
            c->g_grid != grid || c->g_threads != c->threads || c->g_draw != c->tiles_per_draw ||
            c->g_capped != c->capped) {
            if (c->exec) {
                (void)hipGraphExecDestroy(c->exec);
                c->exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return TDES_ERR_HIP;
            const hipError_t le = tdes::launch_batch(ks, hdr, tiles, slots, c->d_counter, base, grid, c->threads,
                                                     c->tiles_per_draw, c->capped, c->capture_stream);
            const hipError_t ce = hipStreamEndCapture(c->capture_stream, &graph);
            if (le != hipSuccess || ce != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return TDES_ERR_HIP;
            }
            const hipError_t ie = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                c->exec = nullptr;
                return TDES_ERR_HIP;
            }
            c->g_sched = sched;
            c->g_base = base;
            c->g_tiles = tiles;
            c->g_slots = slots;
            c->g_grid = grid;
            c->g_threads = c->threads;
            c->g_draw = c->tiles_per_draw;
            c->g_capped = c->capped;
            c->info.graph_captures++;
        }
        if (hipGraphLaunch(c->exec, stream) != hipSuccess) return TDES_ERR_HIP;
    }
    if (hipEventRecord(c->plan_done, stream) != hipSuccess) return TDES_ERR_HIP;
    return TDES_OK;
}

}  // namespace

extern "C" int tdes_ctx_create(tdes_ctx **out, int device) {
    if (!out) return TDES_ERR_NULL;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess) return TDES_ERR_HIP;
    if (device >= n_dev) return TDES_ERR_ARG;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return TDES_ERR_HIP;
    tdes::DeviceGuard guard(device);
    if (!guard.ok()) return TDES_ERR_HIP;
    tdes::DeviceInfo dinfo;
    if (tdes::device_info(&dinfo) != TDES_OK) return TDES_ERR_HIP;
    tdes_ctx *c = new (std::nothrow) tdes_ctx;
    if (!c) return TDES_ERR_NOMEM;
    c->device = dinfo.device;
    c->cu_count = dinfo.cu_count;
    bool ok = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->staging_free, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->plan_done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&c->d_counter, 256) == hipSuccess && hipMemset(c->d_counter, 0, 256) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        tdes_ctx_destroy(c);
        return TDES_ERR_HIP;
    }
    c->info.threads = c->threads;
    c->info.groups_per_cu = c->groups_per_cu;
    c->info.wave_remainder = c->wave_remainder;
    c->info.tiles_per_draw = c->tiles_per_draw;
    *out = c;
    return TDES_OK;
}

extern "C" int tdes_ctx_destroy(tdes_ctx *c) {
    if (!c) return TDES_OK;
    tdes::DeviceGuard guard(c->device);
    if (c->plan_done) (void)hipEventSynchronize(c->plan_done);
    if (c->staging_free) (void)hipEventSynchronize(c->staging_free);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->d_plan) (void)hipFree(c->d_plan);
    if (c->h_plan) (void)hipHostFree(c->h_plan);
    if (c->d_counter) (void)hipFree(c->d_counter);
    if (c->staging_free) (void)hipEventDestroy(c->staging_free);
    if (c->plan_done) (void)hipEventDestroy(c->plan_done);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
    return TDES_OK;
}

extern "C" int tdes_ctx_set_tuning(tdes_ctx *c, uint32_t threads, uint32_t groups_per_cu, uint32_t wave_remainder,
                                   uint32_t tiles_per_draw) {
    if (!c) return TDES_ERR_NULL;
    if (threads == 0 || threads > 256 || threads % 64 != 0 || groups_per_cu == 0 || groups_per_cu > 64)
        return TDES_ERR_ARG;
    if (wave_remainder > kWaveBlocks || tiles_per_draw > kMaxTilesPerDraw) return TDES_ERR_ARG;
    c->threads = threads;
    c->groups_per_cu = groups_per_cu;
    c->wave_remainder = wave_remainder ? wave_remainder : kDefaultWaveRemainder;
    c->tiles_per_draw = tiles_per_draw ? tiles_per_draw : 1;
    c->info.threads = threads;
    c->info.groups_per_cu = groups_per_cu;
    c->info.wave_remainder = c->wave_remainder;
    c->info.tiles_per_draw = c->tiles_per_draw;
    return TDES_OK;
}

namespace tdes {
void ctx_set_capped(tdes_ctx *c, bool capped) { c->capped = capped; }
}  // namespace tdes

extern "C" int tdes_ctx_get_info(const tdes_ctx *c, tdes_batch_info *info) {
    if (!c || !info) return TDES_ERR_NULL;
    *info = c->info;
    return TDES_OK;
}

extern "C" int tdes_ecb_batch(tdes_ctx *c, const tdes_job *jobs, uint32_t n_jobs, const void *dev_sched_table,
                              uint64_t n_scheds, void *dev_base, uint32_t flags, void *stream) {
    if (!c) return TDES_ERR_NULL;
    if (n_jobs == 0) return TDES_OK;
    if (!jobs || !dev_sched_table || !dev_base) return TDES_ERR_NULL;
    if (flags & ~(TDES_BATCH_NO_GRAPH | TDES_BATCH_PER_MESSAGE)) return TDES_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(dev_sched_table) & 3) != 0) return TDES_ERR_ALIGN;
    if (n_scheds == 0 || n_scheds > (1ull << 32) / (TDES_SCHED_BYTES / 4)) return TDES_ERR_SIZE;
    int rc = validate_jobs(jobs, n_jobs, n_scheds, reinterpret_cast<uintptr_t>(dev_base));
    if (rc != TDES_OK) return rc;
    tdes::DeviceGuard guard(c->device);
    if (!guard.ok()) return TDES_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(dev_base);
    const uint32_t *table = static_cast<const uint32_t *>(dev_sched_table);

    if (flags & TDES_BATCH_PER_MESSAGE) {
        // The baseline: one plain launch per message, in order, on the stream.
        for (uint32_t j = 0; j < n_jobs; j++) {
            const tdes_job &x = jobs[j];
            if (x.n_blocks == 0) continue;
            const uint32_t *ks = table + x.sched_idx * (TDES_SCHED_BYTES / 4) + x.direction * tdes::kDirWords;
            if (tdes::launch_auto(ks, base + x.in_off, base + x.out_off, x.n_blocks, s) != hipSuccess)
                return TDES_ERR_HIP;
        }
        return TDES_OK;
    }

    size_t max_tiles, max_slots;
    count_bounds(jobs, n_jobs, c->wave_remainder, &max_tiles, &max_slots);
    if (max_tiles >= (size_t)tdes::kLaneTileBit || max_slots >= (size_t)tdes::kLaneTileBit) return TDES_ERR_SIZE;
    rc = ensure_capacity(c, max_tiles, max_slots);
    if (rc != TDES_OK) return rc;
    // The staging buffer must not change under a previous upload.
    if (hipEventSynchronize(c->staging_free) != hipSuccess) return TDES_ERR_HIP;
    uint32_t n_tiles = 0, n_slots = 0;
    plan_jobs(c, jobs, n_jobs, &n_tiles, &n_slots, &c->info);
    // A previous launch on another stream may still read the device plan.
    if (hipStreamWaitEvent(s, c->plan_done, 0) != hipSuccess) return TDES_ERR_HIP;
    const size_t so = slots_offset(c->cap_tiles);
    if (hipMemcpyAsync(c->d_plan, c->h_plan, 256 + (size_t)n_tiles * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->d_plan + so, c->h_plan + so, (size_t)n_slots * sizeof(tdes::Slot), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipEventRecord(c->staging_free, s) != hipSuccess)
        return TDES_ERR_HIP;
    c->have_plan = true;
    c->last_sched = dev_sched_table;
    c->last_base = base;
    c->last_tiles = n_tiles;
    if (n_tiles == 0) return TDES_OK;
    return launch_plan(c, dev_sched_table, base, !(flags & TDES_BATCH_NO_GRAPH), s);
}

extern "C" int tdes_ecb_batch_replay(tdes_ctx *c, uint32_t flags, void *stream) {
    if (!c) return TDES_ERR_NULL;
    if (flags & ~TDES_BATCH_NO_GRAPH) return TDES_ERR_ARG;
    if (!c->have_plan) return TDES_ERR_STATE;
    if (c->last_tiles == 0) return TDES_OK;
    tdes::DeviceGuard guard(c->device);
    if (!guard.ok()) return TDES_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Order after the plan's upload and the previous launch, whichever streams they ran on.
    if (hipStreamWaitEvent(s, c->staging_free, 0) != hipSuccess || hipStreamWaitEvent(s, c->plan_done, 0) != hipSuccess)
        return TDES_ERR_HIP;
    return launch_plan(c, c->last_sched, c->last_base, !(flags & TDES_BATCH_NO_GRAPH), s);
}
