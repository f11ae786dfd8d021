// k_static.hip -- batched ECB that allocates nothing: tdes_ecb_batch_static.
//
// The same operation as tdes_ecb_batch (every message ECB-EDE'd on its own
// under its own key triple and direction, Abstract and Section II.A), for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  The job table is
// already in device memory, and the only working memory is one file-scope
// device array per GPU, `scratch`, whose address is looked up once per device
// with hipGetSymbolAddress and passed to the kernels from then on.
//
// Two launches on the caller's stream:
//   plan   -- one workgroup reads the jobs, rejects any that is malformed or
//             reaches outside [dev_base, dev_base + base_bytes) (it gets no
//             tiles), and writes the exclusive prefix sum of wave tiles (2048
//             blocks each) per job into scratch, the tile total, the number of
//             rejected jobs, and a zeroed tile counter;
//   cipher -- persistent waves draw tiles (the first by wave index, later
//             ones from the counter), find each tile's job by binary search
//             over the prefix sums and run the bitsliced core on it, with the
//             job's key masks in scalar registers.  A job's last tile may be
//             partial; it takes the core's per-block path.
// Nothing here carries state from one call to the next except scratch, which
// the plan launch rewrites before the cipher launch reads it.
#include <stdint.h>

#include <atomic>
#include <mutex>

#include "bitslice_core.h"
#include "internal.h"

namespace {

using namespace tdes_bs;

constexpr uint32_t kMaxJobs = TDES_STATIC_MAX_JOBS;
constexpr uint32_t kPlanThreads = 1024;
constexpr uint32_t kThreads = 256;
constexpr uint32_t kGroupsPerCU = 4;
constexpr uint64_t kMaxJobBlocks = 1ull << 40;

// scratch: [header, 256 B][tile_start: kMaxJobs + 1 words]
struct StaticHeader {
    uint32_t n_tiles;   // wave tiles of the call (0 if the total overflowed)
    uint32_t rejected;  // jobs given no tiles because they were malformed
    uint32_t pad0[30];
    uint32_t counter;   // tile draws after each wave's first (own 128-byte line)
    uint32_t pad1[31];
};
static_assert(sizeof(StaticHeader) == 256, "header is 256 bytes");
constexpr size_t kScratchBytes = sizeof(StaticHeader) + ((size_t)(kMaxJobs + 1) * 4 + 255) / 256 * 256;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

__device__ __forceinline__ bool job_ok(const tdes_job &x, uint64_t n_scheds, uint64_t base_bytes) {
    if (x.direction > TDES_DECRYPT || x.sched_idx >= n_scheds || x.n_blocks > kMaxJobBlocks) return false;
    if ((x.in_off | x.out_off) & 7) return false;
    const uint64_t bytes = 8 * x.n_blocks;
    if (x.in_off > base_bytes || bytes > base_bytes - x.in_off) return false;
    if (x.out_off > base_bytes || bytes > base_bytes - x.out_off) return false;
    // in place, or no shared byte between input and output
    return x.in_off == x.out_off || x.in_off >= x.out_off + bytes || x.out_off >= x.in_off + bytes;
}

__global__ __launch_bounds__(kPlanThreads) void tdes_static_plan_kernel(const tdes_job *__restrict__ jobs,
                                                                        uint32_t n_jobs, uint64_t n_scheds,
                                                                        uint64_t base_bytes, uint8_t *scr,
                                                                        uint32_t *dev_rejected) {
    __shared__ uint64_t part[kPlanThreads];
    __shared__ uint32_t bad_total;
    StaticHeader *hdr = reinterpret_cast<StaticHeader *>(scr);
    uint32_t *tile_start = reinterpret_cast<uint32_t *>(scr + sizeof(StaticHeader));
    const uint32_t tid = threadIdx.x;
    if (tid == 0) bad_total = 0;
    // thread tid plans jobs [lo, hi)
    const uint32_t per = (n_jobs + kPlanThreads - 1) / kPlanThreads;
    const uint32_t lo = min(n_jobs, tid * per), hi = min(n_jobs, lo + per);
    // first pass: each job's tile count (at most 2^29) into tile_start[j]
    uint64_t sum = 0;
    uint32_t bad = 0;
    for (uint32_t j = lo; j < hi; j++) {
        const tdes_job x = jobs[j];
        uint32_t t = 0;
        if (job_ok(x, n_scheds, base_bytes))
            t = (uint32_t)((x.n_blocks + kTileBlocks - 1) / kTileBlocks);
        else
            bad++;
        tile_start[j] = t;
        sum += t;
    }
    part[tid] = sum;
    __syncthreads();
    if (bad) atomicAdd(&bad_total, bad);
    // inclusive scan of part[] (Hillis-Steele)
    for (uint32_t d = 1; d < kPlanThreads; d <<= 1) {
        const uint64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint64_t total = part[kPlanThreads - 1];
    const bool overflow = total >= (1ull << 31);
    // second pass: counts to exclusive prefix sums, in place
    uint64_t run = part[tid] - sum;
    for (uint32_t j = lo; j < hi; j++) {
        const uint32_t t = tile_start[j];
        tile_start[j] = overflow ? 0 : (uint32_t)run;
        run += t;
    }
    if (tid == 0) {
        tile_start[n_jobs] = overflow ? 0 : (uint32_t)total;
        hdr->n_tiles = overflow ? 0 : (uint32_t)total;
        hdr->counter = 0;
    }
    __syncthreads();
    if (tid == 0) {
        const uint32_t rejected = overflow ? n_jobs : bad_total;
        hdr->rejected = rejected;
        if (dev_rejected) *dev_rejected = rejected;
    }
}

// A wave's tile after its first: n_waves + the counter's old value (none left at or past n_tiles).
__device__ __forceinline__ uint32_t next_ticket(uint32_t *counter, uint32_t n_waves, uint32_t lane) {
    uint32_t d = 0;
    if (lane == 0) d = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return n_waves + __builtin_amdgcn_readfirstlane(d);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(kThreads, kGroupsPerCU) void tdes_static_batch_kernel(
    const tdes_job *__restrict__ jobs, uint32_t n_jobs, const uint32_t *__restrict__ sched, uint8_t *scr,
    uint8_t *base) {
    StaticHeader *hdr = reinterpret_cast<StaticHeader *>(scr);
    const uint32_t *tile_start = reinterpret_cast<const uint32_t *>(scr + sizeof(StaticHeader));
    const uint32_t lane = threadIdx.x % kLanes;
    const uint32_t n_tiles = __builtin_amdgcn_readfirstlane(hdr->n_tiles);
    const uint32_t n_waves = gridDim.x * (blockDim.x / kLanes);
    const uint32_t wave_id = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kLanes) + threadIdx.x / kLanes);
    for (uint32_t ticket = wave_id; ticket < n_tiles; ticket = next_ticket(&hdr->counter, n_waves, lane)) {
        // the job j with tile_start[j] <= ticket < tile_start[j + 1] (tile_start[n_jobs] = n_tiles)
        uint32_t lo = 0, hi = n_jobs;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (__builtin_amdgcn_readfirstlane(tile_start[mid]) <= ticket)
                lo = mid;
            else
                hi = mid;
        }
        const tdes_job &x = jobs[lo];
        const uint64_t n_blocks = uniform64(x.n_blocks);
        const uint64_t first = (uint64_t)(ticket - __builtin_amdgcn_readfirstlane(tile_start[lo])) * kTileBlocks;
        const uint32_t count = (uint32_t)min((uint64_t)kTileBlocks, n_blocks - first);
        const uint32_t *ks = sched + (uint64_t)__builtin_amdgcn_readfirstlane(x.sched_idx) * (TDES_SCHED_BYTES / 4) +
                             __builtin_amdgcn_readfirstlane(x.direction) * tdes::kDirWords;
        const uint8_t *tin = base + uniform64(x.in_off) + 8 * first;
        uint8_t *tout = base + uniform64(x.out_off) + 8 * first;
        const bool full = count == kTileBlocks &&
                          ((reinterpret_cast<uintptr_t>(tin) | reinterpret_cast<uintptr_t>(tout)) & 15) == 0;
        if (full)
            wave_tile<true>(ks, tin, tout, kTileBlocks, lane);
        else
            wave_tile<false>(ks, tin, tout, count, lane);
    }
}

// scratch's device address on each GPU, looked up on the first call there.
constexpr int kMaxDevices = 64;
std::atomic<uint8_t *> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

int scratch_for(int device, uint8_t **out) {
    if (device < 0 || device >= kMaxDevices) return TDES_ERR_ARG;
    uint8_t *p = g_scratch[device].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch[device].load(std::memory_order_relaxed);
        if (!p) {
            // device is current: the address of this GPU's copy of the array
            if (hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch)) != hipSuccess || !p)
                return TDES_ERR_HIP;
            g_scratch[device].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return TDES_OK;
}

}  // namespace

extern "C" int tdes_ecb_batch_static(const tdes_job *dev_jobs, uint32_t n_jobs, const void *dev_sched_table,
                                     uint64_t n_scheds, void *dev_base, uint64_t base_bytes, uint32_t *dev_rejected,
                                     void *stream) {
    if (n_jobs == 0) return TDES_OK;
    if (!dev_jobs || !dev_sched_table || !dev_base) return TDES_ERR_NULL;
    if ((reinterpret_cast<uintptr_t>(dev_jobs) & 7) || (reinterpret_cast<uintptr_t>(dev_sched_table) & 3) ||
        (reinterpret_cast<uintptr_t>(dev_base) & 7) || (reinterpret_cast<uintptr_t>(dev_rejected) & 3))
        return TDES_ERR_ALIGN;
    if (n_jobs > kMaxJobs) return TDES_ERR_SIZE;
    if (n_scheds == 0 || n_scheds > (1ull << 32) / (TDES_SCHED_BYTES / 4)) return TDES_ERR_SIZE;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return TDES_ERR_HIP;
    uint8_t *scr = nullptr;
    int rc = scratch_for(device, &scr);
    if (rc != TDES_OK) return rc;
    tdes::DeviceInfo info;
    if (tdes::device_info(&info) != TDES_OK) return TDES_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(dev_base);
    hipLaunchKernelGGL(tdes_static_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, dev_jobs, n_jobs, n_scheds,
                       base_bytes, scr, dev_rejected);
    if (hipGetLastError() != hipSuccess) return TDES_ERR_HIP;
    hipLaunchKernelGGL(tdes_static_batch_kernel, dim3((uint32_t)info.cu_count * kGroupsPerCU), dim3(kThreads), 0, s,
                       dev_jobs, n_jobs, static_cast<const uint32_t *>(dev_sched_table), scr, base);
    return hipGetLastError() == hipSuccess ? TDES_OK : TDES_ERR_HIP;
}
