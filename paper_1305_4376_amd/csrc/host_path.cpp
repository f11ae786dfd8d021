// host_path.cpp -- ECB over a message in host memory: copies and kernels pipelined in chunks.
//
// The paper copies the whole message to the GPU once, runs every kernel, and
// copies the result back (Listing 1.1; Section II.B), leaving the transfers
// (10.4 s of its 20.4 s total for 512 MB, mostly disk) off the timed path
// (Section III).  Here the message stays in host memory and moves through three
// device slots: while chunk i is enciphered, chunk i+1 is copied in and chunk
// i-1 copied out, each on its own stream, so the rate is bounded by the host
// link rather than by the cipher.  Host buffers should be pinned
// (hipHostMalloc) for the copies to overlap; pageable memory works but the
// runtime then stages each copy synchronously.
#include <stdint.h>

#include "internal.h"

namespace {

constexpr int kSlots = 3;

struct Pipeline {
    hipStream_t in = nullptr, work = nullptr, out = nullptr;
    hipEvent_t loaded[kSlots] = {}, done[kSlots] = {}, freed[kSlots] = {};
    uint8_t *slot[kSlots] = {};

    int init(size_t slot_bytes) {
        if (hipStreamCreateWithFlags(&in, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&work, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&out, hipStreamNonBlocking) != hipSuccess)
            return TDES_ERR_HIP;
        for (int i = 0; i < kSlots; i++) {
            if (hipEventCreateWithFlags(&loaded[i], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&done[i], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&freed[i], hipEventDisableTiming) != hipSuccess)
                return TDES_ERR_HIP;
            if (hipMalloc(&slot[i], slot_bytes) != hipSuccess) return TDES_ERR_NOMEM;
        }
        return TDES_OK;
    }

    ~Pipeline() {
        for (hipStream_t s : {in, work, out})
            if (s) (void)hipStreamSynchronize(s);
        for (int i = 0; i < kSlots; i++) {
            if (slot[i]) (void)hipFree(slot[i]);
            for (hipEvent_t e : {loaded[i], done[i], freed[i]})
                if (e) (void)hipEventDestroy(e);
        }
        for (hipStream_t s : {in, work, out})
            if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

extern "C" int tdes_ecb_host(const void *dev_sched, const void *host_in, void *host_out, uint64_t n_blocks,
                             int direction, uint64_t chunk_blocks, void *stream) {
    if (n_blocks == 0) return TDES_OK;
    if (!dev_sched || !host_in || !host_out) return TDES_ERR_NULL;
    if ((reinterpret_cast<uintptr_t>(dev_sched) & 3) != 0) return TDES_ERR_ALIGN;
    if (direction != TDES_ENCRYPT && direction != TDES_DECRYPT) return TDES_ERR_ARG;
    if (chunk_blocks == 0 || chunk_blocks > (1ull << 31) || n_blocks > (1ull << 58)) return TDES_ERR_SIZE;
    const uintptr_t a = reinterpret_cast<uintptr_t>(host_in), b = reinterpret_cast<uintptr_t>(host_out);
    if (a != b && a < b + n_blocks * 8 && b < a + n_blocks * 8) return TDES_ERR_OVERLAP;
    if (chunk_blocks > n_blocks) chunk_blocks = n_blocks;
    hipStream_t caller = static_cast<hipStream_t>(stream);
    // Work queued on the caller's stream (e.g. the schedule upload) comes first.
    if (hipStreamSynchronize(caller) != hipSuccess) return TDES_ERR_HIP;

    Pipeline p;
    int rc = p.init(chunk_blocks * 8);
    if (rc != TDES_OK) return rc;
    const uint32_t *ks = static_cast<const uint32_t *>(dev_sched) + direction * tdes::kDirWords;
    const uint8_t *src = static_cast<const uint8_t *>(host_in);
    uint8_t *dst = static_cast<uint8_t *>(host_out);
    const uint64_t chunks = (n_blocks + chunk_blocks - 1) / chunk_blocks;
    for (uint64_t c = 0; c < chunks; c++) {
        const int s = (int)(c % kSlots);
        const uint64_t first = c * chunk_blocks;
        const uint64_t n = n_blocks - first < chunk_blocks ? n_blocks - first : chunk_blocks;
        // The slot is free once chunk c - kSlots has been copied out.
        if ((c >= kSlots && hipStreamWaitEvent(p.in, p.freed[s], 0) != hipSuccess) ||
            hipMemcpyAsync(p.slot[s], src + 8 * first, n * 8, hipMemcpyHostToDevice, p.in) != hipSuccess ||
            hipEventRecord(p.loaded[s], p.in) != hipSuccess || hipStreamWaitEvent(p.work, p.loaded[s], 0) != hipSuccess ||
            tdes::launch_bitslice(ks, p.slot[s], p.slot[s], n, p.work) != hipSuccess ||
            hipEventRecord(p.done[s], p.work) != hipSuccess || hipStreamWaitEvent(p.out, p.done[s], 0) != hipSuccess ||
            hipMemcpyAsync(dst + 8 * first, p.slot[s], n * 8, hipMemcpyDeviceToHost, p.out) != hipSuccess ||
            hipEventRecord(p.freed[s], p.out) != hipSuccess)
            return TDES_ERR_HIP;
    }
    if (hipStreamSynchronize(p.out) != hipSuccess) return TDES_ERR_HIP;
    return TDES_OK;
}
