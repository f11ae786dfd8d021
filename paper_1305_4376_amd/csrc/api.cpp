// api.cpp -- the C ABI entry points of libtdes: argument checks and dispatch to the kernels.
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "internal.h"

namespace tdes {

hipError_t launch_auto(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, hipStream_t stream) {
    return n_blocks < kAutoTableBelow ? launch_table(ks, in, out, n_blocks, stream)
                                      : launch_bitslice(ks, in, out, n_blocks, stream);
}

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_dev_once[kMaxDevices];
DeviceInfo g_dev[kMaxDevices];
int g_dev_status[kMaxDevices];
}  // namespace

int device_info(DeviceInfo *info) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TDES_ERR_HIP;
    std::call_once(g_dev_once[dev], [dev] {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
            g_dev_status[dev] = TDES_ERR_HIP;
            return;
        }
        g_dev[dev].cu_count = cus;
        g_dev[dev].device = dev;
        g_dev_status[dev] = TDES_OK;
    });
    if (g_dev_status[dev] != TDES_OK) return g_dev_status[dev];
    *info = g_dev[dev];
    return TDES_OK;
}

}  // namespace tdes

namespace {

constexpr uint64_t kMaxBlocks = 1ull << 58;

int check_buffers(const void *dev_sched, const void *in, const void *out, uint64_t n_blocks) {
    if (!dev_sched || !in || !out) return TDES_ERR_NULL;
    if ((reinterpret_cast<uintptr_t>(dev_sched) & 3) != 0) return TDES_ERR_ALIGN;
    if (((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 7) != 0) return TDES_ERR_ALIGN;
    if (n_blocks > kMaxBlocks) return TDES_ERR_SIZE;
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    const uint64_t bytes = n_blocks * 8;
    if (a != b && a < b + bytes && b < a + bytes) return TDES_ERR_OVERLAP;
    return TDES_OK;
}

// The automatic choice, on MI355X measurements of one launch (encrypt, HIP
// events around the launch): the bitsliced kernel costs about 36 us for
// anything up to 2^18 blocks (one wave runs a whole 2048-block tile through all
// 48 rounds) and then scales at about 900 GB/s; the table kernel costs 8-13 us
// up to 2^16 blocks (14 us at 2^18; the spread is the launch cost of different
// machines) and scales at about 260 GB/s.  At 2^20 blocks the bitsliced kernel
// is already ahead (39 vs 42 us).
int resolve_variant(int variant, uint64_t n_blocks) {
    if (variant == TDES_VARIANT_AUTO) return n_blocks < tdes::kAutoTableBelow ? TDES_VARIANT_TABLE : TDES_VARIANT_BITSLICE;
    return variant;
}

}  // namespace

extern "C" int tdes_ecb_run(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, int direction,
                            int variant, void *stream) {
    const int rc = check_buffers(dev_sched, in, out, n_blocks);
    if (rc != TDES_OK) return rc;
    if (direction != TDES_ENCRYPT && direction != TDES_DECRYPT) return TDES_ERR_ARG;
    if (variant != TDES_VARIANT_AUTO && variant != TDES_VARIANT_TABLE && variant != TDES_VARIANT_BITSLICE)
        return TDES_ERR_ARG;
    if (n_blocks == 0) return TDES_OK;
    const uint32_t *ks = static_cast<const uint32_t *>(dev_sched) + direction * tdes::kDirWords;
    const uint8_t *src = static_cast<const uint8_t *>(in);
    uint8_t *dst = static_cast<uint8_t *>(out);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t err;
    switch (resolve_variant(variant, n_blocks)) {
        case TDES_VARIANT_BITSLICE:
            err = tdes::launch_bitslice(ks, src, dst, n_blocks, s);
            break;
        default:
            err = tdes::launch_table(ks, src, dst, n_blocks, s);
            break;
    }
    return err == hipSuccess ? TDES_OK : TDES_ERR_HIP;
}

extern "C" int tdes_ecb_encrypt(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, void *stream) {
    return tdes_ecb_run(dev_sched, in, out, n_blocks, TDES_ENCRYPT, TDES_VARIANT_AUTO, stream);
}

extern "C" int tdes_ecb_decrypt(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, void *stream) {
    return tdes_ecb_run(dev_sched, in, out, n_blocks, TDES_DECRYPT, TDES_VARIANT_AUTO, stream);
}

extern "C" int tdes_ecb_chunked(const void *dev_sched, const void *in, void *out, uint64_t n_blocks,
                                uint64_t chunk_blocks, int direction, int variant, uint32_t threads, void *stream) {
    const int rc = check_buffers(dev_sched, in, out, n_blocks);
    if (rc != TDES_OK) return rc;
    if (direction != TDES_ENCRYPT && direction != TDES_DECRYPT) return TDES_ERR_ARG;
    if (variant != TDES_VARIANT_AUTO && variant != TDES_VARIANT_TABLE && variant != TDES_VARIANT_BITSLICE)
        return TDES_ERR_ARG;
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        return TDES_ERR_ARG;
    if (chunk_blocks == 0) return TDES_ERR_SIZE;
    const uint32_t *ks = static_cast<const uint32_t *>(dev_sched) + direction * tdes::kDirWords;
    const uint8_t *src = static_cast<const uint8_t *>(in);
    uint8_t *dst = static_cast<uint8_t *>(out);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (uint64_t first = 0; first < n_blocks; first += chunk_blocks) {
        const uint64_t n = n_blocks - first < chunk_blocks ? n_blocks - first : chunk_blocks;
        const hipError_t e = resolve_variant(variant, n) == TDES_VARIANT_BITSLICE
                                 ? tdes::launch_bitslice(ks, src + 8 * first, dst + 8 * first, n, s, threads)
                                 : tdes::launch_table(ks, src + 8 * first, dst + 8 * first, n, s, threads);
        if (e != hipSuccess) return TDES_ERR_HIP;
    }
    return TDES_OK;
}

namespace {

uint64_t iv_value(const uint8_t iv[8]) {
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v = (v << 8) | iv[i];
    return v;
}

}  // namespace

extern "C" int tdes_ctr_crypt(const void *dev_sched, const uint8_t iv[8], const void *in, void *out,
                              uint64_t n_blocks, void *stream) {
    if (!iv) return TDES_ERR_NULL;
    const int rc = check_buffers(dev_sched, in, out, n_blocks);
    if (rc != TDES_OK) return rc;
    if (n_blocks == 0) return TDES_OK;
    const uint32_t *ks = static_cast<const uint32_t *>(dev_sched) + TDES_ENCRYPT * tdes::kDirWords;
    return tdes::launch_ctr(ks, static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out), n_blocks, iv_value(iv),
                            static_cast<hipStream_t>(stream)) == hipSuccess
               ? TDES_OK
               : TDES_ERR_HIP;
}

extern "C" int tdes_cbc_decrypt(const void *dev_sched, const uint8_t iv[8], const void *in, void *out,
                                uint64_t n_blocks, void *stream) {
    if (!iv) return TDES_ERR_NULL;
    const int rc = check_buffers(dev_sched, in, out, n_blocks);
    if (rc != TDES_OK) return rc;
    // Every output block reads the ciphertext block before it, which another
    // wave may already have overwritten if the buffers are the same.
    if (n_blocks && in == out) return TDES_ERR_OVERLAP;
    if (n_blocks == 0) return TDES_OK;
    const uint32_t *ks = static_cast<const uint32_t *>(dev_sched) + TDES_DECRYPT * tdes::kDirWords;
    return tdes::launch_cbc_decrypt(ks, static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out), n_blocks,
                                    iv_value(iv), static_cast<hipStream_t>(stream)) == hipSuccess
               ? TDES_OK
               : TDES_ERR_HIP;
}

extern "C" int tdes_sched_upload(const tdes_sched *host, uint64_t count, void *dev_table, void *stream) {
    if (count == 0) return TDES_OK;
    if (!host || !dev_table) return TDES_ERR_NULL;
    if ((reinterpret_cast<uintptr_t>(dev_table) & 3) != 0) return TDES_ERR_ALIGN;
    if (count > (1ull << 40) / TDES_SCHED_BYTES) return TDES_ERR_SIZE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(dev_table, host, count * TDES_SCHED_BYTES, hipMemcpyHostToDevice, s) != hipSuccess)
        return TDES_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return TDES_ERR_HIP;
    return TDES_OK;
}

extern "C" int tdes_fill_splitmix64(void *dev, uint64_t n_words, uint64_t seed, uint64_t first, void *stream) {
    if (n_words == 0) return TDES_OK;
    if (!dev) return TDES_ERR_NULL;
    if ((reinterpret_cast<uintptr_t>(dev) & 7) != 0) return TDES_ERR_ALIGN;
    const hipError_t err =
        tdes::launch_fill_splitmix64(static_cast<uint64_t *>(dev), n_words, seed, first, static_cast<hipStream_t>(stream));
    return err == hipSuccess ? TDES_OK : TDES_ERR_HIP;
}

extern "C" const char *tdes_status_str(int status) {
    switch (status) {
        case TDES_OK: return "ok";
        case TDES_ERR_NULL: return "a required pointer is NULL";
        case TDES_ERR_ALIGN: return "a buffer is misaligned (blocks need 8 bytes, schedules 4)";
        case TDES_ERR_OVERLAP: return "input and output overlap without being equal";
        case TDES_ERR_SIZE: return "a size is out of range";
        case TDES_ERR_PARITY: return "a key byte does not have odd parity";
        case TDES_ERR_WEAKKEY: return "a key is a weak or semi-weak DES key";
        case TDES_ERR_ARG: return "an invalid flag, direction or variant";
        case TDES_ERR_HIP: return "a HIP runtime call or kernel launch failed";
        case TDES_ERR_NOMEM: return "out of memory";
        case TDES_ERR_BUDGET: return "the request can never fit in the memory budget";
        case TDES_ERR_STATE: return "call made in the wrong state";
        default: return "unknown status";
    }
}
