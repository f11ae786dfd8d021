// internal.h -- declarations shared by libtdes's translation units (not part of the ABI).
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "../../include/tdes.h"

namespace tdes {

// Words of a schedule: the encryption block, then the decryption block, each
// kDirWords long: its kRoundWords round words (round r uses words 2r, the key
// chunks of boxes 1,7,5,3, and 2r+1) followed by the folded key words of the
// bitsliced kernels (bitslice_maps.h).
constexpr int kRounds = 48;
constexpr int kRoundWords = 2 * kRounds;
constexpr int kDirWords = 200;
static_assert(kRoundWords + 104 <= kDirWords && 2 * kDirWords * 4 == TDES_SCHED_BYTES, "schedule layout");

// Per-device properties the launchers need (cached on first use).
struct DeviceInfo {
    int cu_count;
    int device;
};
int device_info(DeviceInfo *info);

// Makes `device` current for the lifetime of the guard and restores the
// caller's device afterwards (no-op when it already is current).
class DeviceGuard {
  public:
    explicit DeviceGuard(int device) {
        ok_ = hipGetDevice(&prev_) == hipSuccess;
        if (ok_ && prev_ != device) {
            ok_ = hipSetDevice(device) == hipSuccess;
            switched_ = ok_;
        }
    }
    ~DeviceGuard() {
        if (switched_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;

  private:
    int prev_ = 0;
    bool ok_ = false, switched_ = false;
};

// Kernel launchers.  Arguments are already validated; n_blocks > 0.
// `ks` points at the words of one direction.  threads: workgroup size, 0 for
// the kernel's own (256); otherwise 64, 128, 256, 512 or 1024
// (hipErrorInvalidValue for anything else).
hipError_t launch_table(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                        hipStream_t stream, uint32_t threads = 0);
hipError_t launch_bitslice(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                           hipStream_t stream, uint32_t threads = 0);
// TDES_VARIANT_AUTO: the table kernel below this many blocks, the bitsliced one from it on.
constexpr uint64_t kAutoTableBelow = 1ull << 20;
hipError_t launch_auto(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, hipStream_t stream);
// Block-parallel modes (bitsliced): ks is the encryption half for CTR and the
// decryption half for CBC decryption; iv is the 8 IV bytes read as a big-endian integer.
hipError_t launch_ctr(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, uint64_t iv,
                      hipStream_t stream);
hipError_t launch_cbc_decrypt(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks, uint64_t iv,
                              hipStream_t stream);
hipError_t launch_fill_splitmix64(uint64_t *dev, uint64_t n_words, uint64_t seed, uint64_t first,
                                  hipStream_t stream);

// Batch contexts of the server launch the 120-VGPR variant of the batch kernel, so that the
// payload fills of later steps run beside it.
void ctx_set_capped(tdes_ctx *c, bool capped);

// A run of serving-payload words (chained generator, k_util.hip) written to base + dst_off, one
// workgroup each; first_word is the run's first word in its request, a multiple of 16384.
struct FillTile {
    uint64_t dst_off;
    uint64_t seed;
    uint64_t first_word;
    uint32_t n_words;
    uint32_t pad;
};
constexpr uint32_t kFillTileWords = 1u << 18;
hipError_t launch_fill_tiles(const FillTile *tiles, uint32_t n_tiles, uint8_t *base, hipStream_t stream);

}  // namespace tdes
