// k_util.hip -- device-side synthetic data (messages and serving payloads made in place in HBM).
//
// Word i of the SplitMix64 stream seeded with s is mix(s + (i + 1) * 0x9E3779B97F4A7C15),
// the SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

constexpr int kThreads = 256;

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// The output function applied to the state s + (i + 1) * gamma of word i.
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each thread walks its words with a fixed stride, so the state advances by stride * gamma (one
// addition instead of a 64-bit multiplication per word).
__global__ __launch_bounds__(kThreads) void fill_kernel(uint64_t *dev, uint64_t n, uint64_t seed, uint64_t first) {
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint64_t z = seed + (first + i + 1) * kGamma;
    const uint64_t step = stride * kGamma;
    for (; i < n; i += stride, z += step) dev[i] = splitmix64_mix(z);
}

}  // namespace

namespace tdes {

hipError_t launch_fill_splitmix64(uint64_t *dev, uint64_t n_words, uint64_t seed, uint64_t first,
                                  hipStream_t stream) {
    DeviceInfo info;
    if (device_info(&info) != TDES_OK) return hipErrorInvalidDevice;
    uint64_t grid = (n_words + kThreads - 1) / kThreads;
    const uint64_t cap = (uint64_t)info.cu_count * 16;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, dev, n_words, seed, first);
    return hipGetLastError();
}

}  // namespace tdes

// ---- batched fill: the serving payloads, many buffers, one stream each ----
//
// Payload word i, with i = 256 * (64 * c + k) + t (column t < 256, chain c, step k < 64), is
// X^k(W), where W is SplitMix64 word 16384 * c + t of the request's stream and X the xorshift64
// step x ^= x << 13, x ^= x >> 7, x ^= x << 17 (Marsaglia, J. Stat. Softw. 8(14), 2003): one
// 64-bit mix (two 64-bit multiplications) per 64 words, three shifts and XORs for the others.

namespace {

constexpr int kFillThreads = 256;
constexpr uint32_t kChainSteps = 64;
static_assert(tdes::kFillTileWords % (kFillThreads * kChainSteps) == 0, "a tile holds whole chains");

__device__ __forceinline__ uint64_t xorshift64(uint64_t x) {
    x ^= x << 13;
    x ^= x >> 7;
    return x ^ (x << 17);
}

// One workgroup per tile; a tile starts at a multiple of 256 * 64 words of its request, so each
// thread's words t, t + 256, ... run along its columns' chains from their heads.
__global__ __launch_bounds__(kFillThreads) void fill_tiles_kernel(const tdes::FillTile *__restrict__ tiles,
                                                                  uint32_t n_tiles, uint8_t *base) {
    if (blockIdx.x >= n_tiles) return;
    const tdes::FillTile t = tiles[blockIdx.x];
    uint64_t *dst = reinterpret_cast<uint64_t *>(base + t.dst_off);
    uint64_t z = t.seed + (t.first_word + threadIdx.x + 1) * kGamma;
    for (uint32_t head = threadIdx.x; head < t.n_words; head += kFillThreads * kChainSteps) {
        uint64_t x = splitmix64_mix(z);
        z += kFillThreads * kChainSteps * kGamma;
        const uint32_t rows = (t.n_words - head + kFillThreads - 1) / kFillThreads;
        const uint32_t steps = rows < kChainSteps ? rows : kChainSteps;
        for (uint32_t k = 0; k < steps; k++, x = xorshift64(x)) dst[head + k * kFillThreads] = x;
    }
}

}  // namespace

namespace tdes {

hipError_t launch_fill_tiles(const FillTile *tiles, uint32_t n_tiles, uint8_t *base, hipStream_t stream) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_tiles_kernel, dim3(n_tiles), dim3(kFillThreads), 0, stream, tiles, n_tiles, base);
    return hipGetLastError();
}

}  // namespace tdes
