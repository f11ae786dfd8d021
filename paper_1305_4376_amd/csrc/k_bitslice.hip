// k_bitslice.hip -- Triple-DES ECB, bitsliced variant.
//
// The paper maps one 64-bit block to one GPU thread and notes that the cipher
// is almost entirely bit operations on integers (Abstract; Section IV).  Here a
// lane instead holds 32 blocks as 64 bit planes: plane f is a 32-bit word
// whose bit j is bit f of the lane's block j.  Then
//   - IP, E, P and IP^-1 are renamings of planes (no instructions);
//   - the subkey XOR is one XOR per S-box input plane with a wave-uniform
//     mask (0 or ~0) held in a scalar register;
//   - each S-box is a circuit of 3-input lookup gates (v_bitop3_b32) on whole
//     planes, generated offline from the standard's tables (sbox_circuits.inc),
//     that XORs its four outputs into the Feistel half;
//   - the block <-> plane conversion is an in-register 32x32 bit transpose of
//     each half of the 32 blocks (five exchange stages; the byte-sized ones
//     are single byte permutes).
// No lookup tables and no LDS are involved, so the cost per block is fixed and
// data-independent.
//
// Memory access: a wave owns a tile of 2048 consecutive blocks (16 KiB).  Lane
// l holds blocks 128k + 2l and 128k + 2l + 1 for k = 0..15, so each of the 16
// loads (and stores) is one 16-byte access per lane covering 1 KiB of
// contiguous memory across the wave.  A short final tile reads and writes
// only its valid blocks (8 bytes at a time).
#include <hip/hip_runtime.h>

#include "des_spec.h"
#include "internal.h"

namespace {

#include "sbox_circuits.inc"

constexpr int kThreads = 256;                // 4 waves per workgroup
constexpr int kLanes = 64;
constexpr int kTileBlocks = 32 * kLanes;     // blocks per wave tile

// ---- compile-time plane maps ----

// Transposed plane that holds block bit f (0-based, bit 0 = MSB of byte 0).
// Half h (bytes 4h..4h+3) is loaded as a little-endian word whose bit i is
// bit 7 - i % 8 of byte i / 8 of the half.
constexpr int plane_of_bit(int f) { return 32 * (f / 32) + 8 * ((f % 32) / 8) + 7 - f % 8; }

struct Maps {
    int l0[32], r0[32];   // plane of IP output bit k (L0, R0)
    int out_src[64];      // for plane p after FP: index into the preoutput R16 || L16 (0..63)
    int e[48];            // R bit feeding S-box input 6s+j
    int p_inv[32];        // f(R) bit receiving S-box output bit q
};

constexpr Maps make_maps() {
    Maps m{};
    for (int k = 0; k < 32; k++) {
        m.l0[k] = plane_of_bit(tdes_spec::ip(k));
        m.r0[k] = plane_of_bit(tdes_spec::ip(32 + k));
    }
    // FP = IP^-1: output bit ip(k) is preoutput bit k.
    for (int k = 0; k < 64; k++) m.out_src[plane_of_bit(tdes_spec::ip(k))] = k;
    for (int i = 0; i < 48; i++) m.e[i] = tdes_spec::expansion(i);
    for (int i = 0; i < 32; i++) m.p_inv[tdes_spec::kP[i]] = i;
    return m;
}

constexpr Maps kMaps = make_maps();

// Key chunk of S-box s sits in schedule word s % 2 at byte ((8 + s % 2 - s) % 8) / 2,
// its first bit at position 5 of the byte (the host layout of keysched.cpp).
constexpr int key_pos(int s, int j) { return 8 * (((8 + s % 2 - s) % 8) / 2) + 5 - j; }

// ---- bit transpose ----

// One exchange stage of the transpose: for rows j and j + S (j & S == 0), swap the
// bits of row j at positions i + S with those of row j + S at positions i, for the
// positions i selected by M.
template <int S, uint32_t M>
__device__ __forceinline__ void exchange_stage(uint32_t (&w)[32]) {
#pragma unroll
    for (int j = 0; j < 32; j++) {
        if (j & S) continue;
        const uint32_t a = w[j], b = w[j + S];
        w[j] = (a & M) | ((b << S) & ~M);
        w[j + S] = ((a >> S) & M) | (b & ~M);
    }
}

// In place: afterwards bit j of w[i] is what bit i of w[j] was.
__device__ __forceinline__ void transpose32(uint32_t (&w)[32]) {
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const uint32_t a = w[j], b = w[j + 16];
        w[j] = __builtin_amdgcn_perm(b, a, 0x05040100u);       // a.lo16 | b.lo16 << 16
        w[j + 16] = __builtin_amdgcn_perm(b, a, 0x07060302u);  // a.hi16 | b.hi16 << 16
    }
#pragma unroll
    for (int j = 0; j < 32; j++) {
        if (j & 8) continue;
        const uint32_t a = w[j], b = w[j + 8];
        w[j] = __builtin_amdgcn_perm(b, a, 0x06020400u);       // bytes a0 b0 a2 b2
        w[j + 8] = __builtin_amdgcn_perm(b, a, 0x07030501u);   // bytes a1 b1 a3 b3
    }
    exchange_stage<4, 0x0F0F0F0Fu>(w);
    exchange_stage<2, 0x33333333u>(w);
    exchange_stage<1, 0x55555555u>(w);
}

// ---- rounds ----

__device__ __forceinline__ uint32_t key_mask(uint32_t word, int pos) {
    return (uint32_t)((int32_t)(word << (31 - pos)) >> 31);
}

template <int S>
__device__ __forceinline__ void sbox_round(uint32_t (&l)[32], const uint32_t (&r)[32], uint32_t kw) {
    const uint32_t x0 = r[kMaps.e[6 * S + 0]] ^ key_mask(kw, key_pos(S, 0));
    const uint32_t x1 = r[kMaps.e[6 * S + 1]] ^ key_mask(kw, key_pos(S, 1));
    const uint32_t x2 = r[kMaps.e[6 * S + 2]] ^ key_mask(kw, key_pos(S, 2));
    const uint32_t x3 = r[kMaps.e[6 * S + 3]] ^ key_mask(kw, key_pos(S, 3));
    const uint32_t x4 = r[kMaps.e[6 * S + 4]] ^ key_mask(kw, key_pos(S, 4));
    const uint32_t x5 = r[kMaps.e[6 * S + 5]] ^ key_mask(kw, key_pos(S, 5));
    uint32_t &o0 = l[kMaps.p_inv[4 * S + 0]];
    uint32_t &o1 = l[kMaps.p_inv[4 * S + 1]];
    uint32_t &o2 = l[kMaps.p_inv[4 * S + 2]];
    uint32_t &o3 = l[kMaps.p_inv[4 * S + 3]];
    if constexpr (S == 0) sbox0(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 1) sbox1(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 2) sbox2(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 3) sbox3(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 4) sbox4(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 5) sbox5(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 6) sbox6(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
    if constexpr (S == 7) sbox7(x0, x1, x2, x3, x4, x5, o0, o1, o2, o3);
}

// L ^= f(R, K) for one round with schedule words (ka, kb).
__device__ __forceinline__ void feistel(uint32_t (&l)[32], const uint32_t (&r)[32], uint32_t ka, uint32_t kb) {
    sbox_round<0>(l, r, ka);
    sbox_round<1>(l, r, kb);
    sbox_round<2>(l, r, ka);
    sbox_round<3>(l, r, kb);
    sbox_round<4>(l, r, ka);
    sbox_round<5>(l, r, kb);
    sbox_round<6>(l, r, ka);
    sbox_round<7>(l, r, kb);
}

// Sixteen rounds: x holds L0 and y holds R0 on entry, L16 and R16 on exit.
__device__ __forceinline__ void des_stage(uint32_t (&x)[32], uint32_t (&y)[32], const uint32_t *__restrict__ ks) {
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        feistel(x, y, ks[2 * r], ks[2 * r + 1]);
        feistel(y, x, ks[2 * r + 2], ks[2 * r + 3]);
    }
}

// ---- kernel ----

// Loads the tile starting at `tin` (wave-uniform) into two 32-word halves.
// Full tiles use 16-byte accesses; a short tile (n_valid < 2048 blocks, or a
// buffer not 16-byte aligned) reads 8 bytes per block and clamps indices past
// the end to the last valid block, so every read stays inside the message.
template <bool kFull>
__device__ __forceinline__ void load_tile(const uint8_t *tin, uint32_t n_valid, int lane, uint32_t (&a)[32],
                                          uint32_t (&b)[32]) {
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (kFull) {
            const uint4 v = *reinterpret_cast<const uint4 *>(tin + 1024 * k + 16 * lane);
            a[2 * k] = v.x; b[2 * k] = v.y; a[2 * k + 1] = v.z; b[2 * k + 1] = v.w;
        } else {
            const uint32_t j = 128 * k + 2 * lane;
            const uint32_t j0 = j < n_valid ? j : n_valid - 1;
            const uint32_t j1 = j + 1 < n_valid ? j + 1 : n_valid - 1;
            const uint2 v0 = *reinterpret_cast<const uint2 *>(tin + 8 * j0);
            const uint2 v1 = *reinterpret_cast<const uint2 *>(tin + 8 * j1);
            a[2 * k] = v0.x; b[2 * k] = v0.y; a[2 * k + 1] = v1.x; b[2 * k + 1] = v1.y;
        }
    }
}

// Stores only the tile's valid blocks.
template <bool kFull>
__device__ __forceinline__ void store_tile(uint8_t *tout, uint32_t n_valid, int lane, const uint32_t (&a)[32],
                                           const uint32_t (&b)[32]) {
#pragma unroll
    for (int k = 0; k < 16; k++) {
        if (kFull) {
            *reinterpret_cast<uint4 *>(tout + 1024 * k + 16 * lane) =
                make_uint4(a[2 * k], b[2 * k], a[2 * k + 1], b[2 * k + 1]);
        } else {
            const uint32_t j = 128 * k + 2 * lane;
            if (j < n_valid) *reinterpret_cast<uint2 *>(tout + 8 * j) = make_uint2(a[2 * k], b[2 * k]);
            if (j + 1 < n_valid) *reinterpret_cast<uint2 *>(tout + 8 * (j + 1)) = make_uint2(a[2 * k + 1], b[2 * k + 1]);
        }
    }
}

// The empty asm statements make the lane index opaque at each use, so the
// compiler recomputes per-block offsets instead of hoisting 32 of them out of
// the tile loop and keeping them live across the rounds.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

template <bool kFull>
__device__ __forceinline__ void tdes_tile(const uint32_t *__restrict__ ks, const uint8_t *tin, uint8_t *tout,
                                          uint32_t n_valid, int lane) {
    uint32_t a[32], b[32];
    load_tile<kFull>(tin, n_valid, opaque(lane), a, b);
    transpose32(a);
    transpose32(b);
    uint32_t l[32], r[32];
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int pl = kMaps.l0[k], pr = kMaps.r0[k];
        l[k] = pl < 32 ? a[pl] : b[pl - 32];
        r[k] = pr < 32 ? a[pr] : b[pr - 32];
    }
    des_stage(l, r, ks);        // E (or D) under the first key
    des_stage(r, l, ks + 32);   // IP^-1 then IP cancel: the halves swap
    des_stage(l, r, ks + 64);
    // Preoutput R16 || L16 = (r, l); FP is a renaming back to block bit planes.
#pragma unroll
    for (int p = 0; p < 64; p++) {
        const int q = kMaps.out_src[p];
        const uint32_t v = q < 32 ? r[q] : l[q - 32];
        if (p < 32) a[p] = v; else b[p - 32] = v;
    }
    transpose32(a);
    transpose32(b);
    store_tile<kFull>(tout, n_valid, opaque(lane), a, b);
}

__global__ __launch_bounds__(kThreads) void tdes_bitslice_kernel(const uint32_t *__restrict__ ks, const uint8_t *in,
                                                                 uint8_t *out, uint64_t n_blocks, int vec16) {
    const int lane = threadIdx.x % kLanes;
    const uint64_t tiles = (n_blocks + kTileBlocks - 1) / kTileBlocks;
    const uint64_t stride = (uint64_t)gridDim.x * (kThreads / kLanes);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    for (uint64_t tile = (uint64_t)blockIdx.x * (kThreads / kLanes) + wave; tile < tiles; tile += stride) {
        const uint64_t first = tile * kTileBlocks;
        const uint64_t left = n_blocks - first;
        const uint32_t n_valid = left < kTileBlocks ? (uint32_t)left : kTileBlocks;
        if (vec16 && n_valid == kTileBlocks)
            tdes_tile<true>(ks, in + 8 * first, out + 8 * first, n_valid, lane);
        else
            tdes_tile<false>(ks, in + 8 * first, out + 8 * first, n_valid, lane);
    }
}

}  // namespace

namespace tdes {

hipError_t launch_bitslice(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                           hipStream_t stream) {
    const uint64_t tiles = (n_blocks + kTileBlocks - 1) / kTileBlocks;
    uint64_t grid = (tiles + kThreads / kLanes - 1) / (kThreads / kLanes);
    if (grid > (1u << 20)) grid = 1u << 20;  // larger messages loop over tiles
    const int vec16 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    hipLaunchKernelGGL(tdes_bitslice_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, ks, in, out, n_blocks,
                       vec16);
    return hipGetLastError();
}

}  // namespace tdes
