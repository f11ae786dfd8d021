// k_table.hip -- Triple-DES ECB, table variant: combined S-box/P lookups in LDS.
//
// Work: one lane owns two adjacent blocks (one 16-byte load, one 16-byte
// store, so a wave touches 1 KiB of contiguous memory per access).  Each
// block goes through IP, the 48 Feistel rounds of E-D-E and IP^-1 (the
// paper's one-thread-per-block mapping of an ECB message, Abstract and
// Listing 1.1; the cipher steps are the standard's).
//
// Round function.  f(R, K) = P(S(E(R) xor K)).  With R rotated left by 5 the
// inputs of boxes 1, 7, 5, 3 sit in bytes 0..3, and rotated by 9 those of
// boxes 2, 8, 6, 4: the key chunks are laid out to match, so E and the key
// XOR cost two XORs and one rotate.  S and P are folded into eight 64-entry
// tables SP[b][x] = P(S_b(x) in its output nibble); f is the XOR of eight
// lookups.  The state stays rotated by 5 through all 48 rounds, and the tables
// hold P's output rotated the same way.
//
// LDS layout.  A lookup index differs per lane, so one table copy would bank-
// conflict.  Each table entry is stored 32 times, copy c in bank c, and lane
// l reads copy l % 32, so the lanes of a half-wave always hit 32 different
// banks.  Entry x of box b, copy c, is at byte
//     (b / 2) * 16384 + x * 256 + (b % 2) * 128 + c * 4        (64 KiB in all).
// With the 6-bit index in byte 1 and c * 4 in byte 0, one byte permute
// (v_perm_b32) of the masked input word and a per-lane constant forms the
// whole address; the box's part is the instruction's immediate offset.  A
// round then costs one rotate, two XOR-and-mask operations, eight permutes,
// eight LDS reads and four three-way XORs (which also fold in L).
//
// IP and IP^-1.  IP is a transposition of the block's 8x8 bit matrix; it is
// done with five exchanges of bit groups between the two 32-bit halves (the
// network found by a search over such exchanges and checked bit-exact against
// the standard's IP table; FP runs the same exchanges in reverse order).
// Between the three DES stages IP^-1 followed by IP cancels, so only the
// swap of the halves remains.
#include <hip/hip_runtime.h>

#include "des_spec.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kCopies = 32;

constexpr uint32_t rotl32(uint32_t x, int n) { return n == 0 ? x : (x << n) | (x >> (32 - n)); }

struct SpTables {
    uint32_t v[8][64];
};

// SP[b][x]: f(R) word (bit 0 of f in bit 31) for box b's output S_b(x), rotated left by 5.
constexpr SpTables make_sp() {
    SpTables t{};
    for (int b = 0; b < 8; b++)
        for (uint32_t x = 0; x < 64; x++) {
            const uint32_t s = tdes_spec::sbox(b, x);
            uint32_t f = 0;
            for (int i = 0; i < 32; i++) {
                const int src = tdes_spec::kP[i];
                if (src / 4 == b) f |= ((s >> (3 - src % 4)) & 1u) << (31 - i);
            }
            t.v[b][x] = rotl32(f, 5);
        }
    return t;
}

__constant__ SpTables g_sp = make_sp();

__device__ __forceinline__ uint32_t rotl(uint32_t x, int n) {
    return __builtin_amdgcn_alignbit(x, x, (32 - n) & 31);
}

// Exchange bits (a >> n) & m with b & m.
__device__ __forceinline__ void exchange(uint32_t &a, uint32_t &b, int n, uint32_t m) {
    const uint32_t t = ((a >> n) ^ b) & m;
    b ^= t;
    a ^= t << n;
}

// IP on a block held as (hi, lo) = bits 0..31, 32..63 of the standard's numbering.
__device__ __forceinline__ void initial_perm(uint32_t &hi, uint32_t &lo) {
    exchange(hi, lo, 4, 0x0F0F0F0Fu);
    exchange(hi, lo, 16, 0x0000FFFFu);
    exchange(lo, hi, 2, 0x33333333u);
    exchange(lo, hi, 8, 0x00FF00FFu);
    exchange(hi, lo, 1, 0x55555555u);
}

__device__ __forceinline__ void final_perm(uint32_t &hi, uint32_t &lo) {
    exchange(hi, lo, 1, 0x55555555u);
    exchange(lo, hi, 8, 0x00FF00FFu);
    exchange(lo, hi, 2, 0x33333333u);
    exchange(hi, lo, 16, 0x0000FFFFu);
    exchange(hi, lo, 4, 0x0F0F0F0Fu);
}

// One round: returns L ^ f(R, K), all words rotated left by 5.  lane4 = (lane % 32) * 4.
__device__ __forceinline__ uint32_t feistel(uint32_t l5, uint32_t r5, uint32_t ka, uint32_t kb, const uint8_t *lds,
                                            uint32_t lane4) {
    constexpr uint32_t kMask = 0x3F3F3F3Fu;
    // (x ^ k) & m as one three-input operation (truth table of x, k, m: 0x28).
    const uint32_t a = __builtin_amdgcn_bitop3_b32(r5, ka, kMask, 0x28);           // boxes 1, 7, 5, 3
    const uint32_t b = __builtin_amdgcn_bitop3_b32(rotl(r5, 4), kb, kMask, 0x28);  // boxes 2, 8, 6, 4
    auto look = [&](int box, uint32_t word, int byte) {
        // byte 0 = lane4, byte 1 = index, bytes 2..3 = 0.
        const uint32_t addr = __builtin_amdgcn_perm(word, lane4, 0x0C0C0000u | ((4u + byte) << 8));
        return *reinterpret_cast<const uint32_t *>(lds + addr + (box / 2) * 16384 + (box % 2) * 128);
    };
    const uint32_t v0 = look(0, a, 0), v6 = look(6, a, 1), v4 = look(4, a, 2), v2 = look(2, a, 3);
    const uint32_t v1 = look(1, b, 0), v7 = look(7, b, 1), v5 = look(5, b, 2), v3 = look(3, b, 3);
    const uint32_t x0 = __builtin_amdgcn_bitop3_b32(v0, v6, v4, 0x96);
    const uint32_t x1 = __builtin_amdgcn_bitop3_b32(v2, v1, v7, 0x96);
    const uint32_t x2 = __builtin_amdgcn_bitop3_b32(l5, v5, v3, 0x96);
    return __builtin_amdgcn_bitop3_b32(x0, x1, x2, 0x96);
}

// Sixteen rounds; x holds L0 and y holds R0 on entry, L16 and R16 on exit.
__device__ __forceinline__ void des_stage(uint32_t &x0, uint32_t &y0, uint32_t &x1, uint32_t &y1,
                                          const uint32_t *__restrict__ ks, const uint8_t *lds,
                                          uint32_t lane4) {
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        const uint32_t ka = ks[2 * r], kb = ks[2 * r + 1];
        x0 = feistel(x0, y0, ka, kb, lds, lane4);
        x1 = feistel(x1, y1, ka, kb, lds, lane4);
        const uint32_t ka2 = ks[2 * r + 2], kb2 = ks[2 * r + 3];
        y0 = feistel(y0, x0, ka2, kb2, lds, lane4);
        y1 = feistel(y1, x1, ka2, kb2, lds, lane4);
    }
}

// One lane, two blocks (w0,w1) and (w2,w3) as loaded (little-endian words).
__device__ __forceinline__ void tdes_two_blocks(uint32_t &w0, uint32_t &w1, uint32_t &w2, uint32_t &w3,
                                                const uint32_t *__restrict__ ks, const uint8_t *lds,
                                                uint32_t lane4) {
    uint32_t l0 = __builtin_bswap32(w0), r0 = __builtin_bswap32(w1);
    uint32_t l1 = __builtin_bswap32(w2), r1 = __builtin_bswap32(w3);
    initial_perm(l0, r0);
    initial_perm(l1, r1);
    l0 = rotl(l0, 5); r0 = rotl(r0, 5); l1 = rotl(l1, 5); r1 = rotl(r1, 5);
    des_stage(l0, r0, l1, r1, ks, lds, lane4);            // stage 1: L0 = l, R0 = r
    des_stage(r0, l0, r1, l1, ks + 32, lds, lane4);       // stage 2: halves swapped (IP^-1 then IP cancel)
    des_stage(l0, r0, l1, r1, ks + 64, lds, lane4);       // stage 3
    // Preoutput R16 L16 = (r, l).
    l0 = rotl(l0, 27); r0 = rotl(r0, 27); l1 = rotl(l1, 27); r1 = rotl(r1, 27);
    final_perm(r0, l0);
    final_perm(r1, l1);
    w0 = __builtin_bswap32(r0); w1 = __builtin_bswap32(l0);
    w2 = __builtin_bswap32(r1); w3 = __builtin_bswap32(l1);
}

template <bool kVec16>
__global__ __launch_bounds__(kThreads) void tdes_table_kernel(const uint32_t *__restrict__ ks, const uint8_t *in,
                                                              uint8_t *out, uint64_t n_blocks) {
    __shared__ uint4 lds4[8 * 64 * kCopies / 4];
    // 16-byte stores of four copies each, consecutive lanes on consecutive 16 bytes (no bank
    // conflicts); word w holds box 2 (w / 4096) + (w / 32) % 2, entry (w / 64) % 64.
#pragma unroll
    for (int i = 0; i < 8 * 64 * kCopies / 4 / kThreads; i++) {
        const int c = i * kThreads + threadIdx.x, w = 4 * c;
        const uint32_t v = g_sp.v[2 * (w / 4096) + (w / 32) % 2][(w / 64) % 64];
        lds4[c] = make_uint4(v, v, v, v);
    }
    __syncthreads();
    const uint32_t *lds = reinterpret_cast<const uint32_t *>(lds4);
    const uint8_t *lbase = reinterpret_cast<const uint8_t *>(lds);
    const uint32_t lane4 = (threadIdx.x % kCopies) * 4;

    const uint64_t n_pairs = n_blocks / 2;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x; p < n_pairs; p += stride) {
        uint32_t w0, w1, w2, w3;
        if (kVec16) {
            const uint4 v = reinterpret_cast<const uint4 *>(in)[p];
            w0 = v.x; w1 = v.y; w2 = v.z; w3 = v.w;
        } else {
            const uint2 a = reinterpret_cast<const uint2 *>(in)[2 * p];
            const uint2 b = reinterpret_cast<const uint2 *>(in)[2 * p + 1];
            w0 = a.x; w1 = a.y; w2 = b.x; w3 = b.y;
        }
        tdes_two_blocks(w0, w1, w2, w3, ks, lbase, lane4);
        if (kVec16) {
            reinterpret_cast<uint4 *>(out)[p] = make_uint4(w0, w1, w2, w3);
        } else {
            reinterpret_cast<uint2 *>(out)[2 * p] = make_uint2(w0, w1);
            reinterpret_cast<uint2 *>(out)[2 * p + 1] = make_uint2(w2, w3);
        }
    }
    // An odd final block: the first lane of the grid takes it alone.
    if ((n_blocks & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint2 a = reinterpret_cast<const uint2 *>(in)[n_blocks - 1];
        uint32_t w0 = a.x, w1 = a.y, w2 = 0, w3 = 0;
        tdes_two_blocks(w0, w1, w2, w3, ks, lbase, lane4);
        reinterpret_cast<uint2 *>(out)[n_blocks - 1] = make_uint2(w0, w1);
    }
}

}  // namespace

namespace tdes {

hipError_t launch_table(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                        hipStream_t stream) {
    DeviceInfo info;
    if (device_info(&info) != TDES_OK) return hipErrorInvalidDevice;
    const uint64_t n_pairs = n_blocks / 2;
    uint64_t grid = (n_pairs + kThreads - 1) / kThreads;
    const uint64_t resident = (uint64_t)info.cu_count * 2;  // 64 KiB of LDS per workgroup
    if (grid > resident) grid = resident;
    if (grid == 0) grid = 1;
    const bool vec16 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (vec16)
        hipLaunchKernelGGL(tdes_table_kernel<true>, dim3((unsigned)grid), dim3(kThreads), 0, stream, ks, in, out,
                           n_blocks);
    else
        hipLaunchKernelGGL(tdes_table_kernel<false>, dim3((unsigned)grid), dim3(kThreads), 0, stream, ks, in, out,
                           n_blocks);
    return hipGetLastError();
}

}  // namespace tdes
