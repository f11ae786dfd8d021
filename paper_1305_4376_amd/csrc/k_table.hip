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

constexpr int kDefaultThreads = 256;
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

// Sixteen rounds on kN blocks side by side (independent chains the scheduler
// interleaves); x[i] holds L0 and y[i] R0 of block i on entry, L16 and R16 on exit.
template <int kN>
__device__ __forceinline__ void round_pair(uint32_t (&x)[kN], uint32_t (&y)[kN], const uint32_t *__restrict__ ks, int r,
                                           const uint8_t *lds, uint32_t lane4) {
    const uint32_t ka = ks[2 * r], kb = ks[2 * r + 1];
#pragma unroll
    for (int i = 0; i < kN; i++) x[i] = feistel(x[i], y[i], ka, kb, lds, lane4);
    const uint32_t ka2 = ks[2 * r + 2], kb2 = ks[2 * r + 3];
#pragma unroll
    for (int i = 0; i < kN; i++) y[i] = feistel(y[i], x[i], ka2, kb2, lds, lane4);
}

// kWritten: the stage written out, so that its 32 key words come in with a few wide scalar loads
// ahead of the rounds instead of a load and its wait before every pair.  Used with one block per
// lane (short messages, where the dependent rounds are the kernel's time): kernel time 7.28 -> 6.44 us
// on 2^13 blocks and 8.04 -> 7.92 us on 2^17 (medians of 180 launches each); with two blocks per
// lane it was slower.
template <int kN, bool kWritten>
__device__ __forceinline__ void des_stage(uint32_t (&x)[kN], uint32_t (&y)[kN], const uint32_t *__restrict__ ks,
                                          const uint8_t *lds, uint32_t lane4) {
    if constexpr (kWritten) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) round_pair<kN>(x, y, ks, r, lds, lane4);
    } else {
#pragma unroll 1
        for (int r = 0; r < 16; r += 2) round_pair<kN>(x, y, ks, r, lds, lane4);
    }
}

// kN blocks of one lane, block i as the little-endian words (w[2i], w[2i+1]) as loaded.
template <int kN, bool kWritten = (kN == 1)>
__device__ __forceinline__ void tdes_blocks(uint32_t (&w)[2 * kN], const uint32_t *__restrict__ ks,
                                            const uint8_t *lds, uint32_t lane4) {
    uint32_t l[kN], r[kN];
#pragma unroll
    for (int i = 0; i < kN; i++) {
        l[i] = __builtin_bswap32(w[2 * i]);
        r[i] = __builtin_bswap32(w[2 * i + 1]);
        initial_perm(l[i], r[i]);
        l[i] = rotl(l[i], 5);
        r[i] = rotl(r[i], 5);
    }
    des_stage<kN, kWritten>(l, r, ks, lds, lane4);       // stage 1: L0 = l, R0 = r
    des_stage<kN, kWritten>(r, l, ks + 32, lds, lane4);  // stage 2: halves swapped (IP^-1 then IP cancel)
    des_stage<kN, kWritten>(l, r, ks + 64, lds, lane4);  // stage 3
#pragma unroll
    for (int i = 0; i < kN; i++) {
        // Preoutput R16 L16 = (r, l).
        l[i] = rotl(l[i], 27);
        r[i] = rotl(r[i], 27);
        final_perm(r[i], l[i]);
        w[2 * i] = __builtin_bswap32(r[i]);
        w[2 * i + 1] = __builtin_bswap32(l[i]);
    }
}

// kPerLane blocks per lane per pass (2: one 16-byte access when kVec16; 1: an
// 8-byte access, twice the lanes for the same message, for short messages,
// where the 48 dependent rounds of one pass are the whole kernel time).  Each
// lane's first load is issued before the LDS table fill so that its memory
// latency overlaps the fill.
template <bool kVec16, int kThreads, int kPerLane>
__global__ __launch_bounds__(kThreads) void tdes_table_kernel(const uint32_t *__restrict__ ks, const uint8_t *in,
                                                              uint8_t *out, uint64_t n_blocks) {
    __shared__ uint4 lds4[8 * 64 * kCopies / 4];
    const uint64_t n_units = n_blocks / kPerLane;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint32_t w[2 * kPerLane];
    auto load = [&](uint64_t q) {
        if (kPerLane == 2 && kVec16) {
            const uint4 v = reinterpret_cast<const uint4 *>(in)[q];
            w[0] = v.x; w[1] = v.y; w[2 % (2 * kPerLane)] = v.z; w[3 % (2 * kPerLane)] = v.w;
        } else {
#pragma unroll
            for (int i = 0; i < kPerLane; i++) {
                const uint2 a = reinterpret_cast<const uint2 *>(in)[kPerLane * q + i];
                w[2 * i] = a.x;
                w[2 * i + 1] = a.y;
            }
        }
    };
    if (p < n_units) load(p);
    // 16-byte stores of four copies each, consecutive lanes on consecutive 16 bytes (no bank
    // conflicts); word w holds box 2 (w / 4096) + (w / 32) % 2, entry (w / 64) % 64.
#pragma unroll
    for (int i = 0; i < 8 * 64 * kCopies / 4 / kThreads; i++) {
        const int c = i * kThreads + threadIdx.x, wd = 4 * c;
        const uint32_t v = g_sp.v[2 * (wd / 4096) + (wd / 32) % 2][(wd / 64) % 64];
        lds4[c] = make_uint4(v, v, v, v);
    }
    __syncthreads();
    const uint8_t *lbase = reinterpret_cast<const uint8_t *>(lds4);
    const uint32_t lane4 = (threadIdx.x % kCopies) * 4;

    for (; p < n_units; p += stride) {
        tdes_blocks<kPerLane>(w, ks, lbase, lane4);
        if (kPerLane == 2 && kVec16) {
            reinterpret_cast<uint4 *>(out)[p] = make_uint4(w[0], w[1], w[2 % (2 * kPerLane)], w[3 % (2 * kPerLane)]);
        } else {
#pragma unroll
            for (int i = 0; i < kPerLane; i++)
                reinterpret_cast<uint2 *>(out)[kPerLane * p + i] = make_uint2(w[2 * i], w[2 * i + 1]);
        }
        if (p + stride < n_units) load(p + stride);
    }
    // An odd final block (two blocks per lane): the first lane of the grid takes it alone.
    if (kPerLane == 2 && (n_blocks & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint2 a = reinterpret_cast<const uint2 *>(in)[n_blocks - 1];
        uint32_t v[2] = {a.x, a.y};
        tdes_blocks<1, false>(v, ks, lbase, lane4);
        reinterpret_cast<uint2 *>(out)[n_blocks - 1] = make_uint2(v[0], v[1]);
    }
}

}  // namespace

namespace tdes {

hipError_t launch_table(const uint32_t *ks, const uint8_t *in, uint8_t *out, uint64_t n_blocks,
                        hipStream_t stream, uint32_t threads) {
    DeviceInfo info;
    if (device_info(&info) != TDES_OK) return hipErrorInvalidDevice;
    if (threads == 0) threads = kDefaultThreads;
    // 64 KiB of LDS per workgroup: two per CU (the compiler fits the registers of every size to that)
    const uint64_t resident = (uint64_t)info.cu_count * 2;
    // One block per lane while one pass of the resident grid covers the message, else two.
    const int per_lane = n_blocks <= resident * threads ? 1 : 2;
    const uint64_t units = n_blocks / per_lane;
    uint64_t grid = (units + threads - 1) / threads;
    if (grid > resident) grid = resident;
    if (grid == 0) grid = 1;
    const bool vec16 = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, stream, ks, in, out, n_blocks);
        return hipGetLastError();
    };
#define TDES_TABLE_CASE(T)                                                              \
    case T:                                                                             \
        if (per_lane == 1) return go(tdes_table_kernel<false, T, 1>);                   \
        return vec16 ? go(tdes_table_kernel<true, T, 2>) : go(tdes_table_kernel<false, T, 2>);
    switch (threads) {
        TDES_TABLE_CASE(64)
        TDES_TABLE_CASE(128)
        TDES_TABLE_CASE(256)
        TDES_TABLE_CASE(512)
        TDES_TABLE_CASE(1024)
        default: return hipErrorInvalidValue;
    }
#undef TDES_TABLE_CASE
}

}  // namespace tdes
