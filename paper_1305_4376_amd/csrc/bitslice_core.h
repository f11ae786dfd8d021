// bitslice_core.h -- the bitsliced Triple-DES round core shared by the plain and batched kernels.
//
// A lane holds 32 blocks as 64 bit planes: plane f is a 32-bit word whose bit j
// is bit f of the lane's block j.  IP, E, P and IP^-1 are renamings of planes;
// the subkey XOR is one XOR per S-box input plane with a mask (0 or ~0) taken
// from the schedule word (a scalar register when the key is the same for the
// whole wave, a vector register when lanes use different keys); each S-box is
// a circuit of 3-input lookup gates (sbox_circuits.inc).  Blocks become planes
// by an in-register 32x32 bit transpose of each 4-byte half of the 32 blocks.
#pragma once
#include <hip/hip_runtime.h>

#include "des_spec.h"

namespace tdes_bs {

#include "sbox_circuits.inc"

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
    return (uint32_t)__builtin_amdgcn_sbfe((int32_t)word, pos, 1);  // bit pos of word as 0 or ~0
}

// Keeps the schedule word live in its register class at each use, so that the
// compiler extracts each key mask right before its XOR instead of hoisting all
// 48 masks of a round (which exhausts scalar registers, or vector registers
// when lanes have their own keys).
template <bool kLaneKeys>
__device__ __forceinline__ uint32_t key_word(uint32_t w) {
    if (kLaneKeys)
        asm volatile("" : "+v"(w));
    else
        asm volatile("" : "+s"(w));
    return w;
}

template <int S, bool kLaneKeys>
__device__ __forceinline__ void sbox_round(uint32_t (&l)[32], const uint32_t (&r)[32], uint32_t kw_in) {
    const uint32_t kw = key_word<kLaneKeys>(kw_in);
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
template <bool kLaneKeys>
__device__ __forceinline__ void feistel(uint32_t (&l)[32], const uint32_t (&r)[32], uint32_t ka, uint32_t kb) {
    sbox_round<0, kLaneKeys>(l, r, ka);
    sbox_round<1, kLaneKeys>(l, r, kb);
    sbox_round<2, kLaneKeys>(l, r, ka);
    sbox_round<3, kLaneKeys>(l, r, kb);
    sbox_round<4, kLaneKeys>(l, r, ka);
    sbox_round<5, kLaneKeys>(l, r, kb);
    sbox_round<6, kLaneKeys>(l, r, ka);
    sbox_round<7, kLaneKeys>(l, r, kb);
}

// Sixteen rounds: x holds L0 and y holds R0 on entry, L16 and R16 on exit.
template <bool kLaneKeys>
__device__ __forceinline__ void des_stage(uint32_t (&x)[32], uint32_t (&y)[32], const uint32_t *__restrict__ ks) {
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        feistel<kLaneKeys>(x, y, ks[2 * r], ks[2 * r + 1]);
        feistel<kLaneKeys>(y, x, ks[2 * r + 2], ks[2 * r + 3]);
    }
}

// ---- kernel ----

// ---- rounds with folded key masks (one key for the whole wave) ----
//
// Between rounds, every plane of a half is kept XORed with the key bit that the
// next round reading it applies at the plane's first E position.  Then
//   - the first E use of a plane needs no key XOR;
//   - a second E use (16 of the 32 bits are read twice) needs one XOR with the
//     difference of its two key bits;
//   - XORing an S-box output into the target half also swaps that half's
//     folded key from round r-1's to round r+1's: one three-way XOR with the
//     mask of (k[r-1] ^ k[r+1]), replacing the plain XOR of the output.
// Each DES stage starts with both halves clean (the half read first gets round
// 0's key folded in) and ends clean (the half read last has round 15's key
// removed): 64 XORs per stage against 32 saved per round.

struct UseMaps {
    int first[32];   // first S-box input position (0..47) reading R bit q
    int second[32];  // second one, or -1
};

constexpr UseMaps make_uses() {
    UseMaps u{};
    for (int q = 0; q < 32; q++) u.first[q] = u.second[q] = -1;
    for (int i = 0; i < 48; i++) {
        const int q = tdes_spec::expansion(i);
        if (u.first[q] < 0) u.first[q] = i; else u.second[q] = i;
    }
    return u;
}

constexpr UseMaps kUses = make_uses();

// Mask of the key bit at S-box input position i (box i / 6) of a round with words (ka, kb).
__device__ __forceinline__ uint32_t key_bit(uint32_t ka, uint32_t kb, int i) {
    return key_mask((i / 6) % 2 ? kb : ka, key_pos(i / 6, i % 6));
}

template <int S>
__device__ __forceinline__ void sbox_round_folded(uint32_t (&x)[32], const uint32_t (&y)[32], uint32_t ka_in,
                                                  uint32_t kb_in, uint32_t pa_in, uint32_t pb_in) {
    const uint32_t ka = key_word<false>(ka_in), kb = key_word<false>(kb_in);
    const uint32_t pa = key_word<false>(pa_in), pb = key_word<false>(pb_in);
    uint32_t in[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const int i = 6 * S + j, q = kMaps.e[i];
        in[j] = kUses.first[q] == i ? y[q] : y[q] ^ (key_bit(ka, kb, kUses.first[q]) ^ key_bit(ka, kb, i));
    }
    constexpr int p0 = kMaps.p_inv[4 * S + 0], p1 = kMaps.p_inv[4 * S + 1];
    constexpr int p2 = kMaps.p_inv[4 * S + 2], p3 = kMaps.p_inv[4 * S + 3];
    const uint32_t m0 = key_bit(pa, pb, kUses.first[p0]), m1 = key_bit(pa, pb, kUses.first[p1]);
    const uint32_t m2 = key_bit(pa, pb, kUses.first[p2]), m3 = key_bit(pa, pb, kUses.first[p3]);
    if constexpr (S == 0) sbox0_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 1) sbox1_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 2) sbox2_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 3) sbox3_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 4) sbox4_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 5) sbox5_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 6) sbox6_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 7) sbox7_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
}

// x ^= f(y) for a round with words (ka, kb); (pa, pb) = previous round's words ^ next round's.
__device__ __forceinline__ void feistel_folded(uint32_t (&x)[32], const uint32_t (&y)[32], uint32_t ka, uint32_t kb,
                                               uint32_t pa, uint32_t pb) {
    sbox_round_folded<0>(x, y, ka, kb, pa, pb);
    sbox_round_folded<1>(x, y, ka, kb, pa, pb);
    sbox_round_folded<2>(x, y, ka, kb, pa, pb);
    sbox_round_folded<3>(x, y, ka, kb, pa, pb);
    sbox_round_folded<4>(x, y, ka, kb, pa, pb);
    sbox_round_folded<5>(x, y, ka, kb, pa, pb);
    sbox_round_folded<6>(x, y, ka, kb, pa, pb);
    sbox_round_folded<7>(x, y, ka, kb, pa, pb);
}

// XOR the key bits of round words (ka, kb) at every plane's first E position.
__device__ __forceinline__ void fold_keys(uint32_t (&h)[32], uint32_t ka_in, uint32_t kb_in) {
    const uint32_t ka = key_word<false>(ka_in), kb = key_word<false>(kb_in);
#pragma unroll
    for (int q = 0; q < 32; q++) h[q] ^= key_bit(ka, kb, kUses.first[q]);
}

// Sixteen rounds with a wave-uniform key: x holds L0 and y holds R0 on entry,
// L16 and R16 on exit (both without folded keys).
__device__ __forceinline__ void des_stage_folded(uint32_t (&x)[32], uint32_t (&y)[32], const uint32_t *__restrict__ ks) {
    fold_keys(y, ks[0], ks[1]);
    uint32_t prev_a = 0, prev_b = 0;  // round r-1's words (none before round 0)
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        const uint32_t ka0 = ks[2 * r], kb0 = ks[2 * r + 1];
        const uint32_t ka1 = ks[2 * r + 2], kb1 = ks[2 * r + 3];
        // Round r + 2's words, or none after round 15 (the index is clamped so the load stays in the stage).
        const int n2 = r + 2 < 16 ? 2 * r + 4 : 30;
        const uint32_t ka2 = r + 2 < 16 ? ks[n2] : 0u, kb2 = r + 2 < 16 ? ks[n2 + 1] : 0u;
        feistel_folded(x, y, ka0, kb0, prev_a ^ ka1, prev_b ^ kb1);
        feistel_folded(y, x, ka1, kb1, ka0 ^ ka2, kb0 ^ kb2);
        prev_a = ka1;
        prev_b = kb1;
    }
    fold_keys(x, ks[30], ks[31]);
}

// ---- the same rounds with every key mask precomputed in LDS ----
//
// Extracting each mask from the schedule words costs scalar instructions (one
// bit-field extract per mask, three per correction), which the compute unit's
// single scalar unit issues at half the rate of its vector instructions.  The
// table below holds every mask of one direction (48 rounds x 8 boxes x 8 words,
// then each stage's two fix-up rows of 32), built once per workgroup; a round
// reads its masks with two broadcast 16-byte LDS reads per S-box.
//   round r, box S, word w: w < 4  mask of output w (k[r-1] ^ k[r+1] at the
//                                  first E position of the plane it updates);
//                           w >= 4 correction of the box's (w-4)-th second-use
//                                  input (k[r] at the plane's first E position
//                                  ^ k[r] at this one), or 0.
constexpr int kMaskRoundWords = 64;
constexpr int kMaskFixOffset = 48 * kMaskRoundWords;
constexpr int kMaskWords = kMaskFixOffset + 3 * 64;
// 16-byte LDS reads: rows and per-wave tables stay 16-byte aligned.
static_assert(kMaskRoundWords % 8 == 0 && kMaskFixOffset % 4 == 0 && kMaskWords % 4 == 0, "mask table alignment");

struct SecondUses {
    int j[8][4];  // box S: the inputs j that are second uses, in order (-1 past the end)
};

constexpr SecondUses make_second_uses() {
    SecondUses u{};
    for (int b = 0; b < 8; b++) {
        int t = 0;
        for (int k = 0; k < 4; k++) u.j[b][k] = -1;
        for (int jj = 0; jj < 6; jj++) {
            const int i = 6 * b + jj;
            if (kUses.first[kMaps.e[i]] != i) u.j[b][t++] = jj;
        }
    }
    return u;
}

constexpr SecondUses kSecond = make_second_uses();

// Cooperative build of the mask table of one direction (ks: its 96 words).
__device__ __forceinline__ void build_mask_table(uint32_t *tab, const uint32_t *__restrict__ ks, int tid, int nthreads) {
    for (int w = tid; w < kMaskWords; w += nthreads) {
        uint32_t m = 0;
        if (w < kMaskFixOffset) {
            const int r = w / kMaskRoundWords, b = (w % kMaskRoundWords) / 8, slot = w % 8;
            const int i = r % 16;
            if (slot < 4) {
                const int q = kMaps.p_inv[4 * b + slot];
                const uint32_t pa = (i > 0 ? ks[2 * r - 2] : 0u) ^ (i < 15 ? ks[2 * r + 2] : 0u);
                const uint32_t pb = (i > 0 ? ks[2 * r - 1] : 0u) ^ (i < 15 ? ks[2 * r + 3] : 0u);
                m = key_bit(pa, pb, kUses.first[q]);
            } else if (kSecond.j[b][slot - 4] >= 0) {
                const int in = 6 * b + kSecond.j[b][slot - 4];
                const uint32_t ka = ks[2 * r], kb = ks[2 * r + 1];
                m = key_bit(ka, kb, kUses.first[kMaps.e[in]]) ^ key_bit(ka, kb, in);
            }
        } else {
            const int f = w - kMaskFixOffset, stage = f / 64, post = (f % 64) / 32, q = f % 32;
            const int r = 16 * stage + (post ? 15 : 0);
            m = key_bit(ks[2 * r], ks[2 * r + 1], kUses.first[q]);
        }
        tab[w] = m;
    }
}

template <int S>
__device__ __forceinline__ void sbox_round_tab(uint32_t (&x)[32], const uint32_t (&y)[32], const uint32_t *rt) {
    const uint4 mo = *reinterpret_cast<const uint4 *>(rt + 8 * S);
    const uint4 mc = *reinterpret_cast<const uint4 *>(rt + 8 * S + 4);
    const uint32_t corr[4] = {mc.x, mc.y, mc.z, mc.w};
    uint32_t in[6];
    int t = 0;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const int i = 6 * S + j, q = kMaps.e[i];
        if (kUses.first[q] == i) {
            in[j] = y[q];
        } else {
            in[j] = y[q] ^ corr[t];
            t++;
        }
    }
    constexpr int p0 = kMaps.p_inv[4 * S + 0], p1 = kMaps.p_inv[4 * S + 1];
    constexpr int p2 = kMaps.p_inv[4 * S + 2], p3 = kMaps.p_inv[4 * S + 3];
    if constexpr (S == 0) sbox0_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 1) sbox1_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 2) sbox2_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 3) sbox3_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 4) sbox4_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 5) sbox5_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 6) sbox6_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
    if constexpr (S == 7) sbox7_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], mo.x, mo.y, mo.z, mo.w);
}

__device__ __forceinline__ void feistel_tab(uint32_t (&x)[32], const uint32_t (&y)[32], const uint32_t *rt) {
    sbox_round_tab<0>(x, y, rt);
    sbox_round_tab<1>(x, y, rt);
    sbox_round_tab<2>(x, y, rt);
    sbox_round_tab<3>(x, y, rt);
    sbox_round_tab<4>(x, y, rt);
    sbox_round_tab<5>(x, y, rt);
    sbox_round_tab<6>(x, y, rt);
    sbox_round_tab<7>(x, y, rt);
}

__device__ __forceinline__ void fold_tab(uint32_t (&h)[32], const uint32_t *fix) {
#pragma unroll
    for (int q = 0; q < 32; q += 4) {
        const uint4 m = *reinterpret_cast<const uint4 *>(fix + q);
        h[q] ^= m.x; h[q + 1] ^= m.y; h[q + 2] ^= m.z; h[q + 3] ^= m.w;
    }
}

// Stage `stage` (0..2) of EDE with masks from the table: as des_stage_folded.
__device__ __forceinline__ void des_stage_tab(uint32_t (&x)[32], uint32_t (&y)[32], const uint32_t *tab, int stage) {
    fold_tab(y, tab + kMaskFixOffset + 64 * stage);
    const uint32_t *rt = tab + 16 * stage * kMaskRoundWords;
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        feistel_tab(x, y, rt + r * kMaskRoundWords);
        feistel_tab(y, x, rt + (r + 1) * kMaskRoundWords);
    }
    fold_tab(x, tab + kMaskFixOffset + 64 * stage + 32);
}

// The whole EDE (or its inverse, by the schedule) on 32 blocks held as two
// arrays of little-endian words: a[j] = bytes 0..3 and b[j] = bytes 4..7 of
// block j.  ks: the 96 schedule words of one direction.
// How the 48 rounds get their key masks:
//   kLaneMasks   per-lane keys: masks extracted from vector registers (lane tiles);
//   kScalarMasks one key per wave, one scalar extract and one XOR per S-box input;
//   kFoldedMasks one key per wave, masks folded into the Feistel XOR (scalar extracts);
//   kTableMasks  as kFoldedMasks with every mask precomputed in an LDS table.
enum KeyMode { kLaneMasks, kScalarMasks, kFoldedMasks, kTableMasks };

// The whole EDE (or its inverse, by the schedule) on 32 blocks held as two
// arrays of little-endian words: a[j] = bytes 0..3 and b[j] = bytes 4..7 of
// block j.  ks: the 96 schedule words of one direction; tab: the mask table
// (kTableMasks only).
template <KeyMode kMode>
__device__ __forceinline__ void tdes_32_blocks(uint32_t (&a)[32], uint32_t (&b)[32], const uint32_t *__restrict__ ks,
                                               const uint32_t *tab) {
    transpose32(a);
    transpose32(b);
    uint32_t l[32], r[32];
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int pl = kMaps.l0[k], pr = kMaps.r0[k];
        l[k] = pl < 32 ? a[pl] : b[pl - 32];
        r[k] = pr < 32 ? a[pr] : b[pr - 32];
    }
    // Three DES stages; between them IP^-1 then IP cancel and only the halves swap.
    if constexpr (kMode == kLaneMasks || kMode == kScalarMasks) {
        des_stage<kMode == kLaneMasks>(l, r, ks);
        des_stage<kMode == kLaneMasks>(r, l, ks + 32);
        des_stage<kMode == kLaneMasks>(l, r, ks + 64);
    } else if constexpr (kMode == kFoldedMasks) {
        des_stage_folded(l, r, ks);
        des_stage_folded(r, l, ks + 32);
        des_stage_folded(l, r, ks + 64);
    } else {
        des_stage_tab(l, r, tab, 0);
        des_stage_tab(r, l, tab, 1);
        des_stage_tab(l, r, tab, 2);
    }
    // Preoutput R16 || L16 = (r, l); FP is a renaming back to block bit planes.
#pragma unroll
    for (int p = 0; p < 64; p++) {
        const int q = kMaps.out_src[p];
        const uint32_t v = q < 32 ? r[q] : l[q - 32];
        if (p < 32) a[p] = v; else b[p - 32] = v;
    }
    transpose32(a);
    transpose32(b);
}

// The empty asm statement makes a value opaque at its use, so the compiler
// recomputes per-block offsets instead of hoisting them out of tile loops and
// keeping them live across the rounds.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// A wave tile: 2048 consecutive blocks starting at `tin`/`tout` (wave-uniform);
// lane l holds blocks 128k + 2l and 128k + 2l + 1 (k = 0..15), so each access is
// 16 bytes per lane over 1 KiB contiguous across the wave.  A short tile
// (n_valid < 2048, or buffers not 16-byte aligned) reads 8 bytes per block,
// clamping indices past the end to the last valid block, and writes only
// valid blocks.
template <bool kFull, KeyMode kMode>
__device__ __forceinline__ void wave_tile(const uint32_t *__restrict__ ks, const uint8_t *tin, uint8_t *tout,
                                          uint32_t n_valid, uint32_t lane, const uint32_t *tab = nullptr) {
    uint32_t a[32], b[32];
    lane = opaque(lane);
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
    tdes_32_blocks<kMode>(a, b, ks, tab);
    lane = opaque(lane);
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

// A lane slot: up to 32 consecutive blocks owned by this lane alone (its own
// message, key and direction).  count = 0 leaves the lane idle.
__device__ __forceinline__ void lane_slot(const uint32_t *ks, const uint8_t *lin, uint8_t *lout, uint32_t count) {
    uint32_t a[32], b[32];
    if (count) {
#pragma unroll
        for (int j = 0; j < 32; j++) {
            const uint32_t jj = opaque(j < (int)count ? j : count - 1);
            const uint2 v = *reinterpret_cast<const uint2 *>(lin + 8 * jj);
            a[j] = v.x; b[j] = v.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 32; j++) a[j] = b[j] = 0;
    }
    tdes_32_blocks<kLaneMasks>(a, b, ks, nullptr);
    if (count) {
#pragma unroll
        for (int j = 0; j < 32; j++)
            if (j < (int)count) *reinterpret_cast<uint2 *>(lout + 8 * opaque(j)) = make_uint2(a[j], b[j]);
    }
}

}  // namespace tdes_bs
