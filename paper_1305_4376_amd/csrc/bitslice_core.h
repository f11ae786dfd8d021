// bitslice_core.h -- the bitsliced Triple-DES round core shared by the plain and batched kernels.
//
// A lane holds 32 blocks as 64 bit planes: plane f is a 32-bit word whose bit j
// is bit f of the lane's block j.  IP, E, P and IP^-1 are renamings of planes
// (bitslice_maps.h); each S-box is a circuit of 3-input lookup gates
// (sbox_circuits.inc).  Key bits enter as masks (0 or ~0): when the key is the
// same for the whole wave, folded into the halves between rounds, from words
// the host precomputes (scalar registers); when lanes have different keys, one
// XOR per S-box input from the round words (vector registers).  Blocks become
// planes by an in-register 32x32 bit transpose of each 4-byte half of the 32
// blocks.
#pragma once
#include <hip/hip_runtime.h>

#include "bitslice_maps.h"

namespace tdes_bs {

#include "sbox_circuits.inc"

constexpr int kLanes = 64;
constexpr int kTileBlocks = 32 * kLanes;     // blocks per wave tile

// ---- bit transpose ----

// One exchange stage of the transpose: for rows j and j + S (j & S == 0), swap the
// bits of row j at positions i + S with those of row j + S at positions i, for the
// positions i selected by M.  On gfx950 v_bfi, v_perm and left shifts issue at half
// the rate of v_bitop3 with vector-register operands, of adds and of right shifts
// (measured), so the selects are v_bitop3 with the mask in a vector register and a
// 1-bit left shift is an add.
template <int S, uint32_t M>
__device__ __forceinline__ void exchange_stage(uint32_t (&w)[32]) {
    uint32_t m;
    asm("v_mov_b32 %0, %1" : "=v"(m) : "i"(M));
#pragma unroll
    for (int j = 0; j < 32; j++) {
        if (j & S) continue;
        const uint32_t a = w[j], b = w[j + S];
        uint32_t bs;
        if constexpr (S == 1)
            asm("v_add_u32 %0, %1, %1" : "=v"(bs) : "v"(b));            // b << 1 (the compiler would turn b + b into a shift)
        else
            bs = b << S;
        w[j] = __builtin_amdgcn_bitop3_b32(a, bs, m, 0xE4);            // m ? a : bs
        w[j + S] = __builtin_amdgcn_bitop3_b32(a >> S, b, m, 0xE4);    // m ? a >> S : b
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

// ---- rounds with folded key masks (one key for the whole wave) ----
//
// The scheme of bitslice_maps.h: the masks come from the direction's folded
// words (32 output masks and 16 corrections per round, one scalar bit-field
// extract each), so a round costs the S-box gates plus 32 three-way XORs and
// 16 corrections, instead of 48 key XORs plus 32 XORs.

template <int S>
__device__ __forceinline__ void sbox_round_folded(uint32_t (&x)[32], const uint32_t (&y)[32], uint32_t out_in,
                                                  uint32_t corr_in) {
    const uint32_t ow = key_word<false>(out_in), cw = key_word<false>(corr_in);
    uint32_t in[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const int i = 6 * S + j, t = kUses.second_of[i];
        in[j] = t < 0 ? y[kMaps.e[i]] : y[kMaps.e[i]] ^ key_mask(cw, t);
    }
    constexpr int p0 = kMaps.p_inv[4 * S + 0], p1 = kMaps.p_inv[4 * S + 1];
    constexpr int p2 = kMaps.p_inv[4 * S + 2], p3 = kMaps.p_inv[4 * S + 3];
    const uint32_t m0 = key_mask(ow, p0), m1 = key_mask(ow, p1), m2 = key_mask(ow, p2), m3 = key_mask(ow, p3);
    if constexpr (S == 0) sbox0_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 1) sbox1_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 2) sbox2_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 3) sbox3_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 4) sbox4_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 5) sbox5_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 6) sbox6_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
    if constexpr (S == 7) sbox7_m(in[0], in[1], in[2], in[3], in[4], in[5], x[p0], x[p1], x[p2], x[p3], m0, m1, m2, m3);
}

// x ^= f(y) for one round, with its output-fold and correction words.
__device__ __forceinline__ void feistel_folded(uint32_t (&x)[32], const uint32_t (&y)[32], uint32_t ow, uint32_t cw) {
    sbox_round_folded<0>(x, y, ow, cw);
    sbox_round_folded<1>(x, y, ow, cw);
    sbox_round_folded<2>(x, y, ow, cw);
    sbox_round_folded<3>(x, y, ow, cw);
    sbox_round_folded<4>(x, y, ow, cw);
    sbox_round_folded<5>(x, y, ow, cw);
    sbox_round_folded<6>(x, y, ow, cw);
    sbox_round_folded<7>(x, y, ow, cw);
}

// h[q] ^= bit q of w, for every plane q.
__device__ __forceinline__ void fold_fix(uint32_t (&h)[32], uint32_t w_in) {
    const uint32_t w = key_word<false>(w_in);
#pragma unroll
    for (int q = 0; q < 32; q++) h[q] ^= key_mask(w, q);
}

// The same two rounds as generated gfx950 assembly (rounds_asm.inc, written
// by gen/gen_rounds.py from the stored circuits and the standard's E and P,
// and checked there against this file's definition by simulation): x ^= f(y)
// with (ow0, cw0), then y ^= f(x) with (ow1, cw1).  The generator assigns the
// registers itself so that an instruction's vector operands sit in different
// register banks (bank = register number mod 4; two operands in one bank
// halve the issue rate, and the compiler's own assignment of this code has
// that in nearly half its instructions).  The 64 planes live in two fixed
// register sets; kSwapped: x in the second set and y in the first, which is
// how the halves lie in the middle DES stage of EDE.
#include "rounds_asm.inc"

template <bool kSwapped>
__device__ __forceinline__ void feistel_pair_asm(uint32_t (&x)[32], uint32_t (&y)[32], uint32_t ow0, uint32_t cw0,
                                                 uint32_t ow1, uint32_t cw1) {
    if constexpr (!kSwapped)
        asm volatile(TDES_ROUNDS_ASM_A
                     : TDES_ROUNDS_OPERANDS_A(x, y)
                     : [ow0] "s"(ow0), [cw0] "s"(cw0), [ow1] "s"(ow1), [cw1] "s"(cw1)
                     : TDES_ROUNDS_CLOBBERS);
    else
        asm volatile(TDES_ROUNDS_ASM_B
                     : TDES_ROUNDS_OPERANDS_B(x, y)
                     : [ow0] "s"(ow0), [cw0] "s"(cw0), [ow1] "s"(ow1), [cw1] "s"(cw1)
                     : TDES_ROUNDS_CLOBBERS);
}

// The 16 rounds of stage `stage` (0..2) with folded masks: x holds L0 and y
// holds R0 on entry, L16 and R16 on exit; y enters folded with the stage's
// first key and x leaves folded with its last.  fold: the direction's folded
// words.  kSwapped: see feistel_pair_asm.
template <bool kSwapped = false>
__device__ __forceinline__ void des_rounds_folded(uint32_t (&x)[32], uint32_t (&y)[32],
                                                  const uint32_t *__restrict__ fold, int stage) {
    const uint32_t *ow = fold + kFoldOut + 16 * stage, *cw = fold + kFoldCorr + 16 * stage;
    // The next pair's words are loaded before this pair's rounds run, so their
    // scalar loads complete behind the rounds instead of stalling the wave.
    uint32_t o0 = ow[0], c0 = cw[0], o1 = ow[1], c1 = cw[1];
#pragma unroll 1
    for (int r = 0; r < 16; r += 2) {
        const uint32_t ko0 = key_word<false>(o0), kc0 = key_word<false>(c0);
        const uint32_t ko1 = key_word<false>(o1), kc1 = key_word<false>(c1);
        const int n = r + 2 < 16 ? r + 2 : r;  // (the last pair reloads its own words)
        o0 = ow[n];
        c0 = cw[n];
        o1 = ow[n + 1];
        c1 = cw[n + 1];
        feistel_pair_asm<kSwapped>(x, y, ko0, kc0, ko1, kc1);
    }
}

// One whole stage, both halves without folded keys on entry and exit.
__device__ __forceinline__ void des_stage_folded(uint32_t (&x)[32], uint32_t (&y)[32],
                                                 const uint32_t *__restrict__ fold, int stage) {
    fold_fix(y, fold[kFoldPre + stage]);
    des_rounds_folded(x, y, fold, stage);
    fold_fix(x, fold[kFoldPost + stage]);
}

// ---- kernel ----

// The whole EDE (or its inverse, by the schedule) on 32 blocks held as two
// arrays of little-endian words: a[j] = bytes 0..3 and b[j] = bytes 4..7 of
// block j.  ks: one direction's schedule words, wave-uniform (kLaneKeys =
// false: the folded words are used) or per lane (kLaneKeys = true: the round
// words, one key XOR per S-box input).
template <bool kLaneKeys>
__device__ __forceinline__ void tdes_32_blocks(uint32_t (&a)[32], uint32_t (&b)[32], const uint32_t *__restrict__ ks) {
    transpose32(a);
    transpose32(b);
    uint32_t l[32], r[32];
#pragma unroll
    for (int k = 0; k < 32; k++) {
        const int pl = kMaps.l0[k], pr = kMaps.r0[k];
        l[k] = pl < 32 ? a[pl] : b[pl - 32];
        r[k] = pr < 32 ? a[pr] : b[pr - 32];
    }
    // Three DES stages; between them IP^-1 then IP cancel and only the halves
    // swap.  With one key per wave the stages are written out (measured 1.3%
    // faster on MI355X than a shared loop); with per-lane keys one loop runs
    // all three, so the batch kernel carries that round code once.
    if constexpr (kLaneKeys) {
#pragma unroll 1
        for (int stage = 0; stage < 3; stage++) {
            des_stage<true>(l, r, ks + 32 * stage);
            if (stage < 2) {
#pragma unroll
                for (int k = 0; k < 32; k++) {
                    const uint32_t t = l[k];
                    l[k] = r[k];
                    r[k] = t;
                }
            }
        }
    } else {
        // stage s ends reading the half that stage s + 1 reads first: one fix-up between them
        const uint32_t *fold = ks + kFoldBase;
        fold_fix(r, fold[kFoldPre + 0]);
        des_rounds_folded(l, r, fold, 0);
        fold_fix(l, fold[kFoldMid + 0]);
        des_rounds_folded<true>(r, l, fold, 1);
        fold_fix(r, fold[kFoldMid + 1]);
        des_rounds_folded(l, r, fold, 2);
        fold_fix(l, fold[kFoldPost + 2]);
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

// Block-parallel modes built on the same core (NIST SP 800-38A, with TDEA as
// the block cipher; the paper itself is ECB only):
//   kEcb        out_j = E(in_j) or D(in_j), by the schedule;
//   kCtr        out_j = in_j xor E(T_j), T_j = iv + j modulo 2^64 as a big-endian block;
//   kCbcDecrypt out_j = D(in_j) xor in_{j-1}, in_{-1} = iv (never in place).
// j is the block index in the message; `iv` holds the 8 IV bytes read as a
// big-endian integer.
enum class TileMode { kEcb, kCtr, kCbcDecrypt };

// The standard's byte order as the two little-endian words a (bytes 0..3), b (bytes 4..7).
__device__ __forceinline__ uint32_t be_hi_word(uint64_t v) { return __builtin_bswap32((uint32_t)(v >> 32)); }
__device__ __forceinline__ uint32_t be_lo_word(uint64_t v) { return __builtin_bswap32((uint32_t)v); }

// A wave tile: 2048 consecutive blocks starting at `tin`/`tout` (wave-uniform),
// blocks first_block.. of the message; lane l holds blocks 128k + 2l and
// 128k + 2l + 1 (k = 0..15), so each access is 16 bytes per lane over 1 KiB
// contiguous across the wave.  kFull: all 2048 blocks valid and both buffers
// 16-byte aligned.  Otherwise (n_valid < 2048, or buffers only 8-byte
// aligned) each block is loaded and stored on its own, at the same
// addresses, only if it is one of the first n_valid; lanes past the end
// compute on zeros.  Whole-tile loads and stores are nontemporal (every block
// is read and written once), except CBC decryption's first read, which is read
// again after the rounds.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <TileMode kMode, bool kFull>
__device__ __forceinline__ void mode_tile(const uint32_t *__restrict__ ks, const uint8_t *tin, uint8_t *tout,
                                          uint32_t n_valid, uint32_t lane, uint64_t first_block, uint64_t iv) {
    uint32_t a[32], b[32];
    lane = opaque(lane);
    if constexpr (kMode == TileMode::kCtr) {
        const uint64_t t0 = iv + first_block;  // wraps modulo 2^64
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const uint64_t t = t0 + (uint32_t)(128 * k + 2 * lane);
            a[2 * k] = be_hi_word(t); b[2 * k] = be_lo_word(t);
            a[2 * k + 1] = be_hi_word(t + 1); b[2 * k + 1] = be_lo_word(t + 1);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const uint8_t *p = tin + 1024 * k + 16 * lane;
            if (kFull) {
                // CBC decryption reads its input a second time after the rounds: keep it cached
                const v4u v = kMode == TileMode::kCbcDecrypt ? *reinterpret_cast<const v4u *>(p)
                                                              : __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
                a[2 * k] = v.x; b[2 * k] = v.y; a[2 * k + 1] = v.z; b[2 * k + 1] = v.w;
            } else {
                const uint32_t j = 128 * k + 2 * lane;
                uint2 v0 = make_uint2(0, 0), v1 = make_uint2(0, 0);
                if (j < n_valid) v0 = *reinterpret_cast<const uint2 *>(p);
                if (j + 1 < n_valid) v1 = *reinterpret_cast<const uint2 *>(p + 8);
                a[2 * k] = v0.x; b[2 * k] = v0.y; a[2 * k + 1] = v1.x; b[2 * k + 1] = v1.y;
            }
        }
    }
    tdes_32_blocks<false>(a, b, ks);
    lane = opaque(lane);
    // CBC decryption of whole tiles: the ciphertext block before the lane's first block j = 128k + 2l
    // is the second block of lane l - 1's pair (one lane over, by a wave-wide DPP shift), and for
    // lane 0 the last block of the previous 128 (carried in scalars; for k = 0 the block before the
    // tile, or the IV at the message's start).
    uint32_t carry_a = be_hi_word(iv), carry_b = be_lo_word(iv);
    if (kMode == TileMode::kCbcDecrypt && kFull && first_block != 0) {
        const uint2 v = *reinterpret_cast<const uint2 *>(tin - 8);
        carry_a = __builtin_amdgcn_readfirstlane(v.x);
        carry_b = __builtin_amdgcn_readfirstlane(v.y);
    }
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const uint32_t j = 128 * k + 2 * lane;
        const uint8_t *p = tin + 1024 * k + 16 * lane;
        if constexpr (kMode == TileMode::kCtr) {  // the keystream meets the data
            if (kFull) {
                const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
                a[2 * k] ^= v.x; b[2 * k] ^= v.y; a[2 * k + 1] ^= v.z; b[2 * k + 1] ^= v.w;
            } else {
                uint2 v0 = make_uint2(0, 0), v1 = make_uint2(0, 0);
                if (j < n_valid) v0 = *reinterpret_cast<const uint2 *>(p);
                if (j + 1 < n_valid) v1 = *reinterpret_cast<const uint2 *>(p + 8);
                a[2 * k] ^= v0.x; b[2 * k] ^= v0.y; a[2 * k + 1] ^= v1.x; b[2 * k + 1] ^= v1.y;
            }
        } else if constexpr (kMode == TileMode::kCbcDecrypt) {  // XOR the preceding ciphertext blocks
            if (kFull) {
                const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));  // blocks j, j + 1
                constexpr int kWaveShr1 = 0x138;  // DPP: lane i reads lane i - 1; lane 0 keeps the old value
                const uint32_t pa = (uint32_t)__builtin_amdgcn_update_dpp((int)carry_a, (int)v.z, kWaveShr1, 0xF, 0xF, false);
                const uint32_t pb = (uint32_t)__builtin_amdgcn_update_dpp((int)carry_b, (int)v.w, kWaveShr1, 0xF, 0xF, false);
                a[2 * k] ^= pa; b[2 * k] ^= pb; a[2 * k + 1] ^= v.x; b[2 * k + 1] ^= v.y;
                carry_a = __builtin_amdgcn_readlane(v.z, kLanes - 1);
                carry_b = __builtin_amdgcn_readlane(v.w, kLanes - 1);
            } else {
                uint2 v0 = make_uint2(be_hi_word(iv), be_lo_word(iv)), v1 = make_uint2(0, 0);
                if (first_block + j != 0 && j < n_valid) v0 = *reinterpret_cast<const uint2 *>(p - 8);
                if (j + 1 < n_valid) v1 = *reinterpret_cast<const uint2 *>(p);
                a[2 * k] ^= v0.x; b[2 * k] ^= v0.y; a[2 * k + 1] ^= v1.x; b[2 * k + 1] ^= v1.y;
            }
        }
        uint8_t *q = tout + 1024 * k + 16 * lane;
        if (kFull) {
            v4u o = {a[2 * k], b[2 * k], a[2 * k + 1], b[2 * k + 1]};
            __builtin_nontemporal_store(o, reinterpret_cast<v4u *>(q));
        } else {
            if (j < n_valid) *reinterpret_cast<uint2 *>(q) = make_uint2(a[2 * k], b[2 * k]);
            if (j + 1 < n_valid) *reinterpret_cast<uint2 *>(q + 8) = make_uint2(a[2 * k + 1], b[2 * k + 1]);
        }
    }
}

// ECB over a wave tile (see mode_tile).
template <bool kFull>
__device__ __forceinline__ void wave_tile(const uint32_t *__restrict__ ks, const uint8_t *tin, uint8_t *tout,
                                          uint32_t n_valid, uint32_t lane) {
    mode_tile<TileMode::kEcb, kFull>(ks, tin, tout, n_valid, lane, 0, 0);
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
    tdes_32_blocks<true>(a, b, ks);
    if (count) {
#pragma unroll
        for (int j = 0; j < 32; j++)
            if (j < (int)count) *reinterpret_cast<uint2 *>(lout + 8 * opaque(j)) = make_uint2(a[j], b[j]);
    }
}

}  // namespace tdes_bs
