// keysched.cpp -- host key expansion of a Triple-DES key triple into the device schedule.
//
// The paper copies 48 subkeys (three keys x 16 rounds) to the device once,
// before the blocks are processed (Listing 1.1).  Each DES subkey follows the
// standard: PC-1 keeps 56 of the 64 key bits as C and D, C and D rotate left
// by the shift schedule, PC-2 picks 48 bits.  The EDE composition of
// Section II.A fixes the order the rounds consume them:
//   encrypt:  K1 rounds 1..16, K2 rounds 16..1, K3 rounds 1..16
//   decrypt:  K3 rounds 16..1, K2 rounds 1..16, K1 rounds 16..1
//
// Round layout (private to the library).  A 48-bit subkey is eight 6-bit
// chunks c0..c7, chunk b being the key bits XORed into S-box b+1's input.  The
// kernels read R rotated so that four chunk positions line up with bytes:
//   word A = c0 | c6 << 8 | c4 << 16 | c2 << 24   (matches rotl(R, 5))
//   word B = c1 | c7 << 8 | c5 << 16 | c3 << 24   (matches rotl(R, 9))
#include <string.h>

#include "bitslice_maps.h"
#include "des_spec.h"
#include "internal.h"

namespace {

using namespace tdes_spec;

static_assert(tdes_bs::kFoldBase == tdes::kRoundWords && tdes::kRoundWords + tdes_bs::kFoldWords <= tdes::kDirWords,
              "folded words follow the round words of each direction");

uint64_t load_be64(const uint8_t k[8]) {
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v = (v << 8) | k[i];
    return v;
}

// Bit i (0-based, 0 = most significant of the 64) of v.
inline uint64_t bit64(uint64_t v, int i) { return (v >> (63 - i)) & 1u; }

// The sixteen 48-bit subkeys of one DES key (subkey bit 0 in bit 47).
void des_subkeys(const uint8_t key[8], uint64_t sub[16]) {
    const uint64_t k = load_be64(key);
    uint32_t c = 0, d = 0;
    for (int i = 0; i < 28; i++) {
        c = (c << 1) | (uint32_t)bit64(k, pc1(i));
        d = (d << 1) | (uint32_t)bit64(k, pc1(28 + i));
    }
    for (int r = 0; r < 16; r++) {
        const int s = kShift[r];
        c = ((c << s) | (c >> (28 - s))) & 0x0FFFFFFFu;
        d = ((d << s) | (d >> (28 - s))) & 0x0FFFFFFFu;
        const uint64_t cd = ((uint64_t)c << 28) | d;  // C bit 0 in bit 55
        uint64_t v = 0;
        for (int i = 0; i < 48; i++) v = (v << 1) | ((cd >> (55 - kPC2[i])) & 1u);
        sub[r] = v;
    }
}

void pack_round(uint64_t sub, uint32_t *w) {
    uint32_t c[8];
    for (int b = 0; b < 8; b++) c[b] = (uint32_t)(sub >> (42 - 6 * b)) & 63u;
    w[0] = c[0] | c[6] << 8 | c[4] << 16 | c[2] << 24;
    w[1] = c[1] | c[7] << 8 | c[5] << 16 | c[3] << 24;
}

// Key bit at E position i (0..47) of a 48-bit subkey (subkey bit 0 in bit 47).
inline uint32_t key_bit(uint64_t sub, int i) { return (uint32_t)(sub >> (47 - i)) & 1u; }

// The folded key words of one direction (layout in bitslice_maps.h) from its 48
// subkeys in round order.
void fold_words(const uint64_t sub[48], uint32_t *w) {
    using tdes_bs::kMaps;
    using tdes_bs::kUses;
    for (int r = 0; r < 48; r++) {
        const int i = r % 16;
        const uint64_t diff = (i > 0 ? sub[r - 1] : 0) ^ (i < 15 ? sub[r + 1] : 0);
        uint32_t out = 0, corr = 0;
        for (int q = 0; q < 32; q++) out |= key_bit(diff, kUses.first[q]) << q;
        for (int t = 0; t < 16; t++) {
            const int pos = kUses.second_pos[t];
            corr |= (key_bit(sub[r], kUses.first[kMaps.e[pos]]) ^ key_bit(sub[r], pos)) << t;
        }
        w[tdes_bs::kFoldOut + r] = out;
        w[tdes_bs::kFoldCorr + r] = corr;
    }
    for (int st = 0; st < 3; st++) {
        uint32_t pre = 0, post = 0;
        for (int q = 0; q < 32; q++) {
            pre |= key_bit(sub[16 * st], kUses.first[q]) << q;
            post |= key_bit(sub[16 * st + 15], kUses.first[q]) << q;
        }
        w[tdes_bs::kFoldPre + st] = pre;
        w[tdes_bs::kFoldPost + st] = post;
    }
    for (int st = 0; st < 2; st++)
        w[tdes_bs::kFoldMid + st] = w[tdes_bs::kFoldPost + st] ^ w[tdes_bs::kFoldPre + st + 1];
}

// C0 and D0 of a key, for the weak-key test.
void des_cd0(const uint8_t key[8], uint32_t *c, uint32_t *d) {
    const uint64_t k = load_be64(key);
    *c = *d = 0;
    for (int i = 0; i < 28; i++) {
        *c = (*c << 1) | (uint32_t)bit64(k, pc1(i));
        *d = (*d << 1) | (uint32_t)bit64(k, pc1(28 + i));
    }
}

// A DES key is weak or semi-weak when C0 and D0 are each all zeros, all ones
// or one of the two alternating patterns: the shift schedule then yields at
// most two distinct subkeys.
bool weak_or_semi_weak(const uint8_t key[8]) {
    uint32_t c, d;
    des_cd0(key, &c, &d);
    auto special = [](uint32_t h) {
        return h == 0u || h == 0x0FFFFFFFu || h == 0x05555555u || h == 0x0AAAAAAAu;
    };
    return special(c) && special(d);
}

bool odd_parity(const uint8_t key[8]) {
    for (int i = 0; i < 8; i++)
        if ((__builtin_popcount(key[i]) & 1) == 0) return false;
    return true;
}

}  // namespace

extern "C" int tdes_expand_key(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8],
                               uint32_t flags, tdes_sched *out) {
    if (!k1 || !k2 || !k3 || !out) return TDES_ERR_NULL;
    if (flags & ~(TDES_CHECK_PARITY | TDES_REJECT_WEAK)) return TDES_ERR_ARG;
    const uint8_t *keys[3] = {k1, k2, k3};
    if (flags & TDES_CHECK_PARITY)
        for (const uint8_t *k : keys)
            if (!odd_parity(k)) return TDES_ERR_PARITY;
    if (flags & TDES_REJECT_WEAK)
        for (const uint8_t *k : keys)
            if (weak_or_semi_weak(k)) return TDES_ERR_WEAKKEY;

    uint64_t sub[3][16];
    for (int i = 0; i < 3; i++) des_subkeys(keys[i], sub[i]);

    // The 48 subkeys of each direction in the order its rounds use them.
    uint64_t order[2][48];
    for (int r = 0; r < 16; r++) {
        order[0][r] = sub[0][r];             // E under K1
        order[0][16 + r] = sub[1][15 - r];   // D under K2
        order[0][32 + r] = sub[2][r];        // E under K3
        order[1][r] = sub[2][15 - r];        // D under K3
        order[1][16 + r] = sub[1][r];        // E under K2
        order[1][32 + r] = sub[0][15 - r];   // D under K1
    }
    tdes_sched s;
    memset(&s, 0, sizeof s);
    for (int d = 0; d < 2; d++) {
        uint32_t *w = s.w + d * tdes::kDirWords;
        for (int r = 0; r < 48; r++) pack_round(order[d][r], w + 2 * r);
        fold_words(order[d], w + tdes::kRoundWords);
    }
    *out = s;
    return TDES_OK;
}
