// bitslice_maps.h -- compile-time maps of the bitsliced round, shared by the
// host key schedule (keysched.cpp) and the kernels (bitslice_core.h).
//
// In the bitsliced layout a lane holds 32 blocks as 64 bit planes, and every
// DES permutation (IP, E, P, IP^-1) is a renaming of planes.  These maps name
// the planes; they are plain constexpr code with no device intrinsics.
#pragma once
#include "des_spec.h"

namespace tdes_bs {

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

// ---- folded key masks ----
//
// E reads 16 of the 32 bits of R twice.  Between rounds the kernel keeps every
// plane of a half XORed with the key bit that the next round reading that half
// applies at the plane's first E position.  Then a first use needs no key XOR;
// a second use needs one XOR with the difference of its two key bits (a
// "correction"); and XORing an S-box output into the target half also moves
// that half's folded key from round r-1's to round r+1's, in one three-way XOR
// with the mask of (k[r-1] xor k[r+1]) at the plane's first E position.  Each
// DES stage starts with the half read first folded with round 0's key and ends
// by removing round 15's key from the half read last.
struct UseMaps {
    int first[32];       // first E position (0..47) reading R bit q
    int second_of[48];   // E position i: index 0..15 of i among the second uses, or -1
    int second_pos[16];  // second use t: its E position
};

constexpr UseMaps make_uses() {
    UseMaps u{};
    for (int q = 0; q < 32; q++) u.first[q] = -1;
    int t = 0;
    for (int i = 0; i < 48; i++) {
        const int q = tdes_spec::expansion(i);
        if (u.first[q] < 0) {
            u.first[q] = i;
            u.second_of[i] = -1;
        } else {
            u.second_of[i] = t;
            u.second_pos[t++] = i;
        }
    }
    return u;
}

constexpr UseMaps kUses = make_uses();

// The folded words of one direction, after its 96 round words (keysched.cpp):
//   [kFoldOut + r]   round r: bit q = (k[r-1] xor k[r+1]) at first[q], both within r's stage (else 0);
//   [kFoldCorr + r]  round r: bit t = k[r] at first[e[second_pos[t]]] xor k[r] at second_pos[t];
//   [kFoldPre + s]   stage s: bit q = k[16s] at first[q]       (folded into the half read first);
//   [kFoldPost + s]  stage s: bit q = k[16s + 15] at first[q]  (removed from the half read last);
//   [kFoldMid + s]   s = 0, 1: [kFoldPost + s] xor [kFoldPre + s + 1].  The half that stage s reads
//                    last is the half that stage s + 1 reads first, so between two stages one pass
//                    exchanges the two folded keys.
constexpr int kFoldBase = 96;  // offset of the folded words in a direction's block
constexpr int kFoldOut = 0;
constexpr int kFoldCorr = 48;
constexpr int kFoldPre = 96;
constexpr int kFoldPost = 99;
constexpr int kFoldMid = 102;
constexpr int kFoldWords = 104;

}  // namespace tdes_bs
