// des_spec.h -- the Data Encryption Standard's constants as the library uses them.
//
// The paper names DES and Triple-DES (Section II.A) but prints none of the
// cipher's internals; they are the standard's (FIPS 46-3).  Everything here is
// 0-based: bit 0 of a block is the most significant bit of its first byte.
// Where a table has a short closed form (IP, E, PC-1) it is generated from
// that form instead of being listed; the S-boxes are stored as one hex digit
// per entry, row by row.  Every value is constexpr so that kernels can build
// their lookup tables at compile time.
#pragma once
#include <stdint.h>

namespace tdes_spec {

// S-box b (0..7), row r (0..3): 16 hex digits, column 0 first.
constexpr const char *kSboxRows[8][4] = {
    {"E4D12FB83A6C5907", "0F74E2D1A6CB9538", "41E8D62BFC973A50", "FC8249175B3EA06D"},
    {"F18E6B34972DC05A", "3D47F28EC01A69B5", "0E7BA4D158C6932F", "D8A13F42B67C05E9"},
    {"A09E63F51DC7B428", "D709346A285ECBF1", "D6498F30B12C5AE7", "1AD069874FE3B52C"},
    {"7DE3069A1285BC4F", "D8B56F03472C1AE9", "A690CB7DF13E5284", "3F06A1D8945BC72E"},
    {"2C417AB6853FD0E9", "EB2C47D150FA3986", "421BAD78F9C5630E", "B8C71E2D6F09A453"},
    {"C1AF92680D34E75B", "AF427C9561DE0B38", "9EF528C3704A1DB6", "432C95FABE17608D"},
    {"4B2EF08D3C975A61", "D0B7491AE35C2F86", "14BDC37EAF680592", "6BD814A7950FE23C"},
    {"D2846FB1A93E50C7", "1FD8A374C56B0E92", "7B419CE206ADF358", "21E74A8DFC90356B"}};

constexpr int hex_digit(char c) { return c <= '9' ? c - '0' : c - 'A' + 10; }

// S-box b applied to a 6-bit input x whose most significant bit is the box's first input.
// Row = first and last input bits, column = the middle four.
constexpr uint32_t sbox(int b, uint32_t x) {
    return (uint32_t)hex_digit(kSboxRows[b][((x >> 4) & 2) | (x & 1)][(x >> 1) & 15]);
}

// P: bit i of f(R) is bit kP[i] of the S-box output word (outputs of box b are bits 4b..4b+3).
constexpr uint8_t kP[32] = {15, 6,  19, 20, 28, 11, 27, 16, 0,  14, 22, 25, 4,  17, 30, 9,
                            1,  7,  23, 13, 31, 26, 2,  8,  18, 12, 29, 5,  21, 10, 3,  24};

// PC-2: bit i of a subkey is bit kPC2[i] of C||D (C = 0..27, D = 28..55).
constexpr uint8_t kPC2[48] = {13, 16, 10, 23, 0,  4,  2,  27, 14, 5,  20, 9,  22, 18, 11, 3,
                              25, 7,  15, 6,  26, 19, 12, 1,  40, 51, 30, 36, 46, 54, 29, 39,
                              50, 44, 32, 47, 43, 48, 38, 55, 33, 52, 45, 41, 49, 35, 28, 31};

// Left rotations of C and D before each of the 16 subkeys.
constexpr uint8_t kShift[16] = {1, 1, 2, 2, 2, 2, 2, 2, 1, 2, 2, 2, 2, 2, 2, 1};

// IP: output bit 8r+c is input bit 8(7-c)+q[r]; it reads the odd bit positions
// of the eight bytes (counting from 0), then the even ones, last byte first.
constexpr int ip(int i) {
    constexpr int q[8] = {1, 3, 5, 7, 0, 2, 4, 6};
    return 8 * (7 - i % 8) + q[i / 8];
}

// E: box b reads the six consecutive bits 4b-1 .. 4b+4 of R, cyclically.
constexpr int expansion(int i) { return (4 * (i / 6) + i % 6 + 31) % 32; }

// PC-1: C reads bit positions 0,1,2 of bytes 7..0 and then position 3 of
// bytes 7..4; D reads positions 6,5,4 of bytes 7..0 and then position 3 of
// bytes 3..0.  The parity bits (position 7) are never read.
constexpr int pc1(int i) {
    if (i < 24) return 8 * (7 - i % 8) + i / 8;
    if (i < 28) return 8 * (7 - (i - 24)) + 3;
    if (i < 52) return 8 * (7 - (i - 28) % 8) + 6 - (i - 28) / 8;
    return 8 * (3 - (i - 52)) + 3;
}

}  // namespace tdes_spec
