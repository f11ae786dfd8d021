/*
 * des_oracle.c -- plain CPU reference for DES and Triple-DES (EDE) in ECB mode,
 * and in the block-parallel modes CBC and CTR.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (libtdes and its kernels) shares no code, header, table or generator with
 * it, and must never call it.
 *
 * What it computes.  The paper states the problem: each 64-bit block of the
 * message is enciphered on its own (ECB, Abstract), by encrypting under the
 * first key, decrypting under the second and encrypting under the third
 * (Section II.A, items a-c); decryption runs the same process in reverse
 * (Section II.A, last paragraph); the three keys give 48 round subkeys
 * (Listing 1.1, the 48-entry key array).  The paper does not print the DES
 * internals, so every table and step below is the Data Encryption Standard
 * (FIPS 46-3) written out literally:
 *   - a block is 64 bits numbered 1..64, bit 1 being the most significant bit
 *     of byte 0 (the standard's byte order);
 *   - key schedule: PC-1 drops the 8 parity bits, C and D (28 bits each) are
 *     rotated left by the shift schedule, PC-2 selects the 48-bit subkey;
 *   - cipher: IP, then 16 rounds L' = R, R' = L xor P(S(E(R) xor K)), then the
 *     final permutation IP^-1 applied to R16 L16;
 *   - decryption uses the subkeys in reverse order.
 * Every permutation works on arrays of single bits, one byte per bit, with
 * no precomputed combined tables, no bit tricks and no skipped steps: each of
 * the three stages of EDE does its own IP and IP^-1.
 *
 * Parity: PC-1 ignores the parity bits, so, as the standard says, they do not
 * affect the result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ---- FIPS 46-3 tables (1-based bit numbers, as printed in the standard) ---- */

/* Initial permutation IP. */
static const unsigned char IP[64] = {
    58, 50, 42, 34, 26, 18, 10, 2,
    60, 52, 44, 36, 28, 20, 12, 4,
    62, 54, 46, 38, 30, 22, 14, 6,
    64, 56, 48, 40, 32, 24, 16, 8,
    57, 49, 41, 33, 25, 17,  9, 1,
    59, 51, 43, 35, 27, 19, 11, 3,
    61, 53, 45, 37, 29, 21, 13, 5,
    63, 55, 47, 39, 31, 23, 15, 7};

/* Final permutation IP^-1. */
static const unsigned char FP[64] = {
    40, 8, 48, 16, 56, 24, 64, 32,
    39, 7, 47, 15, 55, 23, 63, 31,
    38, 6, 46, 14, 54, 22, 62, 30,
    37, 5, 45, 13, 53, 21, 61, 29,
    36, 4, 44, 12, 52, 20, 60, 28,
    35, 3, 43, 11, 51, 19, 59, 27,
    34, 2, 42, 10, 50, 18, 58, 26,
    33, 1, 41,  9, 49, 17, 57, 25};

/* Expansion E: 32 -> 48 bits. */
static const unsigned char E[48] = {
    32,  1,  2,  3,  4,  5,
     4,  5,  6,  7,  8,  9,
     8,  9, 10, 11, 12, 13,
    12, 13, 14, 15, 16, 17,
    16, 17, 18, 19, 20, 21,
    20, 21, 22, 23, 24, 25,
    24, 25, 26, 27, 28, 29,
    28, 29, 30, 31, 32,  1};

/* Permutation P applied to the 32 S-box output bits. */
static const unsigned char P[32] = {
    16,  7, 20, 21,
    29, 12, 28, 17,
     1, 15, 23, 26,
     5, 18, 31, 10,
     2,  8, 24, 14,
    32, 27,  3,  9,
    19, 13, 30,  6,
    22, 11,  4, 25};

/* Permuted choice 1: 64 key bits -> 56 (C = first 28, D = last 28). */
static const unsigned char PC1[56] = {
    57, 49, 41, 33, 25, 17,  9,
     1, 58, 50, 42, 34, 26, 18,
    10,  2, 59, 51, 43, 35, 27,
    19, 11,  3, 60, 52, 44, 36,
    63, 55, 47, 39, 31, 23, 15,
     7, 62, 54, 46, 38, 30, 22,
    14,  6, 61, 53, 45, 37, 29,
    21, 13,  5, 28, 20, 12,  4};

/* Permuted choice 2: C||D (56 bits) -> 48-bit subkey. */
static const unsigned char PC2[48] = {
    14, 17, 11, 24,  1,  5,
     3, 28, 15,  6, 21, 10,
    23, 19, 12,  4, 26,  8,
    16,  7, 27, 20, 13,  2,
    41, 52, 31, 37, 47, 55,
    30, 40, 51, 45, 33, 48,
    44, 49, 39, 56, 34, 53,
    46, 42, 50, 36, 29, 32};

/* Left-rotation amounts of C and D before subkeys 1..16. */
static const unsigned char SHIFTS[16] = {1, 1, 2, 2, 2, 2, 2, 2, 1, 2, 2, 2, 2, 2, 2, 1};

/* Substitution boxes S1..S8: [box][row 0..3][column 0..15]. */
static const unsigned char SBOX[8][4][16] = {
    {{14, 4, 13, 1, 2, 15, 11, 8, 3, 10, 6, 12, 5, 9, 0, 7},
     {0, 15, 7, 4, 14, 2, 13, 1, 10, 6, 12, 11, 9, 5, 3, 8},
     {4, 1, 14, 8, 13, 6, 2, 11, 15, 12, 9, 7, 3, 10, 5, 0},
     {15, 12, 8, 2, 4, 9, 1, 7, 5, 11, 3, 14, 10, 0, 6, 13}},
    {{15, 1, 8, 14, 6, 11, 3, 4, 9, 7, 2, 13, 12, 0, 5, 10},
     {3, 13, 4, 7, 15, 2, 8, 14, 12, 0, 1, 10, 6, 9, 11, 5},
     {0, 14, 7, 11, 10, 4, 13, 1, 5, 8, 12, 6, 9, 3, 2, 15},
     {13, 8, 10, 1, 3, 15, 4, 2, 11, 6, 7, 12, 0, 5, 14, 9}},
    {{10, 0, 9, 14, 6, 3, 15, 5, 1, 13, 12, 7, 11, 4, 2, 8},
     {13, 7, 0, 9, 3, 4, 6, 10, 2, 8, 5, 14, 12, 11, 15, 1},
     {13, 6, 4, 9, 8, 15, 3, 0, 11, 1, 2, 12, 5, 10, 14, 7},
     {1, 10, 13, 0, 6, 9, 8, 7, 4, 15, 14, 3, 11, 5, 2, 12}},
    {{7, 13, 14, 3, 0, 6, 9, 10, 1, 2, 8, 5, 11, 12, 4, 15},
     {13, 8, 11, 5, 6, 15, 0, 3, 4, 7, 2, 12, 1, 10, 14, 9},
     {10, 6, 9, 0, 12, 11, 7, 13, 15, 1, 3, 14, 5, 2, 8, 4},
     {3, 15, 0, 6, 10, 1, 13, 8, 9, 4, 5, 11, 12, 7, 2, 14}},
    {{2, 12, 4, 1, 7, 10, 11, 6, 8, 5, 3, 15, 13, 0, 14, 9},
     {14, 11, 2, 12, 4, 7, 13, 1, 5, 0, 15, 10, 3, 9, 8, 6},
     {4, 2, 1, 11, 10, 13, 7, 8, 15, 9, 12, 5, 6, 3, 0, 14},
     {11, 8, 12, 7, 1, 14, 2, 13, 6, 15, 0, 9, 10, 4, 5, 3}},
    {{12, 1, 10, 15, 9, 2, 6, 8, 0, 13, 3, 4, 14, 7, 5, 11},
     {10, 15, 4, 2, 7, 12, 9, 5, 6, 1, 13, 14, 0, 11, 3, 8},
     {9, 14, 15, 5, 2, 8, 12, 3, 7, 0, 4, 10, 1, 13, 11, 6},
     {4, 3, 2, 12, 9, 5, 15, 10, 11, 14, 1, 7, 6, 0, 8, 13}},
    {{4, 11, 2, 14, 15, 0, 8, 13, 3, 12, 9, 7, 5, 10, 6, 1},
     {13, 0, 11, 7, 4, 9, 1, 10, 14, 3, 5, 12, 2, 15, 8, 6},
     {1, 4, 11, 13, 12, 3, 7, 14, 10, 15, 6, 8, 0, 5, 9, 2},
     {6, 11, 13, 8, 1, 4, 10, 7, 9, 5, 0, 15, 14, 2, 3, 12}},
    {{13, 2, 8, 4, 6, 15, 11, 1, 10, 9, 3, 14, 5, 0, 12, 7},
     {1, 15, 13, 8, 10, 3, 7, 4, 12, 5, 6, 11, 0, 14, 9, 2},
     {7, 11, 4, 1, 9, 12, 14, 2, 0, 6, 10, 13, 15, 3, 5, 8},
     {2, 1, 14, 7, 4, 10, 8, 13, 15, 12, 9, 0, 3, 5, 6, 11}}};

/* ---- bit-array helpers ---- */

/* bytes[0..nbytes) -> bits[0..8*nbytes), bit 1 = MSB of byte 0. */
static void bytes_to_bits(const uint8_t *bytes, int nbytes, unsigned char *bits) {
    for (int i = 0; i < 8 * nbytes; i++) bits[i] = (bytes[i / 8] >> (7 - i % 8)) & 1;
}

static void bits_to_bytes(const unsigned char *bits, int nbytes, uint8_t *bytes) {
    for (int j = 0; j < nbytes; j++) {
        uint8_t v = 0;
        for (int b = 0; b < 8; b++) v = (uint8_t)((v << 1) | bits[8 * j + b]);
        bytes[j] = v;
    }
}

/* out[i] = in[table[i] - 1]: the standard's "bit table[i] of the input". */
static void permute(const unsigned char *in, unsigned char *out, const unsigned char *table, int n) {
    for (int i = 0; i < n; i++) out[i] = in[table[i] - 1];
}

/* ---- key schedule ---- */

/*
 * DES key schedule.  key: 8 bytes in the standard's order (parity bits, the
 * least significant bit of each byte, are ignored by PC-1).  Writes the 16
 * subkeys as bits (subkeys[i][0..47] = K_{i+1}) and, if cd is not NULL, the
 * 56-bit C_i||D_i register after each rotation (cd[i] = C_{i+1}D_{i+1}) and
 * C_0||D_0 to cd0.
 */
void oracle_des_key_schedule(const uint8_t key[8], unsigned char subkeys[16][48],
                             unsigned char cd0[56], unsigned char cd[16][56]) {
    unsigned char kbits[64], c[28], d[28], cdbits[56];
    bytes_to_bits(key, 8, kbits);
    permute(kbits, cdbits, PC1, 56);
    memcpy(c, cdbits, 28);
    memcpy(d, cdbits + 28, 28);
    if (cd0) memcpy(cd0, cdbits, 56);
    for (int i = 0; i < 16; i++) {
        for (int s = 0; s < SHIFTS[i]; s++) {
            unsigned char c0 = c[0], d0 = d[0];
            memmove(c, c + 1, 27);
            memmove(d, d + 1, 27);
            c[27] = c0;
            d[27] = d0;
        }
        memcpy(cdbits, c, 28);
        memcpy(cdbits + 28, d, 28);
        if (cd) memcpy(cd[i], cdbits, 56);
        permute(cdbits, subkeys[i], PC2, 48);
    }
}

/* Subkeys packed as 48-bit integers (bit 1 of the subkey = bit 47), for tests. */
void oracle_des_subkeys_u64(const uint8_t key[8], uint64_t out[16]) {
    unsigned char ks[16][48];
    oracle_des_key_schedule(key, ks, NULL, NULL);
    for (int i = 0; i < 16; i++) {
        uint64_t v = 0;
        for (int b = 0; b < 48; b++) v = (v << 1) | ks[i][b];
        out[i] = v;
    }
}

/* C_0 D_0 and C_i D_i (i = 1..16) as 56-bit integers (C bit 1 = bit 55). */
void oracle_des_cd_u64(const uint8_t key[8], uint64_t out[17]) {
    unsigned char ks[16][48], cd0[56], cd[16][56];
    oracle_des_key_schedule(key, ks, cd0, cd);
    for (int i = 0; i < 17; i++) {
        const unsigned char *src = i == 0 ? cd0 : cd[i - 1];
        uint64_t v = 0;
        for (int b = 0; b < 56; b++) v = (v << 1) | src[b];
        out[i] = v;
    }
}

/* ---- the cipher function and one DES block ---- */

/* f(R, K) = P(S(E(R) xor K)). */
static void cipher_f(const unsigned char r[32], const unsigned char k[48], unsigned char out[32]) {
    unsigned char x[48], s_out[32];
    permute(r, x, E, 48);
    for (int i = 0; i < 48; i++) x[i] ^= k[i];
    for (int box = 0; box < 8; box++) {
        const unsigned char *b = x + 6 * box;
        int row = 2 * b[0] + b[5];
        int col = 8 * b[1] + 4 * b[2] + 2 * b[3] + b[4];
        int v = SBOX[box][row][col];
        for (int j = 0; j < 4; j++) s_out[4 * box + j] = (v >> (3 - j)) & 1;
    }
    permute(s_out, out, P, 32);
}

/*
 * One DES block.  decrypt = 0 uses K1..K16, decrypt = 1 uses K16..K1.
 * If trace is not NULL it receives L_i||R_i for i = 0..16 (17 x 64 bits).
 */
static void des_block_bits(const unsigned char in[64], unsigned char out[64],
                           unsigned char ks[16][48], int decrypt, unsigned char trace[17][64]) {
    unsigned char lr[64], l[32], r[32], f[32], pre[64];
    permute(in, lr, IP, 64);
    memcpy(l, lr, 32);
    memcpy(r, lr + 32, 32);
    if (trace) { memcpy(trace[0], l, 32); memcpy(trace[0] + 32, r, 32); }
    for (int i = 0; i < 16; i++) {
        const unsigned char *k = ks[decrypt ? 15 - i : i];
        cipher_f(r, k, f);
        for (int j = 0; j < 32; j++) {
            unsigned char new_r = l[j] ^ f[j];
            l[j] = r[j];
            r[j] = new_r;
        }
        if (trace) { memcpy(trace[i + 1], l, 32); memcpy(trace[i + 1] + 32, r, 32); }
    }
    /* Preoutput is R16 L16. */
    memcpy(pre, r, 32);
    memcpy(pre + 32, l, 32);
    permute(pre, out, FP, 64);
}

/* Single DES on one 8-byte block. */
void oracle_des_block(const uint8_t key[8], const uint8_t in[8], uint8_t out[8], int decrypt) {
    unsigned char ks[16][48], ib[64], ob[64];
    oracle_des_key_schedule(key, ks, NULL, NULL);
    bytes_to_bits(in, 8, ib);
    des_block_bits(ib, ob, ks, decrypt, NULL);
    bits_to_bytes(ob, 8, out);
}

/* L_i R_i for i = 0..16 of one single-DES block, each as a 64-bit integer (L bit 1 = bit 63). */
void oracle_des_trace(const uint8_t key[8], const uint8_t in[8], int decrypt, uint64_t out[17]) {
    unsigned char ks[16][48], ib[64], ob[64], tr[17][64];
    oracle_des_key_schedule(key, ks, NULL, NULL);
    bytes_to_bits(in, 8, ib);
    des_block_bits(ib, ob, ks, decrypt, tr);
    for (int i = 0; i < 17; i++) {
        uint64_t v = 0;
        for (int b = 0; b < 64; b++) v = (v << 1) | tr[i][b];
        out[i] = v;
    }
}

/* ---- Triple DES, ECB ---- */

typedef struct {
    unsigned char ks[3][16][48];
    const uint8_t *in;
    uint8_t *out;
    uint64_t begin, end;
    int decrypt;
} tdes_job;

/*
 * EDE on one block: C = E_K3(D_K2(E_K1(P))); decryption is the reverse,
 * P = D_K1(E_K2(D_K3(C))).  Each stage is a complete DES with its own IP and
 * IP^-1.
 */
static void tdes_block(unsigned char ks[3][16][48], const uint8_t in[8], uint8_t out[8], int decrypt) {
    unsigned char a[64], b[64];
    bytes_to_bits(in, 8, a);
    if (!decrypt) {
        des_block_bits(a, b, ks[0], 0, NULL);
        des_block_bits(b, a, ks[1], 1, NULL);
        des_block_bits(a, b, ks[2], 0, NULL);
    } else {
        des_block_bits(a, b, ks[2], 1, NULL);
        des_block_bits(b, a, ks[1], 0, NULL);
        des_block_bits(a, b, ks[0], 1, NULL);
    }
    bits_to_bytes(b, 8, out);
}

static void *tdes_worker(void *arg) {
    tdes_job *job = (tdes_job *)arg;
    for (uint64_t i = job->begin; i < job->end; i++)
        tdes_block(job->ks, job->in + 8 * i, job->out + 8 * i, job->decrypt);
    return NULL;
}

/*
 * Triple DES (EDE) in ECB mode over n 8-byte blocks: every block on its own.
 * in and out may be the same buffer.  threads <= 1 runs on the calling
 * thread.  Returns 0, or -1 on a bad argument or thread failure.
 */
int oracle_tdes_ecb(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8],
                    const uint8_t *in, uint8_t *out, uint64_t n, int decrypt, int threads) {
    if ((n && (!in || !out)) || !k1 || !k2 || !k3) return -1;
    tdes_job base;
    oracle_des_key_schedule(k1, base.ks[0], NULL, NULL);
    oracle_des_key_schedule(k2, base.ks[1], NULL, NULL);
    oracle_des_key_schedule(k3, base.ks[2], NULL, NULL);
    base.in = in;
    base.out = out;
    base.decrypt = decrypt;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n) threads = n ? (int)n : 1;
    if (threads == 1) {
        base.begin = 0;
        base.end = n;
        tdes_worker(&base);
        return 0;
    }
    tdes_job *jobs = (tdes_job *)malloc(sizeof(tdes_job) * (size_t)threads);
    pthread_t *tids = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    if (!jobs || !tids) { free(jobs); free(tids); return -1; }
    int started = 0, rc = 0;
    for (int t = 0; t < threads; t++) {
        jobs[t] = base;
        jobs[t].begin = n * (uint64_t)t / (uint64_t)threads;
        jobs[t].end = n * (uint64_t)(t + 1) / (uint64_t)threads;
        if (pthread_create(&tids[t], NULL, tdes_worker, &jobs[t]) != 0) { rc = -1; break; }
        started++;
    }
    for (int t = 0; t < started; t++) pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    return rc;
}

/* ---- Triple DES in the block-parallel modes CBC and CTR ---- */
/*
 * The paper stops at ECB (Abstract).  These follow the modes' definitions in
 * NIST SP 800-38A, with TDEA encryption (EDE, above) as the forward cipher
 * E and its inverse as D, one block at a time, in order:
 *   CBC encrypt: C_1 = E(P_1 xor IV), C_j = E(P_j xor C_{j-1});
 *   CBC decrypt: P_1 = D(C_1) xor IV, P_j = D(C_j) xor C_{j-1};
 *   CTR: T_1 = IV, T_j = T_{j-1} + 1 (the whole 64-bit block read as a
 *        big-endian integer, modulo 2^64), O_j = E(T_j), C_j = P_j xor O_j;
 *        decryption is the same operation.
 * in and out may be the same buffer.  Returns 0, or -1 on a bad argument.
 */
static void key_schedules(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8],
                          unsigned char ks[3][16][48]) {
    oracle_des_key_schedule(k1, ks[0], NULL, NULL);
    oracle_des_key_schedule(k2, ks[1], NULL, NULL);
    oracle_des_key_schedule(k3, ks[2], NULL, NULL);
}

int oracle_tdes_cbc(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8], const uint8_t iv[8],
                    const uint8_t *in, uint8_t *out, uint64_t n, int decrypt) {
    if ((n && (!in || !out)) || !k1 || !k2 || !k3 || !iv) return -1;
    unsigned char ks[3][16][48];
    key_schedules(k1, k2, k3, ks);
    uint8_t prev[8], cur[8], x[8];
    memcpy(prev, iv, 8);
    for (uint64_t j = 0; j < n; j++) {
        memcpy(cur, in + 8 * j, 8);              /* read before writing: in may equal out */
        if (!decrypt) {
            for (int b = 0; b < 8; b++) x[b] = cur[b] ^ prev[b];
            tdes_block(ks, x, out + 8 * j, 0);
            memcpy(prev, out + 8 * j, 8);        /* C_j chains into the next block */
        } else {
            tdes_block(ks, cur, x, 1);
            for (int b = 0; b < 8; b++) out[8 * j + b] = x[b] ^ prev[b];
            memcpy(prev, cur, 8);                /* C_j chains into the next block */
        }
    }
    return 0;
}

int oracle_tdes_ctr(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8], const uint8_t iv[8],
                    const uint8_t *in, uint8_t *out, uint64_t n) {
    if ((n && (!in || !out)) || !k1 || !k2 || !k3 || !iv) return -1;
    unsigned char ks[3][16][48];
    key_schedules(k1, k2, k3, ks);
    uint64_t t = 0;
    for (int b = 0; b < 8; b++) t = (t << 8) | iv[b];
    for (uint64_t j = 0; j < n; j++, t++) {  /* unsigned wrap is the increment modulo 2^64 */
        uint8_t tb[8], o[8];
        for (int b = 0; b < 8; b++) tb[b] = (uint8_t)(t >> (56 - 8 * b));
        tdes_block(ks, tb, o, 0);
        for (int b = 0; b < 8; b++) out[8 * j + b] = in[8 * j + b] ^ o[b];
    }
    return 0;
}

/* ---- table export, so that tests can check the tables' structure ---- */

/* Copies a table by name into out (bytes); returns its length or -1. */
int oracle_table(const char *name, unsigned char *out) {
    struct { const char *n; const unsigned char *p; int len; } t[] = {
        {"IP", IP, 64}, {"FP", FP, 64}, {"E", E, 48}, {"P", P, 32},
        {"PC1", PC1, 56}, {"PC2", PC2, 48}, {"SHIFTS", SHIFTS, 16},
        {"SBOX", &SBOX[0][0][0], 512}};
    for (unsigned i = 0; i < sizeof t / sizeof t[0]; i++)
        if (strcmp(name, t[i].n) == 0) {
            if (out) memcpy(out, t[i].p, (size_t)t[i].len);
            return t[i].len;
        }
    return -1;
}
