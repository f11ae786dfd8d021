/*
 * tdes.h -- C ABI of libtdes: Triple-DES (EDE) in ECB mode on AMD MI355X (gfx950).
 *
 * The operation (the paper's statement of the problem):
 *   - every 64-bit block of a message is enciphered on its own (ECB; Abstract);
 *   - a block is encrypted under K1, decrypted under K2 and encrypted under K3,
 *     and decryption runs the same process in reverse (Section II.A);
 *   - the three keys are expanded once into 48 round subkeys that are copied to
 *     the device before the blocks are processed (Listing 1.1);
 *   - only the kernels are on the timed path; file I/O and host<->device copies
 *     are not (Section III, the paragraph after Table II).
 * The cipher itself is DES as the standard defines it (FIPS 46-3): the paper
 * names it but prints none of its tables.
 *
 * Conventions shared by every call:
 *   - Blocks are 8 bytes in the standard's order: bit 1 is the most significant
 *     bit of byte 0.  Messages are whole blocks (no padding is added).
 *   - Keys are 8 bytes each, parity bit in the least significant bit of every
 *     byte; parity is ignored unless TDES_CHECK_PARITY is passed.  Two-key
 *     (K1 = K3) and one-key (K1 = K2 = K3) triples are accepted.
 *   - Every call returns an int status: TDES_OK (0) or a negative TDES_ERR_*.
 *     Argument errors are detected on the host before anything is enqueued.
 *   - "dev" pointers are device memory of the current HIP device; "host"
 *     pointers are host memory.  The caller owns every buffer it passes.
 *   - Device calls only enqueue work on `stream` (a hipStream_t; NULL is the
 *     null stream) and return; results are visible after the caller
 *     synchronises that stream.  A failed launch returns TDES_ERR_HIP.
 *   - Calls on different streams may run concurrently; the library keeps no
 *     mutable global state on the plain path.
 */
#ifndef TDES_H
#define TDES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define TDES_OK 0
#define TDES_ERR_NULL (-1)     /* a required pointer is NULL */
#define TDES_ERR_ALIGN (-2)    /* a block buffer is not 8-byte aligned (schedule: 4-byte) */
#define TDES_ERR_OVERLAP (-3)  /* in and out overlap without being equal */
#define TDES_ERR_SIZE (-4)     /* a size is out of range */
#define TDES_ERR_PARITY (-5)   /* TDES_CHECK_PARITY and a key byte has even parity */
#define TDES_ERR_WEAKKEY (-6)  /* TDES_REJECT_WEAK and a key is weak or semi-weak */
#define TDES_ERR_ARG (-7)      /* an enumerated argument (flag, direction, variant) is invalid */
#define TDES_ERR_HIP (-8)      /* a HIP runtime call or kernel launch failed */
#define TDES_ERR_NOMEM (-9)    /* the library could not allocate host or device memory */
#define TDES_ERR_BUDGET (-10)  /* serving: a request can never fit in the memory budget */
#define TDES_ERR_STATE (-11)   /* a call made in the wrong state (e.g. an unknown request id) */

/* ---- key schedule ---- */

/* Flags of tdes_expand_key. */
#define TDES_CHECK_PARITY 1u /* reject keys whose bytes do not all have odd parity */
#define TDES_REJECT_WEAK 2u  /* reject weak and semi-weak DES keys */

/* Directions. */
#define TDES_ENCRYPT 0
#define TDES_DECRYPT 1

/* Size in bytes of one expanded schedule (both directions). */
#define TDES_SCHED_BYTES 768

/*
 * An expanded key triple: the 48 round subkeys (3 keys x 16 rounds) in the
 * order the rounds use them, once for encryption and once for decryption.
 * Plain old data; copy it to the device with tdes_sched_upload.  The layout
 * of the words is private to the library.
 */
typedef struct tdes_sched {
    uint32_t w[TDES_SCHED_BYTES / 4];
} tdes_sched;

/*
 * Expand a key triple (Listing 1.1: three keys -> 48 subkeys).
 *   k1, k2, k3: host, 8 bytes each.  flags: 0 or TDES_CHECK_PARITY | TDES_REJECT_WEAK.
 *   out: host, receives the schedule.  Host-only; touches no GPU.
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG (unknown flag bits), TDES_ERR_PARITY,
 * TDES_ERR_WEAKKEY.  On error *out is left unchanged.
 */
int tdes_expand_key(const uint8_t k1[8], const uint8_t k2[8], const uint8_t k3[8], uint32_t flags,
                    tdes_sched *out);

/*
 * Copy `count` schedules from host memory to a device table (count * 768 bytes,
 * 4-byte aligned).  The copy is ordered on `stream` and complete when the call
 * returns, so `host` may be reused at once.  count == 0 is a no-op.
 * Errors: TDES_ERR_NULL, TDES_ERR_ALIGN, TDES_ERR_SIZE, TDES_ERR_HIP.
 */
int tdes_sched_upload(const tdes_sched *host, uint64_t count, void *dev_table, void *stream);

/* ---- plain ECB over one message ---- */

/*
 * Encrypt (decrypt) n_blocks blocks: out[i] = EDE(in[i]) (resp. its inverse).
 *   dev_sched: device, one schedule written by tdes_sched_upload.
 *   in, out:   device, n_blocks * 8 bytes each, 8-byte aligned.  in == out
 *              (in place, as in the paper) is allowed; partial overlap is not.
 *   n_blocks:  0 enqueues nothing; at most 2^58.
 * Errors: TDES_ERR_NULL, TDES_ERR_ALIGN, TDES_ERR_OVERLAP, TDES_ERR_SIZE, TDES_ERR_HIP.
 */
int tdes_ecb_encrypt(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, void *stream);
int tdes_ecb_decrypt(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, void *stream);

/* Kernel variants.  TDES_VARIANT_AUTO is the shipped default (the faster one on MI355X). */
#define TDES_VARIANT_AUTO 0
#define TDES_VARIANT_TABLE 1    /* combined S-box/P tables in LDS, one block per lane */
#define TDES_VARIANT_BITSLICE 2 /* 32 blocks per lane as bit planes, S-boxes as logic circuits */

/*
 * The same operation with an explicit direction and kernel variant, for A/B
 * comparisons.  Errors: as tdes_ecb_encrypt, plus TDES_ERR_ARG.
 */
int tdes_ecb_run(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, int direction,
                 int variant, void *stream);

/* ---- utilities ---- */

/* A short English description of a status code (static storage). */
const char *tdes_status_str(int status);

/*
 * Fill dev[0 .. n_words) with words first .. first+n_words-1 of the SplitMix64
 * stream seeded with `seed` (output i is the mix of seed + (i+1) * 0x9E3779B97F4A7C15;
 * Steele, Lea and Flood, OOPSLA 2014), stored little-endian.  Used to make
 * synthetic messages directly in device memory.  dev must be 8-byte aligned.
 * Errors: TDES_ERR_NULL, TDES_ERR_ALIGN, TDES_ERR_HIP.
 */
int tdes_fill_splitmix64(void *dev, uint64_t n_words, uint64_t seed, uint64_t first, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TDES_H */
