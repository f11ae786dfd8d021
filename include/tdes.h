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
#define TDES_SCHED_BYTES 1600

/*
 * An expanded key triple: the 48 round subkeys (3 keys x 16 rounds) in the
 * order the rounds use them, once for encryption and once for decryption,
 * each followed by key masks precomputed for the bitsliced kernels.  Plain
 * old data; copy it to the device with tdes_sched_upload.  The layout of the
 * words is private to the library.
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
 * Copy `count` schedules from host memory to a device table (count * 1600 bytes,
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

/*
 * Kernel variants.  TDES_VARIANT_AUTO is the shipped default: the faster one on
 * MI355X for the message's size, the table kernel below 2^20 blocks (its
 * latency is lower) and the bitsliced kernel from there on (its throughput is
 * about three times higher).
 */
#define TDES_VARIANT_AUTO 0
#define TDES_VARIANT_TABLE 1    /* combined S-box/P tables in LDS, one block per lane */
#define TDES_VARIANT_BITSLICE 2 /* 32 blocks per lane as bit planes, S-boxes as logic circuits */

/*
 * The same operation with an explicit direction and kernel variant, for A/B
 * comparisons.  Errors: as tdes_ecb_encrypt, plus TDES_ERR_ARG.
 */
int tdes_ecb_run(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, int direction,
                 int variant, void *stream);

/*
 * The paper's host loop (Listing 1.1, Section II.B): the same operation as
 * tdes_ecb_run, issued as consecutive launches of chunk_blocks blocks each
 * (the last one shorter), all on `stream`, each with `variant`
 * (TDES_VARIANT_AUTO chooses by the chunk's size) and workgroups of `threads`
 * threads (0: the kernels' own, 256; else 64, 128, 256, 512 or 1024).  It
 * exists to measure the paper's two launch parameters on this GPU: threads per
 * workgroup (Table I) and blocks per launch (Table II).  Every launch pays the
 * launch overhead and the kernel's latency, which dominate for small chunks;
 * a single launch per message (tdes_ecb_run) or per batch (tdes_ecb_batch)
 * avoids them.
 * Errors: as tdes_ecb_run; TDES_ERR_SIZE if chunk_blocks is 0; TDES_ERR_ARG
 * for any other thread count.
 */
int tdes_ecb_chunked(const void *dev_sched, const void *in, void *out, uint64_t n_blocks, uint64_t chunk_blocks,
                     int direction, int variant, uint32_t threads, void *stream);

/* ---- block-parallel modes on the same round core ---- */

/*
 * The paper is ECB only (Abstract); these run its cipher, unchanged, in the
 * two standard modes whose blocks are independent (NIST SP 800-38A, with
 * Triple-DES EDE as the block cipher).  Blocks, schedules and alignment as in
 * tdes_ecb_encrypt; n_blocks == 0 enqueues nothing.
 *   iv: host, 8 bytes in the standard's byte order, read at the call.
 *
 * CTR: out[j] = in[j] XOR EDE(T_j), with counter block T_j = iv + j modulo
 * 2^64 (the 8 bytes read as a big-endian integer).  The same call encrypts
 * and decrypts.  in == out is allowed.
 */
int tdes_ctr_crypt(const void *dev_sched, const uint8_t iv[8], const void *in, void *out, uint64_t n_blocks,
                   void *stream);

/*
 * CBC decryption: out[j] = EDE^-1(in[j]) XOR in[j-1], with in[-1] = iv.  Each
 * output block reads the ciphertext block before it, so in and out must not
 * overlap at all (in == out gives TDES_ERR_OVERLAP).  CBC encryption is a
 * chain over the blocks and has no parallel form; it is not offered.
 * Errors: as tdes_ecb_encrypt; TDES_ERR_NULL if iv is NULL.
 */
int tdes_cbc_decrypt(const void *dev_sched, const uint8_t iv[8], const void *in, void *out, uint64_t n_blocks,
                     void *stream);

/*
 * ECB over a message held in host memory (the paper's setting, Listing 1.1,
 * with the transfers overlapped instead of done once around the kernels):
 * chunks of chunk_blocks blocks move through three device buffers; the copy
 * in, the bitsliced kernel and the copy out each run on their own stream so
 * that chunks overlap.  Synchronous: returns when host_out holds the result
 * (work already queued on `stream` is waited for first).  Allocates
 * 3 * chunk_blocks * 8 bytes of device memory for the duration of the call.
 * host_in == host_out is allowed.  Host buffers should be pinned
 * (hipHostMalloc) for the copies to overlap.
 * Errors: TDES_ERR_NULL, TDES_ERR_ALIGN, TDES_ERR_ARG, TDES_ERR_SIZE
 * (chunk_blocks 0 or above 2^31), TDES_ERR_OVERLAP, TDES_ERR_NOMEM, TDES_ERR_HIP.
 */
int tdes_ecb_host(const void *dev_sched, const void *host_in, void *host_out, uint64_t n_blocks, int direction,
                  uint64_t chunk_blocks, void *stream);

/* ---- batched ECB: many messages, each with its own key triple and direction ---- */

/*
 * One message of a batch.  Offsets are in bytes from the batch's dev_base;
 * both must leave the message 8-byte aligned.  out_off == in_off works in
 * place.  The caller guarantees that every message lies inside its buffer.
 */
typedef struct tdes_job {
    uint64_t in_off;     /* input of the message */
    uint64_t out_off;    /* output of the message */
    uint64_t n_blocks;   /* length in 8-byte blocks; 0 is allowed; at most 2^40 */
    uint32_t sched_idx;  /* which schedule of the device table (TDES_SCHED_BYTES each) */
    uint32_t direction;  /* TDES_ENCRYPT or TDES_DECRYPT */
} tdes_job;

/* Batch context: device plan buffers, a tile counter, a captured graph and the
 * launch shape.  Not thread-safe: one host thread at a time per context. */
typedef struct tdes_ctx tdes_ctx;

/* Statistics of the last planned batch and the context's launch shape. */
typedef struct tdes_batch_info {
    uint64_t tiles;          /* work items of the last batch */
    uint64_t wave_tiles;     /* ... of up to 2048 blocks of one message */
    uint64_t lane_tiles;     /* ... of 64 lane slots of up to 32 blocks */
    uint64_t slots;          /* slot descriptors uploaded */
    uint64_t blocks;         /* message blocks in the batch */
    uint64_t padded_blocks;  /* block positions computed (tiles x 2048) */
    uint32_t threads;        /* threads per workgroup of the batch kernel */
    uint32_t groups_per_cu;  /* workgroups per compute unit in its grid */
    uint32_t graph_captures; /* graphs captured so far by this context */
    uint32_t wave_remainder; /* a message's last partial tile of at least this many blocks is a wave tile */
    uint32_t tiles_per_draw; /* tiles a wave takes per draw from the work counter */
    uint32_t pad;
} tdes_batch_info;

/* Flags of tdes_ecb_batch. */
#define TDES_BATCH_NO_GRAPH 1u     /* launch the kernel directly instead of replaying a graph */
#define TDES_BATCH_PER_MESSAGE 2u  /* baseline: one plain launch per message, automatic variant (no plan, no graph) */

/*
 * Create a batch context on HIP device `device` (a negative value: the current
 * device).  It allocates ~256 bytes of device memory and a stream there; the
 * plan buffers grow on demand.  Every later call on the context makes that
 * device current for its duration (and restores the caller's), so the stream
 * passed to it must belong to that device.
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG (no such device), TDES_ERR_HIP, TDES_ERR_NOMEM.
 */
int tdes_ctx_create(tdes_ctx **ctx, int device);

/* Destroy a context after its last batch has finished.  NULL is a no-op. */
int tdes_ctx_destroy(tdes_ctx *ctx);

/*
 * Encrypt or decrypt every message of a batch: ECB on each message as in
 * tdes_ecb_encrypt/decrypt, all messages in one launch of a persistent kernel
 * (replayed from a captured graph unless TDES_BATCH_NO_GRAPH).
 *   jobs: host, n_jobs entries; read before the call returns.
 *   dev_sched_table: device, n_scheds schedules written by tdes_sched_upload.
 *   dev_base: device; every offset is relative to it.
 * The host checks every job first: direction and schedule index, alignment,
 * and that no message writes bytes another message reads or writes (only
 * exact in-place is allowed).  The plan is copied to the device on `stream`;
 * the call can block until the previous batch's copy has been read.
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG, TDES_ERR_ALIGN, TDES_ERR_SIZE,
 * TDES_ERR_OVERLAP, TDES_ERR_NOMEM, TDES_ERR_HIP.
 */
int tdes_ecb_batch(tdes_ctx *ctx, const tdes_job *jobs, uint32_t n_jobs, const void *dev_sched_table,
                   uint64_t n_scheds, void *dev_base, uint32_t flags, void *stream);

/*
 * Run the last planned batch again (same messages, keys and buffers) without
 * planning or copying: one graph launch.  flags: 0 or TDES_BATCH_NO_GRAPH.
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG, TDES_ERR_STATE (no batch yet), TDES_ERR_HIP.
 */
int tdes_ecb_batch_replay(tdes_ctx *ctx, uint32_t flags, void *stream);

/*
 * Launch shape and tiling of the batch kernel, chosen by the autotuner (the
 * paper tunes its launch by hand, Tables I and II):
 *   threads:        threads per workgroup (64, 128, 192 or 256);
 *   groups_per_cu:  workgroups per compute unit in the grid (1..64);
 *   wave_remainder: a message's last partial tile of at least this many
 *                   blocks runs as a wave tile (one key per wave), a shorter
 *                   one as lane slots of 32 blocks packed 64 to a tile (one
 *                   key per lane); 1..2048, 0 for the default (1800);
 *   tiles_per_draw: tiles a wave takes per draw from the work counter after
 *                   its first; 1..16, 0 for the default (1).
 * Applies to the next batch (a new plan and graph capture when it changes).
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG.
 */
int tdes_ctx_set_tuning(tdes_ctx *ctx, uint32_t threads, uint32_t groups_per_cu, uint32_t wave_remainder,
                        uint32_t tiles_per_draw);
int tdes_ctx_get_info(const tdes_ctx *ctx, tdes_batch_info *info);

/* ---- batched ECB without allocation ---- */

/* Most jobs one tdes_ecb_batch_static call takes. */
#define TDES_STATIC_MAX_JOBS 65536

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as tdes_ecb_batch on the same jobs, with no context, no host
 * planning, no allocation and no host-device copy.  Its only working memory
 * is a fixed array of about 260 KiB per GPU inside the library (the job
 * plan: one word per job, a tile counter), set up on the first call on each
 * device and held until the process ends.
 *   dev_jobs: device, n_jobs tdes_job entries (8-byte aligned), read by the
 *             kernels; n_jobs at most TDES_STATIC_MAX_JOBS, 0 enqueues nothing.
 *   dev_sched_table: device, n_scheds schedules written by tdes_sched_upload.
 *   dev_base, base_bytes: device buffer (8-byte aligned) holding every input
 *             and output; offsets are relative to it.
 *   dev_rejected: device, one uint32 (may be NULL): receives the number of
 *             jobs the kernels refused -- a direction other than
 *             TDES_ENCRYPT/TDES_DECRYPT, a schedule index >= n_scheds, more
 *             than 2^40 blocks, an offset that is not a multiple of 8, input
 *             or output reaching past base_bytes, or input and output sharing
 *             bytes without being equal.  A refused job's output is not
 *             written.  If the call's wave tiles (2048 blocks each, per job
 *             rounded up) total 2^31 or more, every job is refused.
 * Runs on the current device, on `stream` (which must belong to it): a plan
 * launch, then the cipher launch.  Every call on one GPU uses that GPU's one
 * array, so calls whose launches may overlap on the same GPU race: order
 * them (one stream, or events).  As with tdes_ecb_batch, no message may
 * write bytes another message of the call reads or writes (not checked here).
 * Errors (synchronous, nothing enqueued): TDES_ERR_NULL, TDES_ERR_ALIGN,
 * TDES_ERR_SIZE (n_jobs or n_scheds out of range), TDES_ERR_ARG (device
 * index of 64 or more), TDES_ERR_HIP.
 */
int tdes_ecb_batch_static(const tdes_job *dev_jobs, uint32_t n_jobs, const void *dev_sched_table, uint64_t n_scheds,
                          void *dev_base, uint64_t base_bytes, uint32_t *dev_rejected, void *stream);

/* ---- serving: continuous batching of requests under resident keys ---- */

/* A request.  Its input is n_blocks * 8 bytes: copied from host_in when that
 * is not NULL, otherwise generated on the device from `seed`: block i, with
 * i = 256 * (64 * c + k) + t (t < 256, k < 64), is the little-endian word
 * X^k(W), where W is word 16384 * c + t of the SplitMix64 stream seeded with
 * `seed` (see tdes_fill_splitmix64) and X the xorshift64 step
 * x ^= x << 13, x ^= x >> 7, x ^= x << 17 (Marsaglia, 2003).  If host_out is
 * not NULL the output is copied there before the request completes. */
typedef struct tdes_request {
    uint64_t n_blocks;     /* 1 .. 2^32 */
    uint32_t key_id;       /* index into the server's resident schedule table */
    uint32_t direction;    /* TDES_ENCRYPT or TDES_DECRYPT */
    uint64_t seed;         /* payload stream when host_in is NULL */
    const void *host_in;   /* optional host input (must stay valid until completion) */
    void *host_out;        /* optional host output */
    uint64_t user_tag;     /* returned in the completion */
} tdes_request;

/* Completion record.  Times are seconds on the server's clock (tdes_server_now). */
typedef struct tdes_completion {
    uint64_t id;
    uint64_t user_tag;
    int32_t status;        /* TDES_OK, TDES_ERR_STATE if canceled, or the error that failed it */
    uint32_t pad;
    double t_arrival;      /* submission (or scheduled arrival in a trace) */
    double t_admit;        /* memory granted, placed in a step */
    double t_launch;       /* its step enqueued on the GPU */
    double t_complete;     /* the engine saw its step finish */
    const void *dev_out;   /* device output if the server keeps outputs, else NULL */
} tdes_completion;

typedef struct tdes_serve_config {
    uint64_t budget_bytes;    /* device memory for request inputs and outputs (one allocation) */
    uint32_t max_inflight;    /* steps in flight at once, each on its own stream (1..8) */
    uint32_t max_step_jobs;   /* requests per step */
    uint64_t max_step_blocks; /* blocks per step (a request larger than this runs alone) */
    uint32_t keep_outputs;    /* nonzero: outputs stay in device memory until tdes_server_release */
    uint32_t pad;
    /* Tuning of every step's batch (tdes_ctx_set_tuning); threads == 0 keeps the library's defaults for all four. */
    uint32_t threads, groups_per_cu, wave_remainder, tiles_per_draw;
    /* Backlog-sized steps: while the queue holds more than max_inflight * max_step_blocks blocks, a
       step may take up to (queued blocks / max_inflight) blocks, at most this many.  0, or a value
       not above max_step_blocks: every step is capped at max_step_blocks. */
    uint64_t backlog_step_blocks;
} tdes_serve_config;

typedef struct tdes_serve_stats {
    uint64_t submitted, completed, canceled;
    uint64_t bytes;             /* message bytes processed */
    uint64_t steps;             /* batched launches */
    uint64_t max_step_jobs;     /* largest step */
    uint64_t peak_pool_bytes;   /* most device memory granted at once */
    uint64_t pool_bytes_in_use;
    uint64_t pending;           /* queued, not yet admitted */
} tdes_serve_stats;

typedef struct tdes_server tdes_server;

/*
 * Start a server on the current device: allocates budget_bytes of device
 * memory and max_inflight batch contexts, and starts the engine thread.
 * dev_sched_table holds n_scheds schedules (tdes_sched_upload) and must stay
 * valid and unchanged while the server runs.
 * Errors: TDES_ERR_NULL, TDES_ERR_SIZE, TDES_ERR_ARG, TDES_ERR_NOMEM, TDES_ERR_HIP.
 */
int tdes_server_create(tdes_server **server, const tdes_serve_config *cfg, const void *dev_sched_table,
                       uint64_t n_scheds);

/* Stop the engine and free everything; requests not yet complete are dropped. */
int tdes_server_destroy(tdes_server *server);

/* Seconds since the server started (a monotonic clock). */
double tdes_server_now(const tdes_server *server);

/*
 * Queue a request (thread-safe); *id receives its id.  The request waits until
 * its input and output fit in the budget, then runs in the next free step.
 * Errors: TDES_ERR_NULL, TDES_ERR_ARG, TDES_ERR_SIZE (key id or length),
 * TDES_ERR_BUDGET (input plus output larger than the whole budget).
 */
int tdes_server_submit(tdes_server *server, const tdes_request *req, uint64_t *id);

/* Cancel a request that is still queued; it completes with TDES_ERR_STATE.
 * Errors: TDES_ERR_STATE if it was already admitted, completed or unknown. */
int tdes_server_cancel(tdes_server *server, uint64_t id);

/* Take up to max completion records (non-blocking); *n receives the count. */
int tdes_server_poll(tdes_server *server, tdes_completion *out, uint32_t max, uint32_t *n);

/* Wait until no request is outstanding.  TDES_ERR_STATE on timeout. */
int tdes_server_wait_idle(tdes_server *server, double timeout_s);

/* Free a kept output (keep_outputs).  TDES_ERR_STATE if there is none. */
int tdes_server_release(tdes_server *server, uint64_t id);

int tdes_server_stats(tdes_server *server, tdes_serve_stats *stats);

/*
 * Open-loop driver: submits reqs[i] at arrival[i] seconds after the call
 * starts (arrival non-decreasing), as a client would, and returns when all
 * have completed; out[i] receives request i's completion (latency =
 * t_complete - t_arrival).
 */
int tdes_server_run_trace(tdes_server *server, const tdes_request *reqs, const double *arrival, uint64_t n,
                          tdes_completion *out);

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
