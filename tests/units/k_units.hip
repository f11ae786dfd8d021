// k_units.hip -- unit kernels for the GPU tests: the bitsliced core's pieces on the device.
//
// Test infrastructure, built beside the library (build.py) into
// tests/units/libtdes_units.so and called only from tests/test_gpu_units.py.
// Each entry point launches one single-lane kernel over caller-owned device
// buffers and returns 0, or -1 if the launch failed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../paper_1305_4376_amd/csrc/bitslice_core.h"

namespace {

using namespace tdes_bs;

template <int S>
__device__ void run_box(const uint32_t (&x)[6], uint32_t *o, int variant) {
    uint32_t o0 = 0, o1 = 0, o2 = 0, o3 = 0;
    const uint32_t m = variant == 2 ? ~0u : 0u;
    if (variant == 0) {
        if constexpr (S == 0) sbox0(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 1) sbox1(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 2) sbox2(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 3) sbox3(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 4) sbox4(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 5) sbox5(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 6) sbox6(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
        if constexpr (S == 7) sbox7(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3);
    } else {
        if constexpr (S == 0) sbox0_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 1) sbox1_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 2) sbox2_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 3) sbox3_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 4) sbox4_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 5) sbox5_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 6) sbox6_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
        if constexpr (S == 7) sbox7_m(x[0], x[1], x[2], x[3], x[4], x[5], o0, o1, o2, o3, m, m, m, m);
    }
    o[0] = o0; o[1] = o1; o[2] = o2; o[3] = o3;
}

// out[((box * 3 + variant) * 2 + half) * 4 + j]: output plane j of the box for the 32 inputs
// 32 * half + t (bit t), starting from zero planes; variant 0: plain circuit, 1: masked with
// m = 0, 2: masked with m = ~0.
__global__ void sbox_kernel(uint32_t *out) {
    for (int half = 0; half < 2; half++) {
        uint32_t x[6];
        for (int i = 0; i < 6; i++) {
            x[i] = 0;
            for (int t = 0; t < 32; t++)
                if (((32 * half + t) >> (5 - i)) & 1) x[i] |= 1u << t;
        }
        for (int v = 0; v < 3; v++) {
            run_box<0>(x, out + ((0 * 3 + v) * 2 + half) * 4, v);
            run_box<1>(x, out + ((1 * 3 + v) * 2 + half) * 4, v);
            run_box<2>(x, out + ((2 * 3 + v) * 2 + half) * 4, v);
            run_box<3>(x, out + ((3 * 3 + v) * 2 + half) * 4, v);
            run_box<4>(x, out + ((4 * 3 + v) * 2 + half) * 4, v);
            run_box<5>(x, out + ((5 * 3 + v) * 2 + half) * 4, v);
            run_box<6>(x, out + ((6 * 3 + v) * 2 + half) * 4, v);
            run_box<7>(x, out + ((7 * 3 + v) * 2 + half) * 4, v);
        }
    }
}

__global__ void transpose_kernel(const uint32_t *in, uint32_t *out) {
    uint32_t w[32];
    for (int i = 0; i < 32; i++) w[i] = in[i];
    transpose32(w);
    for (int i = 0; i < 32; i++) out[i] = w[i];
}

// 32 blocks (a[j] = bytes 0..3, b[j] = bytes 4..7 of block j) through `rounds` rounds of one DES
// stage with per-lane round words ks (32 words); out[i * 64 + k]: after round i (i = 0: before the
// first), plane k of the half that started as L (k < 32) or as R (k >= 32).
__global__ void rounds_kernel(const uint32_t *blocks, const uint32_t *ks, int rounds, uint32_t *out) {
    uint32_t a[32], b[32], l[32], r[32];
    for (int j = 0; j < 32; j++) { a[j] = blocks[2 * j]; b[j] = blocks[2 * j + 1]; }
    transpose32(a);
    transpose32(b);
    for (int k = 0; k < 32; k++) {
        const int pl = kMaps.l0[k], pr = kMaps.r0[k];
        l[k] = pl < 32 ? a[pl] : b[pl - 32];
        r[k] = pr < 32 ? a[pr] : b[pr - 32];
    }
    for (int k = 0; k < 32; k++) { out[k] = l[k]; out[32 + k] = r[k]; }
    for (int i = 0; i < rounds; i++) {
        if (i % 2 == 0) feistel<true>(l, r, ks[2 * i], ks[2 * i + 1]);
        else feistel<true>(r, l, ks[2 * i], ks[2 * i + 1]);
        for (int k = 0; k < 32; k++) { out[(i + 1) * 64 + k] = l[k]; out[(i + 1) * 64 + 32 + k] = r[k]; }
    }
}

// One DES stage with folded masks (the wave-key path): out = the 64 planes (L16 then R16).
__global__ void folded_stage_kernel(const uint32_t *blocks, const uint32_t *dir_words, int stage, uint32_t *out) {
    uint32_t a[32], b[32], l[32], r[32];
    for (int j = 0; j < 32; j++) { a[j] = blocks[2 * j]; b[j] = blocks[2 * j + 1]; }
    transpose32(a);
    transpose32(b);
    for (int k = 0; k < 32; k++) {
        const int pl = kMaps.l0[k], pr = kMaps.r0[k];
        l[k] = pl < 32 ? a[pl] : b[pl - 32];
        r[k] = pr < 32 ? a[pr] : b[pr - 32];
    }
    des_stage_folded(l, r, dir_words + kFoldBase, stage);
    for (int k = 0; k < 32; k++) { out[k] = l[k]; out[32 + k] = r[k]; }
}

// ---- VALU issue-rate probe ----
//
// Each wave runs `iters` times a block of 128 VALU instructions of one kind on
// fixed registers (destinations v8..v23, sources v24..v55, never written, so
// no instruction waits on another), between two reads of the shader clock
// counter (s_memtime) and the 100 MHz real-time counter (s_memrealtime).
// A VGPR's bank is its index mod 4; row i's three sources sit in banks 0, 1
// and 2, and its fourth operand is a second bank-0 register.
#define PROBE_ROWS(M) \
    M(8, 24, 37, 46, 28) M(9, 28, 41, 50, 32) M(10, 32, 45, 54, 36) M(11, 36, 49, 26, 40) \
    M(12, 40, 53, 30, 44) M(13, 44, 25, 34, 48) M(14, 48, 29, 38, 52) M(15, 52, 33, 42, 24) \
    M(16, 24, 37, 46, 28) M(17, 28, 41, 50, 32) M(18, 32, 45, 54, 36) M(19, 36, 49, 26, 40) \
    M(20, 40, 53, 30, 44) M(21, 44, 25, 34, 48) M(22, 48, 29, 38, 52) M(23, 52, 33, 42, 24)
#define P_XOR(D, A, B, C, A2) "v_xor_b32 v" #D ", v" #A ", v" #B "\n"
#define P_ADD(D, A, B, C, A2) "v_add_u32 v" #D ", v" #A ", v" #B "\n"
#define P_LSHR(D, A, B, C, A2) "v_lshrrev_b32 v" #D ", 4, v" #A "\n"
#define P_LSHL(D, A, B, C, A2) "v_lshlrev_b32 v" #D ", 4, v" #A "\n"
#define P_BITOP3(D, A, B, C, A2) "v_bitop3_b32 v" #D ", v" #A ", v" #B ", v" #C " bitop3:0x96\n"
#define P_BITOP3_SAME(D, A, B, C, A2) "v_bitop3_b32 v" #D ", v" #A ", v" #A2 ", v" #C " bitop3:0x96\n"
#define P_PERM(D, A, B, C, A2) "v_perm_b32 v" #D ", v" #A ", v" #B ", v" #C "\n"
// Dependent chains: each instruction reads the result of the one d instructions before it (d = 1, 2, 4),
// sources in three banks.
#define PROBE_CHAIN1 "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v53, v34 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v53, v34 bitop3:0x96\n"
#define PROBE_CHAIN2 "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v53, v34 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v53, v34 bitop3:0x96\n"
#define PROBE_CHAIN4 "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v53, v34 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v53, v34 bitop3:0x96\n"
#define PROBE_CHAIN3 "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v53, v34 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v53, v34 bitop3:0x96\n"
#define PROBE_CHAIN8 "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v24, v24, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v28, v28, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v32, v32, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v36, v36, v53, v34 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v12, v12, v29, v42 bitop3:0x96\n" "v_bitop3_b32 v16, v16, v33, v46 bitop3:0x96\n" "v_bitop3_b32 v20, v20, v37, v50 bitop3:0x96\n" "v_bitop3_b32 v24, v24, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v28, v28, v45, v26 bitop3:0x96\n" "v_bitop3_b32 v32, v32, v49, v30 bitop3:0x96\n" "v_bitop3_b32 v36, v36, v53, v34 bitop3:0x96\n"
#define PROBE_CHAIN4R "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v9, v9, v30, v43 bitop3:0x96\n" "v_bitop3_b32 v10, v10, v35, v44 bitop3:0x96\n" "v_bitop3_b32 v11, v11, v36, v49 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v9, v9, v46, v27 bitop3:0x96\n" "v_bitop3_b32 v10, v10, v51, v28 bitop3:0x96\n" "v_bitop3_b32 v11, v11, v52, v33 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v25, v38 bitop3:0x96\n" "v_bitop3_b32 v9, v9, v30, v43 bitop3:0x96\n" "v_bitop3_b32 v10, v10, v35, v44 bitop3:0x96\n" "v_bitop3_b32 v11, v11, v36, v49 bitop3:0x96\n" "v_bitop3_b32 v8, v8, v41, v54 bitop3:0x96\n" "v_bitop3_b32 v9, v9, v46, v27 bitop3:0x96\n" "v_bitop3_b32 v10, v10, v51, v28 bitop3:0x96\n" "v_bitop3_b32 v11, v11, v52, v33 bitop3:0x96\n"
// Independent v_bitop3_b32 with sources in banks 0, 1, 2 and the result in bank 3 or in bank 0.
#define PROBE_DST3 "v_bitop3_b32 v11, v24, v37, v46 bitop3:0x96\n" "v_bitop3_b32 v15, v28, v41, v50 bitop3:0x96\n" "v_bitop3_b32 v19, v32, v45, v54 bitop3:0x96\n" "v_bitop3_b32 v23, v36, v49, v26 bitop3:0x96\n" "v_bitop3_b32 v11, v40, v53, v30 bitop3:0x96\n" "v_bitop3_b32 v15, v44, v25, v34 bitop3:0x96\n" "v_bitop3_b32 v19, v48, v29, v38 bitop3:0x96\n" "v_bitop3_b32 v23, v52, v33, v42 bitop3:0x96\n" "v_bitop3_b32 v11, v24, v37, v46 bitop3:0x96\n" "v_bitop3_b32 v15, v28, v41, v50 bitop3:0x96\n" "v_bitop3_b32 v19, v32, v45, v54 bitop3:0x96\n" "v_bitop3_b32 v23, v36, v49, v26 bitop3:0x96\n" "v_bitop3_b32 v11, v40, v53, v30 bitop3:0x96\n" "v_bitop3_b32 v15, v44, v25, v34 bitop3:0x96\n" "v_bitop3_b32 v19, v48, v29, v38 bitop3:0x96\n" "v_bitop3_b32 v23, v52, v33, v42 bitop3:0x96\n"
#define PROBE_DST0 "v_bitop3_b32 v8, v24, v37, v46 bitop3:0x96\n" "v_bitop3_b32 v12, v28, v41, v50 bitop3:0x96\n" "v_bitop3_b32 v16, v32, v45, v54 bitop3:0x96\n" "v_bitop3_b32 v20, v36, v49, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v40, v53, v30 bitop3:0x96\n" "v_bitop3_b32 v12, v44, v25, v34 bitop3:0x96\n" "v_bitop3_b32 v16, v48, v29, v38 bitop3:0x96\n" "v_bitop3_b32 v20, v52, v33, v42 bitop3:0x96\n" "v_bitop3_b32 v8, v24, v37, v46 bitop3:0x96\n" "v_bitop3_b32 v12, v28, v41, v50 bitop3:0x96\n" "v_bitop3_b32 v16, v32, v45, v54 bitop3:0x96\n" "v_bitop3_b32 v20, v36, v49, v26 bitop3:0x96\n" "v_bitop3_b32 v8, v40, v53, v30 bitop3:0x96\n" "v_bitop3_b32 v12, v44, v25, v34 bitop3:0x96\n" "v_bitop3_b32 v16, v48, v29, v38 bitop3:0x96\n" "v_bitop3_b32 v20, v52, v33, v42 bitop3:0x96\n"
// The round's operand forms: v_bitop3_b32 with a scalar register as its third source (the output
// XORs with their key mask), v_xor_b32 with a scalar first source (the input corrections), and the
// round's mix of one scalar bit-field extract (its result read by the next v_bitop3) per five
// v_bitop3 (s4, s5: any value).
#define P_BITOP3_S(D, A, B, C, A2) "v_bitop3_b32 v" #D ", v" #A ", v" #B ", s4 bitop3:0x96\n"
#define P_XOR_S(D, A, B, C, A2) "v_xor_b32 v" #D ", s4, v" #A "\n"
#define P_BFE_MIX(D, A, B, C, A2) "s_bfe_i32 s72, s5, 0x10003\n" "v_bitop3_b32 v" #D ", v" #A ", v" #B ", s72 bitop3:0x96\n" \
    "v_bitop3_b32 v" #D ", v" #A ", v" #B ", v" #C " bitop3:0x96\n" "v_bitop3_b32 v" #D ", v" #A ", v" #B ", v" #C " bitop3:0x69\n" \
    "v_bitop3_b32 v" #D ", v" #A ", v" #B ", v" #C " bitop3:0x5a\n" "v_bitop3_b32 v" #D ", v" #A ", v" #B ", v" #C " bitop3:0xa5\n"
#define PROBE_CLOBBERS_S PROBE_CLOBBERS, "s72", "scc"
#define PROBE_CASE_S(K, M)                                                                 \
    case K:                                                                                \
        for (int i = 0; i < iters; i++) asm volatile(PROBE_BLOCK(M)::: PROBE_CLOBBERS_S);  \
        break;
#define PROBE_CLOBBERS                                                                                       \
    "v8", "v9", "v10", "v11", "v12", "v13", "v14", "v15", "v16", "v17", "v18", "v19", "v20", "v21", "v22", "v23", \
        "v24", "v25", "v26", "v27", "v28", "v29", "v30", "v31", "v32", "v33", "v34", "v35", "v36", "v37", "v38",   \
        "v39", "v40", "v41", "v42", "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53",   \
        "v54", "v55"
#define PROBE_BLOCK(M) PROBE_ROWS(M) PROBE_ROWS(M) PROBE_ROWS(M) PROBE_ROWS(M) \
    PROBE_ROWS(M) PROBE_ROWS(M) PROBE_ROWS(M) PROBE_ROWS(M)
#define PROBE_CASE(K, M)                                                                   \
    case K:                                                                                \
        for (int i = 0; i < iters; i++) asm volatile(PROBE_BLOCK(M)::: PROBE_CLOBBERS);    \
        break;
#define PROBE_CHAIN_BLOCK(C) C C C C C C C C
#define PROBE_CHAIN_CASE(K, C)                                                             \
    case K:                                                                                \
        for (int i = 0; i < iters; i++) asm volatile(PROBE_CHAIN_BLOCK(C)::: PROBE_CLOBBERS); \
        break;

// clk[6 w + 0..5] for wave w: shader-clock count before and after, real-time count before and
// after, the wave's HW_ID register (SIMD, CU, shader array and engine fields) and its XCC_ID.
__global__ __launch_bounds__(256) void issue_probe_kernel(int op, int iters, uint64_t *clk) {
    const uint64_t c0 = __builtin_readcyclecounter();
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    switch (op) {
        PROBE_CASE(0, P_XOR)
        PROBE_CASE(1, P_ADD)
        PROBE_CASE(2, P_LSHR)
        PROBE_CASE(3, P_LSHL)
        PROBE_CASE(4, P_BITOP3)
        PROBE_CASE(5, P_BITOP3_SAME)
        PROBE_CASE(6, P_PERM)
        PROBE_CHAIN_CASE(7, PROBE_CHAIN1)
        PROBE_CHAIN_CASE(8, PROBE_CHAIN2)
        PROBE_CHAIN_CASE(9, PROBE_CHAIN4)
        PROBE_CHAIN_CASE(10, PROBE_CHAIN3)
        PROBE_CHAIN_CASE(11, PROBE_CHAIN8)
        PROBE_CHAIN_CASE(12, PROBE_CHAIN4R)
        PROBE_CHAIN_CASE(13, PROBE_DST3)
        PROBE_CHAIN_CASE(14, PROBE_DST0)
        PROBE_CASE(15, P_BITOP3_S)
        PROBE_CASE(16, P_XOR_S)
        PROBE_CASE_S(17, P_BFE_MIX)
        default:
            break;
    }
    const uint64_t c1 = __builtin_readcyclecounter();
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    uint32_t hw_id, xcc_id;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw_id));
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc_id));
    if (threadIdx.x % 64 == 0) {
        const uint32_t w = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
        clk[6 * w + 0] = c0;
        clk[6 * w + 1] = c1;
        clk[6 * w + 2] = t0;
        clk[6 * w + 3] = t1;
        clk[6 * w + 4] = hw_id;
        clk[6 * w + 5] = xcc_id;
    }
}

int status() { return hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess ? 0 : -1; }

}  // namespace

// The folded round pair of the bitsliced kernels (generated assembly) alone, `iters` times on planes
// made from the lane index, with the same clock and placement records as issue_probe_kernel; the
// planes are XORed into sink so that nothing is dead.
__global__ __launch_bounds__(256, 4) void rounds_probe_kernel(int iters, uint32_t w0, uint32_t w1, uint64_t *clk,
                                                             uint32_t *sink) {
    uint32_t x[32], y[32];
    for (int q = 0; q < 32; q++) {
        x[q] = threadIdx.x * (2 * q + 1) + blockIdx.x;
        y[q] = (threadIdx.x ^ (0x9E3779B9u * q)) + blockIdx.x;
    }
    const uint64_t c0 = __builtin_readcyclecounter();
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int i = 0; i < iters; i++) feistel_pair_asm<false>(x, y, w0, w1, w1, w0);
    const uint64_t c1 = __builtin_readcyclecounter();
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    uint32_t acc = 0;
    for (int q = 0; q < 32; q++) acc ^= x[q] ^ y[q];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    uint32_t hw_id, xcc_id;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw_id));
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc_id));
    if (threadIdx.x % 64 == 0) {
        const uint32_t w = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
        clk[6 * w + 0] = c0;
        clk[6 * w + 1] = c1;
        clk[6 * w + 2] = t0;
        clk[6 * w + 3] = t1;
        clk[6 * w + 4] = hw_id;
        clk[6 * w + 5] = xcc_id;
    }
}

// groups workgroups of 256 threads; dev_clk holds 6 * 4 * groups words.
extern "C" int units_issue_probe(int op, int groups, int iters, uint64_t *dev_clk) {
    if (op < 0 || op > 17 || groups < 1 || iters < 1) return -1;
    hipLaunchKernelGGL(issue_probe_kernel, dim3(groups), dim3(256), 0, 0, op, iters, dev_clk);
    return status();
}

// groups workgroups of 256 threads; dev_clk: 6 * 4 * groups words; dev_sink: 256 * groups words.
extern "C" int units_rounds_probe(int groups, int iters, uint64_t *dev_clk, uint32_t *dev_sink) {
    if (groups < 1 || iters < 1) return -1;
    hipLaunchKernelGGL(rounds_probe_kernel, dim3(groups), dim3(256), 0, 0, iters, 0x5A3C96E1u, 0x0F1E2D3Cu, dev_clk,
                       dev_sink);
    return status();
}

extern "C" int units_sbox(uint32_t *dev_out) {
    hipLaunchKernelGGL(sbox_kernel, dim3(1), dim3(1), 0, 0, dev_out);
    return status();
}

extern "C" int units_transpose(const uint32_t *dev_in, uint32_t *dev_out) {
    hipLaunchKernelGGL(transpose_kernel, dim3(1), dim3(1), 0, 0, dev_in, dev_out);
    return status();
}

extern "C" int units_rounds(const uint32_t *dev_blocks, const uint32_t *dev_ks, int rounds, uint32_t *dev_out) {
    if (rounds < 0 || rounds > 16) return -1;
    hipLaunchKernelGGL(rounds_kernel, dim3(1), dim3(1), 0, 0, dev_blocks, dev_ks, rounds, dev_out);
    return status();
}

extern "C" int units_folded_stage(const uint32_t *dev_blocks, const uint32_t *dev_dir_words, int stage,
                                  uint32_t *dev_out) {
    if (stage < 0 || stage > 2) return -1;
    hipLaunchKernelGGL(folded_stage_kernel, dim3(1), dim3(1), 0, 0, dev_blocks, dev_dir_words, stage, dev_out);
    return status();
}
