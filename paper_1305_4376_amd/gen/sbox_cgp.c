/*
 * sbox_cgp.c -- shrink an S-box circuit of 3-input lookup gates by evolution
 * (Cartesian genetic programming with a (1 + lambda) strategy and neutral drift).
 *
 * Build-time tool, used by gen_sbox.py after sbox_search.c.  The genome is a
 * fixed array of gates (three operand references to earlier nodes and an
 * 8-bit truth table) plus four output references; only gates reachable from
 * the outputs are "active".  Fitness, compared lexicographically:
 *   1. errors: for each output, the number of the 64 input points where the
 *      output node differs from the S-box bit (an output may be the
 *      complement of its node: the Feistel XOR can absorb the inversion);
 *   2. cost: active gates, plus one per output whose gate cannot also absorb
 *      the XOR into the Feistel half (three distinct operands, or shared).
 * The search starts from a correct circuit, mutates a few genes per child,
 * and accepts a child that is no worse (neutral moves let it drift across
 * equal-cost circuits).  Any improvement is printed; the caller re-checks it
 * on all 64 inputs before using it.
 *
 * Usage: sbox_cgp SEED ITERATIONS SLACK s0..s63 < circuit (format of sbox_circuits.txt, one box)
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t tt;
#define MAXG 96
#define NIN 6

typedef struct {
    int a[MAXG], b[MAXG], c[MAXG];
    uint8_t lut[MAXG];
    int out[4];
    int ng;  /* gates: nodes NIN .. NIN+ng-1 */
} genome_t;

static uint64_t rs = 0x243F6A8885A308D3ull;
static uint64_t rnd(void) {
    uint64_t z = (rs += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int rndint(int n) { return (int)(rnd() % (uint64_t)n); }

static tt IN[NIN];
static tt T[4];

static inline tt lut3(int lut, tt a, tt b, tt c) {
    tt r = 0;
    if (lut & 0x01) r |= ~a & ~b & ~c;
    if (lut & 0x02) r |= ~a & ~b & c;
    if (lut & 0x04) r |= ~a & b & ~c;
    if (lut & 0x08) r |= ~a & b & c;
    if (lut & 0x10) r |= a & ~b & ~c;
    if (lut & 0x20) r |= a & ~b & c;
    if (lut & 0x40) r |= a & b & ~c;
    if (lut & 0x80) r |= a & b & c;
    return r;
}

static void active_set(const genome_t *g, char *act) {
    memset(act, 0, NIN + g->ng);
    for (int j = 0; j < 4; j++) act[g->out[j]] = 1;
    for (int k = NIN + g->ng - 1; k >= NIN; k--)
        if (act[k]) { act[g->a[k - NIN]] = 1; act[g->b[k - NIN]] = 1; act[g->c[k - NIN]] = 1; }
}

/* errors * 1000 + cost */
static long fitness(const genome_t *g) {
    tt v[NIN + MAXG];
    char act[NIN + MAXG];
    active_set(g, act);
    for (int i = 0; i < NIN; i++) v[i] = IN[i];
    int gates = 0;
    for (int k = 0; k < g->ng; k++) {
        int n = NIN + k;
        if (!act[n]) continue;
        gates++;
        v[n] = lut3(g->lut[k], v[g->a[k]], v[g->b[k]], v[g->c[k]]);
    }
    long err = 0;
    for (int j = 0; j < 4; j++) {
        int e0 = __builtin_popcountll(v[g->out[j]] ^ T[j]);
        int e1 = 64 - e0;
        err += e0 < e1 ? e0 : e1;
    }
    int extra = 0;
    for (int j = 0; j < 4; j++) {
        int o = g->out[j];
        int shared = 0;
        for (int i = 0; i < j; i++) if (g->out[i] == o) shared = 1;
        if (o < NIN) { extra++; continue; }
        int k = o - NIN;
        int distinct = 1 + (g->b[k] != g->a[k]) + (g->c[k] != g->a[k] && g->c[k] != g->b[k]);
        for (int m = 0; m < g->ng && !shared; m++)
            if (act[NIN + m] && (g->a[m] == o || g->b[m] == o || g->c[m] == o)) shared = 1;
        if (distinct == 3 || shared) extra++;
    }
    return err * 1000 + gates + extra;
}

static void mutate(genome_t *g, int nmut) {
    for (int m = 0; m < nmut; m++) {
        int r = rndint(100);
        if (r < 4) {
            g->out[rndint(4)] = NIN + rndint(g->ng);
            continue;
        }
        int k = rndint(g->ng);
        int n = NIN + k;
        if (r < 60) {
            int which = rndint(3);
            int ref = rndint(n);
            if (which == 0) g->a[k] = ref; else if (which == 1) g->b[k] = ref; else g->c[k] = ref;
        } else if (r < 85) {
            g->lut[k] ^= (uint8_t)(1u << rndint(8));
        } else {
            g->lut[k] = (uint8_t)rnd();
        }
    }
}

/* Node values of a genome (all gates, active or not). */
static void values(const genome_t *g, tt *v) {
    for (int i = 0; i < NIN; i++) v[i] = IN[i];
    for (int k = 0; k < g->ng; k++) v[NIN + k] = lut3(g->lut[k], v[g->a[k]], v[g->b[k]], v[g->c[k]]);
}

/* Is t a function of (x, y, z)?  Writes its table. */
static int fn_of(tt t, tt x, tt y, tt z, uint8_t *lut) {
    int l = 0;
    for (int m = 0; m < 8; m++) {
        tt cell = ((m & 4) ? x : ~x) & ((m & 2) ? y : ~y) & ((m & 1) ? z : ~z);
        if (!cell) continue;
        tt on = cell & t;
        if (on && on != cell) return 0;
        if (on) l |= 1 << m;
    }
    *lut = (uint8_t)l;
    return 1;
}

/* desc[n] = 1 if node n depends on gate node h (or is h). */
static void descendants(const genome_t *g, int h, char *desc) {
    memset(desc, 0, NIN + g->ng);
    desc[h] = 1;
    for (int k = h - NIN + 1; k < g->ng; k++) {
        int n = NIN + k;
        if (desc[g->a[k]] || desc[g->b[k]] || desc[g->c[k]]) desc[n] = 1;
    }
}

/*
 * Resubstitution: re-express an active gate h as one gate over three nodes that
 * do not depend on h, keeping the change when the fitness (cost) drops because
 * part of h's old fan-in cone is no longer used.  The gate keeps its place in
 * the array; its operands must precede it, so candidates are limited to nodes
 * with a smaller index.  Returns 1 if the genome improved.
 */
static int resub_pass(genome_t *g) {
    tt v[NIN + MAXG];
    char act[NIN + MAXG];
    int improved = 0;
    long f0 = fitness(g);
    for (int k = 0; k < g->ng; k++) {
        int h = NIN + k;
        active_set(g, act);
        if (!act[h]) continue;
        values(g, v);
        const tt t = v[h];
        int done = 0;
        for (int a = 0; a < h && !done; a++)
            for (int b = a + 1; b < h && !done; b++)
                for (int c = b + 1; c < h && !done; c++) {
                    uint8_t lut;
                    if (!fn_of(t, v[a], v[b], v[c], &lut)) continue;
                    genome_t trial = *g;
                    trial.a[k] = a; trial.b[k] = b; trial.c[k] = c; trial.lut[k] = lut;
                    long f = fitness(&trial);
                    if (f < f0) { *g = trial; f0 = f; improved = done = 1; }
                }
    }
    return improved;
}

int main(int argc, char **argv) {
    if (argc < 4 + 64) {
        fprintf(stderr, "usage: sbox_cgp SEED ITERATIONS SLACK s0..s63 < circuit\n");
        return 2;
    }
    rs ^= strtoull(argv[1], NULL, 0) * 0x9E3779B97F4A7C15ull;
    long iters = atol(argv[2]);
    int slack = atoi(argv[3]);
    int sbox[64];
    for (int p = 0; p < 64; p++) sbox[p] = atoi(argv[4 + p]);
    for (int i = 0; i < NIN; i++) {
        IN[i] = 0;
        for (int p = 0; p < 64; p++) if ((p >> (5 - i)) & 1) IN[i] |= 1ull << p;
    }
    for (int j = 0; j < 4; j++) {
        T[j] = 0;
        for (int p = 0; p < 64; p++) if ((sbox[p] >> (3 - j)) & 1) T[j] |= 1ull << p;
    }
    /* read the starting circuit */
    genome_t g;
    memset(&g, 0, sizeof g);
    char line[256];
    int map[NIN + MAXG];
    for (int i = 0; i < NIN; i++) map[i] = i;
    while (fgets(line, sizeof line, stdin)) {
        int node, a, b, c, lut, o0, o1, o2, o3;
        if (sscanf(line, "g %d %d %d %d %d", &node, &a, &b, &c, &lut) == 5) {
            int k = g.ng++;
            g.a[k] = map[a]; g.b[k] = map[b]; g.c[k] = map[c]; g.lut[k] = (uint8_t)lut;
            map[node] = NIN + k;
        } else if (sscanf(line, "out %d %d %d %d", &o0, &o1, &o2, &o3) == 4) {
            g.out[0] = map[o0]; g.out[1] = map[o1]; g.out[2] = map[o2]; g.out[3] = map[o3];
        }
    }
    /* slack: extra inactive gates available to the search */
    for (int s = 0; s < slack && g.ng < MAXG; s++) {
        int k = g.ng++;
        int n = NIN + k;
        g.a[k] = rndint(n); g.b[k] = rndint(n); g.c[k] = rndint(n); g.lut[k] = (uint8_t)rnd();
    }
    long best = fitness(&g);
    if (best >= 1000) { fprintf(stderr, "start circuit is not correct\n"); return 1; }
    while (resub_pass(&g)) {}
    best = fitness(&g);
    fprintf(stderr, "after resubstitution: cost %ld\n", best);
    genome_t bestg = g, parent = g;
    long pf = best;
    const int lambda = 4;
    for (long it = 0; it < iters; it++) {
        genome_t child_best;
        long cf_best = 1L << 60;
        for (int l = 0; l < lambda; l++) {
            genome_t ch = parent;
            mutate(&ch, 1 + rndint(3));
            long f = fitness(&ch);
            if (f <= cf_best) { cf_best = f; child_best = ch; }
        }
        if (cf_best <= pf) { parent = child_best; pf = cf_best; }
        if ((it & 8191) == 0 && pf < 1000) {
            while (resub_pass(&parent)) {}
            pf = fitness(&parent);
        }
        if (pf < best) {
            best = pf;
            bestg = parent;
            fprintf(stderr, "iter %ld: cost %ld\n", it, best);
        }
    }
    /* print the active part of the best circuit, renumbered */
    char act[NIN + MAXG];
    active_set(&bestg, act);
    int ren[NIN + MAXG];
    for (int i = 0; i < NIN; i++) ren[i] = i;
    int next = NIN, gates = 0;
    for (int k = 0; k < bestg.ng; k++) if (act[NIN + k]) { ren[NIN + k] = next++; gates++; }
    printf("cost %ld gates %d\n", best, gates);
    for (int k = 0; k < bestg.ng; k++)
        if (act[NIN + k])
            printf("g %d %d %d %d %d\n", ren[NIN + k], ren[bestg.a[k]], ren[bestg.b[k]], ren[bestg.c[k]], bestg.lut[k]);
    printf("out %d %d %d %d\n", ren[bestg.out[0]], ren[bestg.out[1]], ren[bestg.out[2]], ren[bestg.out[3]]);
    return 0;
}
