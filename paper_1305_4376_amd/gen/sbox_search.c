/*
 * sbox_search.c -- search for small logic circuits of 3-input lookup gates
 * (gfx950's v_bitop3_b32: any Boolean function of three words) computing the
 * four output bits of one 6-to-4 S-box, for the bitsliced kernel.
 *
 * Build-time tool.  Input: the S-box's 64 entries (argument list).  Output
 * (stdout): the best circuit found, one gate per line.  The Python driver
 * (gen_sbox.py) checks every circuit on all 64 inputs before emitting code.
 * Each improvement is printed as it is found; the last block is the best.
 * With IMPROVE set it instead improves a given circuit (large-neighbourhood
 * search: re-realize one output at a time from the others' gates).
 *
 * Functions are truth tables over the 64 input points (bit p = value at input
 * p; input variable x_i is bit 5-i of p, x_0 being the box's first input).
 * Sub-problems are partial functions: a value and a care mask.
 *
 * Method: realize(t, care) returns a node equal to t (or to its complement,
 * which costs nothing: a lookup gate can invert any operand) wherever care is
 * set, by trying in order
 *   0. an existing node;
 *   1. one new gate over three existing nodes (t must be a function of them
 *      on the care set);
 *   2. two new gates: t = F(g, d, e) with g = G(a, b, c), found by fixing the
 *      pair (d, e): on every cell of (d, e) where t is not constant, g must
 *      equal t or its complement, a parity problem over four cells;
 *   3. a decomposition, chosen at random among the options with the lowest
 *      estimated cost (from the sub-problems' support sizes): Shannon on a
 *      node v (an input or an existing gate), t = F(v, A, B) with A = t where
 *      v = 0 and B = t where v = 1; or a bi-decomposition on two nodes,
 *      t = F(a, b, X), where on every cell of (a, b) t is constant or equal to
 *      X or its complement, the polarities picked to make X cheapest.
 * The four outputs are realized in a random order, sharing all nodes (with
 * WIDTH > 1, each output is realized WIDTH times from the same circuit and
 * the attempt that adds the fewest gates is kept); many
 * random restarts run and the circuit with the fewest gates is kept, ties
 * broken by the cost: the gate count plus one for each output whose final gate
 * cannot also absorb the XOR into the Feistel half (a final gate with three
 * operands, or one that is shared).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t tt;

#define MAXN 96

typedef struct {
    int in[3];   /* operand node indices (-1 = unused) */
    int lut;     /* 8-bit table: bit (4a+2b+c) */
} gate_t;

typedef struct {
    tt val[MAXN];
    gate_t g[MAXN];
    int n;       /* nodes 0..5 are inputs */
} circuit_t;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) {
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int rndint(int n) { return (int)(rnd() % (uint64_t)n); }

static tt input_tt(int i) {
    tt v = 0;
    for (int p = 0; p < 64; p++)
        if ((p >> (5 - i)) & 1) v |= 1ull << p;
    return v;
}

static tt lut3(int lut, tt a, tt b, tt c) {
    tt r = 0;
    for (int m = 0; m < 8; m++)
        if ((lut >> m) & 1) r |= ((m & 4) ? a : ~a) & ((m & 2) ? b : ~b) & ((m & 1) ? c : ~c);
    return r;
}

/* Is t (on care) a function of nodes a, b, c?  If so, return the table (don't-care cells random). */
static int function_of(const circuit_t *C, tt t, tt care, int a, int b, int c, int *lut_out) {
    tt va = C->val[a], vb = C->val[b], vc = C->val[c];
    int lut = 0;
    for (int m = 0; m < 8; m++) {
        tt cell = ((m & 4) ? va : ~va) & ((m & 2) ? vb : ~vb) & ((m & 1) ? vc : ~vc) & care;
        if (!cell) {
            if (rnd() & 1) lut |= 1 << m;
            continue;
        }
        tt on = cell & t;
        if (on && on != cell) return 0;
        if (on) lut |= 1 << m;
    }
    *lut_out = lut;
    return 1;
}

static int add_gate(circuit_t *C, int a, int b, int c, int lut) {
    if (C->n >= MAXN) return -1;
    int k = C->n++;
    C->g[k].in[0] = a; C->g[k].in[1] = b; C->g[k].in[2] = c; C->g[k].lut = lut;
    C->val[k] = lut3(lut, C->val[a], C->val[b], C->val[c]);
    return k;
}

/* Support of a partial function: variables i with two cared points differing only in x_i and in value. */
static int support(tt t, tt care) {
    int s = 0;
    for (int i = 0; i < 6; i++) {
        int sh = 5 - i;
        tt lo = ~input_tt(i);  /* points with x_i = 0 */
        tt both = care & (care >> (1 << sh)) & lo;          /* p and p + 2^sh both cared, p has x_i = 0 */
        tt diff = (t ^ (t >> (1 << sh))) & both;
        if (diff) s |= 1 << i;
    }
    return s;
}

static int popc(int x) { return __builtin_popcount(x); }

/* Step 0: an existing node equal to t or its complement on care. */
static int find_existing(const circuit_t *C, tt t, tt care) {
    for (int k = 0; k < C->n; k++) {
        if (((C->val[k] ^ t) & care) == 0) return k;
        if (((~C->val[k] ^ t) & care) == 0) return k;
    }
    return -1;
}

/* Step 1: one gate. */
static int try_one(circuit_t *C, tt t, tt care) {
    int n = C->n, best[3], found = 0, lut = 0;
    /* scan in a random rotation so that ties vary between restarts */
    int off = rndint(n);
    for (int ia = 0; ia < n && !found; ia++) {
        int a = (ia + off) % n;
        for (int b = 0; b < n && !found; b++) {
            if (b == a) continue;
            for (int c = b + 1; c < n; c++) {
                if (c == a) continue;
                if (function_of(C, t, care, a, b, c, &lut)) {
                    best[0] = a; best[1] = b; best[2] = c; found = 1;
                    break;
                }
            }
        }
    }
    if (!found) return -1;
    return add_gate(C, best[0], best[1], best[2], lut);
}

/* Parity union-find over 4 cells. */
static int uf_find(int *par, int *rel, int x, int *p) {
    int acc = 0;
    while (par[x] != x) { acc ^= rel[x]; x = par[x]; }
    *p = acc;
    return x;
}
static int uf_union(int *par, int *rel, int x, int y, int want) {
    int px, py, rx = uf_find(par, rel, x, &px), ry = uf_find(par, rel, y, &py);
    if (rx == ry) return (px ^ py) == want;
    par[rx] = ry; rel[rx] = px ^ py ^ want;
    return 1;
}

/* Step 2: two gates, t = F(g, d, e), g = G(a, b, c). */
static int try_two(circuit_t *C, tt t, tt care, int budget) {
    int n = C->n;
    int tries = 0;
    int offd = rndint(n);
    for (int id = 0; id < n; id++) {
        int d = (id + offd) % n;
        for (int e = d; e < n; e++) {
            tt vd = C->val[d], ve = C->val[e];
            tt cellmask[4]; int live[4], nlive = 0;
            for (int k = 0; k < 4; k++) {
                tt cell = ((k & 2) ? vd : ~vd) & ((k & 1) ? ve : ~ve) & care;
                tt on = cell & t;
                cellmask[k] = cell;
                live[k] = (on && on != cell);
                nlive += live[k];
            }
            if (nlive == 0) continue;
            for (int a = 0; a < n; a++)
                for (int b = a + 1; b < n; b++)
                    for (int c = b + 1; c < n; c++) {
                        if (++tries > budget) return -1;
                        tt va = C->val[a], vb = C->val[b], vc = C->val[c];
                        int par[4] = {0, 1, 2, 3}, rel[4] = {0, 0, 0, 0};
                        int ok = 1;
                        int glut_fixed[8], gval[8];
                        for (int m = 0; m < 8 && ok; m++) {
                            tt cell = ((m & 4) ? va : ~va) & ((m & 2) ? vb : ~vb) & ((m & 1) ? vc : ~vc);
                            int first = -1, fval = 0;
                            glut_fixed[m] = 0;
                            for (int k = 0; k < 4 && ok; k++) {
                                if (!live[k]) continue;
                                tt s = cell & cellmask[k];
                                if (!s) continue;
                                tt on = s & t;
                                if (on && on != s) { ok = 0; break; }
                                int v = on ? 1 : 0;
                                if (first < 0) { first = k; fval = v; }
                                else if (!uf_union(par, rel, k, first, v ^ fval)) ok = 0;
                            }
                            if (first >= 0) { glut_fixed[m] = 1; gval[m] = first * 2 + fval; }
                        }
                        if (!ok) continue;
                        /* choose polarities: roots 0, others by relation */
                        int pol[4];
                        for (int k = 0; k < 4; k++) { int p; uf_find(par, rel, k, &p); pol[k] = p; }
                        int glut = 0;
                        for (int m = 0; m < 8; m++) {
                            int bit;
                            if (glut_fixed[m]) { int k = gval[m] / 2, v = gval[m] & 1; bit = v ^ pol[k]; }
                            else bit = (int)(rnd() & 1);
                            glut |= bit << m;
                        }
                        int g = add_gate(C, a, b, c, glut);
                        int flut;
                        if (g >= 0 && function_of(C, t, care, g, d, e, &flut)) return add_gate(C, g, d, e, flut);
                        if (g >= 0) C->n--;  /* should not happen */
                    }
        }
    }
    return -1;
}

static int realize(circuit_t *C, tt t, tt care, int depth, int budget2);

/* Rough gate cost of a partial function with k support variables. */
static int est_cost(tt t, tt care, const circuit_t *C) {
    static const int cost_by_support[7] = {0, 0, 10, 10, 25, 55, 100};
    if (find_existing(C, t, care) >= 0) return 0;
    return cost_by_support[popc(support(t, care))];
}

/*
 * Step 3: decompose, choosing at random among the cheapest estimated options:
 *   Shannon on a node v:       t = F(v, A, B), A = t where v = 0, B = t where v = 1;
 *   bi-decomposition on (a,b): t = F(a, b, X), where on each of the four cells of
 *       (a, b) t is constant or equal to X or its complement; the polarity of each
 *       cell is chosen to make X cheapest (one sub-problem instead of two).
 */
static int g_allow_bidec = 1;   /* per restart: whether bi-decompositions are offered */

static int decompose(circuit_t *C, tt t, tt care, int depth, int budget2) {
    int n = C->n;
    enum { MAXOPT = 4096 };
    static int opt_kind[MAXOPT], opt_a[MAXOPT], opt_b[MAXOPT], opt_pol[MAXOPT], opt_cost[MAXOPT];
    int nopt = 0, best = 1 << 30;
    for (int v = 0; v < n && nopt < MAXOPT; v++) {
        tt val = C->val[v];
        tt c0 = care & ~val, c1 = care & val;
        if (!c0 || !c1) continue;
        int cost = 10 + est_cost(t, c0, C) + est_cost(t, c1, C) + (int)(rnd() % 6);
        opt_kind[nopt] = 0; opt_a[nopt] = v; opt_cost[nopt] = cost; nopt++;
        if (cost < best) best = cost;
    }
    for (int a = 0; a < n && g_allow_bidec; a++)
        for (int b = a + 1; b < n && nopt < MAXOPT; b++) {
            tt va = C->val[a], vb = C->val[b];
            tt cells[4];
            int live = 0;
            for (int k = 0; k < 4; k++) {
                cells[k] = ((k & 2) ? va : ~va) & ((k & 1) ? vb : ~vb) & care;
                tt on = cells[k] & t;
                if (on && on != cells[k]) live |= 1 << k;
            }
            if (popc(live) < 2) continue;  /* one live cell is a Shannon-like case */
            tt xcare = 0;
            for (int k = 0; k < 4; k++) if (live >> k & 1) xcare |= cells[k];
            const int tsup = popc(support(t, care));
            int bestpol = 0, bestc = 1 << 30;
            for (int pol = 0; pol < 16; pol++) {
                if (pol & ~live) continue;
                if (pol & 1 & live) continue;  /* complement symmetry: fix the first live cell */
                tt x = t;
                for (int k = 0; k < 4; k++) if (pol >> k & 1) x ^= cells[k];
                /* progress: a smaller care set or a smaller support */
                if (xcare == care && popc(support(x, xcare)) >= tsup) continue;
                int c = est_cost(x, xcare, C);
                if (c < bestc) { bestc = c; bestpol = pol; }
            }
            if (bestc >= (1 << 30)) continue;
            int cost = 10 + bestc + (int)(rnd() % 6);
            opt_kind[nopt] = 1; opt_a[nopt] = a; opt_b[nopt] = b; opt_pol[nopt] = bestpol; opt_cost[nopt] = cost; nopt++;
            if (cost < best) best = cost;
        }
    if (!nopt) return -1;
    int cand[MAXOPT], nc = 0;
    for (int i = 0; i < nopt; i++) if (opt_cost[i] <= best) cand[nc++] = i;
    int o = cand[rndint(nc)];
    if (opt_kind[o] == 0) {
        int v = opt_a[o];
        tt val = C->val[v];
        int A = realize(C, t, care & ~val, depth + 1, budget2);
        if (A < 0) return -1;
        int B = realize(C, t, care & val, depth + 1, budget2);
        if (B < 0) return -1;
        int lut;
        if (!function_of(C, t, care, v, A, B, &lut)) return -1;
        return add_gate(C, v, A, B, lut);
    } else {
        int a = opt_a[o], b = opt_b[o];
        tt va = C->val[a], vb = C->val[b];
        tt x = t, xcare = 0;
        for (int k = 0; k < 4; k++) {
            tt cell = ((k & 2) ? va : ~va) & ((k & 1) ? vb : ~vb) & care;
            tt on = cell & t;
            if (on && on != cell) {
                xcare |= cell;
                if (opt_pol[o] >> k & 1) x ^= cell;
            }
        }
        int X = realize(C, x, xcare, depth + 1, budget2);
        if (X < 0) return -1;
        int lut;
        if (!function_of(C, t, care, a, b, X, &lut)) return -1;
        return add_gate(C, a, b, X, lut);
    }
}

static int realize(circuit_t *C, tt t, tt care, int depth, int budget2) {
    int k = find_existing(C, t, care);
    if (k >= 0) return k;
    if ((t & care) == 0 || (t & care) == care) {
        /* constant on care: any node serves as an operand the parent's table ignores */
        return 0;
    }
    if (depth > 12) return -1;
    k = try_one(C, t, care);
    if (k >= 0) return k;
    k = try_two(C, t, care, budget2);
    if (k >= 0) return k;
    return decompose(C, t, care, depth, budget2);
}

static int realize_top(circuit_t *C, tt t, tt care, int budget2) { return realize(C, t, care, 0, budget2); }

static int uses(const circuit_t *C, int node) {
    int u = 0;
    for (int k = 6; k < C->n; k++)
        for (int j = 0; j < 3; j++)
            if (C->g[k].in[j] == node) u++;
    return u;
}

static int distinct_operands(const gate_t *g) {
    int d = 0;
    for (int j = 0; j < 3; j++) {
        int dup = 0;
        for (int i = 0; i < j; i++) if (g->in[i] == g->in[j]) dup = 1;
        if (!dup) d++;
    }
    return d;
}

/* Remove gates no output reaches; returns the new output indices in outs. */
static void prune(circuit_t *C, int outs[4]) {
    int live[MAXN] = {0};
    for (int j = 0; j < 4; j++) live[outs[j]] = 1;
    for (int k = C->n - 1; k >= 6; k--)
        if (live[k])
            for (int j = 0; j < 3; j++) live[C->g[k].in[j]] = 1;
    int map[MAXN], m = 6;
    for (int k = 0; k < 6; k++) map[k] = k;
    circuit_t D = *C;
    for (int k = 6; k < C->n; k++) {
        if (!live[k]) continue;
        gate_t g = C->g[k];
        for (int j = 0; j < 3; j++) g.in[j] = map[g.in[j]];
        D.g[m] = g;
        D.val[m] = C->val[k];
        map[k] = m++;
    }
    D.n = m;
    for (int j = 0; j < 4; j++) outs[j] = map[outs[j]];
    *C = D;
}

static int circuit_cost(const circuit_t *C, const int outs[4]) {
    int extra = 0;
    for (int j = 0; j < 4; j++) {
        int o = outs[j];
        if (o < 6 || distinct_operands(&C->g[o]) == 3 || uses(C, o) > 0) extra++;
        for (int i = 0; i < j; i++) if (outs[i] == o) extra++;
    }
    return C->n - 6 + extra;
}

static void print_circuit(const circuit_t *C, const int outs[4], int cost);

/*
 * Large-neighbourhood search from a circuit read on stdin (the format printed
 * below): repeatedly pick an output (a third of the time two), drop the gates
 * only they use, realize them again from the rest (best of `width` attempts
 * each), and keep the result if it has no more gates (equal ones too, so the
 * circuit drifts).
 */
static int improve(const tt target[4], int iters, int budget2, int width) {
    circuit_t C;
    memset(&C, 0, sizeof C);
    C.n = 6;
    for (int i = 0; i < 6; i++) { C.val[i] = input_tt(i); C.g[i].in[0] = C.g[i].in[1] = C.g[i].in[2] = -1; }
    int outs[4] = {-1, -1, -1, -1};
    char line[256];
    while (fgets(line, sizeof line, stdin)) {
        int node, a, b, c, lut, o0, o1, o2, o3;
        if (sscanf(line, "g %d %d %d %d %d", &node, &a, &b, &c, &lut) == 5) {
            if (node != C.n || a >= node || b >= node || c >= node) { fprintf(stderr, "bad gate line\n"); return 1; }
            add_gate(&C, a, b, c, lut);
        } else if (sscanf(line, "out %d %d %d %d", &o0, &o1, &o2, &o3) == 4) {
            outs[0] = o0; outs[1] = o1; outs[2] = o2; outs[3] = o3;
        }
    }
    for (int j = 0; j < 4; j++)
        if (outs[j] < 0 || outs[j] >= C.n || (C.val[outs[j]] != target[j] && ~C.val[outs[j]] != target[j])) {
            fprintf(stderr, "start circuit is not correct\n");
            return 1;
        }
    int cur_cost = circuit_cost(&C, outs);
    int best_gates = C.n - 6, best_cost = cur_cost;
    fprintf(stderr, "start: gates %d cost %d\n", best_gates, best_cost);
    print_circuit(&C, outs, best_cost);
    for (int it = 0; it < iters; it++) {
        /* drop one output, or two, and realize them again from the rest */
        int drop[4] = {0, 0, 0, 0}, order[2], nd = 1 + (rndint(3) == 0);
        order[0] = rndint(4);
        do { order[1] = rndint(4); } while (order[1] == order[0]);
        for (int d = 0; d < nd; d++) drop[order[d]] = 1;
        circuit_t D = C;
        int o[4];
        memcpy(o, outs, sizeof o);
        int kept[4], m = 0;
        for (int q = 0; q < 4; q++) if (!drop[q]) kept[m++] = o[q];
        for (int q = m; q < 4; q++) kept[q] = kept[0];
        prune(&D, kept);
        for (int q = 0, k = 0; q < 4; q++) if (!drop[q]) o[q] = kept[k++];
        int ok = 1;
        for (int d = 0; d < nd && ok; d++) {
            const int j = order[d];
            circuit_t keep;
            int keep_k = -1;
            for (int w = 0; w < width; w++) {
                circuit_t A = D;
                int k = realize_top(&A, target[j], ~0ull, budget2);
                if (k < 0) continue;
                if (keep_k < 0 || A.n < keep.n) { keep = A; keep_k = k; }
            }
            if (keep_k < 0) { ok = 0; break; }
            D = keep;
            o[j] = keep_k;
        }
        if (!ok) continue;
        circuit_t keep = D;
        prune(&keep, o);
        const int g = keep.n - 6, cost = circuit_cost(&keep, o);
        if (g < C.n - 6 || (g == C.n - 6 && cost <= cur_cost)) {
            C = keep;
            memcpy(outs, o, sizeof o);
            cur_cost = cost;
            if (g < best_gates || (g == best_gates && cost < best_cost)) {
                best_gates = g;
                best_cost = cost;
                fprintf(stderr, "iter %d: gates %d cost %d\n", it, g, cost);
                print_circuit(&C, outs, cost);
            }
        }
    }
    return 0;
}

/* One circuit block on stdout; the last block printed is the best one. */
static void print_circuit(const circuit_t *C, const int outs[4], int cost) {
    printf("cost %d gates %d\n", cost, C->n - 6);
    for (int k = 6; k < C->n; k++)
        printf("g %d %d %d %d %d\n", k, C->g[k].in[0], C->g[k].in[1], C->g[k].in[2], C->g[k].lut);
    printf("out %d %d %d %d\n", outs[0], outs[1], outs[2], outs[3]);
    fflush(stdout);
}

int main(int argc, char **argv) {
    if (argc < 68) {
        fprintf(stderr, "usage: sbox_search SEED TRIALS BUDGET2 s0 .. s63 [WIDTH [IMPROVE]]\n"
                        "  IMPROVE > 0: large-neighbourhood search from a circuit on stdin, TRIALS iterations\n");
        return 2;
    }
    /* argv[4..67]: the 64 table entries; then WIDTH and IMPROVE */
    const int width = argc > 68 ? atoi(argv[68]) : 1;  /* attempts per output, best kept */
    rng_state ^= strtoull(argv[1], NULL, 0);
    int trials = atoi(argv[2]);
    int budget2 = atoi(argv[3]);
    int sbox[64];
    for (int p = 0; p < 64; p++) sbox[p] = atoi(argv[4 + p]);
    tt target[4];
    for (int j = 0; j < 4; j++) {
        target[j] = 0;
        for (int p = 0; p < 64; p++)
            if ((sbox[p] >> (3 - j)) & 1) target[j] |= 1ull << p;
    }
    circuit_t best;
    best.n = 6;
    int best_cost = 1 << 30, best_outs[4] = {0};
    if (argc > 69 && atoi(argv[69]) > 0) return improve(target, trials, budget2, width);
    for (int trial = 0; trial < trials; trial++) {
        g_allow_bidec = (int)(rnd() % 3 == 0);
        circuit_t C;
        memset(&C, 0, sizeof C);
        C.n = 6;
        for (int i = 0; i < 6; i++) { C.val[i] = input_tt(i); C.g[i].in[0] = C.g[i].in[1] = C.g[i].in[2] = -1; }
        int order[4] = {0, 1, 2, 3};
        for (int i = 3; i > 0; i--) { int j = rndint(i + 1); int tmp = order[i]; order[i] = order[j]; order[j] = tmp; }
        int outs[4], ok = 1;
        for (int q = 0; q < 4 && ok; q++) {
            int j = order[q];
            /* best of `width` attempts for this output, each from the same shared circuit */
            circuit_t keep;
            int keep_k = -1;
            for (int w = 0; w < width; w++) {
                circuit_t A = C;
                int k = realize_top(&A, target[j], ~0ull, budget2);
                if (k < 0) continue;
                if (keep_k < 0 || A.n < keep.n) { keep = A; keep_k = k; }
            }
            if (keep_k < 0) { ok = 0; break; }
            C = keep;
            outs[j] = keep_k;
        }
        if (!ok) continue;
        prune(&C, outs);
        int gates = C.n - 6;
        int extra = 0;
        for (int j = 0; j < 4; j++) {
            int o = outs[j];
            if (o < 6 || distinct_operands(&C.g[o]) == 3 || uses(&C, o) > 0) extra++;
            for (int i = 0; i < j; i++) if (outs[i] == o) extra++;
        }
        int cost = gates + extra;
        /* Gates first: the kernels' folded rounds XOR every output with a key mask in a
           three-way gate anyway; the absorbable outputs only help the per-lane-key rounds. */
        if (gates < best.n - 6 || (gates == best.n - 6 && cost < best_cost) || best_cost >= (1 << 30)) {
            best_cost = cost; best = C; memcpy(best_outs, outs, sizeof outs);
            fprintf(stderr, "trial %d: gates %d cost %d\n", trial, gates, cost);
            print_circuit(&best, best_outs, best_cost);  /* every improvement: a long run can be stopped */
        }
    }
    return best_cost >= (1 << 30) ? 1 : 0;
}
