/*
 * sbox_resyn.c -- shrink an S-box circuit of 3-input lookup gates by
 * resynthesis of fanout-free cones.
 *
 * Build-time tool, used by gen_sbox.py after sbox_search.c.  For a gate h, its
 * maximum fanout-free cone (MFFC) is h together with every gate whose paths to
 * the outputs all pass through h: the gates that disappear if h is computed
 * another way.  The pass re-expresses h's function (its full truth table over
 * the 64 input points, or its complement when h is an output, whose polarity
 * is free) as one new gate over three nodes outside the cone and outside h's
 * transitive fanout, or as two new gates (t = F(g, d, e), g = G(a, b, c)), and
 * keeps the change whenever it removes more gates than it adds.  Gates are
 * visited in random order until a whole pass finds nothing; then the circuit
 * is printed in topological order.  Random restarts of the visiting order run
 * for the given number of rounds and the smallest circuit is kept.  The caller
 * re-checks the result on all 64 inputs before using it.
 *
 * Usage: sbox_resyn SEED ROUNDS s0..s63 < circuit   (format of sbox_circuits.txt, one box)
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t tt;
#define NIN 6
#define MAXN 160

typedef struct {
    int a[MAXN], b[MAXN], c[MAXN];  /* operands (nodes < NIN are inputs) */
    int lut[MAXN];
    int alive[MAXN];
    int n;                          /* node slots used */
    int out[4];
} circ_t;

static uint64_t rs = 0x2545F4914F6CDD1Dull;
static uint64_t rnd(void) {
    uint64_t z = (rs += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static tt IN[NIN], T[4];

static tt lut3(int lut, tt a, tt b, tt c) {
    tt r = 0;
    for (int m = 0; m < 8; m++)
        if ((lut >> m) & 1) r |= ((m & 4) ? a : ~a) & ((m & 2) ? b : ~b) & ((m & 1) ? c : ~c);
    return r;
}

/* Values of all live nodes; returns 0 if the graph has a cycle (never expected). */
static int evaluate(const circ_t *C, tt *v) {
    int state[MAXN] = {0}, stack[MAXN], sp = 0;
    for (int i = 0; i < NIN; i++) { v[i] = IN[i]; state[i] = 2; }
    for (int k = NIN; k < C->n; k++) {
        if (!C->alive[k] || state[k] == 2) continue;
        stack[sp++] = k;
        while (sp) {
            int x = stack[sp - 1];
            if (state[x] == 2) { sp--; continue; }
            state[x] = 1;
            int ops[3] = {C->a[x], C->b[x], C->c[x]}, pushed = 0;
            for (int j = 0; j < 3; j++)
                if (state[ops[j]] == 0) { stack[sp++] = ops[j]; pushed = 1; }
                else if (state[ops[j]] == 1 && ops[j] != x) return 0;
            if (!pushed) {
                v[x] = lut3(C->lut[x], v[C->a[x]], v[C->b[x]], v[C->c[x]]);
                state[x] = 2;
                sp--;
            }
        }
    }
    return 1;
}

static int outputs_ok(const circ_t *C) {
    tt v[MAXN];
    if (!evaluate(C, v)) return 0;
    for (int j = 0; j < 4; j++) {
        tt x = v[C->out[j]];
        if (x != T[j] && ~x != T[j]) return 0;
    }
    return 1;
}

static int gate_count(const circ_t *C) {
    int g = 0;
    for (int k = NIN; k < C->n; k++) g += C->alive[k];
    return g;
}

/* Fanout counts of live nodes (outputs count as one use each). */
static void fanouts(const circ_t *C, int *fo) {
    memset(fo, 0, sizeof(int) * MAXN);
    for (int k = NIN; k < C->n; k++)
        if (C->alive[k]) { fo[C->a[k]]++; fo[C->b[k]]++; fo[C->c[k]]++; }
    for (int j = 0; j < 4; j++) fo[C->out[j]]++;
}

/* Remove gates that no output reaches. */
static void sweep(circ_t *C) {
    int live[MAXN] = {0}, changed = 1;
    for (int j = 0; j < 4; j++) live[C->out[j]] = 1;
    while (changed) {
        changed = 0;
        for (int k = NIN; k < C->n; k++)
            if (C->alive[k] && live[k])
                for (int j = 0; j < 3; j++) {
                    int o = j == 0 ? C->a[k] : j == 1 ? C->b[k] : C->c[k];
                    if (!live[o]) { live[o] = 1; changed = 1; }
                }
    }
    for (int k = NIN; k < C->n; k++) if (!live[k]) C->alive[k] = 0;
}

/* mffc[k] = 1 for the gates of h's maximum fanout-free cone. */
static int mffc(const circ_t *C, int h, char *in_cone) {
    int fo[MAXN], size = 0;
    fanouts(C, fo);
    memset(in_cone, 0, MAXN);
    int stack[MAXN], sp = 0;
    in_cone[h] = 1; size = 1; stack[sp++] = h;
    /* reference counting: a fanin leaves with its last reference inside the cone */
    int ref[MAXN];
    memcpy(ref, fo, sizeof ref);
    while (sp) {
        int x = stack[--sp];
        int ops[3] = {C->a[x], C->b[x], C->c[x]};
        for (int j = 0; j < 3; j++) {
            int o = ops[j];
            int dup = 0;
            for (int i = 0; i < j; i++) if (ops[i] == o) dup = 1;
            if (dup) continue;
            if (o < NIN || in_cone[o]) continue;
            int uses = 0;
            for (int i = 0; i < 3; i++) if (ops[i] == o) uses++;
            ref[o] -= uses;
            if (ref[o] == 0) { in_cone[o] = 1; size++; stack[sp++] = o; }
        }
    }
    return size;
}

/* tfo[k] = 1 for h and every node that depends on it. */
static void fanout_cone(const circ_t *C, int h, char *tfo) {
    memset(tfo, 0, MAXN);
    tfo[h] = 1;
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int k = NIN; k < C->n; k++)
            if (C->alive[k] && !tfo[k] && (tfo[C->a[k]] || tfo[C->b[k]] || tfo[C->c[k]])) { tfo[k] = 1; changed = 1; }
    }
}

/* Is t a function of (x, y, z)?  Writes its table (unreachable cells 0). */
static int fn_of(tt t, tt x, tt y, tt z, int *lut) {
    int l = 0;
    for (int m = 0; m < 8; m++) {
        tt cell = ((m & 4) ? x : ~x) & ((m & 2) ? y : ~y) & ((m & 1) ? z : ~z);
        if (!cell) continue;
        tt on = cell & t;
        if (on && on != cell) return 0;
        if (on) l |= 1 << m;
    }
    *lut = l;
    return 1;
}

static int new_slot(circ_t *C) { return C->n < MAXN ? C->n++ : -1; }

/* Re-express node h as one or two new gates over cand[]; on success rewire h's users and outputs. */
static int resynth(circ_t *C, int h, const tt *v, const int *cand, int nc, int max_new, int may_flip) {
    tt targets[2] = {v[h], ~v[h]};
    int ntarg = may_flip ? 2 : 1;
    int found = 0, ga = 0, gb = 0, gc = 0, glut = 0, two = 0, d = 0, e = 0, flut = 0, flip = 0;
    for (int ti = 0; ti < ntarg && !found; ti++) {
        tt t = targets[ti];
        for (int i = 0; i < nc && !found; i++)
            for (int j = i + 1; j < nc && !found; j++)
                for (int k = j + 1; k < nc && !found; k++) {
                    int l;
                    if (fn_of(t, v[cand[i]], v[cand[j]], v[cand[k]], &l)) {
                        found = 1; ga = cand[i]; gb = cand[j]; gc = cand[k]; glut = l; flip = ti;
                    }
                }
    }
    if (!found && max_new >= 2) {
        /* t = F(g, d, e): on each cell of (d, e) where t is not constant, g must be t or ~t. */
        for (int ti = 0; ti < ntarg && !found; ti++) {
            tt t = targets[ti];
            for (int i = 0; i < nc && !found; i++)
                for (int j = i; j < nc && !found; j++) {
                    tt vd = v[cand[i]], ve = v[cand[j]];
                    tt cell[4]; int live[4], nlive = 0;
                    for (int q = 0; q < 4; q++) {
                        cell[q] = ((q & 2) ? vd : ~vd) & ((q & 1) ? ve : ~ve);
                        tt on = cell[q] & t;
                        live[q] = on && on != cell[q];
                        nlive += live[q];
                    }
                    if (!nlive) continue;
                    /* try every polarity assignment of the live cells: g = t ^ (cells flipped) */
                    for (int pol = 0; pol < 16 && !found; pol++) {
                        if (pol & ~((live[0]) | (live[1] << 1) | (live[2] << 2) | (live[3] << 3))) continue;
                        tt care = 0, g = t;
                        for (int q = 0; q < 4; q++) if (live[q]) { care |= cell[q]; if (pol >> q & 1) g ^= cell[q]; }
                        for (int x = 0; x < nc && !found; x++)
                            for (int y = x + 1; y < nc && !found; y++)
                                for (int z = y + 1; z < nc && !found; z++) {
                                    tt vx = v[cand[x]], vy = v[cand[y]], vz = v[cand[z]];
                                    int l = 0, ok = 1;
                                    for (int m = 0; m < 8 && ok; m++) {
                                        tt c8 = ((m & 4) ? vx : ~vx) & ((m & 2) ? vy : ~vy) & ((m & 1) ? vz : ~vz) & care;
                                        if (!c8) { if (rnd() & 1) l |= 1 << m; continue; }
                                        tt on = c8 & g;
                                        if (on && on != c8) ok = 0;
                                        else if (on) l |= 1 << m;
                                    }
                                    if (!ok) continue;
                                    tt gv = lut3(l, vx, vy, vz);
                                    int fl;
                                    if (fn_of(t, gv, vd, ve, &fl)) {
                                        found = 1; two = 1; ga = cand[x]; gb = cand[y]; gc = cand[z]; glut = l;
                                        d = cand[i]; e = cand[j]; flut = fl; flip = ti;
                                    }
                                }
                    }
                }
        }
    }
    if (!found) return 0;
    int g = new_slot(C);
    if (g < 0) return 0;
    C->a[g] = ga; C->b[g] = gb; C->c[g] = gc; C->lut[g] = glut; C->alive[g] = 1;
    int top = g;
    if (two) {
        top = new_slot(C);
        if (top < 0) { C->alive[g] = 0; return 0; }
        C->a[top] = g; C->b[top] = d; C->c[top] = e; C->lut[top] = flut; C->alive[top] = 1;
    }
    /* Users of h take the new node; a flipped replacement is complemented at each use. */
    for (int k = NIN; k < C->n; k++) {
        if (!C->alive[k] || k == g || k == top) continue;
        int *ops[3] = {&C->a[k], &C->b[k], &C->c[k]};
        int mask = 0;
        for (int j = 0; j < 3; j++) if (*ops[j] == h) { *ops[j] = top; mask |= 4 >> j; }
        if (mask && flip) {
            int l = 0;
            for (int m = 0; m < 8; m++) if ((C->lut[k] >> (m ^ mask)) & 1) l |= 1 << m;
            C->lut[k] = l;
        }
    }
    for (int j = 0; j < 4; j++) if (C->out[j] == h) C->out[j] = top;  /* output polarity is free */
    C->alive[h] = 0;
    sweep(C);
    return 1;
}

static int pass(circ_t *C) {
    int improved = 0;
    int order[MAXN], no = 0;
    for (int k = NIN; k < C->n; k++) if (C->alive[k]) order[no++] = k;
    for (int i = no - 1; i > 0; i--) { int j = (int)(rnd() % (uint64_t)(i + 1)); int t = order[i]; order[i] = order[j]; order[j] = t; }
    for (int oi = 0; oi < no; oi++) {
        int h = order[oi];
        if (!C->alive[h]) continue;
        char cone[MAXN], tfo[MAXN];
        int size = mffc(C, h, cone);
        if (size < 2) continue;
        fanout_cone(C, h, tfo);
        tt v[MAXN];
        if (!evaluate(C, v)) return improved;
        int cand[MAXN], nc = 0;
        for (int k = 0; k < C->n; k++)
            if ((k < NIN || C->alive[k]) && !cone[k] && !tfo[k]) cand[nc++] = k;
        int is_out = 0;
        for (int j = 0; j < 4; j++) if (C->out[j] == h) is_out = 1;
        /* h's users can absorb a complement, and so can an output */
        circ_t save = *C;
        const int before = gate_count(C);
        if (resynth(C, h, v, cand, nc, size >= 3 ? 2 : 1, 1)) {
            if (gate_count(C) < before && outputs_ok(C)) { improved = 1; continue; }
        }
        *C = save;
        (void)is_out;
    }
    return improved;
}

static void print_circuit(const circ_t *C) {
    /* topological renumbering */
    int ren[MAXN], next = NIN, done[MAXN] = {0};
    for (int i = 0; i < NIN; i++) { ren[i] = i; done[i] = 1; }
    int order[MAXN], no = 0, progress = 1;
    while (progress) {
        progress = 0;
        for (int k = NIN; k < C->n; k++)
            if (C->alive[k] && !done[k] && done[C->a[k]] && done[C->b[k]] && done[C->c[k]]) {
                done[k] = 1; ren[k] = next++; order[no++] = k; progress = 1;
            }
    }
    printf("gates %d\n", no);
    for (int i = 0; i < no; i++) {
        int k = order[i];
        printf("g %d %d %d %d %d\n", ren[k], ren[C->a[k]], ren[C->b[k]], ren[C->c[k]], C->lut[k]);
    }
    printf("out %d %d %d %d\n", ren[C->out[0]], ren[C->out[1]], ren[C->out[2]], ren[C->out[3]]);
}

int main(int argc, char **argv) {
    if (argc < 3 + 64) {
        fprintf(stderr, "usage: sbox_resyn SEED ROUNDS s0..s63 < circuit\n");
        return 2;
    }
    rs ^= strtoull(argv[1], NULL, 0) * 0x9E3779B97F4A7C15ull;
    int rounds = atoi(argv[2]);
    int sbox[64];
    for (int p = 0; p < 64; p++) sbox[p] = atoi(argv[3 + p]);
    for (int i = 0; i < NIN; i++) {
        IN[i] = 0;
        for (int p = 0; p < 64; p++) if ((p >> (5 - i)) & 1) IN[i] |= 1ull << p;
    }
    for (int j = 0; j < 4; j++) {
        T[j] = 0;
        for (int p = 0; p < 64; p++) if ((sbox[p] >> (3 - j)) & 1) T[j] |= 1ull << p;
    }
    circ_t C;
    memset(&C, 0, sizeof C);
    C.n = NIN;
    int map[MAXN];
    for (int i = 0; i < NIN; i++) map[i] = i;
    char line[256];
    while (fgets(line, sizeof line, stdin)) {
        int node, a, b, c, lut, o0, o1, o2, o3;
        if (sscanf(line, "g %d %d %d %d %d", &node, &a, &b, &c, &lut) == 5) {
            int k = C.n++;
            C.a[k] = map[a]; C.b[k] = map[b]; C.c[k] = map[c]; C.lut[k] = lut; C.alive[k] = 1;
            map[node] = k;
        } else if (sscanf(line, "out %d %d %d %d", &o0, &o1, &o2, &o3) == 4) {
            C.out[0] = map[o0]; C.out[1] = map[o1]; C.out[2] = map[o2]; C.out[3] = map[o3];
        }
    }
    if (!outputs_ok(&C)) { fprintf(stderr, "start circuit is not correct\n"); return 1; }
    circ_t best = C;
    int best_g = gate_count(&C);
    fprintf(stderr, "start: %d gates\n", best_g);
    for (int r = 0; r < rounds; r++) {
        circ_t W = best;
        /* compact slots so that new gates have room */
        while (pass(&W)) {
            if (W.n > MAXN - 8) break;
        }
        int g = gate_count(&W);
        if (g < best_g && outputs_ok(&W)) {
            best = W; best_g = g;
            fprintf(stderr, "round %d: %d gates\n", r, g);
        }
        /* renumber best compactly for the next round */
        {
            circ_t D;
            memset(&D, 0, sizeof D);
            D.n = NIN;
            int ren[MAXN];
            for (int i = 0; i < NIN; i++) ren[i] = i;
            int done[MAXN] = {0}, progress = 1;
            for (int i = 0; i < NIN; i++) done[i] = 1;
            while (progress) {
                progress = 0;
                for (int k = NIN; k < best.n; k++)
                    if (best.alive[k] && !done[k] && done[best.a[k]] && done[best.b[k]] && done[best.c[k]]) {
                        int q = D.n++;
                        D.a[q] = ren[best.a[k]]; D.b[q] = ren[best.b[k]]; D.c[q] = ren[best.c[k]];
                        D.lut[q] = best.lut[k]; D.alive[q] = 1; ren[k] = q; done[k] = 1; progress = 1;
                    }
            }
            for (int j = 0; j < 4; j++) D.out[j] = ren[best.out[j]];
            best = D;
        }
    }
    print_circuit(&best);
    return 0;
}
