"""Generate the bitsliced kernel's folded round pair as gfx950 assembly (csrc/rounds_asm.inc).

    python -m paper_1305_4376_amd.gen.gen_rounds [--seed N] [--check N]

Why.  A VALU instruction reads its vector operands from four register banks
(bank = register number mod 4); two operands in one bank cost an extra issue
cycle: measured on MI355X, v_bitop3_b32 with its three sources in three banks
issues at 0.47 wave-instructions per SIMD per cycle, with two in one bank at
0.25.  The compiler does not model the banks: in its code for the rounds
nearly half the instructions have two operands in one bank.  This generator
does the register assignment of the round pair itself:

  * the 64 bit planes (two halves of 32) get fixed registers, with each
    plane's bank chosen so that the S-box gates that read two planes directly
    find them in different banks as often as possible;
  * every other value of a box (the key-corrected inputs, the gate outputs)
    gets a bank by colouring the graph of operands read together (gate
    sources, and an output gate with the half it is XORed into), then a free
    register of that bank by liveness;
  * a gate that reads one value twice becomes a two-input gate with an inline
    constant as third operand.

What the pair computes is exactly the folded round of bitslice_core.h
(feistel_folded): x ^= f(y) with the round's output-fold and correction words
(ow0, cw0), then y ^= f(x) with (ow1, cw1); the key masks are scalar bit-field
extracts of those words.  --check simulates the emitted instructions on random
planes and words against that definition, written out here from the standard's
E and P (des_spec.h) and the stored circuits, before anything is written.
"""
from __future__ import annotations

import argparse
import os
import random
import re
import sys

from paper_1305_4376_amd.gen import gen_sbox

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
SPEC = os.path.join(PKG, "csrc", "des_spec.h")
OUT = os.path.join(PKG, "csrc", "rounds_asm.inc")

FIRST_VGPR, LAST_VGPR = 8, 95      # registers the asm block may use (the others stay with the compiler)
SGPR_POOL = list(range(72, 84))    # key masks
M32 = 0xFFFFFFFF


# ---- the round's definition (standard's E and P, folded key scheme) ----

def expansion(i: int) -> int:
    """E: S-box input i (box i // 6) reads R bit (4 (i // 6) + i % 6 - 1) mod 32."""
    return (4 * (i // 6) + i % 6 + 31) % 32


def p_table() -> list[int]:
    text = open(SPEC).read()
    body = re.search(r"kP\[32\]\s*=\s*\{([^}]*)\}", text).group(1)
    return [int(v) for v in body.replace("\n", " ").split(",") if v.strip()]


def uses():
    """first[q]: first E position reading R bit q; second_of[i]: index of E position i among the
    second uses (-1 for a first use)."""
    first, second_of, t = [-1] * 32, [-1] * 48, 0
    for i in range(48):
        q = expansion(i)
        if first[q] < 0:
            first[q] = i
        else:
            second_of[i] = t
            t += 1
    return first, second_of


class Round:
    """Everything one folded round needs: circuits, polarities, E, P^-1, correction positions."""

    def __init__(self):
        self.circuits = gen_sbox.load_store()
        tabs = gen_sbox.sbox_tables()
        self.pol = {b: self.circuits[b].polarities(tabs[b]) for b in range(8)}
        kp = p_table()
        self.p_inv = [0] * 32
        for i in range(32):
            self.p_inv[kp[i]] = i
        self.first, self.second_of = uses()

    def reference(self, x, y, ow, cw):
        """x ^= f(y) in the folded form, planes as 32-bit ints (one bit per block)."""
        mask = lambda w, pos: M32 if (w >> pos) & 1 else 0
        x = list(x)
        for s in range(8):
            val = {}
            for j in range(6):
                i = 6 * s + j
                t = self.second_of[i]
                val[j] = y[expansion(i)] ^ (mask(cw, t) if t >= 0 else 0)
            for node, a, b, c, lut in self.circuits[s].gates:
                val[node] = lut3_32(lut, val[a], val[b], val[c])
            for k in range(4):
                p = self.p_inv[4 * s + k]
                v = x[p] ^ val[self.circuits[s].outs[k]] ^ mask(ow, p)
                x[p] = v ^ (M32 if self.pol[s][k] else 0)
        return x


def lut3_32(lut, a, b, c):
    r = 0
    for m in range(8):
        if (lut >> m) & 1:
            r |= (a if m & 4 else ~a) & (b if m & 2 else ~b) & (c if m & 1 else ~c)
    return r & M32


# ---- register assignment ----

def bank(r: int) -> int:
    return r % 4


def plane_banks(rd: Round, rng: random.Random) -> list[int]:
    """Bank of R bit q's planes (the same for both halves), by local search over the gates that read
    two first-use inputs of one box directly: minimise such pairs in one bank."""
    pairs = []
    for s in range(8):
        raw = {j: expansion(6 * s + j) for j in range(6) if rd.second_of[6 * s + j] < 0}
        for _, a, b, c, _ in rd.circuits[s].gates:
            srcs = [raw[v] for v in dict.fromkeys((a, b, c)) if v < 6 and v in raw]
            for u in range(len(srcs)):
                for w in range(u + 1, len(srcs)):
                    pairs.append((srcs[u], srcs[w]))
    best, best_cost = None, None
    for _ in range(40):
        col = [q % 4 for q in range(32)]
        rng.shuffle(col)
        cost = lambda cl: sum(1 for p, q in pairs if cl[p] == cl[q])
        cur = cost(col)
        improved = True
        while improved:
            improved = False
            for p in range(32):
                for q in range(p + 1, 32):
                    if col[p] == col[q]:
                        continue
                    col[p], col[q] = col[q], col[p]   # swaps keep 8 planes per bank
                    c2 = cost(col)
                    if c2 < cur:
                        cur, improved = c2, True
                    else:
                        col[p], col[q] = col[q], col[p]
        if best_cost is None or cur < best_cost:
            best, best_cost = list(col), cur
    return best


class Emitter:
    def __init__(self):
        self.lines = []      # assembly text
        self.prog = []       # (op, dst, srcs, imm) for the simulator

    def valu(self, text, op, dst, srcs, imm=None):
        self.lines.append(text)
        self.prog.append((op, dst, srcs, imm))


def gen_pair(rd: Round, seed: int, swap: bool = False):
    """The round pair with x in register set 0 and y in set 1 (swap: the other way round; the two
    sets have the same bank per plane, so the instructions are the same up to that renaming)."""
    rng = random.Random(seed)
    pb = plane_banks(rd, rng)
    # plane registers: bank pb[q], for half 0 (x) and half 1 (y)
    free = {b: [r for r in range(FIRST_VGPR, LAST_VGPR + 1) if bank(r) == b] for b in range(4)}
    plane_reg = [[0] * 32, [0] * 32]
    for h in range(2):
        for q in range(32):
            plane_reg[h][q] = free[pb[q]].pop(0)
    if swap:
        plane_reg = [plane_reg[1], plane_reg[0]]
    temps = {b: list(free[b]) for b in range(4)}   # registers left for a box's values
    em = Emitter()
    stats = {"valu": 0, "conflicts": 0, "copies": 0}
    sgpr_next = [0]

    def sgpr():
        r = SGPR_POOL[sgpr_next[0] % len(SGPR_POOL)]
        sgpr_next[0] += 1
        return r

    for rnd in range(2):
        xh, yh = (0, 1) if rnd == 0 else (1, 0)      # x ^= f(y), then y ^= f(x)
        ow_op, cw_op = ("%[ow0]", "%[cw0]") if rnd == 0 else ("%[ow1]", "%[cw1]")
        for s in range(8):
            box(rd, s, plane_reg[xh], plane_reg[yh], ow_op, cw_op, rnd, temps, em, stats, sgpr, rng)
    return em, plane_reg, stats


def box(rd, s, xreg, yreg, ow_op, cw_op, rnd, temps, em, stats, sgpr, rng):
    circ = rd.circuits[s]
    # values: ("in", j) inputs, ("g", node) gates; fixed registers for first-use inputs
    gates = []
    for node, a, b, c, lut in circ.gates:
        srcs = list(dict.fromkeys((a, b, c)))
        if len(srcs) < 3:   # a repeated operand: a gate of the distinct ones, constant 0 as the rest
            newlut = 0
            for m in range(8):
                env = {}
                bits = [(m >> 2) & 1, (m >> 1) & 1, m & 1]
                for v, bit in zip(srcs + [None] * (3 - len(srcs)), bits):
                    if v is not None:
                        env[v] = bit
                ok = all(bits[k] == 0 for k in range(len(srcs), 3))
                val = (lut >> ((env[a] << 2) | (env[b] << 1) | env[c])) & 1 if ok else 0
                newlut |= val << m
            gates.append((node, srcs, newlut))
        else:
            gates.append((node, srcs, lut))
    fixed = {}          # value -> register
    corrected = []      # inputs that need a key correction
    for j in range(6):
        i = 6 * s + j
        if rd.second_of[i] < 0:
            fixed[j] = yreg[expansion(i)]
        else:
            corrected.append(j)
    outs = circ.outs
    out_plane = [xreg[rd.p_inv[4 * s + k]] for k in range(4)]
    # co-operand graph over the values that need a register
    free_vals = corrected + [g[0] for g in gates]
    edges = {}
    def add(u, v):
        if u == v:
            return
        key = (min(u, v), max(u, v)) if isinstance(u, int) and isinstance(v, int) else (u, v)
        edges[key] = edges.get(key, 0) + 1
    for node, srcs, _ in gates:
        for u in range(len(srcs)):
            for w in range(u + 1, len(srcs)):
                add(srcs[u], srcs[w])
    # output gate k is XORed into a fixed plane register: a pseudo-node per plane
    for k in range(4):
        add(outs[k], ("plane", out_plane[k]))
    # liveness in program order: corrections, gates, outputs
    order = [("corr", j) for j in corrected] + [("gate", g[0]) for g in gates] + [("out", k) for k in range(4)]
    pos_def = {}
    last_use = {}
    for t, (kind, v) in enumerate(order):
        if kind == "corr":
            pos_def[v] = t
        elif kind == "gate":
            pos_def[v] = t
            srcs = next(g[1] for g in gates if g[0] == v)
            for u in srcs:
                last_use[u] = t
        else:
            last_use[outs[v]] = max(last_use.get(outs[v], 0), t)

    def color(u, col):
        if isinstance(u, tuple):
            return bank(u[1])
        if u in fixed:
            return bank(fixed[u])
        return col[u]

    def conflicts(col):
        return sum(w for (u, v), w in edges.items() if color(u, col) == color(v, col))

    def pressure_ok(col):
        live = {b: 0 for b in range(4)}
        events = []
        for v in free_vals:
            events.append((pos_def[v], 1, v))
            events.append((last_use.get(v, pos_def[v]) + 1, -1, v))
        events.sort(key=lambda e: (e[0], e[1]))
        for _, d, v in events:
            live[col[v]] += d
            if live[col[v]] > len(temps[col[v]]):
                return False
        return True

    best = None
    for attempt in range(200):
        col = {v: rng.randrange(4) for v in free_vals}
        cur = conflicts(col)
        improved = True
        while improved:
            improved = False
            for v in free_vals:
                keep = col[v]
                for c in range(4):
                    if c == keep:
                        continue
                    col[v] = c
                    c2 = conflicts(col)
                    if c2 < cur:
                        cur, keep, improved = c2, c, True
                col[v] = keep
        if not pressure_ok(col):
            continue
        if best is None or cur < best[0]:
            best = (cur, dict(col))
        if cur == 0:
            break
    if best is None:
        raise RuntimeError(f"box {s + 1}: no colouring fits the registers")
    col = best[1]
    # registers by linear scan per bank
    reg = dict(fixed)
    pool = {b: list(temps[b]) for b in range(4)}
    expiring = []
    for t, (kind, v) in enumerate(order):
        for e in [e for e in expiring if e[0] < t]:
            pool[bank(e[1])].append(e[1])
            expiring.remove(e)
        if kind in ("corr", "gate"):
            r = pool[col[v]].pop(0)
            reg[v] = r
            expiring.append((last_use.get(v, t), r))
    # emit: key masks first (scalar), then corrections, gates, outputs
    mreg_out = []
    for k in range(4):
        sg = sgpr()
        p = rd.p_inv[4 * s + k]
        em.lines.append(f"s_bfe_i32 s{sg}, {ow_op}, 0x{0x10000 | p:x}")
        em.prog.append(("mask", sg, (rnd, "ow"), p))
        mreg_out.append(sg)
    for j in corrected:
        sg = sgpr()
        t = rd.second_of[6 * s + j]
        em.lines.append(f"s_bfe_i32 s{sg}, {cw_op}, 0x{0x10000 | t:x}")
        em.prog.append(("mask", sg, (rnd, "cw"), t))
        src = yreg[expansion(6 * s + j)]
        em.valu(f"v_xor_b32 v{reg[j]}, s{sg}, v{src}", "xor_s", reg[j], (sg, src))
        stats["valu"] += 1
    for node, srcs, lut in gates:
        regs = [reg[u] for u in srcs]
        banks = [bank(r) for r in regs]
        if len(set(banks)) < len(banks):
            stats["conflicts"] += 1
        ops = [f"v{r}" for r in regs] + ["0"] * (3 - len(regs))
        em.valu(f"v_bitop3_b32 v{reg[node]}, {', '.join(ops)} bitop3:0x{lut:02x}", "bitop3", reg[node],
                tuple(regs) + (None,) * (3 - len(regs)), lut)
        stats["valu"] += 1
    for k in range(4):
        o = out_plane[k]
        n = reg[outs[k]]
        if bank(o) == bank(n):
            stats["conflicts"] += 1
        lut = 0x69 if rd.pol[s][k] else 0x96
        em.valu(f"v_bitop3_b32 v{o}, v{o}, v{n}, s{mreg_out[k]} bitop3:0x{lut:02x}", "bitop3_s", o, (o, n, mreg_out[k]), lut)
        stats["valu"] += 1


# ---- simulation of the emitted code ----

def simulate(em: Emitter, plane_reg, x, y, words):
    v = {}
    s = {}
    for q in range(32):
        v[plane_reg[0][q]] = x[q]
        v[plane_reg[1][q]] = y[q]
    for op, dst, srcs, imm in em.prog:
        if op == "mask":
            rnd, kind = srcs
            w = words[(rnd, kind)]
            s[dst] = M32 if (w >> imm) & 1 else 0
        elif op == "xor_s":
            v[dst] = s[srcs[0]] ^ v[srcs[1]]
        elif op == "bitop3":
            a, b, c = [v[r] if r is not None else 0 for r in srcs]
            v[dst] = lut3_32(imm, a, b, c)
        elif op == "bitop3_s":
            v[dst] = lut3_32(imm, v[srcs[0]], v[srcs[1]], s[srcs[2]])
    return [v[plane_reg[0][q]] for q in range(32)], [v[plane_reg[1][q]] for q in range(32)]


def check(rd: Round, em, plane_reg, trials: int, seed: int):
    rng = random.Random(seed)
    for _ in range(trials):
        x = [rng.getrandbits(32) for _ in range(32)]
        y = [rng.getrandbits(32) for _ in range(32)]
        words = {(r, k): rng.getrandbits(32) for r in range(2) for k in ("ow", "cw")}
        gx, gy = simulate(em, plane_reg, x, y, words)
        wx = rd.reference(x, y, words[(0, "ow")], words[(0, "cw")])
        wy = rd.reference(y, wx, words[(1, "ow")], words[(1, "cw")])
        if gx != wx or gy != wy:
            raise AssertionError("the emitted round pair differs from the folded round")


def emit_inc(pairs, seed) -> str:
    """pairs: [(em, plane_reg, stats)] for x in set 0 (A) and x in set 1 (B)."""
    em, plane_reg, stats = pairs[0]
    used_v = sorted({r for r in range(FIRST_VGPR, LAST_VGPR + 1)} - set(plane_reg[0]) - set(plane_reg[1]))
    out = ["// Generated by gen/gen_rounds.py (seed %d); do not edit." % seed,
           "// Two folded rounds (x ^= f(y) with ow0/cw0, then y ^= f(x) with ow1/cw1) with bank-aware",
           f"// registers: {stats['valu']} VALU instructions, {stats['conflicts']} with two vector operands in one bank.",
           "// A: x in the first register set, y in the second; B: the other way round.", ""]
    for tag, (em, plane_reg, _) in zip("AB", pairs):
        ops = [f'"+{{v{plane_reg[0][q]}}}"(x[{q}])' for q in range(32)] + \
              [f'"+{{v{plane_reg[1][q]}}}"(y[{q}])' for q in range(32)]
        out.append(f"#define TDES_ROUNDS_OPERANDS_{tag}(x, y) \\")
        for i in range(0, len(ops), 6):
            out.append("    " + ", ".join(ops[i:i + 6]) + (", \\" if i + 6 < len(ops) else ""))
        out.append("")
        out.append(f"#define TDES_ROUNDS_ASM_{tag} \\")
        for l in em.lines:
            out.append(f'    "{l}\\n" \\')
        out.append("")
    out.append("#define TDES_ROUNDS_CLOBBERS \\")
    # s_bfe_i32 also writes SCC
    clob = [f'"v{r}"' for r in used_v] + [f'"s{r}"' for r in SGPR_POOL] + ['"scc"']
    for i in range(0, len(clob), 12):
        out.append("    " + ", ".join(clob[i:i + 12]) + (", \\" if i + 12 < len(clob) else ""))
    out.append("")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--check", type=int, default=200, help="random trials of the simulation check")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    rd = Round()
    pairs = [gen_pair(rd, args.seed, swap) for swap in (False, True)]
    for em, plane_reg, _ in pairs:
        check(rd, em, plane_reg, args.check, args.seed)
    stats = pairs[0][2]
    with open(args.out, "w") as f:
        f.write(emit_inc(pairs, args.seed))
    print(f"wrote {args.out}: {stats['valu']} VALU, {stats['conflicts']} bank conflicts", file=sys.stderr)


if __name__ == "__main__":
    main()
