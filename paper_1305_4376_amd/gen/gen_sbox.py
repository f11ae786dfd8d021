"""Generate the bitsliced kernel's S-box circuits (csrc/sbox_circuits.inc).

    python -m paper_1305_4376_amd.gen.gen_sbox [--search TRIALS] [--budget N] [--seeds K] [--width W]
                                               [--lns ITERATIONS]

Each of the eight DES S-boxes (read from csrc/des_spec.h, the table the other
kernel uses too) becomes a function of six bit planes that XORs its four
output planes into four Feistel planes.  Every gate is one v_bitop3_b32:
any Boolean function of three 32-bit words, given as an 8-bit truth table
whose bit (4a + 2b + c) is the output for operand bits a, b, c.

The circuits come from sbox_search.c (a randomized decomposition search
written for this purpose; see that file).  The chosen ones are stored in
sbox_circuits.txt; with --search the search runs again and a circuit replaces
the stored one only if it has fewer gates (then a lower cost).  --lns runs
the search's large-neighbourhood mode from each stored circuit.  Every
circuit is checked on all 64 inputs before any code is written.
"""
from __future__ import annotations

import argparse
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
SPEC = os.path.join(PKG, "csrc", "des_spec.h")
OUT_INC = os.path.join(PKG, "csrc", "sbox_circuits.inc")
STORE = os.path.join(HERE, "sbox_circuits.txt")
SEARCH_SRC = os.path.join(HERE, "sbox_search.c")

MASK64 = (1 << 64) - 1


def sbox_tables() -> list[list[int]]:
    """The eight S-boxes indexed by the 6-bit input (first input bit = most significant)."""
    rows = re.findall(r'"([0-9A-F]{16})"', open(SPEC).read())
    assert len(rows) == 32
    boxes = []
    for b in range(8):
        tab = []
        for x in range(64):
            row = ((x >> 4) & 2) | (x & 1)
            col = (x >> 1) & 15
            tab.append(int(rows[4 * b + row][col], 16))
        boxes.append(tab)
    return boxes


def input_tt(i: int) -> int:
    return sum(1 << p for p in range(64) if (p >> (5 - i)) & 1)


def lut3(lut: int, a: int, b: int, c: int) -> int:
    r = 0
    for m in range(8):
        if (lut >> m) & 1:
            r |= (a if m & 4 else ~a) & (b if m & 2 else ~b) & (c if m & 1 else ~c)
    return r & MASK64


def target_tt(tab: list[int], j: int) -> int:
    return sum(1 << p for p in range(64) if (tab[p] >> (3 - j)) & 1)


class Circuit:
    def __init__(self, gates, outs):
        self.gates = gates  # list of (node, a, b, c, lut) with node = 6, 7, ...
        self.outs = outs    # node per output bit (0 = first)

    def values(self):
        val = {i: input_tt(i) for i in range(6)}
        for node, a, b, c, lut in self.gates:
            val[node] = lut3(lut, val[a], val[b], val[c])
        return val

    def polarities(self, tab) -> list[int]:
        """0 if the output node equals the S-box bit, 1 if its complement; raises otherwise."""
        val = self.values()
        pol = []
        for j in range(4):
            t = target_tt(tab, j)
            v = val[self.outs[j]]
            if v == t:
                pol.append(0)
            elif v == (~t & MASK64):
                pol.append(1)
            else:
                raise ValueError(f"output {j} is wrong")
        return pol

    def uses(self, node):
        return sum(1 for g in self.gates for x in g[1:4] if x == node)

    def cost(self):
        extra = 0
        for j, o in enumerate(self.outs):
            g = next((g for g in self.gates if g[0] == o), None)
            if g is None or len(set(g[1:4])) == 3 or self.uses(o) > 0 or o in self.outs[:j]:
                extra += 1
        return len(self.gates) + extra

    def dump(self) -> str:
        lines = [f"gates {len(self.gates)} cost {self.cost()}"]
        lines += [f"g {n} {a} {b} {c} {lut}" for n, a, b, c, lut in self.gates]
        lines.append("out " + " ".join(map(str, self.outs)))
        return "\n".join(lines)

    @staticmethod
    def parse(text: str) -> "Circuit":
        gates, outs = [], None
        for line in text.strip().splitlines():
            f = line.split()
            if f[0] == "g":
                gates.append(tuple(int(x) for x in f[1:6]))
            elif f[0] == "out":
                outs = [int(x) for x in f[1:5]]
        return Circuit(gates, outs)


def load_store(path: str = STORE) -> dict[int, Circuit]:
    if not os.path.exists(path):
        return {}
    out = {}
    for block in re.split(r"^box ", open(path).read(), flags=re.M)[1:]:
        head, _, body = block.partition("\n")
        out[int(head.split()[0]) - 1] = Circuit.parse(body)
    return out


def save_store(circuits: dict[int, Circuit], path: str = STORE):
    with open(path, "w") as f:
        f.write("# S-box circuits of 3-input lookup gates, found by sbox_search.c; see gen_sbox.py.\n")
        f.write("# Nodes 0..5 are the box inputs (0 = first); 'g node a b c table'; 'out' lists the nodes\n")
        f.write("# of output bits 1..4 (an output may be the complement of its node).\n")
        for b in sorted(circuits):
            f.write(f"box {b + 1}\n{circuits[b].dump()}\n")


def build_tool(src: str) -> str:
    exe = os.path.join(tempfile.gettempdir(), "tdes_" + os.path.splitext(os.path.basename(src))[0])
    subprocess.check_call(["gcc", "-O2", "-o", exe, src])
    return exe


def run_search(exe, tab, seed, trials, budget, width=1) -> Circuit | None:
    res = subprocess.run([exe, str(seed), str(trials), str(budget)] + [str(v) for v in tab] + [str(width)],
                         stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
    return last_circuit(res.stdout) if res.returncode == 0 else None


def last_circuit(text: str) -> Circuit | None:
    """The last circuit block ("cost ..." header, gate lines, "out" line) of a search's output."""
    blocks = [b for b in re.split(r"^cost .*$", text, flags=re.M) if b.strip()]
    return Circuit.parse(blocks[-1]) if blocks else None


def run_from(exe, args, tab, circuit: Circuit) -> Circuit | None:
    """Feed a stored circuit to the search's large-neighbourhood mode; return the last circuit it printed, or None."""
    res = subprocess.run([exe] + [str(a) for a in args] + [str(v) for v in tab], input=circuit.dump(),
                         stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
    if res.returncode != 0 or "\n" not in res.stdout:
        return None
    return last_circuit(res.stdout)


def emit(circuits: dict[int, Circuit], boxes) -> str:
    out = ["// Generated by gen/gen_sbox.py from gen/sbox_circuits.txt; do not edit.",
           "// sbox<b>(x0..x5, o0..o3): o_j ^= output bit j of S-box b+1 for inputs x0..x5",
           "// (x0 = first input bit, o0 = first output bit), 32 lanes of bits at once.",
           "// sbox<b>_m(x0..x5, o0..o3, m0..m3): o_j ^= output bit j ^ m_j (m_j a key mask, 0 or ~0).",
           "// Each gate is one v_bitop3_b32 (truth table bit 4a+2b+c).", ""]
    total = 0
    for b in range(8):
        c = circuits[b]
        pol = c.polarities(boxes[b])
        total += c.cost()
        head = (f"uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3, uint32_t n4, uint32_t n5, "
                f"uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3")
        outs_set = {}
        for j, o in enumerate(c.outs):
            outs_set.setdefault(o, []).append(j)
        # plain variant: a two-operand output gate also absorbs the XOR into the Feistel plane
        out.append(f"// S{b + 1}: {len(c.gates)} gates, {c.cost()} operations with the output XORs")
        out.append(f"__device__ __forceinline__ void sbox{b}({head}) {{")
        folded = set()
        for node, a, bb, cc, lut in c.gates:
            js = outs_set.get(node, [])
            ops = list(dict.fromkeys([a, bb, cc]))
            if len(js) == 1 and len(ops) <= 2 and c.uses(node) == 0:
                j = js[0]
                while len(ops) < 2:
                    ops.append(ops[0])
                table = 0
                for m in range(8):
                    lv, av, bv = (m >> 2) & 1, (m >> 1) & 1, m & 1
                    env = {ops[0]: av, ops[1]: bv}
                    g = (lut >> ((env[a] << 2) | (env[bb] << 1) | env[cc])) & 1
                    table |= (lv ^ g ^ pol[j]) << m
                out.append(f"    o{j} = __builtin_amdgcn_bitop3_b32(o{j}, n{ops[0]}, n{ops[1]}, 0x{table:02X});")
                folded.add(j)
                continue
            out.append(f"    const uint32_t n{node} = __builtin_amdgcn_bitop3_b32(n{a}, n{bb}, n{cc}, 0x{lut:02X});")
        for j, o in enumerate(c.outs):
            if j in folded:
                continue
            out.append(f"    o{j} = ~(o{j} ^ n{o});" if pol[j] else f"    o{j} ^= n{o};")
        out.append("}")
        out.append("")
        # masked variant: every output is a three-way XOR (Feistel plane, S-box bit, key mask)
        out.append(f"__device__ __forceinline__ void sbox{b}_m({head}, uint32_t m0, uint32_t m1, uint32_t m2, "
                   f"uint32_t m3) {{")
        for node, a, bb, cc, lut in c.gates:
            out.append(f"    const uint32_t n{node} = __builtin_amdgcn_bitop3_b32(n{a}, n{bb}, n{cc}, 0x{lut:02X});")
        for j, o in enumerate(c.outs):
            out.append(f"    o{j} = __builtin_amdgcn_bitop3_b32(o{j}, n{o}, m{j}, 0x{0x69 if pol[j] else 0x96:02X});")
        out.append("}")
        out.append("")
    out.append(f"// Total over the eight boxes: {total} operations; average {total / 8:.2f}.")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--search", type=int, default=0, help="random restarts per seed (0: use stored circuits)")
    ap.add_argument("--budget", type=int, default=200000)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--width", type=int, default=1, help="search: attempts per output, best kept")
    ap.add_argument("--lns", type=int, default=0, help="iterations of the search's large-neighbourhood mode (0: none)")
    ap.add_argument("--boxes", default="1,2,3,4,5,6,7,8")
    ap.add_argument("--store", default=STORE, help="circuit store to read and update")
    ap.add_argument("--out", default=OUT_INC, help="generated HIP include")
    args = ap.parse_args()
    boxes = sbox_tables()
    circuits = load_store(args.store)
    todo = [int(b) - 1 for b in args.boxes.split(",")]

    def accept(b, c, how):
        if c is None:
            return
        c.polarities(boxes[b])  # raises if wrong
        # Fewest gates first (the folded rounds pay one three-way XOR per output anyway),
        # then the cost with the output XORs of the per-lane-key rounds.
        if b not in circuits or (len(c.gates), c.cost()) < (len(circuits[b].gates), circuits[b].cost()):
            circuits[b] = c
            print(f"S{b + 1}: {len(c.gates)} gates, cost {c.cost()} ({how})", file=sys.stderr)

    workers = os.cpu_count() or 4
    if args.search:
        exe = build_tool(SEARCH_SRC)
        jobs = [(b, s) for b in todo for s in range(args.seeds)]
        with ThreadPoolExecutor(max_workers=workers) as pool:
            results = list(pool.map(lambda bs: (bs[0], run_search(exe, boxes[bs[0]], 1000 * bs[0] + bs[1] + 1,
                                                                   args.search, args.budget, args.width)), jobs))
        for b, c in results:
            accept(b, c, "search")
    if args.lns:
        exe = build_tool(SEARCH_SRC)
        jobs = [(b, s) for b in todo if b in circuits for s in range(args.seeds)]
        with ThreadPoolExecutor(max_workers=workers) as pool:
            results = list(pool.map(lambda bs: (bs[0], run_from(
                exe, [7000 * bs[0] + bs[1] + 1, args.lns, args.budget], boxes[bs[0]] + [max(args.width, 1), 1],
                circuits[bs[0]])), jobs))
        for b, c in results:
            accept(b, c, "large-neighbourhood search")
    if args.search or args.lns:
        save_store(circuits, args.store)
    missing = [b + 1 for b in range(8) if b not in circuits]
    if missing:
        sys.exit(f"no circuit stored for boxes {missing}; run with --search")
    for b in range(8):
        circuits[b].polarities(boxes[b])
    with open(args.out, "w") as f:
        f.write(emit(circuits, boxes))
    print(f"wrote {args.out}: {sum(len(c.gates) for c in circuits.values())} gates, "
          f"total cost {sum(c.cost() for c in circuits.values())}")


if __name__ == "__main__":
    main()
