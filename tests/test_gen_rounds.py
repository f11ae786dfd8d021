"""The generated round assembly (csrc/rounds_asm.inc) on the CPU: regenerating it from the stored
circuits and the standard's E and P gives the committed file, and the emitted instructions, simulated
on random planes and key words, compute two folded rounds exactly (the definition the kernels'
C++ rounds follow; the GPU unit tests pin both against the oracle)."""
import os
import random

from paper_1305_4376_amd.gen import gen_rounds

INC = os.path.join(os.path.dirname(gen_rounds.HERE), "csrc", "rounds_asm.inc")


def _seed_of_committed() -> int:
    first = open(INC).readline()
    return int(first.split("(seed ")[1].split(")")[0])


def test_generated_rounds_match_the_committed_file_and_the_round():
    seed = _seed_of_committed()
    rd = gen_rounds.Round()
    pairs = [gen_rounds.gen_pair(rd, seed, swap) for swap in (False, True)]
    for em, plane_reg, _ in pairs:
        gen_rounds.check(rd, em, plane_reg, trials=50, seed=7)
    assert gen_rounds.emit_inc(pairs, seed) == open(INC).read()
    # registers: 64 plane registers, all distinct, inside the block's range
    em, plane_reg, stats = pairs[0]
    regs = plane_reg[0] + plane_reg[1]
    assert len(set(regs)) == 64 and min(regs) >= gen_rounds.FIRST_VGPR and max(regs) <= gen_rounds.LAST_VGPR
    assert stats["valu"] == 2 * (sum(len(c.gates) for c in rd.circuits.values()) + 32 + 16)


def test_check_catches_a_wrong_gate():
    """A planted mistake (one gate's truth table changed) must fail the simulation check."""
    rd = gen_rounds.Round()
    em, plane_reg, _ = gen_rounds.gen_pair(rd, 1)
    k = next(i for i, p in enumerate(em.prog) if p[0] == "bitop3")
    op, dst, srcs, lut = em.prog[k]
    em.prog[k] = (op, dst, srcs, lut ^ 0x10)
    try:
        gen_rounds.check(rd, em, plane_reg, trials=20, seed=3)
    except AssertionError:
        return
    raise AssertionError("the check did not notice a changed gate")


def test_reference_round_is_a_feistel_round():
    """The generator's reference round leaves y alone and is an involution on x for fixed y and words
    (x ^= f(y) twice), which a dropped or doubled XOR would break."""
    rd = gen_rounds.Round()
    rng = random.Random(5)
    x = [rng.getrandbits(32) for _ in range(32)]
    y = [rng.getrandbits(32) for _ in range(32)]
    ow, cw = rng.getrandbits(32), rng.getrandbits(32)
    x1 = rd.reference(x, y, ow, cw)
    assert x1 != x
    assert rd.reference(x1, y, ow, cw) == x
