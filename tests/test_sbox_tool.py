"""The S-box circuit search tool (paper_1305_4376_amd/gen/sbox_search.c), built with gcc and run on the CPU.

A short fresh search and a short large-neighbourhood pass from a stored circuit each print circuits
that compute the S-box on all 64 inputs, checked here against the oracle's S-box table (FIPS 46-3),
with the tool's arguments in their documented order (seed, trials, budget, the 64 table entries,
width, improve).  Nothing is written into the source tree.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GEN = os.path.join(ROOT, "paper_1305_4376_amd", "gen")
sys.path.insert(0, GEN)
import gen_sbox  # noqa: E402  (parsing and evaluation of circuits only)

MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def tool(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sbox_tool") / "sbox_search")
    subprocess.check_call(["gcc", "-O2", "-o", exe, os.path.join(GEN, "sbox_search.c")])
    return exe


def _table(box):
    """S-box box + 1 by its 6-bit input, the first input bit the most significant."""
    t = np.frombuffer(bytes(oracle.table("SBOX")), dtype=np.uint8).reshape(8, 4, 16)
    return [int(t[box, ((x >> 4) & 2) | (x & 1), (x >> 1) & 15]) for x in range(64)]


def _check(circuit, tab):
    val = circuit.values()
    for j in range(4):
        want = sum(1 << p for p in range(64) if (tab[p] >> (3 - j)) & 1)
        assert val[circuit.outs[j]] in (want, ~want & MASK64), f"output {j}"


def _run(tool, args, stdin=""):
    return subprocess.run([tool] + [str(a) for a in args], input=stdin, capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("box", [0, 3, 7])
def test_fresh_search_prints_a_correct_circuit(tool, box):
    tab = _table(box)
    res = _run(tool, [7, 2, 20000] + tab + [2, 0])
    assert res.returncode == 0, res.stderr
    circuit = gen_sbox.last_circuit(res.stdout)
    assert circuit is not None and len(circuit.gates) > 0
    _check(circuit, tab)


def test_improve_pass_keeps_a_correct_circuit(tool):
    store = gen_sbox.load_store()
    tab = _table(4)
    start = store[4]
    _check(start, tab)
    res = _run(tool, [9, 20, 20000] + tab + [2, 1], stdin=start.dump() + "\n")
    assert res.returncode == 0, res.stderr
    assert f"start: gates {len(start.gates)}" in res.stderr
    circuit = gen_sbox.last_circuit(res.stdout)
    _check(circuit, tab)
    assert len(circuit.gates) <= len(start.gates)


def test_improve_pass_rejects_a_wrong_start_circuit(tool):
    store = gen_sbox.load_store()
    res = _run(tool, [9, 5, 20000] + _table(4) + [2, 1], stdin=store[3].dump() + "\n")  # box 4's circuit
    assert res.returncode != 0 and "not correct" in res.stderr
