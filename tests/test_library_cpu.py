"""Host-side checks of libtdes that need no GPU.

  * the library loads and exports every function include/tdes.h declares;
  * host key expansion equals the oracle's subkeys, in the order EDE uses them
    (Section II.A) for both directions;
  * flags, parity and weak-key rejection, and argument errors are reported
    before anything reaches a device;
  * the kernels' compile-time DES constants (des_spec.h) equal the oracle's tables.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdes.h")
SPEC = os.path.join(ROOT, "paper_1305_4376_amd", "csrc", "des_spec.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tdes_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = td.load_library()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    assert td.tdes_status_str(0) == "ok"
    for code in range(-1, -12, -1):
        assert td.tdes_status_str(code) != "unknown status"
    assert td.tdes_status_str(-99) == "unknown status"


DIR_WORDS = td.TDES_SCHED_BYTES // 8  # each direction's block of the schedule, in words


def _decode(sched: np.ndarray):
    """The schedule's private round layout, back to 48-bit subkeys (two directions x 48 rounds)."""
    w = sched.view("<u4")
    out = []
    for d in range(2):
        rounds = []
        for r in range(48):
            a, b = int(w[DIR_WORDS * d + 2 * r]), int(w[DIR_WORDS * d + 2 * r + 1])
            c = [0] * 8
            c[0], c[6], c[4], c[2] = (a & 63), (a >> 8) & 63, (a >> 16) & 63, (a >> 24) & 63
            c[1], c[7], c[5], c[3] = (b & 63), (b >> 8) & 63, (b >> 16) & 63, (b >> 24) & 63
            assert a & 0xC0C0C0C0 == 0 and b & 0xC0C0C0C0 == 0
            v = 0
            for x in c:
                v = (v << 6) | x
            rounds.append(v)
        out.append(rounds)
    return out


@pytest.mark.parametrize("keying", [3, 2, 1])
def test_expand_key_matches_oracle_subkeys(keying):
    for seed in range(6):
        k1, k2, k3 = inputs.key_triple(0x700 + seed, keying)
        enc, dec = _decode(td.tdes_expand_key(k1, k2, k3))
        s1, s2, s3 = oracle.des_subkeys(k1), oracle.des_subkeys(k2), oracle.des_subkeys(k3)
        assert enc == s1 + s2[::-1] + s3
        assert dec == s3[::-1] + s2 + s1[::-1]


def test_expand_key_flags():
    k = inputs.key_triple(0x710)
    base = td.tdes_expand_key(*k)
    assert np.array_equal(td.tdes_expand_key(*k, flags=td.TDES_CHECK_PARITY | td.TDES_REJECT_WEAK), base)
    bad = bytes([k[0][0] ^ 1]) + k[0][1:]
    # Parity is ignored by default (the standard's PC-1 drops those bits) ...
    assert np.array_equal(td.tdes_expand_key(bad, k[1], k[2]), base)
    # ... and rejected on request.
    with pytest.raises(td.TdesError) as e:
        td.tdes_expand_key(bad, k[1], k[2], flags=td.TDES_CHECK_PARITY)
    assert e.value.code == -5
    for weak in ("0101010101010101", "fefefefefefefefe", "e0e0e0e0f1f1f1f1", "01fe01fe01fe01fe", "1fe01fe00ef10ef1"):
        w = bytes.fromhex(weak)
        td.tdes_expand_key(k[0], w, k[2])  # accepted without the flag
        with pytest.raises(td.TdesError) as e:
            td.tdes_expand_key(k[0], w, k[2], flags=td.TDES_REJECT_WEAK)
        assert e.value.code == -6
    with pytest.raises(td.TdesError) as e:
        td.tdes_expand_key(*k, flags=8)
    assert e.value.code == -7


def test_expand_key_null_arguments():
    lib = td.load_library()
    out = np.zeros(td.TDES_SCHED_BYTES, np.uint8)
    k = ctypes.create_string_buffer(b"\x01" * 8, 8)
    assert lib.tdes_expand_key(None, k, k, 0, out.ctypes.data) == -1
    assert lib.tdes_expand_key(k, k, k, 0, None) == -1


def test_argument_errors_are_host_side():
    lib = td.load_library()
    s, a, b = 0x10000, 0x200000, 0x400000
    # zero blocks: nothing is enqueued, no device is touched
    assert lib.tdes_ecb_run(s, a, b, 0, 0, 0, None) == 0
    assert lib.tdes_ecb_encrypt(s, a, a, 0, None) == 0
    assert lib.tdes_ecb_run(None, a, b, 0, 0, 0, None) == -1
    assert lib.tdes_ecb_run(s, None, b, 0, 0, 0, None) == -1
    assert lib.tdes_ecb_run(s, a + 4, b, 0, 0, 0, None) == -2
    assert lib.tdes_ecb_run(s + 2, a, b, 0, 0, 0, None) == -2
    assert lib.tdes_ecb_run(s, a, a + 8, 16, 0, 0, None) == -3
    assert lib.tdes_ecb_run(s, a + 8, a, 16, 0, 0, None) == -3
    assert lib.tdes_ecb_run(s, a, b, (1 << 58) + 1, 0, 0, None) == -4
    assert lib.tdes_ecb_run(s, a, b, 0, 2, 0, None) == -7
    assert lib.tdes_ecb_run(s, a, b, 0, 0, 3, None) == -7
    assert lib.tdes_sched_upload(None, 0, None, None) == 0
    assert lib.tdes_sched_upload(None, 1, b, None) == -1
    assert lib.tdes_fill_splitmix64(None, 0, 1, 0, None) == 0
    assert lib.tdes_fill_splitmix64(a + 4, 8, 1, 0, None) == -2


def _spec_text():
    return open(SPEC).read()


def test_kernel_sboxes_equal_oracle_tables():
    text = _spec_text()
    rows = re.findall(r'"([0-9A-F]{16})"', text)
    assert len(rows) == 32
    flat = [int(ch, 16) for row in rows for ch in row]
    assert flat == oracle.table("SBOX")


def test_kernel_permutations_equal_oracle_tables():
    text = _spec_text()

    def arr(name):
        m = re.search(name + r"\[\d+\]\s*=\s*\{([^}]*)\}", text)
        return [int(v) + 1 for v in m.group(1).replace("\n", " ").split(",") if v.strip()]
    assert arr("kP") == oracle.table("P")
    assert arr("kPC2") == oracle.table("PC2")
    assert [v - 1 for v in arr("kShift")] == oracle.table("SHIFTS")


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's record types have the sizes and field offsets the C header gives them."""
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tdes.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(tdes_job), sizeof(tdes_batch_info),'
        ' sizeof(tdes_request), sizeof(tdes_completion), sizeof(tdes_serve_config), sizeof(tdes_serve_stats),'
        ' offsetof(tdes_request, host_out), offsetof(tdes_completion, t_complete), sizeof(tdes_sched),'
        ' offsetof(tdes_serve_config, backlog_step_blocks)); return 0; }\n')
    exe = tmp_path / "sizes"
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    import ctypes as ct
    want = [td.JOB_DTYPE.itemsize, ct.sizeof(td._BatchInfo), td.REQUEST_DTYPE.itemsize, td.COMPLETION_DTYPE.itemsize,
            ct.sizeof(td._ServeConfig), ct.sizeof(td._ServeStats), td.REQUEST_DTYPE.fields["host_out"][1],
            td.COMPLETION_DTYPE.fields["t_complete"][1], td.TDES_SCHED_BYTES, td._ServeConfig.backlog_step_blocks.offset]
    assert got == want


def test_host_path_argument_errors():
    lib = td.load_library()
    s, a, b = 0x10000, 0x200000, 0x400000
    assert lib.tdes_ecb_host(s, a, b, 0, 0, 1, None) == 0          # nothing to do
    assert lib.tdes_ecb_host(None, a, b, 8, 0, 1, None) == -1
    assert lib.tdes_ecb_host(s + 2, a, b, 8, 0, 1, None) == -2
    assert lib.tdes_ecb_host(s, a, b, 8, 5, 1, None) == -7
    assert lib.tdes_ecb_host(s, a, b, 8, 0, 0, None) == -4
    assert lib.tdes_ecb_host(s, a, a + 8, 8, 0, 4, None) == -3


def _oracle_first_and_second_uses():
    """From the oracle's E table: the first E position reading each R bit, and the second uses in order."""
    e = [x - 1 for x in oracle.table("E")]
    first, second = {}, []
    for i, q in enumerate(e):
        if q in first:
            second.append(i)
        else:
            first[q] = i
    return e, first, second


@pytest.mark.parametrize("keying", [3, 2, 1])
def test_folded_key_words_match_oracle_subkeys(keying):
    """The bitsliced kernels' folded mask words, rebuilt here from the oracle's subkeys and E table."""
    e, first, second = _oracle_first_and_second_uses()
    assert len(second) == 16
    bit = lambda k, i: (k >> (47 - i)) & 1
    for seed in range(4):
        k1, k2, k3 = inputs.key_triple(0x720 + seed, keying)
        s1, s2, s3 = oracle.des_subkeys(k1), oracle.des_subkeys(k2), oracle.des_subkeys(k3)
        w = td.tdes_expand_key(k1, k2, k3).view("<u4")
        for d, order in enumerate((s1 + s2[::-1] + s3, s3[::-1] + s2 + s1[::-1])):
            fold = w[DIR_WORDS * d + 96: DIR_WORDS * d + 96 + 104]
            for r in range(48):
                i = r % 16
                diff = (order[r - 1] if i > 0 else 0) ^ (order[r + 1] if i < 15 else 0)
                assert int(fold[r]) == sum(bit(diff, first[q]) << q for q in range(32)), (d, r)
                corr = sum((bit(order[r], first[e[p]]) ^ bit(order[r], p)) << t for t, p in enumerate(second))
                assert int(fold[48 + r]) == corr, (d, r)
            for st in range(3):
                assert int(fold[96 + st]) == sum(bit(order[16 * st], first[q]) << q for q in range(32))
                assert int(fold[99 + st]) == sum(bit(order[16 * st + 15], first[q]) << q for q in range(32))
            for st in range(2):   # between stages: remove stage st's last key, add stage st + 1's first
                assert int(fold[102 + st]) == sum((bit(order[16 * st + 15], first[q]) ^
                                                   bit(order[16 * st + 16], first[q])) << q for q in range(32))


INC = os.path.join(os.path.dirname(SPEC), "sbox_circuits.inc")


def _eval_circuit_functions():
    """Evaluate every function of the generated S-box include on all 64 inputs, as 64-bit truth
    tables (bit p = input p, input variable i = bit 5 - i of p).  v_bitop3_b32's table bit is
    4a + 2b + c for operand bits a, b, c."""
    full = (1 << 64) - 1
    ins = [sum(1 << p for p in range(64) if (p >> (5 - i)) & 1) for i in range(6)]

    def bitop3(a, b, c, lut):
        r = 0
        for m in range(8):
            if (lut >> m) & 1:
                r |= (a if m & 4 else full ^ a) & (b if m & 2 else full ^ b) & (c if m & 1 else full ^ c)
        return r

    funcs = {}
    for m in re.finditer(r"void (sbox\d(?:_m)?)\(([^)]*)\) \{(.*?)\n\}", open(INC).read(), flags=re.S):
        funcs[m.group(1)] = m.group(3)
    results = {}
    for name, body in funcs.items():
        for mask in ((0, full) if name.endswith("_m") else (0,)):
            env = {f"n{i}": ins[i] for i in range(6)}
            env.update({f"o{j}": 0 for j in range(4)}, **{f"m{j}": mask for j in range(4)})
            for line in body.strip().splitlines():
                line = line.strip().rstrip(";")
                if g := re.fullmatch(r"(?:const uint32_t )?(\w+) = __builtin_amdgcn_bitop3_b32\((\w+), (\w+), (\w+), (0x[0-9A-F]+)\)", line):
                    env[g.group(1)] = bitop3(env[g.group(2)], env[g.group(3)], env[g.group(4)], int(g.group(5), 16))
                elif g := re.fullmatch(r"(\w+) \^= (\w+)", line):
                    env[g.group(1)] ^= env[g.group(2)]
                elif g := re.fullmatch(r"(\w+) = ~\((\w+) \^ (\w+)\)", line):
                    env[g.group(1)] = full ^ (env[g.group(2)] ^ env[g.group(3)])
                else:
                    raise AssertionError(f"unexpected statement in {name}: {line}")
            results[(name, mask)] = [env[f"o{j}"] for j in range(4)]
    return results


def test_generated_sbox_circuits_equal_oracle_tables():
    """The S-box circuits as the kernels compile them (sbox_circuits.inc), on all 64 inputs, plain
    and with key masks 0 and ~0, against the oracle's S-box table."""
    table = oracle.table("SBOX")
    full = (1 << 64) - 1
    results = _eval_circuit_functions()
    assert len(results) == 8 + 16
    for b in range(8):
        want = [0] * 4
        for p in range(64):
            s = table[b * 64 + (((p >> 5) & 1) * 2 + (p & 1)) * 16 + ((p >> 1) & 15)]
            for j in range(4):
                if (s >> (3 - j)) & 1:
                    want[j] |= 1 << p
        assert results[(f"sbox{b}", 0)] == want, b
        assert results[(f"sbox{b}_m", 0)] == want, b
        assert results[(f"sbox{b}_m", full)] == [w ^ full for w in want], b


def test_binding_checks_buffer_sizes_before_the_c_call():
    """Sized buffers (tensors, arrays) smaller than a call would touch raise ValueError in the binding,
    before anything reaches the library or a device (host arrays stand in for device tensors here)."""
    sched = np.zeros(td.TDES_SCHED_BYTES, np.uint8)
    a, b = np.zeros(64, np.uint8), np.zeros(56, np.uint8)
    with pytest.raises(ValueError, match="output"):
        td.tdes_ecb_run(sched, a, b)                       # 8 blocks in, room for 7 out
    with pytest.raises(ValueError, match="input"):
        td.tdes_ecb_encrypt(sched, b, a, n_blocks=8)        # explicit count past the input
    with pytest.raises(ValueError, match="schedule"):
        td.tdes_ecb_decrypt(sched[:800], a, a)
    with pytest.raises(ValueError, match="output"):
        td.tdes_ctr_crypt(sched, b"\0" * 8, a, b)
    with pytest.raises(ValueError, match="output"):
        td.tdes_cbc_decrypt(sched, b"\0" * 8, a, b)
    with pytest.raises(ValueError, match="output"):
        td.tdes_ecb_chunked(sched, a, b, 2)
    with pytest.raises(ValueError, match="output"):
        td.tdes_ecb_host(sched, a, b)
    with pytest.raises(ValueError, match="output"):
        td.tdes_fill_splitmix64(b, 8, 1)
    with pytest.raises(ValueError, match="8-byte"):
        td.tdes_ecb_run(sched, a[:60], a[:60])
    with pytest.raises(ValueError, match="negative"):
        td.tdes_ecb_run(sched, a, a, n_blocks=-1)
    with pytest.raises(ValueError, match="contiguous"):
        td.tdes_ecb_run(sched, a.reshape(8, 8)[:, :4], a)
    with pytest.raises(ValueError, match="schedule table"):
        td.tdes_sched_upload(np.zeros(2 * td.TDES_SCHED_BYTES, np.uint8), sched)
    with pytest.raises(ValueError, match="host bytes"):
        td.tdes_sched_upload(sched, np.zeros(2 * td.TDES_SCHED_BYTES, np.uint8), count=2)
    jobs = np.zeros(2, dtype=td.JOB_DTYPE)
    jobs["n_blocks"] = 4
    jobs["in_off"] = [0, 32]
    jobs["out_off"] = [64, 96]                             # the second output ends at byte 128
    with pytest.raises(ValueError, match="batch base"):
        td.tdes_ecb_batch(0, jobs, sched, 1, np.zeros(120, np.uint8))
    with pytest.raises(ValueError, match="schedule table"):
        td.tdes_ecb_batch(0, jobs, sched, 2, np.zeros(128, np.uint8))
    with pytest.raises(ValueError, match="schedule table"):
        td.tdes_server_create(sched, 2, 1 << 20)


def test_ctx_create_rejects_a_missing_device():
    """tdes_ctx_create takes a device; one past the device count is an argument error (no GPU here:
    the count is 0, so any non-negative device is missing)."""
    lib = td.load_library()
    h = ctypes.c_void_p()
    rc = lib.tdes_ctx_create(ctypes.byref(h), 1 << 20)
    assert rc in (-7, -8) and not h.value     # -8 where the runtime cannot count devices at all
    assert lib.tdes_ctx_create(None, 0) == -1


def test_library_embeds_every_kernel():
    """The built library carries the gfx950 code of every kernel its launchers start (the kernel
    names appear in the embedded code objects): a source left out of the build, or a kernel lost to
    a preprocessor branch, fails here rather than at launch."""
    data = open(td.library_path(), "rb").read()
    for name in (b"tdes_bitslice_kernel", b"tdes_bitslice_tail_kernel", b"tdes_table_kernel", b"tdes_batch_kernel",
                 b"tdes_batch_kernel_capped", b"tdes_static_plan_kernel", b"tdes_static_batch_kernel", b"fill_kernel", b"fill_tiles_kernel"):
        assert name in data, name
    assert b"gfx950" in data
