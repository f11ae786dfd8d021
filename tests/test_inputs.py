"""The seeded input generator: counter-style SplitMix64 equals the sequential generator."""
import numpy as np

from paper_1305_4376_amd import inputs

MASK = (1 << 64) - 1


def _splitmix64_sequential(seed, count):
    # The generator as published: state += gamma, then the output mix of the new state.
    state, out = seed & MASK, []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_counter_form_equals_sequential():
    for seed in (0, 1, 0x3DE50001, MASK):
        want = _splitmix64_sequential(seed, 100)
        assert [int(v) for v in inputs.splitmix64(seed, 0, 100)] == want
        assert [int(v) for v in inputs.splitmix64(seed, 37, 10)] == want[37:47]
        assert [int(v) for v in inputs.splitmix64_at(seed, [5, 99, 0])] == [want[5], want[99], want[0]]


def test_message_layout_and_slices():
    m = inputs.message(7, 64)
    assert m.dtype == np.uint8 and m.size == 512
    assert np.array_equal(inputs.message(7, 16, first_block=10), m[80:208])
    assert np.array_equal(inputs.blocks_at(7, [3, 1]), np.concatenate([m[24:32], m[8:16]]))
    assert int.from_bytes(m[:8].tobytes(), "little") == int(inputs.splitmix64(7, 0, 1)[0])


def test_keys_have_odd_parity_and_keying():
    for keying in (1, 2, 3):
        k1, k2, k3 = inputs.key_triple(11, keying)
        for k in (k1, k2, k3):
            assert all(bin(b).count("1") % 2 == 1 for b in k)
        assert (k1 == k3) == (keying < 3)
        assert (k1 == k2) == (keying == 1)
    t = inputs.key_triples(12, 50)
    assert t.shape == (50, 24)
    assert all(bin(int(b)).count("1") % 2 == 1 for b in t.reshape(-1))


def test_log_uniform_lengths():
    n = inputs.log_uniform_lengths(13, 4096, 131072)
    assert n.min() >= 1 and n.max() <= 131072
    med = np.median(n)
    assert 150 < med < 900  # exp(ln(131073)/2) ~ 362


def _payload_sequential(seed, count):
    # Column t of the payload (words t, t + 256, ...) walks chains of 64 words: each chain opens with
    # the SplitMix64 word at its own index, and each later word is one xorshift64 step on.
    stream = _splitmix64_sequential(seed, count)
    out = [0] * count
    for t in range(min(256, count)):
        x = 0
        for row, i in enumerate(range(t, count, 256)):
            if row % 64 == 0:
                x = stream[i]
            else:
                x ^= (x << 13) & MASK
                x ^= x >> 7
                x ^= (x << 17) & MASK
            out[i] = x
    return out


def test_payload_chains():
    """Served payloads: chain heads are the stream's words, the rest xorshift64 successors; slices
    and sampled indices agree with the whole; no repeated word in a 2^20-word payload."""
    n = 3 * 16384 + 777                     # three whole chains per column, a partial fourth
    want = _payload_sequential(0x5E000001, n)
    got = inputs.payload(0x5E000001, n).view("<u8")
    assert [int(v) for v in got] == want
    idx = np.array([0, 255, 256, 16383, 16384, 16384 + 300, n - 1])
    assert [int(v) for v in inputs.payload_words_at(0x5E000001, idx)] == [want[i] for i in idx]
    big = inputs.payload(17, 1 << 20).view("<u8")
    assert np.unique(big).size == big.size
    assert int(big[0]) == int(inputs.splitmix64(17, 0, 1)[0])
