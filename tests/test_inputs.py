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
