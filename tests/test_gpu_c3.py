"""The keying-option and size sweep: three-key, two-key (K1 = K3) and one-key (K1 = K2 = K3)
triples, messages of 64 KiB, 4 MiB, 256 MiB and 4 GiB, both directions (tolerance 0 bits).

Sizes up to 256 MiB are checked block by block against the oracle (both directions); 4 GiB on
sampled blocks (first and last tiles, tile boundaries, random indices), which the oracle computes
one by one, plus the full round trip on the device.  Keying options follow the standard; the paper uses
three keys (Section I).
"""
import numpy as np
import pytest
import torch

import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests import _gpu

pytestmark = pytest.mark.gpu

SIZES = [1 << 13, 1 << 19, 1 << 25, 1 << 29]


@pytest.mark.parametrize("n_blocks", SIZES)
@pytest.mark.parametrize("keying", [3, 2, 1])
def test_sweep(n_blocks, keying):
    seed = inputs.DATA_SEED_BASE + 3 + 16 * keying
    keys = inputs.key_triple(inputs.KEY_SEED_BASE + 3 + keying, keying)
    sched = _gpu.device_sched(*keys)
    print(f"[c3] n={n_blocks} keying={keying}", flush=True)
    src = _gpu.device_message(seed, n_blocks)
    ct = torch.empty_like(src)
    pt = torch.empty_like(src)
    td.tdes_ecb_encrypt(sched, src, ct, n_blocks)
    td.tdes_ecb_decrypt(sched, ct, pt, n_blocks)
    torch.cuda.synchronize()
    assert torch.equal(pt, src)
    if n_blocks <= 1 << 25:
        host = inputs.message(seed, n_blocks)
        assert np.array_equal(ct.cpu().numpy(), _gpu.oracle_on_blocks(keys, host, False))
        # decryption of an arbitrary message, not only of ciphertext
        td.tdes_ecb_decrypt(sched, src, pt, n_blocks)
        torch.cuda.synchronize()
        assert np.array_equal(pt.cpu().numpy(), _gpu.oracle_on_blocks(keys, host, True))
    else:
        idx = _gpu.sample_indices(n_blocks, 1 << 14, keying, boundaries=[k << 20 for k in range(1, n_blocks >> 20, 13)])
        host_in = inputs.blocks_at(seed, idx)
        assert np.array_equal(_gpu.gather_blocks(ct, idx), _gpu.oracle_on_blocks(keys, host_in, False))
        td.tdes_ecb_decrypt(sched, src, pt, n_blocks)
        torch.cuda.synchronize()
        assert np.array_equal(_gpu.gather_blocks(pt, idx), _gpu.oracle_on_blocks(keys, host_in, True))
    del src, ct, pt
    torch.cuda.empty_cache()
