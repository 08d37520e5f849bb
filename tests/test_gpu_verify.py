"""One-launch verification: zero mismatches for a correct stego, and the
exact number of corrupted bytes otherwise (counted against the oracle)."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import api, inputs

from gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("n,off", [(33, 0), (1000, 0), (65543, 0), (1 << 20, 5), (3000001, 0)])
def test_verify_counts(k, n, off):
    cover = inputs.random_bytes(n, 2001, k, n)
    cap = oracle.capacity(n, k)
    if cap < 0:
        pytest.skip("no room for a header")
    msg = inputs.random_bytes(int(inputs.rng(2002, k, n).integers(0, cap + 1)), 2003, k, n)
    rc, stego = oracle.embed(cover, msg, k)
    c_d, m_d = to_dev(cover, pad_before=off, pad_after=16), to_dev(msg)
    assert int(api.verify(c_d, to_dev(stego, pad_before=off, pad_after=16), m_d, k).item()) == 0
    bad = stego.copy()
    idx = inputs.rng(2004, k, n).choice(n, size=min(n, 37), replace=False)
    bad[idx] ^= 0x10 | (inputs.rng(2005).integers(1, 256, size=idx.size).astype(np.uint8) & 0xEF)
    want = int(np.count_nonzero(bad != stego))
    assert int(api.verify(c_d, to_dev(bad, pad_before=off, pad_after=16), m_d, k).item()) == want


def test_verify_after_device_embed_and_in_place():
    n, k = 201326592, 1
    cover = torch.empty(n, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(cover, 2011)
    msg = torch.empty(api.capacity(n, k), dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(msg, 2012)
    stego = api.embed(cover, msg, k)
    assert int(api.verify(cover, stego, msg, k).item()) == 0
    buf = cover.clone()
    api.embed(buf, msg, k, out=buf)
    assert torch.equal(buf, stego)
    stego[123456789] ^= 1
    assert int(api.verify(cover, stego, msg, k).item()) == 1
