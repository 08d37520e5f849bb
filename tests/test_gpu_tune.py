"""The autotuner on the GPU: lsb_autotune times its candidate launch shapes
for one (op, k, size bucket), installs the fastest in the table and reports
it; launches with the installed shape stay bit-exact against the oracle.  The
table entry is restored afterwards."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import OK, OP_EMBED, OP_EXTRACT

from gpu_helpers import DEV, assert_bytes_equal, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,k", [(OP_EMBED, 1), (OP_EXTRACT, 1), (OP_EMBED, 3), (OP_EXTRACT, 5)])
def test_autotune_installs_a_valid_shape(op, k):
    n = (1 << 20) + 37  # size bucket 20, a ragged tail
    bucket = 20
    before = api.tune_get(op, k, n)
    cap = oracle.capacity(n, k)
    cover = torch.empty(n, dtype=torch.uint8, device=DEV)
    stego = torch.empty(n, dtype=torch.uint8, device=DEV)
    msg = torch.empty(cap, dtype=torch.uint8, device=DEV)
    try:
        cfg, us = api.autotune(op, k, cover, stego, msg, reps=2)
        assert us > 0
        assert cfg["block"] in (256, 512, 1024) and cfg["unroll"] in (1, 2, 4)
        assert cfg["blocks_per_cu"] in (0, 1, 2, 4, 8, 16) and cfg["nontemporal"] in (0, 1)
        assert cfg["pack"] in ((0, 1) if (op == OP_EXTRACT and k == 1) else (0,)) and cfg["order"] in (0, 1)
        assert api.tune_get(op, k, n) == cfg, "the fastest shape is installed for the bucket"
        # launches now use the tuned shape: bit-exact against the oracle
        cover_np = inputs.random_bytes(n, 2701, op, k)
        msg_np = inputs.random_bytes(cap - 11, 2702, op, k)
        rc, want = oracle.embed(cover_np, msg_np, k)
        assert rc == OK
        got = api.embed(to_dev(cover_np), to_dev(msg_np), k)
        assert_bytes_equal(to_host(got), want, "embed with the tuned shape (k=%d)" % k)
        out, ls = api.extract(got, k)
        ls = ls.cpu().numpy()
        assert ls[1] == OK and int(np.uint32(ls[0])) == msg_np.size
        assert_bytes_equal(to_host(out)[:msg_np.size], msg_np, "extract with the tuned shape (k=%d)" % k)
    finally:
        api.tune_set(op, k, bucket, before["block"], before["unroll"], before["blocks_per_cu"],
                     before["nontemporal"], before["pack"])
    assert api.tune_get(op, k, n) == before


def test_autotune_argument_errors():
    cover = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    stego = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    msg = torch.zeros(508, dtype=torch.uint8, device=DEV)
    for op, k, reps in [(7, 1, 2), (OP_EMBED, 0, 2), (OP_EMBED, 9, 2), (OP_EMBED, 1, 0), (OP_EXTRACT, 1, 1001)]:
        with pytest.raises(Exception):
            api.autotune(op, k, cover, stego, msg, reps=reps)
