"""lsb_time_next_launch: a timing request is taken by the next launch of a
timed call, and a call that fails or has nothing to launch clears it without
recording, so the events never reach a later, untimed call."""
import numpy as np
import pytest
import torch

from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import lib

from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def _recorded_pair():
    """Two timing events recorded around a ~1 GiB fill, so that their
    interval is far from that of a small kernel."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    big = torch.empty(1 << 30, dtype=torch.uint8, device=DEV)
    a.record()
    big.fill_(7)
    b.record()
    torch.cuda.synchronize()
    del big
    return a, b


def _small_embed():
    cover = torch.from_numpy(inputs.random_bytes(1 << 20, 3301)).to(DEV)
    msg = torch.from_numpy(inputs.random_bytes(1000, 3302)).to(DEV)
    api.embed(cover, msg, 1)
    torch.cuda.synchronize()


def test_timed_launch_records_the_kernel():
    n = 64 << 20
    cover = torch.from_numpy(inputs.random_bytes(n, 3303)).to(DEV)
    msg = torch.from_numpy(inputs.random_bytes(1 << 20, 3304)).to(DEV)
    a, b = _recorded_pair()
    before = a.elapsed_time(b)
    lib().lsb_time_next_launch(a, b)
    api.embed(cover, msg, 1)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    assert ms != before, "the events were not recorded by the launch"
    # the kernel's own span: more than a microsecond for 2n bytes (the cover
    # may still sit in the 256 MB last-level cache, so no HBM bound is
    # assumed), and far below the 1 GiB fill the events first spanned
    assert 0.001 < ms < min(1.0, before), (ms, before)


@pytest.mark.parametrize("case", ["bad k", "empty raw slice", "capacity", "no stream bits to extract"])
def test_unused_request_is_cleared(case):
    a, b = _recorded_pair()
    before = a.elapsed_time(b)
    cover = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    lib().lsb_time_next_launch(a, b)
    if case == "bad k":
        with pytest.raises(Exception):
            api.embed(cover, torch.zeros(10, dtype=torch.uint8, device=DEV), 9)
    elif case == "empty raw slice":
        api.embed_raw(cover[:0], 0, torch.zeros(16, dtype=torch.uint8, device=DEV), 64, 1)
    elif case == "capacity":
        with pytest.raises(Exception):
            api.embed(cover, torch.zeros(600, dtype=torch.uint8, device=DEV), 1)
    else:  # the slice starts past the stream's end: nothing to extract
        out = torch.zeros(16, dtype=torch.uint8, device=DEV)
        api.extract_raw(cover, 1024, out, 64, 1)
    torch.cuda.synchronize()
    # an untimed launch afterwards must not record the events
    _small_embed()
    assert a.elapsed_time(b) == before, "a cleared request reached a later launch (%s)" % case
    del cover
    assert np.isfinite(before)
