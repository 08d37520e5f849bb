"""Randomised single-plane and paper-layout calls (hypothesis, derandomised):
any channel count 1..6 (the vector kernels take 1..4 on 16-byte aligned
buffers, the others the per-byte kernels), any plane, any k, messages up to
capacity, buffers at byte offsets 0..15, in place or not, and output
buffers larger or smaller than the message.  Every byte is compared with
the oracle, and bytes around the outputs must stay untouched."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import OK

from gpu_helpers import assert_bytes_equal, empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

FILL = 0xA5
SETTINGS = settings(max_examples=60, deadline=None, derandomize=True, database=None,
                    suppress_health_check=list(HealthCheck))
offsets = st.integers(0, 15)


@SETTINGS
@given(k=st.integers(1, 8), pixels=st.one_of(st.integers(1, 64), st.integers(65, 200_000)), c=st.integers(1, 6),
       plane_frac=st.floats(0, 0.999), frac=st.floats(0, 1), co=offsets, so=offsets, mo=offsets, oo=offsets,
       inplace=st.booleans(), short=st.booleans(), seed=st.integers(0, 2**31 - 1))
def test_plane_round_trip(k, pixels, c, plane_frac, frac, co, so, mo, oo, inplace, short, seed):
    cap = oracle.capacity(pixels, k)
    if cap < 0:
        return
    plane = int(plane_frac * c)
    ln = int(frac * cap)
    g = inputs.rng(seed)
    cover_np = g.integers(0, 256, pixels * c, dtype=np.uint8)
    msg_np = g.integers(0, 256, ln, dtype=np.uint8)
    rc, want = oracle.embed_plane(cover_np, c, plane, msg_np, k)
    assert rc == OK
    tag = "k=%d pixels=%d c=%d plane=%d len=%d offs=%s inplace=%d" % (k, pixels, c, plane, ln, (co, so, mo, oo), inplace)
    msg = to_dev(msg_np, pad_before=mo, pad_after=16)
    if inplace:
        stego = to_dev(cover_np, pad_before=co, pad_after=16)
        api.embed_plane(stego, c, plane, msg, k, out=stego)
    else:
        stego = empty_dev(pixels * c, pad_before=so)
        api.embed_plane(to_dev(cover_np, pad_before=co, pad_after=16), c, plane, msg, k, out=stego)
    assert_bytes_equal(to_host(stego), want, "plane embed " + tag)
    # extract into a buffer one byte short of the message (if asked) or larger
    out_cap = ln - 1 if (short and ln > 0) else ln + 8
    orc, oln, omsg = oracle.extract_plane(want, c, plane, k, out_cap=out_cap)
    out = to_dev(np.full(max(out_cap, 1), FILL, np.uint8), pad_before=oo, pad_after=16)[:out_cap]
    out, ls = api.extract_plane(stego, c, plane, k, out=out)
    lsn = ls.cpu().numpy()
    assert lsn[1] == orc and int(np.uint32(lsn[0])) == oln, tag + ": len/status %s want %d/%d" % (lsn, oln, orc)
    got = to_host(out)
    if orc == OK:
        assert_bytes_equal(got[:ln], omsg, "plane extract " + tag)
        assert np.all(got[ln:] == FILL), tag + ": bytes past the message written"
    else:
        assert np.all(got == FILL), tag + ": a failed extract wrote its output"


@SETTINGS
@given(h=st.integers(1, 300), w=st.integers(1, 900), c=st.integers(1, 6), plane_frac=st.floats(0, 0.999),
       frac=st.floats(0, 1), co=offsets, so=offsets, do=offsets, oo=offsets, inplace=st.booleans(),
       seed=st.integers(0, 2**31 - 1))
def test_paper_layout_round_trip(h, w, c, plane_frac, frac, co, so, do, oo, inplace, seed):
    plane = int(plane_frac * c)
    cap = oracle.paper_capacity(h, w)
    ln = int(frac * cap)
    g = inputs.rng(seed)
    cover_np = g.integers(0, 256, h * w * c, dtype=np.uint8)
    data_np = g.integers(0, 256, ln, dtype=np.uint8)
    rc, want = oracle.paper_embed(cover_np, h, w, c, plane, data_np)
    assert rc == OK
    tag = "h=%d w=%d c=%d plane=%d len=%d offs=%s inplace=%d" % (h, w, c, plane, ln, (co, so, do, oo), inplace)
    data = to_dev(data_np, pad_before=do, pad_after=16)
    if inplace:
        stego = to_dev(cover_np, pad_before=co, pad_after=16)
        api.paper_embed(stego, h, w, c, plane, data, out=stego)
    else:
        stego = empty_dev(h * w * c, pad_before=so)
        api.paper_embed(to_dev(cover_np, pad_before=co, pad_after=16), h, w, c, plane, data, out=stego)
    assert_bytes_equal(to_host(stego), want, "paper embed " + tag)
    orc, odata = oracle.paper_extract(want, h, w, c, plane, ln)
    assert orc == OK
    out = to_dev(np.full(ln + 16, FILL, np.uint8), pad_before=oo)
    api.paper_extract(stego, h, w, c, plane, ln, out=out[:ln])
    got = to_host(out)
    assert_bytes_equal(got[:ln], odata, "paper extract " + tag)
    assert_bytes_equal(odata, data_np, "oracle round trip " + tag)
    assert np.all(got[ln:] == FILL), tag + ": bytes past the data written"
