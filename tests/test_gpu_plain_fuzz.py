"""Randomised plain calls (hypothesis, derandomised): raw slices at any t0
and stream length, header embed/extract of any length up to capacity, every
k, and buffers at byte offsets 0..15 from aligned allocations (so both the
vector and the per-byte kernels, and the dword and byte stream paths, run).
Outputs are compared with the oracle byte for byte, and the bytes around
each output must stay untouched."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import OK

from gpu_helpers import assert_bytes_equal, empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

FILL = 0xA5  # gpu_helpers pads with this byte
SETTINGS = settings(max_examples=80, deadline=None, derandomize=True, database=None,
                    suppress_health_check=list(HealthCheck))

sizes = st.one_of(st.integers(1, 40), st.integers(41, 3000), st.integers(3001, 400_000))
offsets = st.integers(0, 15)


@SETTINGS
@given(k=st.integers(1, 8), n=sizes, t0=st.integers(0, 1 << 20), frac=st.floats(0, 1.3),
       co=offsets, so=offsets, mo=offsets, seed=st.integers(0, 2**31 - 1))
def test_raw_embed(k, n, t0, frac, co, so, mo, seed):
    """Any t0 (field k*t0 need not start a byte); the stream ends before,
    inside or after the slice."""
    bits = int(frac * k * (t0 + n))
    g = inputs.rng(seed)
    cover_np = g.integers(0, 256, n, dtype=np.uint8)
    stream_np = g.integers(0, 256, max((bits + 7) // 8, 1), dtype=np.uint8)
    rc, want = oracle.embed_raw(cover_np, t0, stream_np, bits, k)
    assert rc == OK
    cover = to_dev(cover_np, pad_before=co, pad_after=16)
    stream = to_dev(stream_np, pad_before=mo, pad_after=16)
    stego = empty_dev(n, pad_before=so)
    api.embed_raw(cover, t0, stream, bits, k, out=stego)
    assert_bytes_equal(to_host(stego), want, "raw embed k=%d n=%d t0=%d bits=%d offs=%s" % (
        k, n, t0, bits, (co, so, mo)))


@SETTINGS
@given(k=st.integers(1, 8), n=sizes, t0q=st.integers(0, 1 << 17), frac=st.floats(0, 1.3),
       so=offsets, oo=offsets, seed=st.integers(0, 2**31 - 1))
def test_raw_extract(k, n, t0q, frac, so, oo, seed):
    """t0 with k*t0 on a byte; the slice ends on a byte or at the stream's
    end.  Only the slice's stream bytes are written."""
    t0 = 8 * t0q  # k*t0 is a whole number of bytes for every k
    total = k * (t0 + n)
    bits = int(frac * total)
    end = min(total, bits)
    if end > k * t0 and end % 8 and end != bits:
        bits = total
        end = total
    g = inputs.rng(seed)
    stego_np = g.integers(0, 256, n, dtype=np.uint8)
    nb = (bits + 7) // 8
    rc, want = oracle.extract_raw(stego_np, t0, bits, k)
    assert rc == OK
    stego = to_dev(stego_np, pad_before=so, pad_after=16)
    out = to_dev(np.full(max(nb, 1), FILL, np.uint8), pad_before=oo, pad_after=16)
    api.extract_raw(stego, t0, out, bits, k)
    got = to_host(out)
    lo, hi = (k * t0 // 8, (end + 7) // 8) if end > k * t0 else (0, 0)
    tag = "raw extract k=%d n=%d t0=%d bits=%d offs=%s" % (k, n, t0, bits, (so, oo))
    assert_bytes_equal(got[lo:hi], want[lo:hi], tag)
    assert np.all(got[:lo] == FILL) and np.all(got[hi:] == FILL), tag + ": bytes outside the slice written"


@SETTINGS
@given(k=st.integers(1, 8), n=sizes, frac=st.floats(0, 1), co=offsets, so=offsets, mo=offsets, oo=offsets,
       inplace=st.booleans(), seed=st.integers(0, 2**31 - 1))
def test_header_round_trip(k, n, frac, co, so, mo, oo, inplace, seed):
    cap = oracle.capacity(n, k)
    if cap < 0:
        return
    ln = int(frac * cap)
    g = inputs.rng(seed)
    cover_np = g.integers(0, 256, n, dtype=np.uint8)
    msg_np = g.integers(0, 256, ln, dtype=np.uint8)
    rc, want = oracle.embed(cover_np, msg_np, k)
    assert rc == OK
    msg = to_dev(msg_np, pad_before=mo, pad_after=16)
    if inplace:
        stego = to_dev(cover_np, pad_before=co, pad_after=16)
        api.embed(stego, msg, k, out=stego)
    else:
        stego = empty_dev(n, pad_before=so)
        api.embed(to_dev(cover_np, pad_before=co, pad_after=16), msg, k, out=stego)
    tag = "k=%d n=%d len=%d offs=%s inplace=%d" % (k, n, ln, (co, so, mo, oo), inplace)
    assert_bytes_equal(to_host(stego), want, "embed " + tag)
    out = to_dev(np.full(max(ln, 1) + 8, FILL, np.uint8), pad_before=oo)
    out, ls = api.extract(stego, k, out=out)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and int(np.uint32(ls[0])) == ln, tag
    got = to_host(out)
    assert_bytes_equal(got[:ln], msg_np, "extract " + tag)
    assert np.all(got[ln:] == FILL), tag + ": bytes past the message written"
