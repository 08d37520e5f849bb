"""GPU parity of the plain embed / extract path against the CPU oracle.

Every comparison is bit-exact (the method is integer bit placement).  Inputs
come from paper_0912_0947_amd.inputs; expected values from the oracle only.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import E_ARG, E_BUFFER, E_CAPACITY, E_HEADER, OK, LsbError

import oracle_pool
from gpu_helpers import DEV, assert_bytes_equal, empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _gpu_roundtrip(cover_np, msg_np, k, inplace=False):
    cover = to_dev(cover_np)
    msg = to_dev(msg_np)
    if inplace:
        stego = cover.clone()
        api.embed(stego, msg, k, out=stego)
    else:
        stego = api.embed(cover, msg, k)
    out, ls = api.extract(stego, k)
    torch.cuda.synchronize()
    ls = ls.cpu().numpy()
    return to_host(stego), to_host(out), int(np.uint32(ls[0])), int(ls[1])


def _check(cover_np, msg_np, k, what):
    rc, want = oracle.embed(cover_np, msg_np, k)
    assert rc == oracle.OK
    for inplace in (False, True):
        stego, out, ln, status = _gpu_roundtrip(cover_np, msg_np, k, inplace)
        tag = "%s k=%d n=%d len=%d inplace=%d" % (what, k, cover_np.size, msg_np.size, inplace)
        assert_bytes_equal(stego, want, "stego " + tag)
        assert status == OK and ln == msg_np.size, tag
        assert_bytes_equal(out[:ln], msg_np, "message " + tag)


def test_config1_image_parity():
    """512x512x3 uniform cover, 32768-byte message, k = 1."""
    cover = inputs.uniform_cover((512, 512, 3), 101)
    msg = inputs.random_bytes(32768, 102)
    _check(cover, msg, 1, "cfg1")


SIZES = [1, 5, 15, 16, 17, 31, 33, 100, 1000, 4099, 65543, (1 << 20) + 13, 3000001]


@pytest.mark.parametrize("k", range(1, 9))
@pytest.mark.parametrize("n", SIZES)
def test_sizes_and_k(k, n):
    cover = inputs.random_bytes(n, 201, k, n)
    cap = oracle.capacity(n, k)
    if cap < 0:
        # no room for the header: embed refuses, extract reports a header error
        with pytest.raises(LsbError) as ei:
            api.embed(to_dev(cover), to_dev(np.zeros(0, np.uint8)), k)
        assert ei.value.code == E_CAPACITY
        out, ls = api.extract(to_dev(cover), k, out=torch.zeros(1, dtype=torch.uint8, device=DEV))
        ls = ls.cpu().numpy()
        assert ls[1] == E_HEADER
        return
    g = inputs.rng(202, k, n)
    for ln in sorted({0, cap, int(g.integers(0, cap + 1))}):
        msg = inputs.random_bytes(ln, 203, k, n, ln)
        _check(cover, msg, k, "sweep")


@pytest.mark.parametrize("k", [1, 3, 4, 8])
@pytest.mark.parametrize("offs", [(1, 0, 0, 0), (0, 3, 0, 0), (5, 5, 1, 2), (0, 0, 2, 0), (0, 0, 0, 1),
                                  (7, 9, 3, 5), (15, 15, 15, 15), (8, 8, 4, 4)])
def test_misaligned_pointers(k, offs):
    """Cover, stego, message and output at byte offsets 0..15 from aligned
    allocations: same bytes as the oracle (per-byte or vector kernels)."""
    co, so, mo, oo = offs
    n = 10007
    cover_np = inputs.random_bytes(n, 301, k)
    cap = oracle.capacity(n, k)
    msg_np = inputs.random_bytes(cap - 3, 302, k)
    rc, want = oracle.embed(cover_np, msg_np, k)
    cover = to_dev(cover_np, pad_before=co, pad_after=16)
    msg = to_dev(msg_np, pad_before=mo, pad_after=16)
    stego = empty_dev(n, pad_before=so)
    api.embed(cover, msg, k, out=stego)
    assert_bytes_equal(to_host(stego), want, "stego offs=%s" % (offs,))
    out = empty_dev(cap, pad_before=oo)
    out, ls = api.extract(stego, k, out=out)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and ls[0] == msg_np.size
    assert_bytes_equal(to_host(out)[:msg_np.size], msg_np, "msg offs=%s" % (offs,))
    # in place on a misaligned buffer
    buf = to_dev(cover_np, pad_before=co, pad_after=16)
    api.embed(buf, msg, k, out=buf)
    assert_bytes_equal(to_host(buf), want, "in-place offs=%s" % (offs,))


@pytest.mark.parametrize("k", [1, 2, 5, 8])
def test_capacity_plus_one_leaves_output(k):
    n = 4096 + 7
    cap = oracle.capacity(n, k)
    cover = to_dev(inputs.random_bytes(n, 401, k))
    stego = torch.full((n,), 0x77, dtype=torch.uint8, device=DEV)
    with pytest.raises(LsbError) as ei:
        api.embed(cover, to_dev(inputs.random_bytes(cap + 1, 402)), k, out=stego)
    assert ei.value.code == E_CAPACITY
    assert bool((stego == 0x77).all())
    api.embed(cover, to_dev(inputs.random_bytes(cap, 402)), k, out=stego)  # exactly full: fine


@pytest.mark.parametrize("k", [1, 2, 3, 7, 8])
def test_extract_status_codes(k):
    n = 2048 + 3
    cap = oracle.capacity(n, k)
    cover_np = inputs.random_bytes(n, 501, k)
    for claim, want_status in [(cap, OK), (cap + 1, E_HEADER), (0xFFFFFFFF, E_HEADER), (0, OK)]:
        hdr = np.frombuffer(int(claim).to_bytes(4, "big"), np.uint8)
        rc, st_np = oracle.embed_raw(cover_np, 0, hdr, 32, k)
        orc, oln, omsg = oracle.extract(st_np, k)
        assert orc == want_status
        out = torch.full((cap,), 0x5C, dtype=torch.uint8, device=DEV)
        out, ls = api.extract(to_dev(st_np), k, out=out)
        ls = ls.cpu().numpy()
        assert int(ls[1]) == want_status and int(np.uint32(ls[0])) == claim
        got = to_host(out)
        if want_status == OK:
            assert_bytes_equal(got[:claim], omsg, "payload")
        else:
            assert (got == 0x5C).all(), "message buffer written despite a header error"
    # output buffer too small: E_BUFFER, decoded length still reported
    msg_np = inputs.random_bytes(100, 502, k)
    rc, st_np = oracle.embed(cover_np, msg_np, k)
    out = torch.full((99,), 0x5C, dtype=torch.uint8, device=DEV)
    out, ls = api.extract(to_dev(st_np), k, out=out)
    ls = ls.cpu().numpy()
    assert ls[1] == E_BUFFER and ls[0] == 100
    assert bool((out == 0x5C).all())
    with pytest.raises(LsbError) as ei:
        api.extract_sync(to_dev(st_np), k, out=torch.empty(99, dtype=torch.uint8, device=DEV))
    assert ei.value.code == E_BUFFER
    got = api.extract_sync(to_dev(st_np), k)
    assert_bytes_equal(to_host(got), msg_np, "extract_sync")


def test_header_does_not_fit():
    for k in range(1, 9):
        n = -(-32 // k) - 1  # one byte short of holding the header
        out, ls = api.extract(to_dev(np.full(max(n, 1), 0xFF, np.uint8))[:n], k,
                              out=torch.zeros(4, dtype=torch.uint8, device=DEV))
        ls = ls.cpu().numpy()
        assert ls[1] == E_HEADER and ls[0] == 0


def test_argument_errors():
    buf = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    msg = torch.zeros(10, dtype=torch.uint8, device=DEV)
    for k in (0, 9, -1):
        with pytest.raises(LsbError) as ei:
            api.embed(buf[:1000], msg, k, out=buf[2000:3000])
        assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # partial overlap of cover and stego
        api.embed(buf[:1000], msg, 2, out=buf[1:1001])
    assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # message inside the stego buffer
        api.embed(buf[:1000], buf[1500:1510], 2, out=buf[1000:2000])
    assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # raw extract with k*t0 not byte aligned
        api.extract_raw(buf[:64], 3, buf[1000:1100], 600, 3)
    assert ei.value.code == E_ARG


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8])
def test_raw_frames_match_whole_clip(k):
    """A small clip: per-frame raw slices (t0 = f * frame bytes) give the same
    stego bytes as one call over the whole clip, and both match the oracle;
    per-frame raw extraction reassembles the stream."""
    frames, h, w = 7, 36, 64
    clip = inputs.video_frames(frames, h, w, device="cpu").numpy().reshape(-1)
    fb = h * w * 3
    stream_bits = (clip.size * k) // 2 + 5  # about half capacity, ragged
    stream_np = inputs.random_bytes((stream_bits + 7) // 8, 601, k)
    rc, want = oracle.embed_raw(clip, 0, stream_np, stream_bits, k)
    clip_d = to_dev(clip)
    stream_d = to_dev(stream_np)
    whole = api.embed_raw(clip_d, 0, stream_d, stream_bits, k)
    per = torch.empty_like(clip_d)
    for f in range(frames):
        api.embed_raw(clip_d[f * fb:(f + 1) * fb], f * fb, stream_d, stream_bits, k,
                      out=per[f * fb:(f + 1) * fb])
    assert_bytes_equal(to_host(whole), want, "whole clip k=%d" % k)
    assert_bytes_equal(to_host(per), want, "per frame k=%d" % k)
    out = torch.zeros_like(stream_d)
    for f in range(frames):
        api.extract_raw(whole[f * fb:(f + 1) * fb], f * fb, out, stream_bits, k)
    rc, want_stream = oracle.extract_raw(want, 0, stream_bits, k)
    assert_bytes_equal(to_host(out), want_stream, "per-frame extract k=%d" % k)
    out2 = torch.zeros_like(stream_d)
    api.extract_raw(whole, 0, out2, stream_bits, k)
    assert_bytes_equal(to_host(out2), want_stream, "whole extract k=%d" % k)


@pytest.mark.parametrize("k", [1, 3, 5, 7])
@pytest.mark.parametrize("t0", [1, 5, 13, 1003])
def test_embed_raw_unaligned_t0(k, t0):
    """Raw embed where k*t0 is not a whole number of bytes (bit-shifted
    stream reads)."""
    n = 5000 + t0
    cover = inputs.random_bytes(n, 701, k, t0)
    stream_bits = k * (t0 + n) - 11
    stream = inputs.random_bytes((stream_bits + 7) // 8, 702, k, t0)
    rc, want = oracle.embed_raw(cover, t0, stream, stream_bits, k)
    got = api.embed_raw(to_dev(cover), t0, to_dev(stream), stream_bits, k)
    assert_bytes_equal(to_host(got), want, "k=%d t0=%d" % (k, t0))


@pytest.fixture(scope="module")
def cfg2_cover():
    return inputs.smooth_cover(8192, 8192, 3).reshape(-1)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_config2_full_size(k, cfg2_cover):
    """8192x8192x3 smooth cover, message at full capacity, k = 1, 2, 4:
    the whole stego image and the whole message are compared."""
    n = cfg2_cover.size
    cap = oracle.capacity(n, k)
    msg_np = inputs.random_bytes(cap, 203, k)
    rc, want = oracle.embed(cfg2_cover, msg_np, k)
    assert rc == 0
    cover = to_dev(cfg2_cover)
    msg = to_dev(msg_np)
    stego = api.embed(cover, msg, k)
    assert_bytes_equal(to_host(stego), want, "cfg2 stego k=%d" % k)
    out, ls = api.extract(stego, k)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and ls[0] == cap
    assert_bytes_equal(to_host(out), msg_np, "cfg2 message k=%d" % k)


def test_config3_video_full_clip():
    """600 frames of 1080x1920x3 (3.73 GB, device resident), k = 1, one
    message at 50 % capacity (|S| = 233,280,000 bytes, ending exactly at the
    end of frame 299).  Every frame of the whole-clip embed is compared with
    the oracle's raw-slice embed of that frame (Section VI step 7), and the
    stream the oracle extracts from those frames (Section VII step 6) with
    the device's whole-clip and per-frame extracts, byte for byte; 600
    per-frame raw calls also equal the whole-clip calls."""
    frames, h, w = 600, 1080, 1920
    fb = h * w * 3
    clip = inputs.video_frames(frames, h, w, device=DEV).view(-1)
    n = clip.numel()
    ln = (n * 1) // 8 // 2 - 4  # |S| = half the clip's capacity in bytes
    assert 4 + ln == 233_280_000
    bits = 8 * (4 + ln)
    msg = torch.empty(ln, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(msg, 303)
    whole = api.embed(clip, msg, 1)
    # the same stream as raw bytes: 4 header bytes (big endian) then the message
    stream = torch.empty(4 + ln, dtype=torch.uint8, device=DEV)
    stream[:4] = torch.tensor(list(ln.to_bytes(4, "big")), dtype=torch.uint8)
    stream[4:] = msg
    per = torch.empty_like(clip)
    for f in range(frames):
        api.embed_raw(clip[f * fb:(f + 1) * fb], f * fb, stream, bits, 1, out=per[f * fb:(f + 1) * fb])
    assert torch.equal(per, whole), "per-frame raw embed differs from the whole-clip embed"
    del per
    out = api.extract_sync(whole, 1)
    assert out.numel() == ln
    back = torch.zeros_like(stream)
    for f in range(frames):
        api.extract_raw(whole[f * fb:(f + 1) * fb], f * fb, back, bits, 1)
    # every frame against the oracle, 40 frames (249 MB) at a time
    stream_np = to_host(stream)
    want_stream = np.zeros(4 + ln, np.uint8)
    group = 40
    stage = oracle_pool.Staging(group * fb, count=2)
    for f0 in range(0, frames, group):
        f1 = min(frames, f0 + group)
        clip_h = stage.fetch(0, clip, f0 * fb, f1 * fb)
        stego_h = stage.fetch(1, whole, f0 * fb, f1 * fb)

        def one(f):
            sl = slice((f - f0) * fb, (f - f0 + 1) * fb)
            rc, want = oracle.embed_raw(clip_h[sl], f * fb, stream_np, bits, 1)
            assert rc == oracle.OK
            got = stego_h[sl]
            if not np.array_equal(got, want):
                bad = np.nonzero(got != want)[0]
                raise AssertionError("frame %d: %d bytes differ from the oracle, first at %d"
                                     % (f, bad.size, int(bad[0])))
            rc, _ = oracle.extract_raw(got, f * fb, bits, 1, stream_out=want_stream)
            assert rc == oracle.OK
            return f

        assert oracle_pool.run(one, range(f0, f1)) == list(range(f0, f1))
    assert_bytes_equal(want_stream, stream_np, "oracle extraction of the clip")
    assert_bytes_equal(to_host(back), want_stream, "per-frame raw extract vs oracle")
    assert_bytes_equal(to_host(out), want_stream[4:], "whole-clip extract vs oracle")


@pytest.mark.parametrize("k", [4, 8])
def test_maximum_message_length(k):
    """The longest message the 32-bit header allows, 2^32 - 1 bytes, in the
    smallest cover that holds it (n = 8 (2^32 + 3) / k, so every byte carries
    the stream and stream offsets pass 2^32).  Closed forms over the whole
    buffer: at k = 8 the stego is the stream BE32(len) || msg itself; at k = 4
    its high nibbles are the cover's and its low nibbles the stream's, most
    significant first.  The last 64 KiB also match the oracle, and extraction
    reports length 2^32 - 1 with the message whole."""
    ln = 0xFFFFFFFF
    n = 8 * (4 + ln) // k
    assert api.capacity(n, k) == ln and api.capacity(n - 1, k) == ln - 1
    cover = torch.empty(n, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(cover, 2101)
    msg = torch.empty(ln, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(msg, 2102)
    stego = api.embed(cover, msg, k)
    ff = torch.full((4,), 0xFF, dtype=torch.uint8, device=DEV)
    if k == 8:
        assert torch.equal(stego[:4], ff) and torch.equal(stego[4:], msg)
    else:
        assert torch.equal(stego & 0xF0, cover & 0xF0)
        assert torch.equal(stego[0:8:2] & 0x0F, ff >> 4) and torch.equal(stego[1:8:2] & 0x0F, ff & 0x0F)
        assert torch.equal(stego[8::2] & 0x0F, msg >> 4)
        assert torch.equal(stego[9::2] & 0x0F, msg & 0x0F)
    m = 1 << 16
    t0 = n - m
    s_first = k * t0 // 8  # stream bytes of the last m fields: all message bytes
    tail = to_host(msg[s_first - 4:])
    # the oracle takes the stream from byte 0: pass the tail as a shorter
    # stream shifted to start at field 0 (t0' = 0, same bits)
    rc, want = oracle.embed_raw(to_host(cover[t0:]), 0, tail, 8 * tail.size, k)
    assert rc == 0
    assert_bytes_equal(to_host(stego[t0:]), want, "k=%d last %d bytes" % (k, m))
    del cover
    out, ls = api.extract(stego, k)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and int(np.uint32(ls[0])) == ln
    assert torch.equal(out[:ln], msg)


@pytest.mark.parametrize("k", [1, 8])
def test_cover_beyond_4gib(k):
    """A cover of 2^32 + 4109 bytes (byte offsets past 32 bits): the stego
    around the 2^32 boundary, at the start and at the end equals the oracle
    run on those slices (raw slices of the same logical stream), and the
    message comes back whole.  At k = 8 the capacity is capped at 2^32 - 1 by
    the header width."""
    n = (1 << 32) + 4109
    cover = torch.empty(n, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(cover, 1901)
    cap = api.capacity(n, k)
    assert cap == min((n * k) // 8 - 4, 0xFFFFFFFF)
    ln = cap if k == 1 else (1 << 31) + 12345
    msg = torch.empty(ln, dtype=torch.uint8, device=DEV)
    inputs.fill_uniform(msg, 1902)
    stego = api.embed(cover, msg, k)
    hdr = np.frombuffer(int(ln).to_bytes(4, "big"), np.uint8)
    bits = 8 * (4 + ln)
    F = -(-bits // k)
    for t0, m in [(0, 1 << 16), ((1 << 32) - 40000, 80000), (F - 50000, 100000), (n - 70000, 70000)]:
        t0 = max(0, min(t0, n - m))
        # the stream bytes this slice needs, as a slice of the logical stream S
        s_first = (k * t0) // 8
        s_last = min((k * (t0 + m) + 7) // 8, 4 + ln)
        s_np = np.zeros(max(s_last, 1), np.uint8)
        if s_last > s_first:
            lo = max(s_first, 4)
            if s_first < 4:
                s_np[s_first:4] = hdr[s_first:4]
            if s_last > lo:
                s_np[lo:s_last] = to_host(msg[lo - 4:s_last - 4])
        rc, want = oracle.embed_raw(to_host(cover[t0:t0 + m]), t0, s_np, min(bits, 8 * s_last), k)
        assert rc == 0
        if 8 * s_last < bits and k * (t0 + m) > 8 * s_last:
            want = want[: (8 * s_last) // k]  # compare only fields fully covered by the copied stream
        assert_bytes_equal(to_host(stego[t0:t0 + want.size]), want, "k=%d slice at %d" % (k, t0))
    out, ls = api.extract(stego, k)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and int(np.uint32(ls[0])) == ln
    assert torch.equal(out[:ln], msg)


@pytest.mark.parametrize("block,unroll,nt", [(256, 1, 0), (512, 2, 1), (1024, 4, 1), (256, 4, 0)])
def test_ballot_packing_parity(block, unroll, nt):
    """k = 1 extraction with wavefront-ballot packing (LDS-staged) gives the
    oracle's message on aligned, ragged and misaligned outputs."""
    from paper_0912_0947_amd import tune
    try:
        api.tune_set(api.OP_EXTRACT, 1, -1, block, unroll, 0, nt, pack=1)
        for n, off in [(786432, 0), (1000003, 0), (65536 * 3 + 17, 4), (100000, 1), (33, 0)]:
            cover = inputs.random_bytes(n, 1951, n)
            cap = oracle.capacity(n, 1)
            for ln in sorted({cap, cap // 3, 0}):
                msg = inputs.random_bytes(ln, 1952, n, ln)
                rc, st = oracle.embed(cover, msg, 1)
                out = empty_dev(max(cap, 1), pad_before=off)
                out, ls = api.extract(to_dev(st), 1, out=out[:cap] if cap else out[:0])
                ls = ls.cpu().numpy()
                assert ls[1] == OK and ls[0] == ln
                assert_bytes_equal(to_host(out)[:ln], msg, "ballot n=%d len=%d off=%d" % (n, ln, off))
    finally:
        tune.load()


@pytest.mark.parametrize("k", [1, 3, 8])
def test_every_launch_shape(k):
    """Every launch shape the tuner can install (block, vectors per lane, grid
    cap, streaming loads/stores, and for the k = 1 extract the packing) gives
    the oracle's stego and message on a ragged size with a partial last
    field, so a re-tuned table cannot change results."""
    from paper_0912_0947_amd import tune
    n = 1000003
    cover = inputs.random_bytes(n, 1961, k)
    cap = oracle.capacity(n, k)
    ln = cap - 5
    msg = inputs.random_bytes(ln, 1962, k)
    rc, want = oracle.embed(cover, msg, k)
    assert rc == 0
    cd, md, st = to_dev(cover), to_dev(msg), to_dev(want)
    out = empty_dev(cap)
    packs = (0, 1) if k == 1 else (0,)
    try:
        for order in tune.ORDERS:
            for block in tune.BLOCKS:
                for unroll in tune.UNROLLS:
                    for capb in tune.CAPS:
                        for nt in (0, 1):
                            shape = (block, unroll, capb, nt, order)
                            api.tune_set(api.OP_EMBED, k, -1, block, unroll, capb, nt, order=order)
                            got = api.embed(cd, md, k)
                            assert torch.equal(got, st), "embed k=%d shape %s" % (k, shape)
                            for pack in packs:
                                api.tune_set(api.OP_EXTRACT, k, -1, block, unroll, capb, nt, pack=pack, order=order)
                                out.fill_(0)
                                o, ls = api.extract(st, k, out=out)
                                assert ls.cpu().tolist() == [ln, OK]
                                assert torch.equal(o[:ln], md), "extract k=%d shape %s pack %d" % (k, shape, pack)
    finally:
        tune.load()
