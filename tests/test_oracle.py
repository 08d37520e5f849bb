"""Pins for the CPU oracle, checked against facts other than the oracle itself.

Each test names the paper passage or mathematical fact it relies on:
  * hand-worked examples (tests/golden/hand_examples.txt);
  * special cases that reduce to numpy's packbits / unpackbits (k = 1, 2, 4, 8);
  * brute force of the per-byte field operation over all 256 cover bytes;
  * invariants: round trip, only the low k bits change, |stego - cover| is at
    most 2^k - 1, bytes past the stream unchanged;
  * the capacity closed form n*k bits (Section VI step 5 at k = 2);
  * the expected squared change (4^k - 1)/6 for uniform cover and stream.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import ref
from paper_0912_0947_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")


def _golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, cover, msg, want = [p.strip().replace(" ", "") for p in line.split("|")]
            cases.append((int(k), bytes.fromhex(cover), bytes.fromhex(msg), bytes.fromhex(want)))
    return cases


# ---------------------------------------------------------------- golden ----
@pytest.mark.parametrize("k,cover,msg,want", _golden_cases())
def test_golden_hand_examples(oracle_lib, k, cover, msg, want):
    rc, stego = oracle.embed(np.frombuffer(cover, np.uint8), np.frombuffer(msg, np.uint8), k)
    assert rc == oracle.OK
    assert stego.tobytes() == want
    assert ref.embed(cover, msg, k) == want
    rc, ln, got = oracle.extract(stego, k)
    assert rc == oracle.OK and ln == len(msg) and got.tobytes() == msg


# --------------------------------------------------- numpy library pins ----
def _stream(msg: np.ndarray) -> np.ndarray:
    return np.concatenate([np.frombuffer(len(msg).to_bytes(4, "big"), np.uint8), msg])


@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_numpy_reduction(oracle_lib, k, seed):
    """For k | 8 the embed is unpackbits -> group k bits -> write into the low
    bits; the extract is the inverse through packbits (bitorder big)."""
    n = 4096 + 13 * seed
    cover = inputs.random_bytes(n, 11, seed)
    cap = oracle.capacity(n, k)
    ln = [cap, cap // 3, 0][seed]
    msg = inputs.random_bytes(ln, 12, seed)
    s = _stream(msg)
    bits = np.unpackbits(s, bitorder="big")
    fields = bits.reshape(-1, k) @ (1 << np.arange(k - 1, -1, -1))
    want = cover.copy()
    F = fields.size
    low = (1 << k) - 1
    want[:F] = (cover[:F] & (0xFF ^ low)) | fields.astype(np.uint8)
    rc, stego = oracle.embed(cover, msg, k)
    assert rc == 0
    np.testing.assert_array_equal(stego, want)
    # extract via numpy: fields -> bits -> packbits
    got_fields = (stego[:F] & low).astype(np.int64)
    got_bits = ((got_fields[:, None] >> np.arange(k - 1, -1, -1)) & 1).reshape(-1)
    np.testing.assert_array_equal(np.packbits(got_bits.astype(np.uint8), bitorder="big"), s)
    rc, ln2, out = oracle.extract(stego, k)
    assert rc == 0 and ln2 == ln
    np.testing.assert_array_equal(out, msg)


# ------------------------------------------------------------ brute force ----
@pytest.mark.parametrize("k", range(1, 9))
def test_field_brute_force(oracle_lib, k):
    """Every cover byte c and field value v: a single full field becomes
    (c with its low k bits cleared) | v, and reads back as v."""
    for v in range(1 << k):
        stream = np.array([(v << (8 - k)) & 0xFF], np.uint8)  # v's k bits, MSB first
        cover = np.arange(256, dtype=np.uint8)
        for c in range(256):
            rc, st = oracle.embed_raw(cover[c:c + 1], 0, stream, k, k)
            assert rc == 0
            assert int(st[0]) == (c & ~((1 << k) - 1) & 0xFF) | v
            rc, out = oracle.extract_raw(st, 0, k, k)
            assert rc == 0 and (int(out[0]) >> (8 - k)) == v


@pytest.mark.parametrize("k", range(1, 9))
def test_every_one_byte_message(oracle_lib, k):
    n = -(-40 // k) + 3
    cover = inputs.random_bytes(n, 21, k)
    for m in range(256):
        msg = np.array([m], np.uint8)
        rc, stego = oracle.embed(cover, msg, k)
        assert rc == 0
        assert stego.tobytes() == ref.embed(cover.tobytes(), bytes([m]), k)
        rc, ln, got = oracle.extract(stego, k)
        assert rc == 0 and ln == 1 and int(got[0]) == m


# -------------------------------------------------------------- invariants ----
@pytest.mark.parametrize("k", range(1, 9))
@pytest.mark.parametrize("seed", range(4))
def test_invariants(oracle_lib, k, seed):
    n = int(inputs.rng(31, k, seed).integers(5, 3000))
    cover = inputs.random_bytes(n, 32, k, seed)
    cap = oracle.capacity(n, k)
    if cap < 0:
        pytest.skip("cover too small for a header")
    ln = int(inputs.rng(33, k, seed).integers(0, cap + 1))
    msg = inputs.random_bytes(ln, 34, k, seed)
    rc, stego = oracle.embed(cover, msg, k)
    assert rc == 0
    low = (1 << k) - 1
    assert np.all(((stego ^ cover) & (0xFF ^ low)) == 0), "only the low k bits may change"
    assert np.all(np.abs(stego.astype(int) - cover.astype(int)) <= low)
    F = -(-(8 * (4 + ln)) // k)
    np.testing.assert_array_equal(stego[F:], cover[F:])
    rc, ln2, got = oracle.extract(stego, k)
    assert rc == 0 and ln2 == ln
    np.testing.assert_array_equal(got, msg)
    # in-place form gives the same bytes
    buf = cover.copy()
    rc, same = oracle.embed(buf, msg, k, out=buf)
    assert rc == 0
    np.testing.assert_array_equal(buf, stego)


@pytest.mark.parametrize("k", [3, 5, 6, 7])
def test_partial_last_field_keeps_cover_bits(oracle_lib, k):
    """When k does not divide the stream length, the last field carries
    nb < k bits in its top bits and keeps the cover's remaining low bits."""
    for ln in range(0, 12):
        Lb = 8 * (4 + ln)
        if Lb % k == 0:
            continue
        F = -(-Lb // k)
        cover = inputs.random_bytes(F + 2, 41, k, ln)
        msg = inputs.random_bytes(ln, 42, k, ln)
        rc, stego = oracle.embed(cover, msg, k)
        assert rc == 0
        nb = Lb - k * (F - 1)
        keep = (1 << (k - nb)) - 1
        assert (int(stego[F - 1]) & keep) == (int(cover[F - 1]) & keep)
        assert (int(stego[F - 1]) >> k) == (int(cover[F - 1]) >> k)
        assert stego.tobytes() == ref.embed(cover.tobytes(), msg.tobytes(), k)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_mean_squared_change(oracle_lib, k):
    """Uniform cover and uniform stream: E[(stego - cover)^2] over fully used
    fields is 2*Var(U{0..2^k-1}) = (4^k - 1)/6 (0.5, 2.5, 42.5)."""
    n = 1 << 20
    cover = inputs.random_bytes(n, 51, k)
    msg = inputs.random_bytes(oracle.capacity(n, k), 52, k)
    rc, stego = oracle.embed(cover, msg, k)
    assert rc == 0
    d = stego.astype(np.float64) - cover.astype(np.float64)
    want = (4 ** k - 1) / 6
    assert abs(np.mean(d * d) - want) < 0.01 * want


# -------------------------------------------------------------- capacity ----
@pytest.mark.parametrize("k", range(1, 9))
def test_capacity_closed_form(oracle_lib, k):
    for n in [0, 1, 3, 4, 5, 31, 32, 33, 100, 1024, 786432, 201326592]:
        room = (n * k) // 8
        want = room - 4 if room >= 4 else oracle.E_CAPACITY
        assert oracle.capacity(n, k) == want
    assert oracle.capacity(10, 0) == oracle.E_ARG
    assert oracle.capacity(10, 9) == oracle.E_ARG
    assert oracle.capacity(1 << 40, 8) == 0xFFFFFFFF  # header width caps it


def test_capacity_paper_rule(oracle_lib):
    """Section VI step 5: at 2 bits per byte, size(B)*4 <= size(A); with the
    4-byte header the message capacity is size(A)/4 - 4."""
    for n in [1024, 4096, 786432]:
        assert oracle.capacity(n, 2) == n // 4 - 4


@pytest.mark.parametrize("k", range(1, 9))
def test_full_capacity_and_one_more(oracle_lib, k):
    n = 777
    cap = oracle.capacity(n, k)
    cover = inputs.random_bytes(n, 61, k)
    msg = inputs.random_bytes(cap + 1, 62, k)
    rc, stego = oracle.embed(cover, msg[:cap], k)
    assert rc == 0
    rc, ln, got = oracle.extract(stego, k)
    assert rc == 0 and ln == cap
    np.testing.assert_array_equal(got, msg[:cap])
    rc, stego2 = oracle.embed(cover, msg, k)
    assert rc == oracle.E_CAPACITY
    np.testing.assert_array_equal(stego2, cover)


def test_extract_errors(oracle_lib):
    # header that claims more than fits -> E_HEADER (len still reported)
    k = 1
    cover = np.zeros(64, np.uint8)
    stego = cover.copy()
    stego[:32] |= 1  # len = 0xFFFFFFFF
    rc, ln, got = oracle.extract(stego, k)
    assert rc == oracle.E_HEADER and ln == 0xFFFFFFFF and got is None
    # too small for the header at all
    rc, ln, _ = oracle.extract(np.zeros(31, np.uint8), 1)
    assert rc == oracle.E_HEADER and ln == 0
    # output buffer too small -> E_BUFFER with len reported
    msg = inputs.random_bytes(10, 71)
    rc, stego = oracle.embed(inputs.random_bytes(200, 72), msg, 2)
    rc, ln, got = oracle.extract(stego, 2, out_cap=9)
    assert rc == oracle.E_BUFFER and ln == 10 and got is None
    rc, ln, got = oracle.extract(stego, 2, out_cap=10)
    assert rc == 0 and ln == 10


def test_bad_k(oracle_lib):
    cover = np.zeros(64, np.uint8)
    assert oracle.embed(cover, np.zeros(1, np.uint8), 0)[0] == oracle.E_ARG
    assert oracle.embed(cover, np.zeros(1, np.uint8), 9)[0] == oracle.E_ARG
    assert oracle.extract(cover, 0)[0] == oracle.E_ARG


# ------------------------------------------------------------- raw slices ----
@pytest.mark.parametrize("k", range(1, 9))
def test_raw_slices_compose(oracle_lib, k):
    """Embedding slice by slice at offsets t0 equals embedding the whole
    cover; extracting byte-aligned slices reassembles the stream."""
    n = 1000
    cover = inputs.random_bytes(n, 81, k)
    stream_bits = n * k - 5 if k > 1 else n * k - 3
    stream = inputs.random_bytes((stream_bits + 7) // 8, 82, k)
    rc, whole = oracle.embed_raw(cover, 0, stream, stream_bits, k)
    assert rc == 0
    cuts = [0, 8, 136, 400, 808, n]  # multiples of 8: k*t0 % 8 == 0 for any k
    parts = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        rc, st = oracle.embed_raw(cover[a:b], a, stream, stream_bits, k)
        assert rc == 0
        parts.append(st)
    np.testing.assert_array_equal(np.concatenate(parts), whole)
    out = np.zeros_like(stream)
    for a, b in zip(cuts[:-1], cuts[1:]):
        rc, _ = oracle.extract_raw(whole[a:b], a, stream_bits, k, stream_out=out)
        assert rc == 0
    want = stream.copy()
    if stream_bits % 8:
        want[-1] &= (0xFF << (8 - stream_bits % 8)) & 0xFF  # pad bits read as zero
    np.testing.assert_array_equal(out, want)
    # unaligned embed slices are allowed
    rc, st = oracle.embed_raw(cover[3:17], 3, stream, stream_bits, k)
    assert rc == 0 and st.tobytes() == whole[3:17].tobytes()


def test_raw_extract_alignment_rules(oracle_lib):
    stego = np.zeros(64, np.uint8)
    # k*t0 not byte aligned
    assert oracle.extract_raw(stego[:8], 3, 64 * 3, 3)[0] == oracle.E_ARG
    # slice end inside a byte that the next slice also needs
    assert oracle.extract_raw(stego[:5], 0, 64 * 3, 3)[0] == oracle.E_ARG
    # ... unless the stream ends there
    assert oracle.extract_raw(stego[:5], 0, 15, 3)[0] == oracle.OK


# ------------------------------------------------------------- C vs Python ----
@pytest.mark.parametrize("k", range(1, 9))
def test_c_matches_pure_python(oracle_lib, k):
    for seed in range(5):
        g = inputs.rng(91, k, seed)
        n = int(g.integers(40, 400))
        cap = oracle.capacity(n, k)
        if cap < 0:
            continue
        ln = int(g.integers(0, cap + 1))
        cover = inputs.random_bytes(n, 92, k, seed)
        msg = inputs.random_bytes(ln, 93, k, seed)
        rc, stego = oracle.embed(cover, msg, k)
        assert rc == 0
        assert stego.tobytes() == ref.embed(cover.tobytes(), msg.tobytes(), k)
        assert ref.extract(stego.tobytes(), k) == msg.tobytes()


def test_paper_worked_shape(oracle_lib):
    """Section VIII: a 7x8 payload (56 bytes) into a 1024-byte row at 2 bits
    per byte.  224 cover bytes hold the payload (56*4 <= 1024); the header adds
    16 more, so exactly the first 240 bytes may change."""
    cover = inputs.random_bytes(1024, 101)
    payload = inputs.random_bytes(56, 102)
    rc, stego = oracle.embed(cover, payload, 2)
    assert rc == 0
    changed = np.nonzero(stego != cover)[0]
    assert changed.max() < 240
    np.testing.assert_array_equal(stego[240:], cover[240:])
    assert oracle.extract(stego, 2)[2].tobytes() == payload.tobytes()


@pytest.mark.parametrize("k", range(1, 9))
def test_header_boundary(oracle_lib, k):
    """A decoded length of exactly the capacity is accepted; one more is a
    header error (8*(4+len) > n*k), with the decoded length still reported."""
    n = 301
    cap = oracle.capacity(n, k)
    cover = inputs.random_bytes(n, 111, k)
    for claim, want in [(cap, oracle.OK), (cap + 1, oracle.E_HEADER)]:
        hdr = np.frombuffer(int(claim).to_bytes(4, "big"), np.uint8)
        rc, stego = oracle.embed_raw(cover, 0, hdr, 32, k)
        assert rc == 0
        rc, ln, _ = oracle.extract(stego, k)
        assert rc == want and ln == claim
