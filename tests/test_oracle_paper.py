"""Pins for the oracle of the paper's own layout (Section VI steps 2-7,
Section VII steps 2-6): hand-worked examples, an independent numpy
formulation of a full row, round trips, invariants and the capacity rule."""
import os

import numpy as np
import pytest

import oracle
from paper_0912_0947_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_layout_examples.txt")


def _cases():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        h, w, c, plane, cover, data, want = [p.strip() for p in line.split("|")]
        out.append((int(h), int(w), int(c), int(plane), bytes.fromhex(cover), bytes.fromhex(data),
                    bytes.fromhex(want)))
    return out


@pytest.mark.parametrize("h,w,c,plane,cover,data,want", _cases())
def test_golden(oracle_lib, h, w, c, plane, cover, data, want):
    rc, st = oracle.paper_embed(np.frombuffer(cover, np.uint8), h, w, c, plane, np.frombuffer(data, np.uint8))
    assert rc == 0 and st.tobytes() == want
    rc, got = oracle.paper_extract(st, h, w, c, plane, len(data))
    assert rc == 0 and got.tobytes() == data


def _numpy_embed(cover, h, w, c, plane, data):
    """Independent formulation: a row of L data bytes becomes the 4 x L array
    of bit pairs (B >> 2i) & 3, laid out row-major (pixel L*i + j)."""
    img = cover.reshape(h, w, c).copy()
    q = w // 4
    off = 0
    for y in range(h):
        L = min(q, data.size - off)
        if L <= 0:
            break
        B = data[off:off + L].astype(np.int64)
        pairs = (B[None, :] >> (2 * np.arange(4))[:, None]) & 3  # [i, j]
        px = img[y, :4 * L, plane].astype(np.int64)
        img[y, :4 * L, plane] = ((px & 0xFC) | pairs.reshape(-1)).astype(np.uint8)
        off += L
    return img.reshape(-1)


@pytest.mark.parametrize("seed", range(12))
def test_numpy_formulation_and_round_trip(oracle_lib, seed):
    g = inputs.rng(1201, seed)
    h, w, c = int(g.integers(1, 40)), int(g.integers(1, 70)), int(g.integers(1, 5))
    plane = int(g.integers(0, c))
    cap = oracle.paper_capacity(h, w)
    assert cap == h * (w // 4)
    ln = [cap, 0, int(g.integers(0, cap + 1))][seed % 3]
    cover = inputs.random_bytes(h * w * c, 1202, seed)
    data = inputs.random_bytes(ln, 1203, seed)
    rc, st = oracle.paper_embed(cover, h, w, c, plane, data)
    assert rc == 0
    np.testing.assert_array_equal(st, _numpy_embed(cover, h, w, c, plane, data))
    rc, got = oracle.paper_extract(st, h, w, c, plane, ln)
    assert rc == 0
    np.testing.assert_array_equal(got, data)
    # invariants: only the chosen plane, only its low two bits
    diff = (st ^ cover).reshape(h, w, c)
    others = np.delete(diff, plane, axis=2)
    assert not others.any()
    assert not (diff[:, :, plane] & 0xFC).any()


def test_capacity_rule(oracle_lib):
    """Section VI step 5: size(B)*4 <= size(A) per row, so h * floor(w/4)."""
    h, w, c = 5, 23, 3
    cap = oracle.paper_capacity(h, w)
    assert cap == 5 * 5
    cover = inputs.random_bytes(h * w * c, 1211)
    assert oracle.paper_embed(cover, h, w, c, 0, inputs.random_bytes(cap, 1212))[0] == 0
    assert oracle.paper_embed(cover, h, w, c, 0, inputs.random_bytes(cap + 1, 1212))[0] == oracle.E_CAPACITY
    assert oracle.paper_embed(cover, h, w, c, 3, inputs.random_bytes(1, 1212))[0] == oracle.E_ARG


def test_paper_session_shape(oracle_lib):
    """Section VIII: a 7x8 payload (56 bytes) into a 1024x1 row: only the
    first 56*4 = 224 pixels may change and the payload comes back."""
    cover = inputs.random_bytes(1024, 1221)
    payload = inputs.random_bytes(56, 1222)
    rc, st = oracle.paper_embed(cover, 1, 1024, 1, 0, payload)
    assert rc == 0
    assert np.nonzero(st != cover)[0].max() < 224
    np.testing.assert_array_equal(st[224:], cover[224:])
    assert oracle.paper_extract(st, 1, 1024, 1, 0, 56)[1].tobytes() == payload.tobytes()


def test_greedy_rows(oracle_lib):
    """Rows fill in order: with w = 8 (2 bytes per row) and 5 data bytes, rows
    0 and 1 carry 2 bytes each, row 2 carries 1 byte in pixels 0..3, rows 3+
    are untouched."""
    h, w = 6, 8
    cover = np.zeros(h * w, np.uint8)
    data = np.full(5, 0xFF, np.uint8)  # every pair = 11
    rc, st = oracle.paper_embed(cover, h, w, 1, 0, data)
    img = st.reshape(h, w)
    assert (img[0] == 3).all() and (img[1] == 3).all()
    assert (img[2, :4] == 3).all() and (img[2, 4:] == 0).all()
    assert not img[3:].any()
