"""Pins for single-plane embedding with the general method and for the
squared-error / PSNR functions (Section VIII)."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_0912_0947_amd import inputs

HERE = os.path.dirname(__file__)


def test_sse_matches_numpy(oracle_lib):
    for seed in range(5):
        n = int(inputs.rng(1501, seed).integers(0, 5000))
        a = inputs.random_bytes(n, 1502, seed)
        b = inputs.random_bytes(n, 1503, seed)
        want = int(np.sum((a.astype(np.int64) - b.astype(np.int64)) ** 2))
        assert oracle.sse(a, b) == want


def test_psnr_closed_forms(oracle_lib):
    # MSE = 1 for 8-bit data is the textbook 20*log10(255) = 48.1308 dB
    assert abs(oracle.psnr(1000, 1000) - 20 * math.log10(255)) < 1e-9
    assert abs(oracle.psnr(4, 1) - 10 * math.log10(255 ** 2 / 4)) < 1e-9
    assert math.isinf(oracle.psnr(0, 10))


def test_paper_psnr_gap(oracle_lib):
    """Reading: MSE is taken over every byte of the cover.  Then the same
    squared error over a 3-plane cover gives a PSNR exactly 10*log10(3)
    higher than over one plane -- the gap between the paper's two values."""
    vals = {}
    for line in open(os.path.join(HERE, "golden", "paper_psnr.txt")):
        if line.strip() and not line.startswith("#"):
            bpp, db = [p.strip() for p in line.split("|")]
            vals[int(bpp)] = float(db)
    gap = 10 * math.log10(3)
    assert abs((vals[24] - vals[8]) - gap) < 1e-3
    for sse in (1, 453, 10 ** 6):
        assert abs((oracle.psnr(sse, 3 * 1024) - oracle.psnr(sse, 1024)) - gap) < 1e-9


def test_plane_golden(oracle_lib):
    """msg 0x41 at k = 1 into plane 1 of a 40-pixel RGB cover of FF: plane 1
    takes the bytes of the hand-worked k = 1 example (set stream bits 31, 33,
    39), planes 0 and 2 stay FF."""
    cover = np.full(40 * 3, 0xFF, np.uint8)
    rc, st = oracle.embed_plane(cover, 3, 1, np.array([0x41], np.uint8), 1)
    assert rc == 0
    img = st.reshape(40, 3)
    want = np.full(40, 0xFE, np.uint8)
    want[[31, 33, 39]] = 0xFF
    np.testing.assert_array_equal(img[:, 1], want)
    assert (img[:, 0] == 0xFF).all() and (img[:, 2] == 0xFF).all()
    rc, ln, got = oracle.extract_plane(st, 3, 1, 1)
    assert rc == 0 and got.tobytes() == b"\x41"


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_plane_round_trip_and_invariants(oracle_lib, k):
    for seed in range(3):
        g = inputs.rng(1511, k, seed)
        pixels, c = int(g.integers(10, 3000)), int(g.integers(1, 5))
        plane = int(g.integers(0, c))
        cap = oracle.capacity(pixels, k)
        if cap < 0:
            continue
        cover = inputs.random_bytes(pixels * c, 1512, k, seed)
        msg = inputs.random_bytes(int(g.integers(0, cap + 1)), 1513, k, seed)
        rc, st = oracle.embed_plane(cover, c, plane, msg, k)
        assert rc == 0
        d = (st ^ cover).reshape(pixels, c)
        assert not np.delete(d, plane, axis=1).any()
        assert not (d[:, plane] & (0xFF ^ ((1 << k) - 1))).any()
        rc, ln, got = oracle.extract_plane(st, c, plane, k)
        assert rc == 0 and got.tobytes() == msg.tobytes()
        # the plane on its own is the plain method on that plane
        rc, want = oracle.embed(cover.reshape(pixels, c)[:, plane].copy(), msg, k)
        np.testing.assert_array_equal(st.reshape(pixels, c)[:, plane], want)


def test_plane_capacity(oracle_lib):
    pixels, c, k = 1000, 3, 2
    cap = oracle.capacity(pixels, k)
    cover = inputs.random_bytes(pixels * c, 1521)
    assert oracle.embed_plane(cover, c, 0, inputs.random_bytes(cap + 1, 1522), k)[0] == oracle.E_CAPACITY
    assert oracle.embed_plane(cover, c, 3, inputs.random_bytes(1, 1522), k)[0] == oracle.E_ARG
