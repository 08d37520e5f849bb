"""GPU parity of single-plane embedding (general method) and of the
on-device squared error / PSNR against the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import E_BUFFER, E_HEADER, OK

from gpu_helpers import DEV, assert_bytes_equal, empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_plane_golden():
    cover = np.full(40 * 3, 0xFF, np.uint8)
    rc, want = oracle.embed_plane(cover, 3, 1, np.array([0x41], np.uint8), 1)
    got = api.embed_plane(to_dev(cover), 3, 1, to_dev(np.array([0x41], np.uint8)), 1)
    assert_bytes_equal(to_host(got), want, "plane golden")
    out, ls = api.extract_plane(got, 3, 1, 1)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and ls[0] == 1 and to_host(out)[0] == 0x41


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("seed", range(4))
def test_plane_random(k, seed):
    g = inputs.rng(1601, k, seed)
    pixels, c = int(g.integers(20, 200000)), int(g.integers(1, 5))
    plane = int(g.integers(0, c))
    cap = oracle.capacity(pixels, k)
    if cap < 0:
        pytest.skip("too small")
    cover = inputs.random_bytes(pixels * c, 1602, k, seed)
    msg = inputs.random_bytes([cap, int(g.integers(0, cap + 1)), 0, cap // 2][seed], 1603, k, seed)
    rc, want = oracle.embed_plane(cover, c, plane, msg, k)
    assert rc == 0
    co, so = [(0, 0), (1, 0), (0, 3), (5, 5)][seed]
    st = empty_dev(cover.size, pad_before=so)
    api.embed_plane(to_dev(cover, pad_before=co, pad_after=16), c, plane, to_dev(msg), k, out=st)
    assert_bytes_equal(to_host(st), want, "plane embed k=%d c=%d plane=%d" % (k, c, plane))
    out, ls = api.extract_plane(st, c, plane, k)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and ls[0] == msg.size
    assert_bytes_equal(to_host(out)[:msg.size], msg, "plane extract")
    buf = to_dev(cover)
    api.embed_plane(buf, c, plane, to_dev(msg), k, out=buf)
    assert_bytes_equal(to_host(buf), want, "plane embed in place")


@pytest.mark.parametrize("c", [2, 3, 4])
@pytest.mark.parametrize("seed", range(8))
def test_plane_vector_kernels(c, seed):
    """The vector kernels (aligned buffers, 2-4 channels): many wave groups of
    1024 pixels, a ragged tail, every k and plane, messages at each offset
    mod 4, full and partial capacity, in place and out of place."""
    k = 1 + seed
    g = inputs.rng(1611, c, seed)
    plane = seed % c
    pixels = int(g.integers(1024 * 3, 1024 * 60)) + int(g.integers(0, 1024))
    cap = oracle.capacity(pixels, k)
    ln = cap if seed % 2 == 0 else int(g.integers(cap // 3, cap))
    cover = inputs.random_bytes(pixels * c, 1612, c, seed)
    msg = inputs.random_bytes(ln, 1613, c, seed)
    rc, want = oracle.embed_plane(cover, c, plane, msg, k)
    assert rc == 0
    mo = seed % 4
    st = api.embed_plane(to_dev(cover), c, plane, to_dev(msg, pad_before=mo, pad_after=3), k)
    assert_bytes_equal(to_host(st), want, "plane vec embed k=%d c=%d plane=%d pixels=%d" % (k, c, plane, pixels))
    out = empty_dev(ln + 64, pad_before=(mo + 1) % 4)
    _, ls = api.extract_plane(st, c, plane, k, out=out)
    ls = ls.cpu().numpy()
    assert ls[1] == OK and ls[0] == ln
    assert_bytes_equal(to_host(out)[:ln], msg, "plane vec extract")
    buf = to_dev(cover)
    api.embed_plane(buf, c, plane, to_dev(msg), k, out=buf)
    assert_bytes_equal(to_host(buf), want, "plane vec embed in place")


def test_plane_status_codes():
    pixels, c, k = 3000, 3, 2
    cap = oracle.capacity(pixels, k)
    cover = inputs.random_bytes(pixels * c, 1611)
    hdr = np.frombuffer(int(cap + 1).to_bytes(4, "big"), np.uint8)
    plane_np = cover.reshape(pixels, c)[:, 1].copy()
    rc, plane_st = oracle.embed_raw(plane_np, 0, hdr, 32, k)
    bad = cover.reshape(pixels, c).copy()
    bad[:, 1] = plane_st
    out, ls = api.extract_plane(to_dev(bad.reshape(-1)), c, 1, k)
    assert ls.cpu().numpy()[1] == E_HEADER
    rc, st = oracle.embed_plane(cover, c, 1, inputs.random_bytes(50, 1612), k)
    out, ls = api.extract_plane(to_dev(st), c, 1, k, out=torch.empty(49, dtype=torch.uint8, device=DEV))
    ls = ls.cpu().numpy()
    assert ls[1] == E_BUFFER and ls[0] == 50


@pytest.mark.parametrize("n,off", [(0, 0), (1, 0), (15, 3), (1000, 0), (65537, 7), (201326592, 0)])
def test_sse_matches_oracle(n, off):
    a = inputs.random_bytes(n, 1621, n)
    b = a.copy()
    if n:
        idx = inputs.rng(1622, n).integers(0, n, size=max(1, n // 7))
        b[idx] = inputs.random_bytes(idx.size, 1623, n)
    got = int(api.sse(to_dev(a, pad_before=off, pad_after=16), to_dev(b)).cpu().item())
    assert got == oracle.sse(a, b)


def test_psnr_of_a_single_plane_embed():
    """The paper's PSNR situation at 2 bits per byte: data in one plane of an
    RGB cover.  The device squared error equals the oracle's; the PSNR over
    the whole cover exceeds the one over the plane by exactly 10*log10(3)
    (Section VIII's two figures differ by that amount)."""
    h = w = 2048
    cover = inputs.smooth_cover(h, w, 3).reshape(-1)
    pixels = h * w
    msg = inputs.random_bytes(oracle.capacity(pixels, 2), 1631)
    rc, want = oracle.embed_plane(cover, 3, 0, msg, 2)
    st = api.embed_plane(to_dev(cover), 3, 0, to_dev(msg), 2)
    sse_dev = int(api.sse(st, to_dev(cover)).cpu().item())
    assert sse_dev == oracle.sse(want, cover)
    p8, p24 = api.psnr(sse_dev, pixels), api.psnr(sse_dev, 3 * pixels)
    assert abs((p24 - p8) - 10 * math.log10(3)) < 1e-9
    assert abs(p8 - oracle.psnr(sse_dev, pixels)) < 1e-9
    # uniform low bits: mean squared change per field (4^k - 1)/6 = 2.5 at k = 2
    assert abs(sse_dev / pixels - 2.5) < 0.05
