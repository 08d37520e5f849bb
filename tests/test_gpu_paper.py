"""GPU parity of the paper's own layout (2 bits per byte, one plane, greedy
rows, bit pair i of data byte j in pixel L*i + j) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import E_ARG, E_CAPACITY, LsbError

from gpu_helpers import DEV, assert_bytes_equal, empty_dev, to_dev, to_host
from test_oracle_paper import _cases

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h,w,c,plane,cover,data,want", _cases())
def test_golden(h, w, c, plane, cover, data, want):
    st = api.paper_embed(to_dev(np.frombuffer(cover, np.uint8)), h, w, c, plane, to_dev(np.frombuffer(data, np.uint8)))
    assert to_host(st).tobytes() == want
    assert to_host(api.paper_extract(st, h, w, c, plane, len(data))).tobytes() == data


@pytest.mark.parametrize("seed", range(24))
def test_random_shapes(seed):
    g = inputs.rng(1301, seed)
    h, w, c = int(g.integers(1, 200)), int(g.integers(1, 700)), int(g.integers(1, 5))
    plane = int(g.integers(0, c))
    cap = oracle.paper_capacity(h, w)
    ln = [cap, 0, int(g.integers(0, cap + 1))][seed % 3]
    cover = inputs.random_bytes(h * w * c, 1302, seed)
    data = inputs.random_bytes(ln, 1303, seed)
    rc, want = oracle.paper_embed(cover, h, w, c, plane, data)
    assert rc == 0
    co, so = [(0, 0), (3, 0), (0, 5), (7, 7)][seed % 4]
    st = empty_dev(cover.size, pad_before=so)
    api.paper_embed(to_dev(cover, pad_before=co, pad_after=16), h, w, c, plane, to_dev(data), out=st)
    assert_bytes_equal(to_host(st), want, "paper embed h=%d w=%d c=%d plane=%d len=%d" % (h, w, c, plane, ln))
    got = api.paper_extract(st, h, w, c, plane, ln)
    assert_bytes_equal(to_host(got), data, "paper extract")
    buf = to_dev(cover)
    api.paper_embed(buf, h, w, c, plane, to_dev(data), out=buf)  # in place
    assert_bytes_equal(to_host(buf), want, "paper embed in place")


@pytest.mark.parametrize("seed", range(20))
def test_row_kernel_shapes(seed):
    """Rows of a multiple of 16 bytes with 16-byte aligned image pointers take
    the row-per-block kernel: every channel count 1..5, a data pointer at each
    offset mod 4, a partial last data row, no data, and in-place."""
    g = inputs.rng(1331, seed)
    c = 1 + seed % 5
    w = 16 * int(g.integers(1, 80))
    h = int(g.integers(1, 120))
    plane = int(g.integers(0, c))
    cap = oracle.paper_capacity(h, w)
    ln = [cap, int(g.integers(1, cap + 1)), 0, int(g.integers(0, w // 4 + 1))][seed % 4]
    cover = inputs.random_bytes(h * w * c, 1332, seed)
    data = inputs.random_bytes(ln, 1333, seed)
    rc, want = oracle.paper_embed(cover, h, w, c, plane, data)
    assert rc == 0
    dm = seed % 4
    st = api.paper_embed(to_dev(cover), h, w, c, plane, to_dev(data, pad_before=dm, pad_after=3))
    assert_bytes_equal(to_host(st), want, "row kernel h=%d w=%d c=%d plane=%d len=%d dm=%d" % (h, w, c, plane, ln, dm))
    buf = to_dev(cover)
    api.paper_embed(buf, h, w, c, plane, to_dev(data, pad_before=3 - dm), out=buf)  # in place
    assert_bytes_equal(to_host(buf), want, "row kernel in place")
    assert_bytes_equal(to_host(api.paper_extract(st, h, w, c, plane, ln)), data, "row kernel extract")


def test_wide_rows_fall_back():
    """A row whose data chunk exceeds the row kernels' LDS limit takes the
    per-vector embed and per-byte extract (w = 262,144 pixels: 65,536 data
    bytes per row)."""
    h, w, c = 3, 262144, 1
    cap = oracle.paper_capacity(h, w)
    ln = cap - 1000
    cover = inputs.random_bytes(h * w * c, 1341)
    data = inputs.random_bytes(ln, 1342)
    rc, want = oracle.paper_embed(cover, h, w, c, 0, data)
    st = api.paper_embed(to_dev(cover), h, w, c, 0, to_dev(data))
    assert_bytes_equal(to_host(st), want, "wide rows")
    assert_bytes_equal(to_host(api.paper_extract(st, h, w, c, 0, ln)), data, "wide rows extract")


def test_session_shape():
    """Section VIII: 56 bytes into a 1024x1 row."""
    cover = inputs.random_bytes(1024, 1311)
    payload = inputs.random_bytes(56, 1312)
    rc, want = oracle.paper_embed(cover, 1, 1024, 1, 0, payload)
    st = api.paper_embed(to_dev(cover), 1, 1024, 1, 0, to_dev(payload))
    assert_bytes_equal(to_host(st), want, "session shape")
    assert to_host(api.paper_extract(st, 1, 1024, 1, 0, 56)).tobytes() == payload.tobytes()


@pytest.mark.parametrize("plane", [0, 2])
def test_large_image_full_capacity(plane):
    """8192x8192x3 smooth cover, one plane filled to capacity (16,777,216 bytes)."""
    h = w = 8192
    cover = inputs.smooth_cover(h, w, 3).reshape(-1)
    cap = oracle.paper_capacity(h, w)
    data = inputs.random_bytes(cap, 1321, plane)
    rc, want = oracle.paper_embed(cover, h, w, 3, plane, data)
    st = api.paper_embed(to_dev(cover), h, w, 3, plane, to_dev(data))
    assert_bytes_equal(to_host(st), want, "8192^2 plane %d" % plane)
    assert_bytes_equal(to_host(api.paper_extract(st, h, w, 3, plane, cap)), data, "8192^2 extract")


def test_errors():
    buf = torch.zeros(8 * 8 * 3, dtype=torch.uint8, device=DEV)
    with pytest.raises(LsbError) as ei:
        api.paper_embed(buf, 8, 8, 3, 3, torch.zeros(1, dtype=torch.uint8, device=DEV))
    assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:
        api.paper_embed(buf, 8, 8, 3, 0, torch.zeros(17, dtype=torch.uint8, device=DEV))
    assert ei.value.code == E_CAPACITY
    with pytest.raises(LsbError) as ei:
        api.paper_extract(buf, 8, 8, 3, 0, 17)
    assert ei.value.code == E_CAPACITY
