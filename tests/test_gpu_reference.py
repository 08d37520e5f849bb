"""The reference streams (measurement aid) move the bytes they claim to:
outputs against numpy for every traffic mix (k = 1, 2, 4) and launch shape,
on vector counts that leave ragged grid-stride tails, and argument errors."""
import numpy as np
import pytest

from paper_0912_0947_amd import api, inputs
from paper_0912_0947_amd._lib import E_ARG, REF_COPY, REF_EMBED_MIX, REF_EXTRACT_MIX, LsbError

from gpu_helpers import assert_bytes_equal, empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(256, 1, 0), (512, 2, 0), (1024, 4, 0), (256, 2, 3), (256, 4, 1), (1024, 1, 2)]


def _want(kind, src, side, k):
    v = src.view(np.uint32).reshape(-1, 4).copy()
    if kind == REF_COPY:
        return v.view(np.uint8).reshape(-1)
    if kind == REF_EMBED_MIX:
        if k == 1:
            v[:, 0] ^= side.view(np.uint16).astype(np.uint32)
        elif k == 2:
            v[:, 0] ^= side.view(np.uint32)
        else:
            v[:, :2] ^= side.view(np.uint32).reshape(-1, 2)
        return v.view(np.uint8).reshape(-1)
    x = v[:, 0] ^ v[:, 1] ^ v[:, 2] ^ v[:, 3]
    if k == 1:
        return (x & 0xFFFF).astype(np.uint16).view(np.uint8)
    if k == 2:
        return x.view(np.uint8)
    return np.stack([v[:, 0] ^ v[:, 1], v[:, 2] ^ v[:, 3]], axis=1).reshape(-1).view(np.uint8)


@pytest.mark.parametrize("kind,k", [(REF_COPY, 1), (REF_EMBED_MIX, 1), (REF_EMBED_MIX, 2), (REF_EMBED_MIX, 4),
                                    (REF_EXTRACT_MIX, 1), (REF_EXTRACT_MIX, 2), (REF_EXTRACT_MIX, 4)])
@pytest.mark.parametrize("nv", [1, 63, 4097, 70001])
@pytest.mark.parametrize("shape", SHAPES)
def test_outputs(kind, k, nv, shape):
    block, unroll, grid = shape
    n = 16 * nv
    src = inputs.random_bytes(n, 1901, nv)
    side = inputs.random_bytes(n * k // 8, 1902, nv)
    dst = empty_dev(n * k // 8 if kind == REF_EXTRACT_MIX else n)
    api.stream_reference(kind, to_dev(src), dst, to_dev(side) if kind == REF_EMBED_MIX else None,
                         block=block, unroll=unroll, grid=grid, k=k)
    assert_bytes_equal(to_host(dst), _want(kind, src, side, k),
                       "kind %d k %d nv %d shape %s" % (kind, k, nv, shape))


def test_argument_errors():
    src = to_dev(np.zeros(4096, np.uint8))
    dst = empty_dev(4096)
    for kw, bad in [({"block": 128}, None), ({"unroll": 3}, None), ({"k": 3}, None), ({}, "kind")]:
        with pytest.raises(LsbError) as ei:
            api.stream_reference(7 if bad == "kind" else REF_COPY, src, dst, **kw)
        assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # misaligned source
        api.stream_reference(REF_COPY, to_dev(np.zeros(4096, np.uint8), pad_before=4), dst)
    assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # n not a multiple of 16
        api.stream_reference(REF_COPY, to_dev(np.zeros(4100, np.uint8)), empty_dev(4100))
    assert ei.value.code == E_ARG
    with pytest.raises(LsbError) as ei:  # output overlaps the input
        api.stream_reference(REF_COPY, src, src)
    assert ei.value.code == E_ARG
