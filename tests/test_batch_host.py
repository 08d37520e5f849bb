"""Host side of the batched binding: the arena extents that Plan checks
before a run (one past the furthest byte any job reads or writes in the
cover, stego and message arenas), worked out by hand for each kind of job."""
import numpy as np
import pytest

from paper_0912_0947_amd import batch
from paper_0912_0947_amd._lib import JOB_RAW, OP_EMBED, OP_EXTRACT, OP_MIXED


def _job(**kw):
    j = batch.make_jobs(1)
    for key, v in kw.items():
        j[key] = v
    return j


def test_header_embed():
    # n = 1000 at k = 1: room 125 bytes, capacity 121
    j = _job(cover_off=0, stego_off=256, msg_off=512, n=1000, k=1, len=50, op=OP_EMBED)
    assert batch._extents(j, OP_MIXED) == (1000, 1256, 562)
    # a message over capacity reads nothing (the job fails with a status)
    j["len"] = 122
    assert batch._extents(j, OP_MIXED) == (1000, 1256, 0)


def test_header_extract_is_bounded_by_capacity_and_msg_cap():
    # n = 4096 at k = 2: room 1024, capacity 1020
    j = _job(cover_off=1 << 40, stego_off=1024, msg_off=256, n=4096, k=2, msg_cap=10**9, op=OP_EXTRACT)
    assert batch._extents(j, OP_MIXED) == (0, 1024 + 4096, 256 + 1020)  # the cover arena is not read
    j["msg_cap"] = 100
    assert batch._extents(j, OP_MIXED) == (0, 1024 + 4096, 256 + 100)


def test_raw_slices():
    # embed: fields [100, 150) at k = 3 carry stream bits [300, 450): bytes up to ceil(450/8) = 57
    e = _job(cover_off=0, stego_off=0, msg_off=768, n=50, k=3, t0=100, stream_bits=10**6, flags=JOB_RAW,
             op=OP_EMBED)
    assert batch._extents(e, OP_MIXED) == (50, 50, 768 + 57)
    # the stream ends inside the slice: bits [300, 310) -> 39 bytes
    e["stream_bits"] = 310
    assert batch._extents(e, OP_MIXED) == (50, 50, 768 + 39)
    # an extract slice that starts past the stream's end writes nothing
    x = _job(stego_off=256, msg_off=512, n=10, k=1, t0=1000, stream_bits=64, flags=JOB_RAW, op=OP_EXTRACT)
    assert batch._extents(x, OP_MIXED) == (0, 266, 0)


def test_plan_kind_overrides_the_op_field_and_maxima_combine():
    jobs = np.concatenate([
        _job(cover_off=0, stego_off=0, msg_off=0, n=1000, k=1, len=50, op=OP_EXTRACT),
        _job(cover_off=4096, stego_off=8192, msg_off=256, n=512, k=8, len=500, op=OP_EXTRACT),
        _job(cover_off=1 << 50, stego_off=1 << 50, msg_off=1 << 50, n=0, k=1, op=OP_EMBED),  # empty: ignored
    ])
    # read as embeds: 4096 + 512, 8192 + 512, 256 + 500 (capacity 508)
    assert batch._extents(jobs, OP_EMBED) == (4608, 8704, 756)
    # read as their own op field (extracts, msg_cap 0): no message bytes at all
    assert batch._extents(jobs, OP_MIXED) == (0, 8704, 0)
    assert batch._extents(batch.make_jobs(0), OP_MIXED) == (0, 0, 0)


def test_offsets_beyond_any_arena_are_refused():
    j = _job(cover_off=1 << 62, n=16, k=1, op=OP_EMBED)
    with pytest.raises(ValueError):
        batch._extents(j, OP_MIXED)
