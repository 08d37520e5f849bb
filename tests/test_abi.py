"""The C ABI library builds, loads without a GPU and exports every function
that include/lsb.h declares.  Only host-side calls are made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|int64_t|void|char)\s*\*?\s*(lsb_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_0912_0947_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_0912_0947_amd import build
        build.build()
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["lsb_capacity", "lsb_embed", "lsb_extract", "lsb_extract_sync", "lsb_embed_raw",
                 "lsb_extract_raw", "lsb_plan_create", "lsb_plan_update", "lsb_plan_run", "lsb_embed_batch", "lsb_extract_batch",
                 "lsb_plan_destroy", "lsb_last_error", "lsb_autotune", "lsb_tune_set", "lsb_tune_get"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, "declared in lsb.h but not exported: %s" % missing


def test_binding_covers_the_header():
    from paper_0912_0947_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_capacity_is_host_only(lib):
    import oracle
    for k in range(1, 9):
        for n in [0, 3, 31, 32, 33, 1000, 786432, 201326592, 3732480000]:
            assert lib.lsb_capacity(n, k) == oracle.capacity(n, k)
    assert lib.lsb_capacity(100, 0) == -1
    assert b"outside" in lib.lsb_last_error()


def test_tune_table_roundtrip(lib):
    from paper_0912_0947_amd._lib import LaunchCfg
    old27, old26 = LaunchCfg(), LaunchCfg()
    assert lib.lsb_tune_get(0, 1, 1 << 27, ctypes.byref(old27)) == 0
    assert lib.lsb_tune_get(0, 1, 1 << 26, ctypes.byref(old26)) == 0
    new = LaunchCfg(512, 4, 2, 1)
    assert lib.lsb_tune_set(0, 1, 27, ctypes.byref(new)) == 0
    got = LaunchCfg()
    lib.lsb_tune_get(0, 1, (1 << 27) + 5, ctypes.byref(got))
    assert got.as_dict() == new.as_dict()
    lib.lsb_tune_get(0, 1, 1 << 26, ctypes.byref(got))
    assert got.as_dict() == old26.as_dict()  # other buckets untouched
    assert lib.lsb_tune_set(0, 1, 27, ctypes.byref(old27)) == 0
    bad = LaunchCfg(100, 3, 0, 0)
    assert lib.lsb_tune_set(0, 1, 27, ctypes.byref(bad)) == -1


def test_stored_tuning_table_is_valid():
    """The committed table loads, covers every (op, k) and holds valid
    configurations only."""
    import json

    from paper_0912_0947_amd import tune
    table = json.load(open(tune.TABLE))
    assert {(e["op"], e["k"]) for e in table["entries"]} == {(op, k) for op in (0, 1) for k in range(1, 9)}
    assert tune.load() is True


def test_no_cpu_fallback(monkeypatch, tmp_path):
    """Without the built library every operation raises instead of running
    anywhere else."""
    from paper_0912_0947_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.lib()


def test_binding_refuses_integers_that_would_wrap(lib):
    """ctypes would pass 2**32 + 5 to a uint32 parameter as 5; the binding
    refuses any integer outside its parameter's range instead."""
    assert lib.lsb_capacity(786432, 1) == 98300
    import numpy as np
    assert lib.lsb_capacity(np.uint64(786432), np.int64(1)) == 98300
    for args in [(786432, 2**32 + 1), (-1, 1), (2**64, 1)]:
        with pytest.raises(ctypes.ArgumentError):
            lib.lsb_capacity(*args)
    assert lib.lsb_paper_capacity(7, 1024) == 7 * 256
    with pytest.raises(ctypes.ArgumentError):
        lib.lsb_paper_capacity(2**32 + 7, 1024)


def test_image_sizes_that_would_overflow_are_refused(lib):
    """h*w*c and pixels*c are formed in 64 bits; sizes past the stated
    limits are LSB_E_ARG before anything else is looked at (no GPU call)."""
    E_ARG = -1
    # 2^31 x 2^31 x 2^16 wraps to 0 in 64 bits: refused, not taken as empty
    assert lib.lsb_paper_embed(None, None, 2**31, 2**31, 2**16, 0, None, 0, None) == E_ARG
    assert lib.lsb_paper_extract(None, 2**31, 2**31, 2**16, 0, None, 1, None) == E_ARG
    assert b"2^48" in lib.lsb_last_error()
    assert lib.lsb_embed_plane(None, None, 16, 65537, 0, None, 0, 1, None) == E_ARG
    assert lib.lsb_embed_plane(None, None, 2**48 + 1, 3, 0, None, 0, 1, None) == E_ARG


def test_binding_checks_stream_buffer_sizes_before_calling(lib):
    """A raw slice reads (embed) or writes (extract) stream bytes up to
    ceil(min(k*(t0+n), stream_bits)/8); the binding refuses shorter stream
    buffers before anything reaches the library (CPU tensors suffice: the
    size check comes first)."""
    import torch

    from paper_0912_0947_amd import api

    cover = torch.zeros(100, dtype=torch.uint8)
    # k = 3, t0 = 100, n = 100: bits [300, 600) -> bytes up to 75
    with pytest.raises(ValueError, match="75"):
        api.embed_raw(cover, 100, torch.zeros(74, dtype=torch.uint8), 10**6, 3)
    with pytest.raises(ValueError, match="75"):
        api.extract_raw(cover, 100, torch.zeros(74, dtype=torch.uint8), 10**6, 3)
    # the stream ends at bit 310: 39 bytes are enough, and the next check is the device one
    with pytest.raises(TypeError, match="GPU"):
        api.embed_raw(cover, 100, torch.zeros(39, dtype=torch.uint8), 310, 3)
    with pytest.raises(ValueError):
        api.paper_extract(torch.zeros(48, dtype=torch.uint8), 4, 4, 3, 0, 4, out=torch.zeros(3, dtype=torch.uint8))
