"""CPU oracle for k-bit LSB embedding / extraction (arXiv:0912.0947).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
(``__graft_entry__.smoke``) and the benchmark's ``cpu_baseline`` leg may import
this package.  It shares no code with the GPU library and imports nothing from
the product package.

Two implementations of the same plain definition live here:

* ``lsb_oracle.c`` -- bit-by-bit C, fast enough for full-size inputs; loaded
  through ctypes (``embed``, ``extract``, ``embed_raw``, ``extract_raw``,
  ``capacity``).
* ``ref`` -- the same definition in pure-Python loops, for tiny inputs only.

Paper passages: Section VI step 7 (embedding), Section VII step 6
(extraction), Section VI step 5 / VII step 4 (capacity).  The readings where
the paper is silent (MSB-first stream, BE32 length header, sequential
placement over every channel byte, partial last field, bytes past the stream
unchanged) are stated in ``lsb_oracle.h``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

OK = 0
E_ARG = -1
E_CAPACITY = -2
E_HEADER = -3
E_BUFFER = -4
E_NOMEM = -6

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsb_oracle.c")
_LIB = os.path.join(_HERE, "liblsb_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``oracle/liblsb_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    u8p = ctypes.c_void_p
    lib.oracle_capacity.restype = ctypes.c_int64
    lib.oracle_capacity.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.oracle_embed.restype = ctypes.c_int
    lib.oracle_embed.argtypes = [u8p, u8p, ctypes.c_uint64, u8p,
                                 ctypes.c_uint32, ctypes.c_int]
    lib.oracle_extract.restype = ctypes.c_int
    lib.oracle_extract.argtypes = [u8p, ctypes.c_uint64, ctypes.c_int,
                                   u8p, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_uint32)]
    lib.oracle_embed_raw.restype = ctypes.c_int
    lib.oracle_embed_raw.argtypes = [u8p, u8p, ctypes.c_uint64,
                                     ctypes.c_uint64, u8p,
                                     ctypes.c_uint64, ctypes.c_int]
    lib.oracle_extract_raw.restype = ctypes.c_int
    lib.oracle_extract_raw.argtypes = [u8p, ctypes.c_uint64,
                                       ctypes.c_uint64, u8p,
                                       ctypes.c_uint64, ctypes.c_int]
    lib.oracle_paper_capacity.restype = ctypes.c_uint64
    lib.oracle_paper_capacity.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_paper_embed.restype = ctypes.c_int
    lib.oracle_paper_embed.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, u8p, ctypes.c_uint64]
    lib.oracle_paper_extract.restype = ctypes.c_int
    lib.oracle_paper_extract.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32, u8p, ctypes.c_uint64]
    lib.oracle_embed_plane.restype = ctypes.c_int
    lib.oracle_embed_plane.argtypes = [u8p, u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u8p,
                                       ctypes.c_uint32, ctypes.c_int]
    lib.oracle_extract_plane.restype = ctypes.c_int
    lib.oracle_extract_plane.argtypes = [u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                         u8p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)]
    lib.oracle_sse.restype = ctypes.c_uint64
    lib.oracle_sse.argtypes = [u8p, u8p, ctypes.c_uint64]
    lib.oracle_psnr.restype = ctypes.c_double
    lib.oracle_psnr.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            override = os.environ.get("LSB_ORACLE_LIB")  # mutation tests, sanitizer builds
            if override:
                _lib = _bind(override)
            else:
                if not os.path.exists(_LIB):
                    build()
                _lib = _bind(_LIB)
    return _lib


def use_library(path: str | None):
    """Point this module at another build of ``lsb_oracle.c`` (the mutation
    tests load deliberately broken copies); ``None`` restores the default."""
    global _lib
    with _lock:
        _lib = _bind(path) if path else None


def _u8(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8)).reshape(-1)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


def capacity(n: int, k: int) -> int:
    """floor(n*k/8) - 4 message bytes, or a negative error code."""
    return int(_load().oracle_capacity(n, k))


def embed(cover, msg, k: int, out=None):
    """Header-mode embed.  Returns (status, stego); stego is a fresh array
    (or ``out``, which may be ``cover`` itself for the in-place form)."""
    cover = _u8(cover)
    msg = _u8(msg)
    stego = np.empty_like(cover) if out is None else out
    if out is None:
        stego[...] = cover  # untouched on error, like the library
    rc = _load().oracle_embed(_ptr(cover), _ptr(stego), cover.size, _ptr(msg),
                              msg.size, k)
    return rc, stego


def extract(stego, k: int, out_cap: int | None = None):
    """Header-mode extract.  Returns (status, len, msg bytes or None)."""
    stego = _u8(stego)
    if out_cap is None:
        cap = capacity(stego.size, k)
        out_cap = max(cap, 0)
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    ln = ctypes.c_uint32(0)
    rc = _load().oracle_extract(_ptr(stego), stego.size, k, _ptr(out), out_cap,
                                ctypes.byref(ln))
    msg = out[: ln.value].copy() if rc == OK else None
    return rc, int(ln.value), msg


def embed_raw(cover, t0: int, stream, stream_bits: int, k: int):
    """Raw-slice embed.  Returns (status, stego)."""
    cover = _u8(cover)
    stream = _u8(stream)
    stego = cover.copy()
    rc = _load().oracle_embed_raw(_ptr(cover), _ptr(stego), cover.size, t0,
                                  _ptr(stream), stream_bits, k)
    return rc, stego


def extract_raw(stego, t0: int, stream_bits: int, k: int, stream_out=None):
    """Raw-slice extract into ``stream_out`` (a logical-stream-sized buffer,
    zeros if not given).  Returns (status, stream_out)."""
    stego = _u8(stego)
    if stream_out is None:
        stream_out = np.zeros((stream_bits + 7) // 8, dtype=np.uint8)
    rc = _load().oracle_extract_raw(_ptr(stego), stego.size, t0,
                                    _ptr(stream_out), stream_bits, k)
    return rc, stream_out


# ---------------------------------------------------------------------------
# The paper's own layout (2 bits per byte, one plane, greedy rows, strided
# bit pairs).
def paper_capacity(h: int, w: int) -> int:
    return int(_load().oracle_paper_capacity(h, w))


def paper_embed(cover, h: int, w: int, c: int, plane: int, data):
    """Returns (status, stego) for an h x w x c cover (flat or shaped)."""
    cover = _u8(cover)
    data = _u8(data)
    stego = cover.copy()
    rc = _load().oracle_paper_embed(_ptr(cover), _ptr(stego), h, w, c, plane, _ptr(data), data.size)
    return rc, stego


def paper_extract(stego, h: int, w: int, c: int, plane: int, length: int):
    """Returns (status, data bytes)."""
    stego = _u8(stego)
    out = np.zeros(max(length, 1), dtype=np.uint8)
    rc = _load().oracle_paper_extract(_ptr(stego), h, w, c, plane, _ptr(out), length)
    return rc, out[:length]


# ---------------------------------------------------------------------------
# One colour plane with the general method; squared error and PSNR.
def embed_plane(cover, c: int, plane: int, msg, k: int):
    cover = _u8(cover)
    msg = _u8(msg)
    stego = cover.copy()
    rc = _load().oracle_embed_plane(_ptr(cover), _ptr(stego), cover.size // c, c, plane, _ptr(msg), msg.size, k)
    return rc, stego


def extract_plane(stego, c: int, plane: int, k: int, out_cap: int | None = None):
    stego = _u8(stego)
    pixels = stego.size // c
    if out_cap is None:
        out_cap = max(capacity(pixels, k), 0)
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    ln = ctypes.c_uint32(0)
    rc = _load().oracle_extract_plane(_ptr(stego), pixels, c, plane, k, _ptr(out), out_cap, ctypes.byref(ln))
    return rc, int(ln.value), (out[: ln.value].copy() if rc == OK else None)


def sse(a, b) -> int:
    a = _u8(a)
    b = _u8(b)
    assert a.size == b.size
    return int(_load().oracle_sse(_ptr(a), _ptr(b), a.size))


def psnr(sse_value: int, count: int) -> float:
    return float(_load().oracle_psnr(sse_value, count))
