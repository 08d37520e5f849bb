"""Python API over liblsb.so for torch uint8 device tensors.

Thin marshalling only: every operation runs in the HIP kernels of liblsb.so
on the tensor's device and the caller's (or torch's current) stream.  Names
follow include/lsb.h.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (E_ARG, OK, OP_EMBED, OP_EXTRACT, LaunchCfg, LsbError, check, lib)

__all__ = ["capacity", "embed", "extract", "extract_sync", "embed_raw", "extract_raw",
           "paper_capacity", "paper_embed", "paper_extract", "embed_plane", "extract_plane", "sse", "psnr",
           "video_embed_host", "verify", "embed_verify", "stream_reference",
           "tune_get", "tune_set", "autotune", "LsbError", "OK", "OP_EMBED", "OP_EXTRACT"]


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _u8(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8:
        raise TypeError("%s must be a torch.uint8 tensor" % name)
    if not t.is_cuda:
        raise TypeError("%s must live on a GPU (no CPU path exists)" % name)
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    if t.device.index != torch.cuda.current_device():
        # the library launches on the current device
        raise ValueError("%s is on %s but the current device is cuda:%d (use torch.cuda.device)"
                         % (name, t.device, torch.cuda.current_device()))
    return t.data_ptr() if t.numel() else 0


def _len_status_ptr(t: torch.Tensor) -> int:
    """Device address of a [length, status] pair: two int32 words that the
    kernel writes."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or t.numel() < 2 or not t.is_cuda \
            or not t.is_contiguous():
        raise TypeError("len_status must be a contiguous int32 device tensor of 2 elements")
    if t.device.index != torch.cuda.current_device():
        raise ValueError("len_status is on %s but the current device is cuda:%d" % (t.device,
                                                                                   torch.cuda.current_device()))
    return t.data_ptr()


def _word64_ptr(t: torch.Tensor, name: str) -> ctypes.c_void_p:
    """Device address of one 64-bit result word that a kernel writes."""
    if not isinstance(t, torch.Tensor) or t.dtype not in (torch.int64, torch.uint64) or t.numel() < 1 \
            or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous 64-bit integer device tensor of at least 1 element" % name)
    if t.device.index != torch.cuda.current_device():
        raise ValueError("%s is on %s but the current device is cuda:%d" % (name, t.device,
                                                                           torch.cuda.current_device()))
    return ctypes.c_void_p(t.data_ptr())


def _slice_stream_end(k: int, t0: int, n: int, stream_bits: int) -> int:
    """One past the last stream byte that cover bytes [t0, t0 + n) touch, or
    0 when they carry no bit (lsb_slice_stream_bytes)."""
    return check(lib().lsb_slice_stream_bytes(k, t0, n, stream_bits))


def capacity(n: int, k: int) -> int:
    """Message capacity in bytes of an n-byte cover at k bits per byte."""
    return check(lib().lsb_capacity(n, k))


def embed(cover: torch.Tensor, msg: torch.Tensor, k: int, out: torch.Tensor | None = None,
          stream=None) -> torch.Tensor:
    """stego = cover with BE32(len(msg)) || msg in its low k bits.  ``out`` may
    be ``cover`` itself (in place)."""
    stego = torch.empty_like(cover) if out is None else out
    if stego.numel() != cover.numel():
        raise ValueError("out must have as many bytes as cover")
    check(lib().lsb_embed(_u8(cover, "cover"), _u8(stego, "out"), cover.numel(), _u8(msg, "msg"),
                          msg.numel(), k, _stream_ptr(stream)))
    return stego


def extract(stego: torch.Tensor, k: int, out: torch.Tensor | None = None,
            len_status: torch.Tensor | None = None, stream=None):
    """Asynchronous extract.  Returns (out, len_status): ``out`` holds the
    message bytes, ``len_status`` an int32 device tensor [decoded length,
    status] that is valid once the stream gets there."""
    if out is None:
        cap = lib().lsb_capacity(stego.numel(), k)
        out = torch.empty(max(int(cap), 0), dtype=torch.uint8, device=stego.device)
    if len_status is None:
        len_status = torch.empty(2, dtype=torch.int32, device=stego.device)
    base = _len_status_ptr(len_status)
    check(lib().lsb_extract(_u8(stego, "stego"), stego.numel(), k,
                            _u8(out, "out") if out.numel() else None, out.numel(),
                            ctypes.c_void_p(base), ctypes.c_void_p(base + 4), _stream_ptr(stream)))
    return out, len_status


def extract_sync(stego: torch.Tensor, k: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Extract and wait; returns the message as a view of ``out``.  Raises
    LsbError for a header or buffer error."""
    if out is None:
        cap = lib().lsb_capacity(stego.numel(), k)
        out = torch.empty(max(int(cap), 0), dtype=torch.uint8, device=stego.device)
    ln = ctypes.c_uint32(0)
    check(lib().lsb_extract_sync(_u8(stego, "stego"), stego.numel(), k,
                                 _u8(out, "out") if out.numel() else None, out.numel(),
                                 ctypes.byref(ln), _stream_ptr(stream)))
    return out[: ln.value]


def embed_raw(cover: torch.Tensor, t0: int, stream_bytes: torch.Tensor, stream_bits: int, k: int,
              out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Embed logical-stream bits into cover bytes [t0, t0+n) of a longer
    logical cover (no header)."""
    stego = torch.empty_like(cover) if out is None else out
    if stego.numel() != cover.numel():
        raise ValueError("out must have as many bytes as cover")
    if 1 <= k <= 8 and stream_bytes.numel() < _slice_stream_end(k, t0, cover.numel(), stream_bits):
        raise ValueError("stream_bytes holds %d bytes; the slice reads up to byte %d"
                         % (stream_bytes.numel(), _slice_stream_end(k, t0, cover.numel(), stream_bits)))
    check(lib().lsb_embed_raw(_u8(cover, "cover"), _u8(stego, "out"), cover.numel(), t0,
                              _u8(stream_bytes, "stream_bytes"), stream_bits, k, _stream_ptr(stream)))
    return stego


def extract_raw(stego: torch.Tensor, t0: int, stream_out: torch.Tensor, stream_bits: int, k: int,
                stream=None) -> torch.Tensor:
    """Extract the stream bits carried by cover bytes [t0, t0+n) into the
    logical-stream buffer ``stream_out``."""
    if 1 <= k <= 8 and stream_out.numel() < _slice_stream_end(k, t0, stego.numel(), stream_bits):
        raise ValueError("stream_out holds %d bytes; the slice writes up to byte %d"
                         % (stream_out.numel(), _slice_stream_end(k, t0, stego.numel(), stream_bits)))
    check(lib().lsb_extract_raw(_u8(stego, "stego"), stego.numel(), t0, _u8(stream_out, "stream_out"),
                                stream_bits, k, _stream_ptr(stream)))
    return stream_out


def paper_capacity(h: int, w: int) -> int:
    """h * floor(w/4): data bytes the paper's layout holds in one plane."""
    return int(lib().lsb_paper_capacity(h, w))


def paper_embed(cover: torch.Tensor, h: int, w: int, c: int, plane: int, data: torch.Tensor,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The paper's own layout: 2 bits per byte in one plane, greedy rows,
    bit pair i of data byte j in pixel L*i + j.  ``out`` may be ``cover``."""
    if cover.numel() != h * w * c:
        raise ValueError("cover must hold h*w*c bytes")
    stego = torch.empty_like(cover) if out is None else out
    check(lib().lsb_paper_embed(_u8(cover, "cover"), _u8(stego, "out"), h, w, c, plane, _u8(data, "data"),
                                data.numel(), _stream_ptr(stream)))
    return stego


def paper_extract(stego: torch.Tensor, h: int, w: int, c: int, plane: int, length: int,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Inverse of paper_embed for ``length`` data bytes."""
    if stego.numel() != h * w * c:
        raise ValueError("stego must hold h*w*c bytes")
    if out is None:
        out = torch.empty(length, dtype=torch.uint8, device=stego.device)
    if out.numel() < length:
        raise ValueError("out must hold the %d data bytes" % length)
    check(lib().lsb_paper_extract(_u8(stego, "stego"), h, w, c, plane, _u8(out, "out") if length else None,
                                  length, _stream_ptr(stream)))
    return out


def embed_plane(cover: torch.Tensor, c: int, plane: int, msg: torch.Tensor, k: int,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """General method on one colour plane of an HWC image (fields = bytes
    p*c + plane); other planes copied.  ``out`` may be ``cover``."""
    if cover.numel() % c:
        raise ValueError("cover bytes must be a multiple of the channel count")
    stego = torch.empty_like(cover) if out is None else out
    check(lib().lsb_embed_plane(_u8(cover, "cover"), _u8(stego, "out"), cover.numel() // c, c, plane,
                                _u8(msg, "msg"), msg.numel(), k, _stream_ptr(stream)))
    return stego


def extract_plane(stego: torch.Tensor, c: int, plane: int, k: int, out: torch.Tensor | None = None,
                  len_status: torch.Tensor | None = None, stream=None):
    """Asynchronous single-plane extract; returns (out, len_status) like extract."""
    pixels = stego.numel() // c
    if out is None:
        cap = lib().lsb_capacity(pixels, k)
        out = torch.empty(max(int(cap), 0), dtype=torch.uint8, device=stego.device)
    if len_status is None:
        len_status = torch.empty(2, dtype=torch.int32, device=stego.device)
    base = _len_status_ptr(len_status)
    check(lib().lsb_extract_plane(_u8(stego, "stego"), pixels, c, plane, k, _u8(out, "out") if out.numel() else None,
                                  out.numel(), ctypes.c_void_p(base), ctypes.c_void_p(base + 4),
                                  _stream_ptr(stream)))
    return out, len_status


def sse(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Sum of squared byte differences as an int64 device tensor of 1 element."""
    if a.numel() != b.numel():
        raise ValueError("a and b must have the same size")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=a.device)
    check(lib().lsb_sse(_u8(a, "a"), _u8(b, "b"), a.numel(), _word64_ptr(out, "out"), _stream_ptr(stream)))
    return out


def psnr(sse_value: int, count: int) -> float:
    """10*log10(255^2 / (sse / count)) in dB (host arithmetic on a reduced value)."""
    import math
    return math.inf if sse_value == 0 else 10.0 * math.log10(255.0 * 255.0 * count / sse_value)


def video_embed_host(host_frames: torch.Tensor, host_stego: torch.Tensor, frame_bytes: int,
                     stream_bytes: torch.Tensor, stream_bits: int, k: int, ring: torch.Tensor, streams):
    """Pipeline frames from pinned host memory through the device ring: frame
    f goes to ``streams[f % len(streams)]``, which copies it in, embeds it in
    place (raw slice t0 = f * frame_bytes) and copies it out.  The ring's slot
    count is rounded down to a multiple of the stream count.  Returns after
    enqueueing; synchronize every stream before reading host_stego."""
    for t, name in ((host_frames, "host_frames"), (host_stego, "host_stego")):
        if t.is_cuda or not t.is_pinned() or t.dtype != torch.uint8 or not t.is_contiguous():
            raise TypeError("%s must be a contiguous pinned uint8 host tensor" % name)
    if host_frames.numel() % frame_bytes or host_stego.numel() != host_frames.numel():
        raise ValueError("host buffers must hold whole frames, stego as many bytes as frames")
    frames = host_frames.numel() // frame_bytes
    if 1 <= k <= 8 and stream_bytes.numel() < _slice_stream_end(k, 0, frames * frame_bytes, stream_bits):
        raise ValueError("stream_bytes holds %d bytes; the clip reads up to byte %d"
                         % (stream_bytes.numel(), _slice_stream_end(k, 0, frames * frame_bytes, stream_bits)))
    streams = list(streams)
    slots = ring.numel() // frame_bytes // len(streams) * len(streams)
    if slots < 1:
        raise ValueError("ring must hold at least one frame per stream")
    arr = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
    check(lib().lsb_video_embed_host(ctypes.c_void_p(host_frames.data_ptr()), ctypes.c_void_p(host_stego.data_ptr()),
                                     frame_bytes, host_frames.numel() // frame_bytes, _u8(stream_bytes, "stream_bytes"),
                                     stream_bits, k, _u8(ring, "ring"), slots, arr, len(streams)))


def verify(cover: torch.Tensor, stego: torch.Tensor, msg: torch.Tensor, k: int,
           out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Count (on the device, int64 tensor of 1 element) the stego bytes that
    fail the round-trip check against ``cover`` and ``msg`` (lsb_verify);
    0 means verified."""
    if cover.numel() != stego.numel():
        raise ValueError("cover and stego must have the same size")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=cover.device)
    check(lib().lsb_verify(_u8(cover, "cover"), _u8(stego, "stego"), cover.numel(), _u8(msg, "msg"), msg.numel(), k,
                           _word64_ptr(out, "out"), _stream_ptr(stream)))
    return out


def embed_verify(cover: torch.Tensor, msg: torch.Tensor, k: int, out: torch.Tensor | None = None,
                 mismatches: torch.Tensor | None = None, stream=None):
    """Embed as ``embed`` and, in the same launch, check every written byte
    through extraction.  Returns (stego, mismatches): ``mismatches`` is an
    int64 device tensor of 1 element holding the number of wrong bytes (0
    for a correct embedding).  ``out`` may be ``cover`` itself (in place)."""
    stego = torch.empty_like(cover) if out is None else out
    if stego.numel() != cover.numel():
        raise ValueError("out must have as many bytes as cover")
    if mismatches is None:
        mismatches = torch.empty(1, dtype=torch.int64, device=cover.device)
    check(lib().lsb_embed_verify(_u8(cover, "cover"), _u8(stego, "out"), cover.numel(), _u8(msg, "msg"),
                                 msg.numel(), k, _word64_ptr(mismatches, "mismatches"), _stream_ptr(stream)))
    return stego, mismatches


def stream_reference(kind: int, src: torch.Tensor, dst: torch.Tensor, side: torch.Tensor | None = None,
                     block: int = 256, unroll: int = 1, grid: int = 0, stream=None, k: int = 1) -> torch.Tensor:
    """Reference stream with the traffic mix ``kind`` (REF_COPY, REF_EMBED_MIX,
    REF_EXTRACT_MIX) of k bits per cover byte (1, 2 or 4) over ``src``; a
    measurement aid that computes nothing of the method.  ``dst`` holds
    src.numel() bytes (src.numel() * k // 8 for REF_EXTRACT_MIX); ``side``
    holds src.numel() * k // 8 bytes for REF_EMBED_MIX."""
    n = src.numel()
    want = n * k // 8 if kind == 2 else n
    if dst.numel() != want:
        raise ValueError("dst must hold %d bytes" % want)
    if kind == 1 and (side is None or side.numel() != n * k // 8):
        raise ValueError("side must hold %d bytes" % (n * k // 8))
    sp = _u8(side, "side") if side is not None else None
    check(lib().lsb_stream_reference(kind, k, _u8(src, "src"), _u8(dst, "dst"), sp, n, block, unroll, grid,
                                     _stream_ptr(stream)))
    return dst


def tune_get(op: int, k: int, n: int) -> dict:
    cfg = LaunchCfg()
    check(lib().lsb_tune_get(op, k, n, ctypes.byref(cfg)))
    return cfg.as_dict()


def tune_set(op: int, k: int, bucket: int, block: int, unroll: int, blocks_per_cu: int, nontemporal: int,
             pack: int = 0, order: int = 0):
    cfg = LaunchCfg(block, unroll, blocks_per_cu, nontemporal, pack, order)
    check(lib().lsb_tune_set(op, k, bucket, ctypes.byref(cfg)))


def autotune(op: int, k: int, cover: torch.Tensor, stego: torch.Tensor, msg: torch.Tensor,
             reps: int = 10, stream=None):
    """Time every launch configuration for (op, k, cover size) and install the
    fastest.  Returns (config dict, mean kernel microseconds)."""
    best = LaunchCfg()
    us = ctypes.c_double(0.0)
    check(lib().lsb_autotune(op, k, cover.numel(), _u8(cover, "cover"), _u8(stego, "stego"),
                             _u8(msg, "msg"), reps, ctypes.byref(best), ctypes.byref(us),
                             _stream_ptr(stream)))
    return best.as_dict(), us.value


_ = (E_ARG, LsbError)
