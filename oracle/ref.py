"""Pure-Python twin of the C oracle, for tiny inputs only.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Written from the same plain definition
(paper Section VI step 7 and Section VII step 6, generalised to k bits, with
the readings stated in ``lsb_oracle.h``) but independently of the C code, so
that the two can be compared on small cases.  Works on Python lists/bytes.
"""
from __future__ import annotations


def stream_of(msg: bytes) -> bytes:
    """S = BE32(len) || msg."""
    return len(msg).to_bytes(4, "big") + bytes(msg)


def bits_msb_first(data: bytes) -> list[int]:
    out = []
    for byte in data:
        for r in range(8):
            out.append((byte >> (7 - r)) & 1)
    return out


def embed_stream(cover: bytes, stream_bits: list[int], k: int, t0: int = 0) -> bytes:
    """Byte t of ``cover`` (logical field t0+t) takes stream bits
    k*(t0+t) .. k*(t0+t)+k-1, first bit highest; a short last field fills the
    top of the field; fields past the stream are unchanged."""
    assert 1 <= k <= 8
    out = bytearray(cover)
    for t in range(len(cover)):
        first = k * (t0 + t)
        piece = stream_bits[first:first + k]
        if not piece:
            continue
        value = 0
        for b in piece:
            value = value * 2 + b
        shift = k - len(piece)
        field_mask = (2 ** len(piece) - 1) * 2 ** shift
        out[t] = (cover[t] - (cover[t] & field_mask)) + value * 2 ** shift
    return bytes(out)


def extract_bits(stego: bytes, k: int, nbits: int) -> list[int]:
    """Read the first ``nbits`` stream bits back out of the fields."""
    bits = []
    for t in range(len(stego)):
        for q in range(k):
            if len(bits) == nbits:
                return bits
            bits.append((stego[t] // 2 ** (k - 1 - q)) % 2)
    return bits


def bits_to_bytes(bits: list[int]) -> bytes:
    out = bytearray()
    for i in range(0, len(bits), 8):
        chunk = bits[i:i + 8] + [0] * (8 - len(bits[i:i + 8]))
        value = 0
        for b in chunk:
            value = value * 2 + b
        out.append(value)
    return bytes(out)


def embed(cover: bytes, msg: bytes, k: int) -> bytes:
    cap_bits = len(cover) * k
    s = stream_of(msg)
    if 8 * len(s) > cap_bits:
        raise ValueError("message does not fit")
    return embed_stream(cover, bits_msb_first(s), k)


def extract(stego: bytes, k: int) -> bytes:
    if len(stego) * k < 32:
        raise ValueError("header does not fit")
    header = bits_to_bytes(extract_bits(stego, k, 32))
    n = int.from_bytes(header, "big")
    if 8 * (4 + n) > len(stego) * k:
        raise ValueError("decoded length does not fit")
    s = bits_to_bytes(extract_bits(stego, k, 8 * (4 + n)))
    return s[4:]
