"""Device-resident batched workloads (uneven covers in shared arenas).

The arena layout packs every cover, stego buffer and message at 256-byte
aligned offsets, as the batched entry points require.  Message lengths are
drawn as a fraction of each cover's capacity; the capacity function is
passed in by the caller so that this module holds none of the method's
arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import inputs
from .batch import ALIGN, JOB_DTYPE, OP_EMBED, OP_EXTRACT, align_up


class BatchWorkload:
    """Uneven covers (width, height ~ U{lo..hi}, 1 or 3 channels, k in ks,
    message = floor(u * capacity), u ~ U[0.1, 1]) laid out in arenas:
    cover arena (covers), stego arena (one stego buffer per cover) and message
    arena (messages; extract outputs go to a second message arena)."""

    def __init__(self, count: int, cap_fn, seed: int = 401, lo: int = 64, hi: int = 4096, ks=(1, 2)):
        sh = inputs.batch_shapes(count, seed=seed, lo=lo, hi=hi, ks=ks)
        self.count = count
        self.n = sh["n"].astype(np.int64)
        self.k = sh["k"].astype(np.int64)
        caps = np.array([cap_fn(int(n), int(k)) for n, k in zip(self.n, self.k)], dtype=np.int64)
        self.len = np.floor(sh["u"] * caps).astype(np.int64)
        self.cap = caps
        self.cover_off = np.zeros(count, np.int64)
        self.msg_off = np.zeros(count, np.int64)
        off = 0
        for i, n in enumerate(self.n):
            self.cover_off[i] = off
            off = align_up(off + int(n))
        self.cover_bytes = off
        off = 0
        for i, ln in enumerate(self.len):
            self.msg_off[i] = off
            off = align_up(off + max(int(ln), 1))
        self.msg_bytes = off

    def jobs(self, op: int, order=None) -> np.ndarray:
        """Job table: embed reads cover -> writes stego (same offsets) with the
        message at msg_off; extract reads stego -> writes msg_off."""
        j = np.zeros(self.count, dtype=JOB_DTYPE)
        j["cover_off"] = self.cover_off
        j["stego_off"] = self.cover_off
        j["msg_off"] = self.msg_off
        j["n"] = self.n
        j["k"] = self.k
        j["op"] = op
        if op == OP_EMBED:
            j["len"] = self.len
        else:
            j["msg_cap"] = self.len
        if order is not None:
            j = j[order]
        return j

    def allocate(self, device, pixel_seed: int = 402, msg_seed: int = 403):
        """Cover, stego, message and output arenas on the device; covers and
        messages filled with seeded uniform bytes."""
        import torch

        cover = torch.empty(self.cover_bytes, dtype=torch.uint8, device=device)
        stego = torch.empty(self.cover_bytes, dtype=torch.uint8, device=device)
        msg = torch.empty(self.msg_bytes, dtype=torch.uint8, device=device)
        out = torch.zeros(self.msg_bytes, dtype=torch.uint8, device=device)
        inputs.fill_uniform(cover, pixel_seed)
        inputs.fill_uniform(msg, msg_seed)
        # zero the alignment gaps between messages so that whole-arena
        # comparisons of messages and extract outputs are meaningful
        ends = self.msg_off + self.len
        starts = np.append(self.msg_off[1:], self.msg_bytes)
        for a, b in zip(ends, starts):
            if b > a:
                msg[int(a):int(b)].zero_()
        return cover, stego, msg, out


_ = (ALIGN, OP_EXTRACT)
