"""Run the CPU oracle over many independent jobs on several host threads.

The oracle's C functions release the GIL (ctypes), so a thread pool runs
them in parallel.  The pool is sized to the cores this process may use,
at most 16 (the share of a one-GPU host).  Device results are brought to
the host in chunks through one pinned staging buffer, so full-size
workloads (tens of GB) are compared byte for byte without holding them in
host memory at once.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run(fn, items) -> list:
    """fn(item) for every item on the pool; the first exception propagates."""
    items = list(items)
    if not items:
        return []
    with ThreadPoolExecutor(min(threads(), len(items))) as pool:
        return list(pool.map(fn, items))


def chunks(offsets, sizes, limit: int):
    """Split job indices (in order) into runs whose byte span
    [offsets[first], offsets[last] + sizes[last]) stays within ``limit``
    (a single larger job forms a run of its own)."""
    out, cur, start = [], [], None
    for i, (o, s) in enumerate(zip(offsets, sizes)):
        o, s = int(o), int(s)
        if cur and o + s - start > limit:
            out.append(cur)
            cur = []
        if not cur:
            start = o
        cur.append(i)
    if cur:
        out.append(cur)
    return out


class Staging:
    """Pinned host buffers that device byte ranges are copied into."""

    def __init__(self, nbytes: int, count: int = 1):
        import torch

        self.bufs = [torch.empty(int(nbytes), dtype=torch.uint8, pin_memory=True) for _ in range(count)]

    def fetch(self, slot: int, tensor, begin: int, end: int) -> np.ndarray:
        """Device bytes tensor[begin:end] as a host array (valid until the
        slot is fetched into again)."""
        import torch

        n = int(end) - int(begin)
        host = self.bufs[slot][:n]
        host.copy_(tensor[int(begin):int(end)])
        torch.cuda.synchronize()
        return host.numpy()
