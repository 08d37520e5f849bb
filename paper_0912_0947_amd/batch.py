"""Batched embed/extract: many covers of uneven size and k in one persistent,
graph-replayed launch (lsb_plan_* in include/lsb.h).  Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import JOB_RAW, OP_EMBED, OP_EXTRACT, OP_MIXED, Job, LaunchCfg, check, lib

ALIGN = 256

JOB_DTYPE = np.dtype([("cover_off", "<u8"), ("stego_off", "<u8"), ("msg_off", "<u8"), ("n", "<u8"),
                      ("msg_cap", "<u8"), ("t0", "<u8"), ("stream_bits", "<u8"), ("len", "<u4"), ("k", "u1"),
                      ("op", "u1"), ("flags", "u1"), ("reserved", "u1")])
assert JOB_DTYPE.itemsize == ctypes.sizeof(Job)


def align_up(x: int, a: int = ALIGN) -> int:
    return (x + a - 1) // a * a


def make_jobs(count: int) -> np.ndarray:
    return np.zeros(count, dtype=JOB_DTYPE)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("arenas and status buffers must be device tensors")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owns an lsb_plan: a device job table, its pinned host mirror and the
    HIP graph {table upload, prologue, persistent kernel}."""

    def __init__(self, max_jobs: int, op: int = OP_MIXED, jobs: np.ndarray | None = None):
        """Room for ``max_jobs`` jobs; ``op`` = OP_EMBED / OP_EXTRACT makes
        every job that kind, OP_MIXED keeps each job's op field.  ``jobs``,
        if given, is installed at creation (lsb_plan_create)."""
        self._p = ctypes.c_void_p()
        ptr = None
        if jobs is not None:
            jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
            if jobs.size != max_jobs:
                raise ValueError("jobs given at creation must number max_jobs")
            ptr = jobs.ctypes.data_as(ctypes.POINTER(Job))
        check(lib().lsb_plan_create(ctypes.byref(self._p), ptr, int(max_jobs), int(op)))
        self.max_jobs = int(max_jobs)
        self.n_jobs = int(max_jobs) if jobs is not None else 0

    def set_jobs(self, jobs: np.ndarray) -> None:
        """Replace the job list (lsb_plan_update)."""
        jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
        ptr = jobs.ctypes.data_as(ctypes.POINTER(Job)) if jobs.size else None
        check(lib().lsb_plan_update(self._p, ptr, int(jobs.size)))
        self.n_jobs = int(jobs.size)

    update = set_jobs

    def embed_batch(self, cover_arena, stego_arena, msg_arena, status_dev, stream=None) -> None:
        """lsb_embed_batch: every job of the plan must be an embed."""
        if stream is None:
            stream = torch.cuda.current_stream()
        check(lib().lsb_embed_batch(self._p, _ptr(cover_arena), _ptr(stego_arena), _ptr(msg_arena),
                                    _ptr(status_dev), ctypes.c_void_p(stream.cuda_stream)))

    def extract_batch(self, stego_arena, msg_arena, len_dev, status_dev, stream=None) -> None:
        """lsb_extract_batch: every job of the plan must be an extract."""
        if stream is None:
            stream = torch.cuda.current_stream()
        check(lib().lsb_extract_batch(self._p, _ptr(stego_arena), _ptr(msg_arena), _ptr(len_dev),
                                      _ptr(status_dev), ctypes.c_void_p(stream.cuda_stream)))

    @property
    def tiles(self) -> int:
        return int(check(lib().lsb_plan_tiles(self._p)))

    def run(self, cover_arena, stego_arena, msg_arena, len_dev, status_dev, stream=None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream()
        check(lib().lsb_plan_run(self._p, _ptr(cover_arena), _ptr(stego_arena), _ptr(msg_arena),
                                 _ptr(len_dev), _ptr(status_dev), ctypes.c_void_p(stream.cuda_stream)))

    def close(self) -> None:
        if self._p:
            lib().lsb_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_get():
    cfg = LaunchCfg()
    tv = ctypes.c_int64()
    check(lib().lsb_batch_tune_get(ctypes.byref(cfg), ctypes.byref(tv)))
    return cfg.as_dict(), int(tv.value)


def tune_set(block: int, unroll: int, blocks_per_cu: int, nontemporal: int, tile_vectors: int) -> None:
    cfg = LaunchCfg(block, unroll, blocks_per_cu, nontemporal, 0)
    check(lib().lsb_batch_tune_set(ctypes.byref(cfg), int(tile_vectors)))


__all__ = ["Plan", "make_jobs", "align_up", "JOB_DTYPE", "JOB_RAW", "OP_EMBED", "OP_EXTRACT", "OP_MIXED", "tune_get",
           "tune_set"]
