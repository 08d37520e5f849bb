"""Batched embed/extract: many covers of uneven size and k in one persistent
launch (lsb_plan_* in include/lsb.h).  Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import JOB_RAW, OP_EMBED, OP_EXTRACT, OP_MIXED, STATIC_MAX_JOBS, Job, LaunchCfg, check, lib

ALIGN = 256

JOB_DTYPE = np.dtype([("cover_off", "<u8"), ("stego_off", "<u8"), ("msg_off", "<u8"), ("n", "<u8"),
                      ("msg_cap", "<u8"), ("t0", "<u8"), ("stream_bits", "<u8"), ("len", "<u4"), ("k", "u1"),
                      ("op", "u1"), ("flags", "u1"), ("reserved", "u1")])
assert JOB_DTYPE.itemsize == ctypes.sizeof(Job)


def align_up(x: int, a: int = ALIGN) -> int:
    return (x + a - 1) // a * a


def make_jobs(count: int) -> np.ndarray:
    return np.zeros(count, dtype=JOB_DTYPE)


def _extents(jobs: np.ndarray, op_mode: int) -> tuple[int, int, int]:
    """Bytes that the cover, stego and message arenas must hold for ``jobs``:
    one past the furthest byte that any job reads or writes in each, as the
    library computes it (lsb_job_extents)."""
    if not jobs.size:
        return 0, 0, 0
    jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
    if max(int(jobs[f].max()) for f in ("cover_off", "stego_off", "msg_off")) >= 1 << 62:
        raise ValueError("a job offset lies beyond any device arena")
    ext = (ctypes.c_uint64 * 3)()
    check(lib().lsb_job_extents(jobs.ctypes.data_as(ctypes.POINTER(Job)), int(jobs.size), int(op_mode), ext))
    return int(ext[0]), int(ext[1]), int(ext[2])


def _ptr(t, name: str, need: int = 0, dtypes=(torch.uint8,)):
    """Device pointer of ``t`` after checking it: dtype, contiguous, on the
    current device, and at least ``need`` elements.  None passes as NULL
    when nothing is needed from it."""
    if t is None:
        if need:
            raise ValueError("%s is required by the plan's jobs" % name)
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s must be of dtype %s" % (name, " or ".join(str(d) for d in dtypes)))
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    if t.device.index != torch.cuda.current_device():
        raise ValueError("%s is on %s but the current device is cuda:%d" % (name, t.device,
                                                                            torch.cuda.current_device()))
    if t.numel() < need:
        raise ValueError("%s holds %d elements; the plan's jobs need %d" % (name, t.numel(), need))
    return ctypes.c_void_p(t.data_ptr())


_WORD = (torch.int32, torch.uint32) if hasattr(torch, "uint32") else (torch.int32,)


class Plan:
    """Owns an lsb_plan: a device job table and its pinned host mirror (a
    run uploads the table when it changed, then launches the persistent
    kernel).  Before each run
    the binding checks that the arenas hold every byte the jobs name and
    that the status and length arrays have an entry per job (the C call
    takes base pointers only and trusts the caller on this)."""

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
        self.op = int(op)
        self.n_jobs = 0
        self._need = (0, 0, 0)
        if jobs is not None:
            self._installed(jobs)

    def _installed(self, jobs: np.ndarray) -> None:
        self.n_jobs = int(jobs.size)
        self._need = _extents(jobs, self.op)

    def set_jobs(self, jobs: np.ndarray) -> None:
        """Replace the job list (lsb_plan_update)."""
        jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
        ptr = jobs.ctypes.data_as(ctypes.POINTER(Job)) if jobs.size else None
        check(lib().lsb_plan_update(self._p, ptr, int(jobs.size)))
        self._installed(jobs)

    update = set_jobs

    def embed_batch(self, cover_arena, stego_arena, msg_arena, status_dev, stream=None) -> None:
        """lsb_embed_batch: every job of the plan must be an embed."""
        if stream is None:
            stream = torch.cuda.current_stream()
        c, st, m = self._need
        check(lib().lsb_embed_batch(self._p, _ptr(cover_arena, "cover_arena", c), _ptr(stego_arena, "stego_arena", st),
                                    _ptr(msg_arena, "msg_arena", m), _ptr(status_dev, "status_dev", self.n_jobs, _WORD),
                                    ctypes.c_void_p(stream.cuda_stream)))

    def extract_batch(self, stego_arena, msg_arena, len_dev, status_dev, stream=None) -> None:
        """lsb_extract_batch: every job of the plan must be an extract."""
        if stream is None:
            stream = torch.cuda.current_stream()
        _, st, m = self._need
        check(lib().lsb_extract_batch(self._p, _ptr(stego_arena, "stego_arena", st), _ptr(msg_arena, "msg_arena", m),
                                      _ptr(len_dev, "len_dev", self.n_jobs, _WORD),
                                      _ptr(status_dev, "status_dev", self.n_jobs, _WORD),
                                      ctypes.c_void_p(stream.cuda_stream)))

    @property
    def tiles(self) -> int:
        return int(check(lib().lsb_plan_tiles(self._p)))

    def run(self, cover_arena, stego_arena, msg_arena, len_dev, status_dev, stream=None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream()
        c, st, m = self._need
        check(lib().lsb_plan_run(self._p, _ptr(cover_arena, "cover_arena", c), _ptr(stego_arena, "stego_arena", st),
                                 _ptr(msg_arena, "msg_arena", m),
                                 _ptr(len_dev, "len_dev", self.n_jobs if len_dev is not None else 0, _WORD),
                                 _ptr(status_dev, "status_dev", self.n_jobs, _WORD),
                                 ctypes.c_void_p(stream.cuda_stream)))

    def close(self) -> None:
        if self._p:
            lib().lsb_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_static(jobs: np.ndarray, op: int, cover_arena, stego_arena, msg_arena, len_dev, status_dev,
               stream=None) -> None:
    """lsb_batch_run_static: run ``jobs`` (at most STATIC_MAX_JOBS) as a plan
    created with ``op`` would, without allocating anything: the job table
    goes to the library's fixed device array.  Same checks of the arenas and
    result arrays as Plan.run."""
    jobs = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
    if stream is None:
        stream = torch.cuda.current_stream()
    c, st, m = _extents(jobs, int(op))
    n = int(jobs.size)
    check(lib().lsb_batch_run_static(jobs.ctypes.data_as(ctypes.POINTER(Job)) if n else None, n, int(op),
                                     _ptr(cover_arena, "cover_arena", c), _ptr(stego_arena, "stego_arena", st),
                                     _ptr(msg_arena, "msg_arena", m),
                                     _ptr(len_dev, "len_dev", n if len_dev is not None else 0, _WORD),
                                     _ptr(status_dev, "status_dev", n, _WORD), ctypes.c_void_p(stream.cuda_stream)))


def tune_get():
    cfg = LaunchCfg()
    tv = ctypes.c_int64()
    check(lib().lsb_batch_tune_get(ctypes.byref(cfg), ctypes.byref(tv)))
    return cfg.as_dict(), int(tv.value)


def tune_set(block: int, unroll: int, blocks_per_cu: int, nontemporal: int, tile_vectors: int) -> None:
    """Set the launch shape of every plan (embed and extract) and the tile size."""
    cfg = LaunchCfg(block, unroll, blocks_per_cu, nontemporal, 0)
    check(lib().lsb_batch_tune_set(ctypes.byref(cfg), int(tile_vectors)))


def tune_get_op(op: int) -> dict:
    """Launch shape of plans with embed jobs (OP_EMBED) or of extract-only plans (OP_EXTRACT)."""
    cfg = LaunchCfg()
    check(lib().lsb_batch_tune_get_op(int(op), ctypes.byref(cfg)))
    return cfg.as_dict()


def tune_set_op(op: int, block: int, unroll: int, blocks_per_cu: int, nontemporal: int) -> None:
    cfg = LaunchCfg(block, unroll, blocks_per_cu, nontemporal, 0)
    check(lib().lsb_batch_tune_set_op(int(op), ctypes.byref(cfg)))


def set_tile_vectors(tile_vectors: int) -> None:
    """Change the tile size only (both launch shapes stay)."""
    state = tune_state()
    tune_restore((state[0], state[1], int(tile_vectors)))


def tune_state():
    """Both launch shapes and the tile size, for tune_restore."""
    return tune_get_op(OP_EMBED), tune_get_op(OP_EXTRACT), tune_get()[1]


def tune_restore(state) -> None:
    emb, ext, tv = state
    tune_set(emb["block"], emb["unroll"], emb["blocks_per_cu"], emb["nontemporal"], tv)
    tune_set_op(OP_EXTRACT, ext["block"], ext["unroll"], ext["blocks_per_cu"], ext["nontemporal"])


__all__ = ["Plan", "make_jobs", "align_up", "run_static", "JOB_DTYPE", "JOB_RAW", "OP_EMBED", "OP_EXTRACT", "OP_MIXED",
           "STATIC_MAX_JOBS", "tune_get", "tune_set", "tune_get_op", "tune_set_op", "tune_state", "tune_restore",
           "set_tile_vectors"]
