"""Serving loop (lsb_serve in include/lsb.h): open-loop request streams
served with continuous batching under an HBM budget.  Marshalling and
request-stream drawing only; the loop itself runs in liblsb.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import inputs
from ._lib import OP_EMBED, OP_EXTRACT, REQUEST_BYTES, RESULT_BYTES, ServerCfg, ServeStats, check, lib

REQ_DTYPE = np.dtype([("arrival_s", "<f8"), ("cover_off", "<u8"), ("n", "<u8"), ("msg_off", "<u8"),
                      ("len", "<u4"), ("k", "u1"), ("op", "u1"), ("reserved", "<u2"), ("target", "<i8")])
RES_DTYPE = np.dtype([("admit_s", "<f8"), ("launch_s", "<f8"), ("done_s", "<f8"), ("out_off", "<u8"),
                      ("status", "<i4"), ("len", "<u4"), ("target", "<i8"), ("op_run", "u1"), ("k", "u1"),
                      ("reserved", "u1", (6,))])
assert REQ_DTYPE.itemsize == REQUEST_BYTES and RES_DTYPE.itemsize == RESULT_BYTES
FREED = np.iinfo(np.uint64).max


def poisson_requests(workload, rate: float, count: int, seed: int = 501, extract_frac: float = 0.5):
    """Open-loop stream: Poisson arrivals at ``rate`` req/s; each request
    picks a cover of the pool uniformly; embed or extract with probability
    1 - extract_frac / extract_frac (an extract reads the oldest resident
    stego buffer, or is served as an embed when there is none)."""
    g = inputs.rng(seed, int(rate), count)
    req = np.zeros(count, dtype=REQ_DTYPE)
    req["arrival_s"] = inputs.poisson_arrivals(rate, count, seed)
    ids = g.integers(0, workload.count, size=count)
    req["cover_off"] = workload.cover_off[ids]
    req["n"] = workload.n[ids]
    req["msg_off"] = workload.msg_off[ids]
    req["len"] = workload.len[ids]
    req["k"] = workload.k[ids]
    req["op"] = np.where(g.random(count) < extract_frac, OP_EXTRACT, OP_EMBED)
    req["target"] = -1
    return req, ids


def serve(arena: torch.Tensor, cover_pool: torch.Tensor, msg_pool: torch.Tensor, requests: np.ndarray,
          max_batch: int = 256, n_slots: int = 4, keep_outputs: bool = False):
    """Run the serving loop over ``requests`` on the current device.
    Returns (results structured array, stats dict)."""
    requests = np.ascontiguousarray(requests, dtype=REQ_DTYPE)
    results = np.zeros(requests.size, dtype=RES_DTYPE)
    for name, t in (("arena", arena), ("cover_pool", cover_pool), ("msg_pool", msg_pool)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 or not t.is_contiguous():
            raise TypeError("%s must be a contiguous torch.uint8 device tensor" % name)
        if t.device.index != torch.cuda.current_device():
            raise ValueError("%s is on %s but the current device is cuda:%d" % (name, t.device,
                                                                                torch.cuda.current_device()))
    # any request may run as an embed (an extract with nothing resident does),
    # so every request's cover and message must lie inside the pools
    if requests.size:
        if int((requests["cover_off"] + requests["n"]).max()) > cover_pool.numel() or \
                max(int(requests["cover_off"].max()), int(requests["n"].max())) >= 1 << 62:
            raise ValueError("a request's cover lies outside cover_pool")
        if int((requests["msg_off"] + requests["len"]).max()) > msg_pool.numel() or \
                int(requests["msg_off"].max()) >= 1 << 62:
            raise ValueError("a request's message lies outside msg_pool")
    cfg = ServerCfg(arena.data_ptr(), arena.numel(), cover_pool.data_ptr(), msg_pool.data_ptr(),
                    int(max_batch), int(n_slots), int(bool(keep_outputs)), 0)
    stats = ServeStats()
    torch.cuda.synchronize()
    check(lib().lsb_serve(ctypes.byref(cfg), ctypes.c_void_p(requests.ctypes.data), int(requests.size),
                          ctypes.c_void_p(results.ctypes.data), ctypes.byref(stats)))
    return results, stats.as_dict()


def simulate(requests: np.ndarray, budget: int, max_batch: int = 256, n_slots: int = 4,
             keep_outputs: bool = False, launch_us: float = 10.0, device_gbps: float = 5000.0):
    """Run the serving scheduler on the host with modelled launches (no GPU,
    no data): each launch takes launch_us plus its algorithmic bytes at
    device_gbps.  Returns (results, stats) like serve()."""
    requests = np.ascontiguousarray(requests, dtype=REQ_DTYPE)
    results = np.zeros(requests.size, dtype=RES_DTYPE)
    cfg = ServerCfg(None, int(budget), None, None, int(max_batch), int(n_slots), int(bool(keep_outputs)), 0)
    stats = ServeStats()
    check(lib().lsb_serve_simulate(ctypes.byref(cfg), ctypes.c_void_p(requests.ctypes.data), int(requests.size),
                                   ctypes.c_void_p(results.ctypes.data), ctypes.byref(stats),
                                   float(launch_us), float(device_gbps)))
    return results, stats.as_dict()


__all__ = ["REQ_DTYPE", "RES_DTYPE", "FREED", "poisson_requests", "serve", "simulate"]
