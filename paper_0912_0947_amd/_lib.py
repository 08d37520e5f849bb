"""ctypes binding of liblsb.so (argument marshalling only).

Every entry point of ``include/lsb.h`` is declared here with its C types.
Loading fails loudly if the library has not been built: there is no CPU
fallback for any operation.
"""
from __future__ import annotations

import ctypes
import numbers
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsb.so")

OK = 0
E_ARG = -1
E_CAPACITY = -2
E_HEADER = -3
E_BUFFER = -4
E_HIP = -5
E_NOMEM = -6
OP_EMBED = 0
OP_EXTRACT = 1
OP_MIXED = 2
JOB_RAW = 1  # lsb_job.flags: raw slice, no header
STATIC_MAX_JOBS = 4096  # LSB_STATIC_MAX_JOBS
REF_COPY, REF_EMBED_MIX, REF_EXTRACT_MIX = 0, 1, 2

ERROR_NAMES = {
    OK: "LSB_OK", E_ARG: "LSB_E_ARG", E_CAPACITY: "LSB_E_CAPACITY", E_HEADER: "LSB_E_HEADER",
    E_BUFFER: "LSB_E_BUFFER", E_HIP: "LSB_E_HIP", E_NOMEM: "LSB_E_NOMEM",
}


class LaunchCfg(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("pack", ctypes.c_int32), ("order", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("cover_off", ctypes.c_uint64), ("stego_off", ctypes.c_uint64),
                ("msg_off", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("msg_cap", ctypes.c_uint64), ("t0", ctypes.c_uint64), ("stream_bits", ctypes.c_uint64),
                ("len", ctypes.c_uint32), ("k", ctypes.c_uint8), ("op", ctypes.c_uint8),
                ("flags", ctypes.c_uint8), ("reserved", ctypes.c_uint8)]


assert ctypes.sizeof(Job) == 64


class ServerCfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64),
                ("cover_pool", ctypes.c_void_p), ("msg_pool", ctypes.c_void_p),
                ("max_batch", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("keep_outputs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("makespan_s", ctypes.c_double), ("bytes", ctypes.c_double), ("gbps", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("launches", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("admission_stalls", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("peak_arena_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


assert ctypes.sizeof(ServerCfg) == 48 and ctypes.sizeof(ServeStats) == 104
REQUEST_BYTES = 48
RESULT_BYTES = 56

_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_I = ctypes.c_int

SIGNATURES = {
    "lsb_capacity": (_I64, [_U64, _I]),
    "lsb_embed": (_I, [_P, _P, _U64, _P, _U32, _I, _P]),
    "lsb_extract": (_I, [_P, _U64, _I, _P, _U64, _P, _P, _P]),
    "lsb_extract_sync": (_I, [_P, _U64, _I, _P, _U64, ctypes.POINTER(_U32), _P]),
    "lsb_embed_raw": (_I, [_P, _P, _U64, _U64, _P, _U64, _I, _P]),
    "lsb_extract_raw": (_I, [_P, _U64, _U64, _P, _U64, _I, _P]),
    "lsb_paper_capacity": (_I64, [_U32, _U32]),
    "lsb_paper_embed": (_I, [_P, _P, _U32, _U32, _U32, _U32, _P, _U64, _P]),
    "lsb_paper_extract": (_I, [_P, _U32, _U32, _U32, _U32, _P, _U64, _P]),
    "lsb_embed_plane": (_I, [_P, _P, _U64, _U32, _U32, _P, _U32, _I, _P]),
    "lsb_extract_plane": (_I, [_P, _U64, _U32, _U32, _I, _P, _U64, _P, _P, _P]),
    "lsb_sse": (_I, [_P, _P, _U64, _P, _P]),
    "lsb_video_embed_host": (_I, [_P, _P, _U64, _U64, _P, _U64, _I, _P, _U32, ctypes.POINTER(_P), _I]),
    "lsb_verify": (_I, [_P, _P, _U64, _P, _U32, _I, _P, _P]),
    "lsb_embed_verify": (_I, [_P, _P, _U64, _P, _U32, _I, _P, _P]),
    "lsb_plan_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(Job), _I, _I]),
    "lsb_plan_update": (_I, [_P, ctypes.POINTER(Job), _I]),
    "lsb_plan_run": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "lsb_embed_batch": (_I, [_P, _P, _P, _P, _P, _P]),
    "lsb_extract_batch": (_I, [_P, _P, _P, _P, _P, _P]),
    "lsb_plan_tiles": (_I64, [_P]),
    "lsb_batch_run_static": (_I, [ctypes.POINTER(Job), _I, _I, _P, _P, _P, _P, _P, _P]),
    "lsb_job_extents": (_I, [ctypes.POINTER(Job), _I, _I, ctypes.POINTER(_U64)]),
    "lsb_slice_stream_bytes": (_I64, [_I, _U64, _U64, _U64]),
    "lsb_plan_destroy": (None, [_P]),
    "lsb_tune_get": (_I, [_I, _I, _U64, ctypes.POINTER(LaunchCfg)]),
    "lsb_tune_set": (_I, [_I, _I, _I, ctypes.POINTER(LaunchCfg)]),
    "lsb_autotune": (_I, [_I, _I, _U64, _P, _P, _P, _I, ctypes.POINTER(LaunchCfg),
                          ctypes.POINTER(ctypes.c_double), _P]),
    "lsb_batch_tune_get": (_I, [ctypes.POINTER(LaunchCfg), ctypes.POINTER(_I64)]),
    "lsb_batch_tune_set": (_I, [ctypes.POINTER(LaunchCfg), _I64]),
    "lsb_batch_tune_get_op": (_I, [_I, ctypes.POINTER(LaunchCfg)]),
    "lsb_batch_tune_set_op": (_I, [_I, ctypes.POINTER(LaunchCfg)]),
    "lsb_serve": (_I, [ctypes.POINTER(ServerCfg), _P, _I, _P, ctypes.POINTER(ServeStats)]),
    "lsb_serve_simulate": (_I, [ctypes.POINTER(ServerCfg), _P, _I, _P, ctypes.POINTER(ServeStats),
                                ctypes.c_double, ctypes.c_double]),
    "lsb_time_next_launch": (_I, [_P, _P]),
    "lsb_stream_reference": (_I, [_I, _I, _P, _P, _P, _U64, _I, _I, _U32, _P]),
    "lsb_roundtrip_latency": (_I, [_P, _P, _U64, _P, _U32, _I, _P, _I, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), _P]),
    "lsb_last_error": (ctypes.c_char_p, []),
    "lsb_version": (ctypes.c_char_p, []),
}

def _range_checked(base, bits: int, signed: bool):
    """An argument type that refuses integers outside ``base``'s range
    instead of letting ctypes wrap them (a 2**32 + 5 byte length would
    otherwise reach the library as 5)."""
    lo, hi = (-(1 << (bits - 1)), (1 << (bits - 1)) - 1) if signed else (0, (1 << bits) - 1)

    class Checked(base):
        @classmethod
        def from_param(cls, v):
            if isinstance(v, numbers.Integral) and not isinstance(v, bool):
                v = int(v)
                if not lo <= v <= hi:
                    raise OverflowError("%d is outside the range of %s" % (v, base.__name__))
                return base(v)
            return base.from_param(v)

    Checked.__name__ = base.__name__
    return Checked


_CHECKED = {_U64: _range_checked(_U64, 64, False), _I64: _range_checked(_I64, 64, True),
            _U32: _range_checked(_U32, 32, False), _I: _range_checked(_I, 32, True)}

_lock = threading.Lock()
_lib = None


class LsbError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, message))


def lib():
    """The loaded liblsb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(
                        "liblsb.so is not built (%s); run `python -m paper_0912_0947_amd.build` "
                        "or __graft_entry__.build() -- there is no CPU fallback" % LIB_PATH)
                handle = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(handle, name)
                    fn.restype = res
                    fn.argtypes = [_CHECKED.get(a, a) for a in args]
                from . import tune
                tune.load(handle)  # stored launch configurations, if any
                _lib = handle
    return _lib


def check(rc: int) -> int:
    """Raise LsbError for a negative return code."""
    if rc < 0:
        raise LsbError(rc, lib().lsb_last_error().decode(errors="replace"))
    return rc
