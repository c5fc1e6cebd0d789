"""Python binding of ``libtdct.so``, the MI355X (gfx950) block codec built on
the 14-addition approximate DCT of Bayer and Cintra.

Argument marshalling only: every function here has the name of a C-ABI
entry point declared in ``include/tdct.h`` and forwards to it, turning torch
tensors into device pointers and torch streams into ``hipStream_t`` handles.
All computation happens in the HIP library; if it is not built, importing
this package raises. PyTorch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtdct.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("paper_1702_00817_amd: %s is not built; run __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950)" % LIB_PATH)

# torch ships its own HIP runtime (SONAME libamdhip64.so.7, requested by
# torch under another name). Loading torch first makes libtdct.so bind to that
# same runtime instead of pulling a second one into the process, so tensors,
# streams and kernels all live in one HIP context.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

TDCT_OK, TDCT_EINVAL, TDCT_EDIM, TDCT_EQTAB = 0, -1, -2, -3
TDCT_ENOMEM, TDCT_EDEVICE, TDCT_EBUSY, TDCT_ENOTFOUND = -4, -5, -6, -7
OP_ENCODE, OP_DECODE, OP_ROUNDTRIP, OP_ENCODE_I8ZZ, OP_FORWARD = 0, 1, 2, 3, 4


class TdctError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.tdct_strerror(status).decode()
        if status == TDCT_EDEVICE:
            msg += " (" + _lib.tdct_last_error().decode() + ")"
        super().__init__("%s: %s [%d]" % (where, msg, status))
        self.status = status


class tdct_qtable(ctypes.Structure):
    _fields_ = [("q", ctypes.c_uint16 * 64)]


class tdct_image_desc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("qtab", ctypes.c_int32), ("keep", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("src", ctypes.c_void_p), ("src_stride", ctypes.c_int64),
                ("coef", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("dst_stride", ctypes.c_int64)]


class tdct_tune(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32),
                ("tile_waves", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("pixel_cache", ctypes.c_int32)]

    def as_dict(self):
        return {"waves_per_group": self.waves_per_group, "groups_per_cu": self.groups_per_cu,
                "tile_waves": self.tile_waves, "xcd_remap": self.xcd_remap,
                "pixel_cache": self.pixel_cache}


class tdct_plan_info(ctypes.Structure):
    _fields_ = [("images", ctypes.c_int64), ("blocks", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("pixels", ctypes.c_int64), ("table_bytes", ctypes.c_int64), ("tune", tdct_tune)]


class tdct_server_cfg(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_wait_us", ctypes.c_int32),
                ("batching", ctypes.c_int32), ("max_batch_px", ctypes.c_int64), ("tune", tdct_tune),
                ("fake_device_us", ctypes.c_int32), ("fake_fail_every", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("resident_workers", ctypes.c_int32),
                ("resident_idle_us", ctypes.c_int32), ("resident_jobs", ctypes.c_int32),
                ("resident_tiles", ctypes.c_int32), ("resident_reserved", ctypes.c_int32),
                ("tune_cache", ctypes.c_int32), ("idle_poll_us", ctypes.c_int32)]


class tdct_tune_cache_stats(ctypes.Structure):
    _fields_ = [("on", ctypes.c_int32), ("reserved", ctypes.c_int32), ("entries", ctypes.c_int64),
                ("hits", ctypes.c_int64), ("misses", ctypes.c_int64), ("stores", ctypes.c_int64),
                ("write_errors", ctypes.c_int64), ("batch_hits", ctypes.c_int64),
                ("batch_misses", ctypes.c_int64)]


class tdct_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("input", ctypes.c_void_p), ("in_stride", ctypes.c_int64),
                ("Q", tdct_qtable), ("host_io", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("host_output", ctypes.c_void_p)]


class tdct_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("output", ctypes.c_void_p), ("output_bytes", ctypes.c_int64),
                ("submit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class tdct_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("pixels_done", ctypes.c_int64),
                ("arena_bytes_in_use", ctypes.c_int64), ("arena_high_water", ctypes.c_int64),
                ("busy_us", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("p999_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("mean_batch", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_PQ = ctypes.POINTER(tdct_qtable)
_SIG = {
    "tdct_forward": [_P, _i64, _i32, _i32, _P, _P],
    "tdct_quantise": [_P, _i64, _i32, _i32, _PQ, _i32, _P, _P],
    "tdct_inverse": [_P, _PQ, _i32, _i32, _P, _i64, _P],
    "tdct_roundtrip": [_P, _i64, _i32, _i32, _PQ, _i32, _P, _P, _i64, _P],
    "tdct_quantise_i8_zigzag": [_P, _i64, _i32, _i32, _PQ, _P, _P],
    "tdct_sse": [_P, _i64, _P, _i64, _i32, _i32, _P, _P],
    "tdct_stream_probe": [_i32, _P, _P, _i64, _P],
    "tdct_batch_plan": [ctypes.POINTER(tdct_image_desc), _i32, _PQ, _i32,
                        ctypes.POINTER(tdct_tune), ctypes.POINTER(_P)],
    "tdct_batch_run": [_P, _P],
    "tdct_batch_graph": [_P, _P],
    "tdct_autotune": [_P, _P, _i32, ctypes.POINTER(tdct_tune)],
    "tdct_plan_info_get": [_P, ctypes.POINTER(tdct_plan_info)],
    "tdct_tune_cache_open": [ctypes.c_char_p],
    "tdct_tune_cache_info": [ctypes.POINTER(tdct_tune_cache_stats)],
    "tdct_run_per_image": [ctypes.POINTER(tdct_image_desc), _i32, _PQ, _i32, _P],
    "tdct_batch_run_static": [ctypes.POINTER(tdct_image_desc), _i32, _PQ, _i32,
                              ctypes.POINTER(tdct_tune), _P],
    "tdct_server_create": [ctypes.POINTER(tdct_server_cfg), ctypes.POINTER(_P)],
    "tdct_server_submit": [_P, ctypes.POINTER(tdct_request), ctypes.POINTER(ctypes.c_uint64)],
    "tdct_server_poll": [_P, ctypes.c_uint64, ctypes.POINTER(tdct_result)],
    "tdct_server_wait": [_P, ctypes.c_uint64, ctypes.POINTER(tdct_result)],
    "tdct_server_release": [_P, ctypes.c_uint64],
    "tdct_server_drain": [_P],
    "tdct_server_stats": [_P, ctypes.POINTER(tdct_stats)],
    "tdct_server_replay": [_P, ctypes.POINTER(tdct_request), ctypes.POINTER(ctypes.c_double), _i32,
                           _i32, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
}
for _name, _args in _SIG.items():
    getattr(_lib, _name).argtypes = _args
    getattr(_lib, _name).restype = ctypes.c_int
_lib.tdct_log_level.argtypes = [ctypes.c_int]
_lib.tdct_log_level.restype = ctypes.c_int
_lib.tdct_strerror.argtypes = [ctypes.c_int]
_lib.tdct_strerror.restype = ctypes.c_char_p
_lib.tdct_last_error.restype = ctypes.c_char_p
_lib.tdct_plan_free.argtypes = [_P]
_lib.tdct_plan_free.restype = None
_lib.tdct_server_destroy.argtypes = [_P]
_lib.tdct_server_destroy.restype = None
_lib.tdct_server_last_error.argtypes = [_P]
_lib.tdct_server_last_error.restype = ctypes.c_char_p


def lib():
    return _lib


# ---- marshalling helpers -------------------------------------------------

def _ptr(x):
    """Device pointer of a torch tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    """hipStream_t of a torch stream (None: torch's current stream)."""
    if isinstance(s, int):
        return s
    import torch
    if s is None:
        s = torch.cuda.current_stream()
    return s.cuda_stream


def qtable(Q) -> tdct_qtable:
    if isinstance(Q, tdct_qtable):
        return Q
    import numpy as np
    a = np.asarray(Q).reshape(-1)
    if a.size != 64:
        raise ValueError("a quantisation table has 64 entries")
    t = tdct_qtable()
    for k in range(64):
        t.q[k] = int(a[k])
    return t


def _check(st, where):
    if st != TDCT_OK:
        raise TdctError(st, where)


def _qref(Q):
    return ctypes.byref(qtable(Q)) if Q is not None else None


# ---- plain calls -----------------------------------------------------------

def tdct_forward(src, src_stride, w, h, coef, stream=None):
    _check(_lib.tdct_forward(_ptr(src), src_stride, w, h, _ptr(coef), _stream(stream)),
           "tdct_forward")


def tdct_quantise(src, src_stride, w, h, Q, keep, q, stream=None):
    _check(_lib.tdct_quantise(_ptr(src), src_stride, w, h, _qref(Q), keep, _ptr(q),
                              _stream(stream)), "tdct_quantise")


def tdct_inverse(q, Q, w, h, dst, dst_stride, stream=None):
    _check(_lib.tdct_inverse(_ptr(q), _qref(Q), w, h, _ptr(dst), dst_stride, _stream(stream)),
           "tdct_inverse")


def tdct_roundtrip(src, src_stride, w, h, Q, keep, q_or_null, dst, dst_stride, stream=None):
    _check(_lib.tdct_roundtrip(_ptr(src), src_stride, w, h, _qref(Q), keep, _ptr(q_or_null),
                               _ptr(dst), dst_stride, _stream(stream)), "tdct_roundtrip")


def tdct_quantise_i8_zigzag(src, src_stride, w, h, Q, out, stream=None):
    _check(_lib.tdct_quantise_i8_zigzag(_ptr(src), src_stride, w, h, _qref(Q), _ptr(out),
                                        _stream(stream)), "tdct_quantise_i8_zigzag")


def tdct_sse(a, a_stride, b, b_stride, w, h, sse_dev, stream=None):
    _check(_lib.tdct_sse(_ptr(a), a_stride, _ptr(b), b_stride, w, h, _ptr(sse_dev),
                         _stream(stream)), "tdct_sse")


PROBE_COPY, PROBE_READ, PROBE_WRITE, PROBE_R1W2, PROBE_R2W1, PROBE_R1W3 = 0, 1, 2, 3, 4, 5


def tdct_stream_probe(kind, src, dst, units, stream=None):
    _check(_lib.tdct_stream_probe(kind, _ptr(src), _ptr(dst), units, _stream(stream)),
           "tdct_stream_probe")


def tdct_strerror(status: int) -> str:
    return _lib.tdct_strerror(status).decode()


def tdct_last_error() -> str:
    return _lib.tdct_last_error().decode()


# ---- batch form --------------------------------------------------------------

def image_desc(op, w, h, qtab=0, keep=64, src=None, src_stride=0, coef=None, dst=None,
               dst_stride=0) -> tdct_image_desc:
    d = tdct_image_desc()
    d.op, d.w, d.h, d.qtab, d.keep = op, w, h, qtab, keep
    d.src, d.src_stride = _ptr(src), src_stride
    d.coef = _ptr(coef)
    d.dst, d.dst_stride = _ptr(dst), dst_stride
    return d


def _desc_array(descs):
    arr = (tdct_image_desc * max(1, len(descs)))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def _q_array(qtabs):
    arr = (tdct_qtable * max(1, len(qtabs)))()
    for i, q in enumerate(qtabs):
        arr[i] = qtable(q)
    return arr


def tdct_batch_plan(descs, qtabs, tune=None):
    """Returns an opaque plan handle (int)."""
    da, qa = _desc_array(descs), _q_array(qtabs)
    t = None
    if tune is not None:
        t = tdct_tune(**tune) if isinstance(tune, dict) else tune
    h = ctypes.c_void_p()
    _check(_lib.tdct_batch_plan(da, len(descs), qa, len(qtabs),
                                ctypes.byref(t) if t is not None else None, ctypes.byref(h)),
           "tdct_batch_plan")
    return h.value


def tdct_batch_run(plan, stream=None):
    _check(_lib.tdct_batch_run(plan, _stream(stream)), "tdct_batch_run")


def tdct_batch_graph(plan, stream=None):
    _check(_lib.tdct_batch_graph(plan, _stream(stream)), "tdct_batch_graph")


def tdct_autotune(plan, stream=None, reps=3) -> dict:
    t = tdct_tune()
    _check(_lib.tdct_autotune(plan, _stream(stream), reps, ctypes.byref(t)), "tdct_autotune")
    return t.as_dict()


def tdct_log_level(level=-1) -> int:
    """Sets the library's diagnostic level on stderr (0 silent .. 3 every
    server batch) when level >= 0; returns the previous level."""
    return _lib.tdct_log_level(level)


def tdct_tune_cache_open(path):
    """Opens the autotune cache file at `path` (None or "": cache off)."""
    _check(_lib.tdct_tune_cache_open(os.fsencode(path) if path else None), "tdct_tune_cache_open")


def tdct_tune_cache_info() -> dict:
    st = tdct_tune_cache_stats()
    _check(_lib.tdct_tune_cache_info(ctypes.byref(st)), "tdct_tune_cache_info")
    return {k: getattr(st, k) for k in ("on", "entries", "hits", "misses", "stores", "write_errors",
                                        "batch_hits", "batch_misses")}


def tdct_plan_info_get(plan) -> dict:
    i = tdct_plan_info()
    _check(_lib.tdct_plan_info_get(plan, ctypes.byref(i)), "tdct_plan_info_get")
    return {"images": i.images, "blocks": i.blocks, "tiles": i.tiles, "pixels": i.pixels,
            "table_bytes": i.table_bytes, "tune": i.tune.as_dict()}


def tdct_plan_free(plan):
    _lib.tdct_plan_free(plan)


def tdct_run_per_image(descs, qtabs, stream=None):
    da, qa = _desc_array(descs), _q_array(qtabs)
    _check(_lib.tdct_run_per_image(da, len(descs), qa, len(qtabs), _stream(stream)),
           "tdct_run_per_image")


def tdct_batch_run_static(descs, qtabs, tune=None, stream=None):
    da, qa = _desc_array(descs), _q_array(qtabs)
    t = None
    if tune is not None:
        t = tdct_tune(**tune) if isinstance(tune, dict) else tune
    _check(_lib.tdct_batch_run_static(da, len(descs), qa, len(qtabs),
                                      ctypes.byref(t) if t is not None else None, _stream(stream)),
           "tdct_batch_run_static")


# ---- serving form ------------------------------------------------------------

def server_cfg(budget_bytes, streams=4, max_batch=64, max_wait_us=0, batching=1, tune=None,
               fake_device_us=0, fake_fail_every=0, max_batch_px=0, resident=0, resident_workers=0,
               resident_idle_us=0, resident_jobs=0, resident_tiles=0, tune_cache=0,
               idle_poll_us=0) -> tdct_server_cfg:
    c = tdct_server_cfg()
    c.budget_bytes, c.streams, c.max_batch = budget_bytes, streams, max_batch
    c.max_wait_us, c.batching, c.max_batch_px = max_wait_us, batching, max_batch_px
    if tune:
        c.tune = tdct_tune(**tune)
    c.fake_device_us, c.fake_fail_every = fake_device_us, fake_fail_every
    c.resident, c.resident_workers, c.resident_idle_us = resident, resident_workers, resident_idle_us
    c.resident_jobs, c.resident_tiles = resident_jobs, resident_tiles
    c.tune_cache, c.idle_poll_us = tune_cache, idle_poll_us
    return c


def request(op, w, h, inp, Q, keep=64, in_stride=None, host_output=None) -> tdct_request:
    """A serving request; with host_output given, input and output are pinned
    host buffers (host_io)."""
    r = tdct_request()
    r.op, r.w, r.h, r.keep = op, w, h, keep
    r.input = _ptr(inp)
    r.in_stride = w if in_stride is None else in_stride
    r.Q = qtable(Q)
    if host_output is not None:
        r.host_io = 1
        r.host_output = _ptr(host_output)
    return r


def tdct_server_create(cfg: tdct_server_cfg):
    h = ctypes.c_void_p()
    _check(_lib.tdct_server_create(ctypes.byref(cfg), ctypes.byref(h)), "tdct_server_create")
    return h.value


def tdct_server_submit(server, req: tdct_request) -> int:
    t = ctypes.c_uint64()
    _check(_lib.tdct_server_submit(server, ctypes.byref(req), ctypes.byref(t)),
           "tdct_server_submit")
    return t.value


def tdct_server_poll(server, ticket) -> tdct_result:
    r = tdct_result()
    _check(_lib.tdct_server_poll(server, ticket, ctypes.byref(r)), "tdct_server_poll")
    return r


def tdct_server_wait(server, ticket) -> tdct_result:
    r = tdct_result()
    _check(_lib.tdct_server_wait(server, ticket, ctypes.byref(r)), "tdct_server_wait")
    return r


def tdct_server_release(server, ticket):
    _check(_lib.tdct_server_release(server, ticket), "tdct_server_release")


def tdct_server_drain(server):
    _check(_lib.tdct_server_drain(server), "tdct_server_drain")


def tdct_server_stats(server) -> dict:
    s = tdct_stats()
    _check(_lib.tdct_server_stats(server, ctypes.byref(s)), "tdct_server_stats")
    return s.as_dict()


def tdct_server_last_error(server) -> str:
    return _lib.tdct_server_last_error(server).decode()


def tdct_server_destroy(server):
    _lib.tdct_server_destroy(server)


def request_array(n):
    """A ctypes array of n requests (filled by the caller)."""
    return (tdct_request * n)()


def tdct_server_replay(server, reqs, arrival_us, keep_outputs=False, with_batch=False):
    """Returns (tickets, latency_us, status) as lists, and the batch sizes as
    a fourth list when with_batch. `reqs` is a sequence of tdct_request or an
    array made by request_array."""
    n = len(reqs)
    if isinstance(reqs, ctypes.Array):
        ra = reqs
    else:
        ra = request_array(n)
        for i, r in enumerate(reqs):
            ra[i] = r
    at = (ctypes.c_double * max(1, n))(*arrival_us)
    tk = (ctypes.c_uint64 * max(1, n))()
    lat = (ctypes.c_double * max(1, n))()
    st = (ctypes.c_int32 * max(1, n))()
    bs = (ctypes.c_int32 * max(1, n))()
    _check(_lib.tdct_server_replay(server, ra, at, n, int(keep_outputs), tk, lat, st, bs),
           "tdct_server_replay")
    out = (list(tk)[:n], list(lat)[:n], list(st)[:n])
    return out + (list(bs)[:n],) if with_batch else out
