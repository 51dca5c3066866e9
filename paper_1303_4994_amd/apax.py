"""Python binding of libapax.so (argument marshalling only).

Names follow the C ABI in include/apax.h.  Arrays are torch tensors on the
GPU; every call runs on the current torch stream unless one is given.  The
compute runs in the HIP library: if libapax.so is missing this module raises
at import time -- there is no CPU fallback.

Parameters are dicts:
    {"mode": "lossless" | "fixed_rate" | "fixed_quality" | "adaptive_rate",
     "brick": (..), "stream_mask": 0, "rate": 4.0, "target_corr": 0.99999,
     "code": 0}
dtype and dims come from the tensor.
"""
from __future__ import annotations

import ctypes as C
import os
import struct

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapax.so")

I8, I16, I32, F32, F64 = 1, 2, 3, 4, 5
LOSSLESS, FIXED_RATE, FIXED_QUALITY, ADAPTIVE_RATE = 0, 1, 2, 3
OK, E_INVALID, E_UNSUPPORTED, E_CAPACITY, E_CORRUPT, E_NONFINITE, E_HIP, E_INTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7
NEAR_TIE = 1
NCURVE = 17
FLAG_LAGGED = 1  # apax_params.flags: lagged stream choice (lossless)
CODE_PROFILED = -(1 << 31)  # apax_encode: adopt the code and mask of the profile in ws

_DT = {torch.int8: I8, torch.int16: I16, torch.int32: I32, torch.float32: F32,
       torch.float64: F64}
_TORCH_OF = {v: k for k, v in _DT.items()}
_MODES = {"lossless": LOSSLESS, "fixed_rate": FIXED_RATE, "fixed_quality": FIXED_QUALITY,
          "adaptive_rate": ADAPTIVE_RATE}


class ApaxError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {code} ({_errstr(code)})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("dtype", C.c_uint32), ("ndim", C.c_uint32),
                ("mode", C.c_uint32), ("dims", C.c_uint64 * 3), ("brick", C.c_uint32 * 3),
                ("stream_mask", C.c_uint32), ("rate", C.c_double),
                ("target_corr", C.c_double), ("code", C.c_int32), ("flags", C.c_uint32)]


class Metrics(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "r", "one_minus_r", "snr_db", "rms_pct", "rms_db", "mean_x", "mean_y", "mean_d",
        "std_x", "std_y", "std_d", "max_abs_d", "sxx", "syy", "sdd", "sds", "sum_x",
        "sum_y", "sum_d", "ratio")] + [("n", C.c_uint64), ("enc_bytes", C.c_uint64)]


class CurvePoint(C.Structure):
    _fields_ = [("code", C.c_int32), ("pad", C.c_int32), ("ratio", C.c_double),
                ("r", C.c_double)]


class ProfileResult(C.Structure):
    _fields_ = [("size", C.c_uint32), ("code", C.c_int32), ("stream_mask", C.c_uint32),
                ("flags", C.c_uint32), ("c_floor", C.c_int32), ("c_cap", C.c_int32),
                ("n_sub", C.c_uint32), ("n_probes", C.c_uint32),
                ("curve", CurvePoint * NCURVE), ("m", Metrics)]


class BatchItem(C.Structure):
    _fields_ = [("p", Params), ("d_in", C.c_void_p), ("d_out", C.c_void_p),
                ("in_bytes", C.c_uint64), ("cap", C.c_uint64), ("d_nbytes", C.c_void_p),
                ("h_hdr", C.c_void_p)]


REQ_AFTER = 1


class Request(C.Structure):
    _fields_ = [("op", C.c_int32), ("flags", C.c_uint32), ("item", BatchItem), ("tag", C.c_uint64),
                ("after", C.c_void_p)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int32), ("slot", C.c_uint32),
                ("latency_s", C.c_double)]


class Tune(C.Structure):
    _fields_ = [("waves_per_wg", C.c_uint32), ("wgs_per_cu", C.c_uint32),
                ("tiles_per_ticket", C.c_uint32), ("reserved", C.c_uint32)]


OP_ENCODE, OP_DECODE = 0, 1


class Spectral(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("peak_x", "floor_x", "peak_y", "floor_y", "peak_d", "floor_d",
                                           "resid_mean", "dr", "srr", "fft_s2r_margin")] + \
               [("segments", C.c_uint64)]


class Monitor(C.Structure):
    _fields_ = [("acf", C.c_double * 17)] + \
               [(f, C.c_double) for f in ("center_freq", "peak_db", "floor_db", "snr_db", "gain_db")] + \
               [(f, C.c_int32) for f in ("peak_bin", "stride", "sign", "pad")] + [("segments", C.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, P, u64 = C.c_void_p, C.POINTER, C.c_uint64
    L.apax_encode_bound.argtypes = [P(Params), P(u64)]
    L.apax_workspace_size.argtypes = [P(Params), P(u64)]
    L.apax_profile.argtypes = [vp, P(Params), P(ProfileResult), vp, u64, vp]
    L.apax_profile_async.argtypes = [vp, P(Params), vp, u64, vp]
    L.apax_profile_async_point.argtypes = [vp, P(Params), vp, u64, vp, vp]
    L.apax_adopt_point.argtypes = [vp, vp, vp]
    L.apax_profile_encode_async.argtypes = [vp, P(Params), vp, u64, vp, u64, vp, vp, vp, vp, vp]
    L.apax_s2r_margin.argtypes = [vp, P(Params), P(C.c_double), P(C.c_double), vp, u64, vp]
    L.apax_decode_dot.argtypes = [vp, vp, u64, vp, vp, vp, u64, vp]
    L.apax_dot.argtypes = [vp, vp, C.c_uint32, u64, vp, vp, u64, vp]
    L.apax_spectral_workspace_bytes.argtypes = []
    L.apax_spectral_workspace_bytes.restype = u64
    L.apax_spectral_metrics.argtypes = [vp, vp, C.c_uint32, u64, P(Spectral), vp, u64, vp]
    L.apax_signal_monitor.argtypes = [vp, C.c_uint32, u64, P(Monitor), vp, u64, vp]
    L.apax_profile_timed.argtypes = [vp, P(Params), P(ProfileResult), P(C.c_float), vp, u64, vp]
    L.apax_profile_encode_timed.argtypes = [vp, P(Params), P(ProfileResult), P(C.c_float), vp, u64, vp, u64,
                                            vp, vp]
    L.apax_profile_read.argtypes = [P(Params), P(ProfileResult), vp, vp]
    L.apax_encode.argtypes = [vp, P(Params), vp, u64, vp, vp, u64, vp]
    L.apax_encode_noalloc.argtypes = [vp, P(Params), vp, u64, vp, vp, vp]
    L.apax_decode.argtypes = [vp, vp, u64, vp, u64, vp, u64, vp]
    L.apax_stream_info.argtypes = [vp, u64, P(Params)]
    L.apax_stream_size.argtypes = [vp, u64, P(u64)]
    L.apax_status_clear.argtypes = [vp, vp]
    L.apax_status.argtypes = [vp, vp]
    L.apax_batch_create.argtypes = [C.c_int, P(BatchItem), C.c_uint32, P(Tune), P(vp), P(u64)]
    L.apax_batch_upload.argtypes = [vp, vp, u64, vp]
    L.apax_batch_run.argtypes = [vp, vp]
    L.apax_batch_capture.argtypes = [vp]
    L.apax_batch_launch.argtypes = [vp, vp]
    L.apax_batch_destroy.argtypes = [vp]
    L.apax_server_create.argtypes = [u64, C.c_uint32, C.c_uint32, u64, P(Tune), P(vp)]
    L.apax_server_submit.argtypes = [vp, P(Request), P(u64)]
    L.apax_server_poll.argtypes = [vp, P(Completion), C.c_uint32, P(C.c_uint32)]
    L.apax_server_stats.argtypes = [vp, P(u64), P(u64), P(u64)]
    L.apax_server_destroy.argtypes = [vp]
    L.apax_server_destroy.restype = None
    L.apax_batch_destroy.restype = None
    L.apax_strerror.argtypes = [C.c_int]
    L.apax_strerror.restype = C.c_char_p
    return L


lib = _load()


def _errstr(code):
    return lib.apax_strerror(int(code)).decode()


def _check(rc, what):
    if rc != 0:
        raise ApaxError(rc, what)


_PCACHE: dict = {}


def make_params(dtype: torch.dtype, shape, params: dict) -> Params:
    """apax_params for (dtype, shape, params); marshalled structs are cached
    (callers never modify them)."""
    try:
        key = (dtype, tuple(shape), tuple(sorted((k, tuple(v) if isinstance(v, (list, tuple)) else v)
                                                  for k, v in params.items())))
        hit = _PCACHE.get(key)
    except TypeError:
        key, hit = None, None
    if hit is not None:
        return hit
    p = _make_params(dtype, shape, params)
    if key is not None:
        if len(_PCACHE) > 4096:
            _PCACHE.clear()
        _PCACHE[key] = p
    return p


def _make_params(dtype: torch.dtype, shape, params: dict) -> Params:
    p = Params()
    p.size = C.sizeof(Params)
    p.dtype = _DT[dtype]
    p.ndim = len(shape)
    for i, d in enumerate(shape):
        p.dims[i] = int(d)
    brick = params.get("brick", (256,) if len(shape) == 1 else None)
    if brick is None or len(brick) != len(shape):
        raise ApaxError(E_INVALID, "brick must have one extent per dimension")
    for i, b in enumerate(brick):
        p.brick[i] = int(b)
    p.mode = _MODES[params.get("mode", "lossless")]
    p.stream_mask = int(params.get("stream_mask", 0))
    p.rate = float(params.get("rate", 0.0))
    p.target_corr = float(params.get("target_corr", 0.99999))
    p.code = int(params.get("code", 0))
    p.flags = FLAG_LAGGED if params.get("lagged", False) else 0
    f = params.get("filter")  # (stride k, sign s): the 1-d filter stream x[n] - s x[n-k]
    if f:
        p.flags |= filter_flags(*f)
    if int(params.get("group", 4)) == 8:  # APAX_FLAG_GROUP8: 8 samples per exponent
        p.flags |= 0x4000
    return p


def filter_flags(k: int, sign: int) -> int:
    """APAX_FILTER(k, sign < 0)."""
    return (int(k) << 8) | (0x2000 if sign < 0 else 0)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else C.c_void_p(0)


def apax_encode_bound(dtype, shape, params) -> int:
    p = make_params(dtype, shape, params)
    b = C.c_uint64()
    _check(lib.apax_encode_bound(C.byref(p), C.byref(b)), "apax_encode_bound")
    return b.value


def apax_workspace_size(dtype, shape, params) -> int:
    p = make_params(dtype, shape, params)
    b = C.c_uint64()
    _check(lib.apax_workspace_size(C.byref(p), C.byref(b)), "apax_workspace_size")
    return b.value


def workspace(dtype, shape, params, device="cuda") -> torch.Tensor:
    n = apax_workspace_size(dtype, shape, params)
    return torch.empty(max(n, 16), dtype=torch.uint8, device=device)


def apax_status_clear(ws: torch.Tensor, stream=None):
    _check(lib.apax_status_clear(_dev_ptr(ws), _stream_ptr(stream)), "apax_status_clear")


def apax_status(ws: torch.Tensor, stream=None) -> int:
    return lib.apax_status(_dev_ptr(ws), _stream_ptr(stream))


def apax_profile(x: torch.Tensor, params: dict, ws: torch.Tensor | None = None, stream=None) -> dict:
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    if ws is None:
        ws = workspace(x.dtype, tuple(x.shape), params, x.device)
    r = ProfileResult()
    _check(lib.apax_profile(_dev_ptr(x), C.byref(p), C.byref(r), _dev_ptr(ws), ws.numel(),
                            _stream_ptr(stream)), "apax_profile")
    return profile_dict(r)


def apax_profile_async(x: torch.Tensor, params: dict, ws: torch.Tensor, stream=None):
    """Enqueue the profile of x on the stream; the result stays in ws.  An
    apax_encode of x with code=CODE_PROFILED on the same ws and stream adopts
    its code and stream mask on the device."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    _check(lib.apax_profile_async(_dev_ptr(x), C.byref(p), _dev_ptr(ws), ws.numel(),
                                  _stream_ptr(stream)), "apax_profile_async")


PASS_NAMES = ["max", "probe1", "probe2", "probe3", "probe4", "probe5", "probe6", "probe7", "probe8",
              "probe9", "hist", "curve", "metrics", "centred"]


def _event_ptr(ev):
    if ev.cuda_event == 0:  # torch creates the event at its first record
        ev.record()
    return C.c_void_p(ev.cuda_event)


def apax_profile_async_point(x: torch.Tensor, params: dict, ws: torch.Tensor, point_ready, stream=None):
    """apax_profile_async that records the torch.cuda.Event point_ready once
    the operating point is final (after the stream histogram)."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    ev = _event_ptr(point_ready)
    _check(lib.apax_profile_async_point(_dev_ptr(x), C.byref(p), _dev_ptr(ws), ws.numel(),
                                        _stream_ptr(stream), ev), "apax_profile_async_point")


def apax_adopt_point(ws_from: torch.Tensor, ws_to: torch.Tensor, stream=None):
    """Copy the profiled operating point of ws_from into ws_to (enqueued)."""
    _check(lib.apax_adopt_point(_dev_ptr(ws_from), _dev_ptr(ws_to), _stream_ptr(stream)), "apax_adopt_point")


def apax_profile_timed(x: torch.Tensor, params: dict, ws: torch.Tensor, stream=None):
    """apax_profile plus the duration (ms, HIP events on the stream) of the
    kernel of each pass that ran: returns (result dict, {pass name: ms})."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    r = ProfileResult()
    ms = (C.c_float * len(PASS_NAMES))()
    _check(lib.apax_profile_timed(_dev_ptr(x), C.byref(p), C.byref(r), ms, _dev_ptr(ws), ws.numel(),
                                  _stream_ptr(stream)), "apax_profile_timed")
    return profile_dict(r), {n: ms[i] for i, n in enumerate(PASS_NAMES) if ms[i] >= 0}


def apax_profile_encode_timed(x: torch.Tensor, params: dict, ws: torch.Tensor, out=None, nbytes=None,
                              stream=None):
    """apax_profile_encode_async on one stream with the duration (ms) of the
    kernel of each pass (fixed rate: the metrics pass writes the blocks);
    returns (result dict, {pass name: ms}, stream buffer, nbytes tensor)."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    bound = apax_encode_bound(x.dtype, tuple(x.shape), dict(params, code=0))
    if out is None:
        out = torch.empty(max(bound, 64), dtype=torch.uint8, device=x.device)
    if nbytes is None:
        nbytes = torch.zeros(1, dtype=torch.int64, device=x.device)
    r = ProfileResult()
    ms = (C.c_float * len(PASS_NAMES))()
    _check(lib.apax_profile_encode_timed(_dev_ptr(x), C.byref(p), C.byref(r), ms, _dev_ptr(ws), ws.numel(),
                                         _dev_ptr(out), out.numel(), _dev_ptr(nbytes), _stream_ptr(stream)),
           "apax_profile_encode_timed")
    return profile_dict(r), {n: ms[i] for i, n in enumerate(PASS_NAMES) if ms[i] >= 0}, out, nbytes


def apax_s2r_margin(x: torch.Tensor, params: dict, ws: torch.Tensor, stream=None):
    """2-sigma S2R margin (ratio, dB) at the operating point of the profile
    of x that ws holds (apax_profile / apax_profile_async with params)."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    ratio, db = C.c_double(), C.c_double()
    _check(lib.apax_s2r_margin(_dev_ptr(x), C.byref(p), C.byref(ratio), C.byref(db), _dev_ptr(ws),
                               ws.numel(), _stream_ptr(stream)), "apax_s2r_margin")
    return ratio.value, db.value


DOT_WGS = 1024


def apax_decode_dot(stream_buf: torch.Tensor, nbytes: int, hdr: bytes, w: torch.Tensor,
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Decode-on-read dot product with w; returns a device float64 tensor (1,)."""
    assert stream_buf.is_cuda and w.is_cuda and w.is_contiguous()
    info = apax_stream_info(hdr)
    if ws is None:
        params = {"mode": info["mode"], "brick": info["brick"], "rate": info["rate"],
                  "code": info["code"], "target_corr": 0.5}
        ws = workspace(info["dtype"], info["shape"], params, w.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=w.device)
    h = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
    _check(lib.apax_decode_dot(C.cast(h, C.c_void_p), _dev_ptr(stream_buf), int(nbytes), _dev_ptr(w),
                               _dev_ptr(out), _dev_ptr(ws), ws.numel(), _stream_ptr(stream)), "apax_decode_dot")
    return out


def apax_dot(x: torch.Tensor, w: torch.Tensor, out: torch.Tensor | None = None,
             ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The same consumer on an uncompressed array: sum x * w in binary64."""
    assert x.is_cuda and w.is_cuda and x.dtype == w.dtype and x.numel() == w.numel()
    if ws is None:
        ws = torch.empty(DOT_WGS * 8, dtype=torch.uint8, device=x.device)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib.apax_dot(_dev_ptr(x), _dev_ptr(w), _DT[x.dtype], x.numel(), _dev_ptr(out), _dev_ptr(ws),
                        ws.numel(), _stream_ptr(stream)), "apax_dot")
    return out


def apax_spectral_metrics(x: torch.Tensor, y: torch.Tensor, ws: torch.Tensor | None = None,
                          stream=None) -> dict:
    """Welch-spectrum metrics of x and its decoded array y (Sec. 4 Windows 3-4)."""
    assert x.is_cuda and y.is_cuda and x.dtype == y.dtype and x.numel() == y.numel()
    assert x.is_contiguous() and y.is_contiguous()
    if ws is None:
        ws = torch.empty(int(lib.apax_spectral_workspace_bytes()), dtype=torch.uint8, device=x.device)
    r = Spectral()
    _check(lib.apax_spectral_metrics(_dev_ptr(x), _dev_ptr(y), _DT[x.dtype], x.numel(), C.byref(r),
                                     _dev_ptr(ws), ws.numel(), _stream_ptr(stream)), "apax_spectral_metrics")
    return {f: getattr(r, f) for f, _ in Spectral._fields_}


def apax_signal_monitor(x: torch.Tensor, ws: torch.Tensor | None = None, stream=None) -> dict:
    """Signal monitor of x (Sec. 6): center bin and frequency, SNR, lags
    0..16 autocorrelation, the correlated neighbour's stride and sign and
    the gain of that filter."""
    assert x.is_cuda and x.is_contiguous()
    if ws is None:
        ws = torch.empty(int(lib.apax_spectral_workspace_bytes()), dtype=torch.uint8, device=x.device)
    r = Monitor()
    _check(lib.apax_signal_monitor(_dev_ptr(x), _DT[x.dtype], x.numel(), C.byref(r), _dev_ptr(ws), ws.numel(),
                                   _stream_ptr(stream)), "apax_signal_monitor")
    out = {f: getattr(r, f) for f, _ in Monitor._fields_ if f not in ("acf", "pad")}
    out["acf"] = [r.acf[i] for i in range(17)]
    return out


def apax_profile_read(x: torch.Tensor, params: dict, ws: torch.Tensor, stream=None) -> dict:
    """Wait for the stream and read the profile that ws holds (x: the array
    that was profiled, for its dtype and shape)."""
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    r = ProfileResult()
    _check(lib.apax_profile_read(C.byref(p), C.byref(r), _dev_ptr(ws), _stream_ptr(stream)),
           "apax_profile_read")
    return profile_dict(r)


def profile_dict(r: ProfileResult) -> dict:
    m = {f: getattr(r.m, f) for f, _ in Metrics._fields_}
    return {"code": r.code, "stream_mask": r.stream_mask, "flags": r.flags,
            "c_floor": r.c_floor, "c_cap": r.c_cap, "n_sub": r.n_sub, "n_probes": r.n_probes,
            "curve": [(r.curve[i].code, r.curve[i].ratio, r.curve[i].r) for i in range(NCURVE)],
            "metrics": m}


def apax_encode(x: torch.Tensor, params: dict, out: torch.Tensor | None = None,
                nbytes: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                stream=None, clear_status: bool = True):
    """Encode x; returns (stream buffer, device int64 tensor holding the byte length)."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), params)
    bound = C.c_uint64()
    _check(lib.apax_encode_bound(C.byref(p), C.byref(bound)), "apax_encode_bound")
    if out is None:
        out = torch.empty(max(bound.value, 64), dtype=torch.uint8, device=x.device)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=x.device)
    if ws is None:
        ws = workspace(x.dtype, tuple(x.shape), params, x.device)
    sp = _stream_ptr(stream)
    if clear_status:
        _check(lib.apax_status_clear(_dev_ptr(ws), sp), "apax_status_clear")
    _check(lib.apax_encode(_dev_ptr(x), C.byref(p), _dev_ptr(out), out.numel(),
                           _dev_ptr(nbytes), _dev_ptr(ws), ws.numel(), sp), "apax_encode")
    return out, nbytes


def apax_profile_encode_async(x: torch.Tensor, params: dict, ws: torch.Tensor, out: torch.Tensor | None = None,
                              nbytes: torch.Tensor | None = None, encoded=None, stream=None, side=None,
                              forked=None):
    """Profile x and encode it at the profiled operating point in one launch
    sequence (the encode from the profile's per-block results); records the
    torch.cuda.Event `encoded` once the stream is complete.  side (a
    torch.cuda.Stream) with forked (a torch.cuda.Event): the profile's centred
    and curve passes run on `side` beside the encode; join `side` before
    reading the profile.  Returns (stream buffer, device int64 byte length);
    the profile stays in ws (apax_profile_read)."""
    assert x.is_cuda and x.is_contiguous()
    p = make_params(x.dtype, tuple(x.shape), dict(params, code=0))
    bound = C.c_uint64()
    _check(lib.apax_encode_bound(C.byref(p), C.byref(bound)), "apax_encode_bound")
    if out is None:
        out = torch.empty(max(bound.value, 64), dtype=torch.uint8, device=x.device)
    if nbytes is None:
        nbytes = torch.empty(1, dtype=torch.int64, device=x.device)
    ev = _event_ptr(encoded) if encoded is not None else None
    sd = _stream_ptr(side) if side is not None else None
    fk = _event_ptr(forked) if forked is not None else None
    _check(lib.apax_profile_encode_async(_dev_ptr(x), C.byref(p), _dev_ptr(ws), ws.numel(), _dev_ptr(out),
                                         out.numel(), _dev_ptr(nbytes), _stream_ptr(stream), ev, sd, fk),
           "apax_profile_encode_async")
    return out, nbytes


def apax_encode_noalloc(x: torch.Tensor, params: dict, out: torch.Tensor, nbytes: torch.Tensor,
                        status: torch.Tensor | None = None, stream=None):
    """Encode x into the caller's buffers with the library's own scratch
    (no workspace, nothing allocated by the call).  out: uint8 stream buffer
    of at least apax_encode_bound bytes; nbytes: device int64[1]; status:
    device int32[1] or None, set to 0 or an APAX_E_* code on the device."""
    assert x.is_cuda and x.is_contiguous() and out.dtype == torch.uint8
    p = make_params(x.dtype, tuple(x.shape), params)
    sp = _stream_ptr(stream)
    st = _dev_ptr(status) if status is not None else None
    _check(lib.apax_encode_noalloc(_dev_ptr(x), C.byref(p), _dev_ptr(out), out.numel(),
                                   _dev_ptr(nbytes), st, sp), "apax_encode_noalloc")
    return out, nbytes


def apax_stream_info(hdr: bytes) -> dict:
    b = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
    p = Params()
    _check(lib.apax_stream_info(C.cast(b, C.c_void_p), 64, C.byref(p)), "apax_stream_info")
    names = {v: k for k, v in _MODES.items()}
    return {"dtype": _TORCH_OF[p.dtype], "shape": tuple(int(p.dims[i]) for i in range(p.ndim)),
            "mode": names[p.mode], "brick": tuple(int(p.brick[i]) for i in range(p.ndim)),
            "stream_mask": p.stream_mask, "rate": p.rate, "code": p.code,
            "filter": ((p.flags >> 8) & 0x1F, -1 if p.flags & 0x2000 else 1) if (p.flags >> 8) & 0x1F else None,
            "group": 8 if p.flags & 0x4000 else 4}


def stream_nbytes(hdr: bytes) -> int:
    """Whole stream length from its 64-byte header (apax_stream_size)."""
    b = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
    n = C.c_uint64(0)
    _check(lib.apax_stream_size(C.cast(b, C.c_void_p), 64, C.byref(n)), "apax_stream_size")
    return int(n.value)


def apax_decode(stream_buf: torch.Tensor, nbytes: int | None = None, hdr: bytes | None = None,
                y: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None,
                clear_status: bool = True) -> torch.Tensor:
    assert stream_buf.is_cuda
    if hdr is None:
        hdr = bytes(stream_buf[:64].cpu().numpy().tobytes())
    info = apax_stream_info(hdr)
    if nbytes is None:
        nbytes = stream_nbytes(hdr)
    params = {"mode": info["mode"], "brick": info["brick"], "rate": info["rate"],
              "code": info["code"], "target_corr": 0.5}
    if y is None:
        y = torch.empty(info["shape"], dtype=info["dtype"], device=stream_buf.device)
    if ws is None:
        ws = workspace(info["dtype"], info["shape"], params, stream_buf.device)
    sp = _stream_ptr(stream)
    hb = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
    if clear_status:
        _check(lib.apax_status_clear(_dev_ptr(ws), sp), "apax_status_clear")
    _check(lib.apax_decode(C.cast(hb, C.c_void_p), _dev_ptr(stream_buf), int(nbytes), _dev_ptr(y),
                           y.numel() * y.element_size(), _dev_ptr(ws), ws.numel(), sp),
           "apax_decode")
    return y


# ---------------------------------------------------------------- batches

def apax_batch_create(op: int, items, tune: dict | None = None):
    """Plan for a list of BatchItem; returns (handle, workspace bytes)."""
    arr = (BatchItem * max(1, len(items)))(*items)
    t = Tune()
    for k, v in (tune or {}).items():
        setattr(t, k, int(v))
    h = C.c_void_p()
    nb = C.c_uint64()
    _check(lib.apax_batch_create(int(op), arr, len(items), C.byref(t), C.byref(h), C.byref(nb)),
           "apax_batch_create")
    return h, nb.value


def apax_batch_upload(h, ws: torch.Tensor, stream=None):
    _check(lib.apax_batch_upload(h, _dev_ptr(ws), ws.numel(), _stream_ptr(stream)),
           "apax_batch_upload")


def apax_batch_run(h, stream=None):
    _check(lib.apax_batch_run(h, _stream_ptr(stream)), "apax_batch_run")


def apax_batch_capture(h):
    _check(lib.apax_batch_capture(h), "apax_batch_capture")


def apax_batch_launch(h, stream=None):
    _check(lib.apax_batch_launch(h, _stream_ptr(stream)), "apax_batch_launch")


def apax_batch_destroy(h):
    lib.apax_batch_destroy(h)


class Batch:
    """Encode (or decode) many device arrays with one persistent launch.

    encode: Batch.encode([(tensor, params), ...]) -> outputs in .outs /
            .nbytes (device int64 per item);
    decode: Batch.decode([(stream_buffer, nbytes, header_bytes), ...]).
    run() enqueues the batch, capture() records it as a hipGraph, launch()
    replays it.  tune: dict of Tune fields (launch geometry only)."""

    def __init__(self, op, items, keep, outs, nbytes, tune=None, device="cuda", ws=None,
                 stream=None):
        self.op = op
        self._keep = keep
        self.outs = outs
        self.nbytes = nbytes
        self.stream = stream
        self.handle, wsb = apax_batch_create(op, items, tune)
        if ws is None or ws.numel() < wsb:
            ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=device)
        self.ws = ws
        apax_batch_upload(self.handle, self.ws, stream)

    @staticmethod
    def workspace_bytes(op, items, tune=None) -> int:
        h, n = apax_batch_create(op, items, tune)
        apax_batch_destroy(h)
        return n

    @classmethod
    def encode(cls, arrays, tune=None, device="cuda", ws=None, stream=None, outs=None):
        items, keep = [], []
        given = outs is not None
        outs = list(outs) if given else []
        nbytes = torch.empty(max(1, len(arrays)), dtype=torch.int64, device=device)
        for i, (x, params) in enumerate(arrays):
            assert x.is_cuda and x.is_contiguous()
            p = make_params(x.dtype, tuple(x.shape), params)
            bound = apax_encode_bound(x.dtype, tuple(x.shape), params)
            out = outs[i] if given else torch.empty(max(bound, 64), dtype=torch.uint8, device=device)
            it = BatchItem()
            it.p = p
            it.d_in = x.data_ptr() if x.numel() else None
            it.d_out = out.data_ptr()
            it.cap = out.numel()
            it.d_nbytes = nbytes.data_ptr() + 8 * i
            items.append(it)
            keep.append(x)
            if not given:
                outs.append(out)
        return cls(OP_ENCODE, items, keep, outs, nbytes, tune, device, ws, stream)

    @classmethod
    def decode(cls, streams, tune=None, device="cuda", ws=None, stream=None, outs=None):
        items, keep = [], []
        given = outs is not None
        outs = list(outs) if given else []
        for k, (buf, n, hdr) in enumerate(streams):
            info = apax_stream_info(hdr)
            y = outs[k] if given else torch.empty(info["shape"], dtype=info["dtype"], device=device)
            hb = (C.c_uint8 * 64).from_buffer_copy(bytes(hdr[:64]))
            it = BatchItem()
            it.d_in = buf.data_ptr()
            it.d_out = y.data_ptr() if y.numel() else None
            it.in_bytes = int(n)
            it.cap = y.numel() * y.element_size()
            it.h_hdr = C.cast(hb, C.c_void_p)
            items.append(it)
            keep += [buf, hb]
            if not given:
                outs.append(y)
        return cls(OP_DECODE, items, keep, outs, None, tune, device, ws, stream)

    def run(self, stream=None):
        apax_batch_run(self.handle, stream if stream is not None else self.stream)

    def capture(self):
        apax_batch_capture(self.handle)

    def launch(self, stream=None):
        apax_batch_launch(self.handle, stream if stream is not None else self.stream)

    def status(self, stream=None) -> int:
        return apax_status(self.ws, stream)

    def close(self):
        if self.handle:
            apax_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
