"""ctypes binding of the CPU oracle (test infrastructure only).

Everything here works on host numpy arrays.  Parameters are plain dicts:
    {"mode": "lossless" | "fixed_rate" | "fixed_quality" | "adaptive_rate",
     "brick": (..), "stream_mask": 0, "rate": 4.0, "target_corr": 0.99999,
     "code": 0}
The array's dtype and shape give the dtype and dims.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

I8, I16, I32, F32, F64 = 1, 2, 3, 4, 5
LOSSLESS, FIXED_RATE, FIXED_QUALITY, ADAPTIVE_RATE = 0, 1, 2, 3
ADAPT_HALF = 32  # the adaptive loop's window: start code - 32 .. start code + 31
E_INVALID, E_UNSUPPORTED, E_CAPACITY, E_CORRUPT, E_NONFINITE = -1, -2, -3, -4, -5
NEAR_TIE = 1
NCURVE = 17

DTYPES = {np.dtype(np.int8): I8, np.dtype(np.int16): I16, np.dtype(np.int32): I32,
          np.dtype(np.float32): F32, np.dtype(np.float64): F64}
NP_OF = {v: k for k, v in DTYPES.items()}
MODES = {"lossless": LOSSLESS, "fixed_rate": FIXED_RATE, "fixed_quality": FIXED_QUALITY,
         "adaptive_rate": ADAPTIVE_RATE}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
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


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        vp, P = C.c_void_p, C.POINTER
        L.orc_encode_bound.argtypes = [P(Params), P(C.c_uint64)]
        L.orc_encode.argtypes = [vp, P(Params), vp, C.c_uint64, P(C.c_uint64)]
        L.orc_decode.argtypes = [vp, C.c_uint64, vp, C.c_uint64]
        L.orc_stream_info.argtypes = [vp, C.c_uint64, P(Params)]
        L.orc_profile.argtypes = [vp, P(Params), P(ProfileResult)]
        L.orc_gain.argtypes = [C.c_int32]
        L.orc_gain.restype = C.c_double
        L.orc_inv_gain_mantissa.argtypes = [C.c_int32]
        L.orc_inv_gain_mantissa.restype = C.c_double
        L.orc_block_bracket.argtypes = [vp, P(Params), C.c_int64, P(C.c_double),
                                        P(C.c_int32), P(C.c_int32)]
        L.orc_encode_block.argtypes = [vp, P(Params), C.c_int64, vp, C.c_int32,
                                       P(C.c_int32), P(C.c_int32), P(C.c_int32),
                                       P(C.c_int32)]
        L.orc_stream_values.argtypes = [vp, vp, C.c_int32, C.c_int32, vp]
        L.orc_group_eps.argtypes = [vp, C.c_int32, C.c_int32, vp]
        L.orc_stream_values_f.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_stream_inverse.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
        L.orc_jee_tokens.argtypes = [vp, C.c_int32, vp, P(C.c_int32)]
        L.orc_stats.argtypes = [vp, vp, C.c_uint64, P(Metrics)]
        L.orc_corr_at.argtypes = [vp, P(Params), C.c_int32, P(C.c_double)]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def make_params(x_or_dtype, shape, params) -> Params:
    dt = np.dtype(x_or_dtype)
    p = Params()
    p.size = C.sizeof(Params)
    p.dtype = DTYPES[dt]
    p.ndim = len(shape)
    for i, d in enumerate(shape):
        p.dims[i] = int(d)
    brick = params.get("brick", (256,) if len(shape) == 1 else None)
    for i, b in enumerate(brick):
        p.brick[i] = int(b)
    p.mode = MODES[params.get("mode", "lossless")]
    p.stream_mask = int(params.get("stream_mask", 0))
    p.rate = float(params.get("rate", 0.0))
    p.target_corr = float(params.get("target_corr", 0.99999))
    p.code = int(params.get("code", 0))
    p.flags = 1 if params.get("lagged", False) else 0  # ORC_FLAG_LAGGED
    f = params.get("filter")  # (stride k, sign s): the stream x[n] - s x[n-k] (1-d)
    if f:
        p.flags |= filter_flags(*f)
    if int(params.get("group", 4)) == 8:  # ORC_FLAG_GROUP8: 8 samples per exponent
        p.flags |= 0x4000
    return p


def filter_flags(k: int, sign: int) -> int:
    """ORC_FILTER(k, sign < 0)."""
    return (int(k) << 8) | (0x2000 if sign < 0 else 0)


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def encode_bound(dtype, shape, params) -> int:
    p = make_params(dtype, shape, params)
    b = C.c_uint64()
    _check(lib().orc_encode_bound(C.byref(p), C.byref(b)), "encode_bound")
    return b.value


def encode(x: np.ndarray, params) -> np.ndarray:
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, x.shape, params)
    b = C.c_uint64()
    _check(lib().orc_encode_bound(C.byref(p), C.byref(b)), "encode_bound")
    out = np.zeros(b.value, np.uint8)
    nb = C.c_uint64()
    _check(lib().orc_encode(_ptr(x), C.byref(p), _ptr(out), b.value, C.byref(nb)), "encode")
    return out[: nb.value].copy()


def stream_info(buf: np.ndarray) -> Params:
    buf = np.ascontiguousarray(buf, np.uint8)
    p = Params()
    _check(lib().orc_stream_info(_ptr(buf), buf.size, C.byref(p)), "stream_info")
    return p


def decode(buf: np.ndarray) -> np.ndarray:
    buf = np.ascontiguousarray(buf, np.uint8)
    p = stream_info(buf)
    shape = tuple(int(p.dims[i]) for i in range(p.ndim))
    y = np.zeros(shape, NP_OF[p.dtype])
    _check(lib().orc_decode(_ptr(buf), buf.size, _ptr(y), y.nbytes), "decode")
    return y


def decode_rc(buf: np.ndarray, y: np.ndarray) -> int:
    buf = np.ascontiguousarray(buf, np.uint8)
    return lib().orc_decode(_ptr(buf), buf.size, _ptr(y), y.nbytes)


def profile(x: np.ndarray, params) -> ProfileResult:
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, x.shape, dict(params, code=0))
    r = ProfileResult()
    _check(lib().orc_profile(_ptr(x), C.byref(p), C.byref(r)), "profile")
    return r


def profile_dict(r: ProfileResult) -> dict:
    m = {f: getattr(r.m, f) for f, _ in Metrics._fields_}
    return {"code": r.code, "stream_mask": r.stream_mask, "flags": r.flags,
            "c_floor": r.c_floor, "c_cap": r.c_cap, "n_sub": r.n_sub, "n_probes": r.n_probes,
            "curve": [(r.curve[i].code, r.curve[i].ratio, r.curve[i].r) for i in range(NCURVE)],
            "metrics": m}


def gain(c: int) -> float:
    return lib().orc_gain(int(c))


def inv_gain_mantissa(f: int) -> float:
    return lib().orc_inv_gain_mantissa(int(f))


def block_bracket(x: np.ndarray, params, j: int):
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, x.shape, params)
    M, cf, cc = C.c_double(), C.c_int32(), C.c_int32()
    _check(lib().orc_block_bracket(_ptr(x), C.byref(p), int(j), C.byref(M), C.byref(cf),
                                   C.byref(cc)), "block_bracket")
    return M.value, cf.value, cc.value


def encode_block(x: np.ndarray, params, j: int, cap_words: int = 20000):
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, x.shape, params)
    w = np.zeros(cap_words, np.uint32)
    nw, st, cj, ub = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().orc_encode_block(_ptr(x), C.byref(p), int(j), _ptr(w), cap_words,
                                  C.byref(nw), C.byref(st), C.byref(cj), C.byref(ub)),
           "encode_block")
    return w[: nw.value].copy(), st.value, cj.value, ub.value


def stream_values(a: np.ndarray, brick, W: int, s: int) -> np.ndarray:
    a = np.ascontiguousarray(a, np.int64).ravel()
    b = np.ones(3, np.uint32)
    b[3 - len(brick):] = brick
    v = np.zeros_like(a)
    _check(lib().orc_stream_values(_ptr(a), _ptr(b), int(W), int(s), _ptr(v)), "stream_values")
    return v


def stream_values_f(a: np.ndarray, brick, W: int, s: int, k: int, sign: int) -> np.ndarray:
    """Stream s with the filter (k, sign) (k = 0: none)."""
    a = np.ascontiguousarray(a, np.int64).ravel()
    b = np.ones(3, np.uint32)
    b[3 - len(brick):] = brick
    v = np.zeros_like(a)
    _check(lib().orc_stream_values_f(_ptr(a), _ptr(b), int(W), int(s), int(k), 1 if sign < 0 else 0, _ptr(v)),
           "stream_values_f")
    return v


def stream_inverse(v: np.ndarray, brick, W: int, s: int, k: int = 0, sign: int = 1) -> np.ndarray:
    """The decoder's inverse of stream s (with the filter (k, sign) for s = 3 in 1-d)."""
    v = np.ascontiguousarray(v, np.int64).ravel()
    b = np.ones(3, np.uint32)
    b[3 - len(brick):] = brick
    a = np.zeros_like(v)
    _check(lib().orc_stream_inverse(_ptr(v), _ptr(b), int(W), int(s), int(k), 1 if sign < 0 else 0, _ptr(a)),
           "stream_inverse")
    return a


def group_eps(v: np.ndarray, W: int) -> np.ndarray:
    v = np.ascontiguousarray(v, np.int64).ravel()
    G = v.size // 4
    e = np.zeros(G, np.int32)
    _check(lib().orc_group_eps(_ptr(v), G, int(W), _ptr(e)), "group_eps")
    return e


def jee_tokens(eps) -> list:
    e = np.ascontiguousarray(eps, np.int32)
    nib = np.zeros(2 * max(e.size, 1), np.uint8)
    n = C.c_int32()
    _check(lib().orc_jee_tokens(_ptr(e), e.size, _ptr(nib), C.byref(n)), "jee_tokens")
    return [int(t) for t in nib[: n.value]]


def stats(x: np.ndarray, y: np.ndarray) -> dict:
    x = np.ascontiguousarray(x, np.float64).ravel()
    y = np.ascontiguousarray(y, np.float64).ravel()
    m = Metrics()
    _check(lib().orc_stats(_ptr(x), _ptr(y), x.size, C.byref(m)), "stats")
    return {f: getattr(m, f) for f, _ in Metrics._fields_}


def corr_at(x: np.ndarray, params, code: int) -> float:
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, x.shape, dict(params, code=0))
    r = C.c_double()
    _check(lib().orc_corr_at(_ptr(x), C.byref(p), int(code), C.byref(r)), "corr_at")
    return r.value


# ---------------------------------------------------------------- Sec. 4, Window 4
# The 2-sigma signal-to-residual margin: the per-sample ratio |x| / |d| of the
# input to the residual d = x - y of the decoded array y, taken at the level
# that 95.5 % of the samples reach or exceed (the 4.5th percentile, nearest
# rank: the ceil(0.045 n)-th smallest ratio), in dB.  A sample with d = 0 has
# an infinite ratio; one with x = 0 and d != 0 has ratio 0 (-inf dB).
S2R_P = 0.045


def s2r_ratios(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per-sample |x| / |x - y| in binary64 (x, y as binary64)."""
    xd = np.ascontiguousarray(x, np.float64).ravel()
    yd = np.ascontiguousarray(y, np.float64).ravel()
    d = xd - yd
    out = np.full(xd.shape, np.inf)
    nz = d != 0
    out[nz] = np.abs(xd[nz]) / np.abs(d[nz])
    return out


def s2r_margin_xy(x: np.ndarray, y: np.ndarray, p: float = S2R_P):
    """(ratio, dB) at the nearest-rank p-quantile of s2r_ratios(x, y)."""
    r = s2r_ratios(x, y)
    if r.size == 0:
        return float("nan"), float("nan")
    # nearest rank ceil(p n), computed exactly for p = 45/1000
    k = (45 * r.size + 999) // 1000 if p == S2R_P else int(math.ceil(p * r.size))
    k = min(max(k, 1), r.size)
    v = float(np.partition(r, k - 1)[k - 1])
    if v == 0.0:
        return v, float("-inf")
    return v, (float("inf") if math.isinf(v) else 20.0 * math.log10(v))


def s2r_margin(x: np.ndarray, params):
    """2-sigma S2R margin of encoding x at the operating point in params
    (code, stream mask), against the decoded array."""
    y = decode(encode(x, params))
    return s2r_margin_xy(x, y)


# ---------------------------------------------------------------- Sec. 4, Windows 3-4 (spectra)
# Spectral reading (the paper names the metrics but not the estimator): a
# Welch power spectrum of the array in memory order -- segments of L = 1024
# samples, hop L/2, periodic Hann window w_i = sin^2(pi i / L), one-sided
# bins f = 1..L/2 (DC excluded), P[f] = mean over segments of |DFT(w s)[f]|^2.
# Of x, y and d = x - y: peak = max P (dB), floor = the L/4-th smallest bin
# (nearest-rank median of the L/2 bins, dB); residual mean = mean of P_d (dB);
# DR = peak_x - floor_x, SRR = peak_x - residual mean, FFT S2R margin =
# floor_x - residual mean.  Fewer than L samples: no segment (NaN).
PSD_L = 1024


def _db(p):
    return 10.0 * math.log10(p) if p > 0 else float("-inf")


def welch_psd(s: np.ndarray) -> np.ndarray:
    """P[f], f = 1..L/2, of the binary64 sequence s (segments L, hop L/2)."""
    s = np.ascontiguousarray(s, np.float64).ravel()
    L = PSD_L
    K = 1 + (s.size - L) // (L // 2)
    w = np.sin(np.pi * np.arange(L) / L) ** 2
    acc = np.zeros(L // 2 + 1)
    for k in range(K):
        seg = s[k * (L // 2): k * (L // 2) + L] * w
        acc += np.abs(np.fft.rfft(seg)) ** 2
    return acc[1:] / K


def spectral_metrics(x: np.ndarray, y: np.ndarray) -> dict:
    xd = np.ascontiguousarray(x, np.float64).ravel()
    yd = np.ascontiguousarray(y, np.float64).ravel()
    keys = ("peak_x", "floor_x", "peak_y", "floor_y", "peak_d", "floor_d", "resid_mean",
            "dr", "srr", "fft_s2r_margin")
    if xd.size < PSD_L:
        out = {k: float("nan") for k in keys}
        out["segments"] = 0
        return out
    out = {"segments": 1 + (xd.size - PSD_L) // (PSD_L // 2)}
    rank = PSD_L // 4  # nearest-rank median of the L/2 bins
    for name, s in (("x", xd), ("y", yd), ("d", xd - yd)):
        P = welch_psd(s)
        out[f"peak_{name}"] = _db(float(P.max()))
        out[f"floor_{name}"] = _db(float(np.partition(P, rank - 1)[rank - 1]))
        if name == "d":
            out["resid_mean"] = _db(float(P.mean()))
    out["dr"] = out["peak_x"] - out["floor_x"]
    out["srr"] = out["peak_x"] - out["resid_mean"]
    out["fft_s2r_margin"] = out["floor_x"] - out["resid_mean"]
    return out


# ---------------------------------------------------------------- Sec. 6, signal monitor
# Reading (the paper names the monitor's outputs, center frequency and SNR,
# and says the center frequency tells which nearby elements are correlated,
# without formulas): of the array x in memory order, binary64,
#   R[k] = sum_{n >= k} x[n] x[n - k], k = 0..16, and the normalised
#   acf[k] = (R[k] / (N - k)) / (R[0] / N), each lag's mean product over that
#   of lag 0 (all zero when R[0] = 0; lags >= N zero);
#   peak_bin b = the first largest bin of the Welch spectrum above (1..512),
#   center_freq = b / 1024 cycles per sample, peak / floor in dB as above,
#   snr = 10 log10(mean P / floor);
#   correlated neighbour: the lag phase of bin b at lag k is m = b k mod 1024
#   (units of 1/1024 turn); a tone there is cancelled by x[n] - x[n - k] when m
#   is a multiple of 1024 and by x[n] + x[n - k] when m is 512 off one.  The
#   stride is the smallest k in 1..16 whose m is nearest a multiple of 512;
#   sign = +1 (difference) when m is nearer 0 mod 1024 (ties at a quarter turn
#   go to +1), else -1 (sum);
#   gain = 10 log10(sum_{n >= k} x[n]^2 / sum_{n >= k} (x[n] - sign x[n - k])^2)
#   at k = stride: what the filter takes out of the samples it applies to
#   (+inf for a zero residual, NaN when both sums are zero).
# Fewer than 1024 samples: no spectrum (NaN fields, peak_bin = stride = sign = 0).
MON_LAGS = 16


def autocorr(x: np.ndarray, lags: int = MON_LAGS) -> np.ndarray:
    """R[k] = sum_{n >= k} x[n] x[n - k], k = 0..lags, binary64."""
    s = np.ascontiguousarray(x, np.float64).ravel()
    R = np.zeros(lags + 1)
    for k in range(min(lags, s.size - 1) + 1):
        R[k] = float(np.dot(s[k:], s[:s.size - k]))
    return R


def monitor_stride(b: int):
    """(stride, sign) that the center bin b selects (0, 0 for no bin)."""
    if b <= 0:
        return 0, 0
    best_k, best_dist = 0, PSD_L
    for k in range(1, MON_LAGS + 1):
        r = (b * k) % (PSD_L // 2)
        dist = min(r, PSD_L // 2 - r)
        if dist < best_dist:
            best_k, best_dist = k, dist
    m = (b * best_k) % PSD_L
    sign = 1 if (m <= PSD_L // 4 or m >= 3 * PSD_L // 4) else -1
    return best_k, sign


def signal_monitor(x: np.ndarray) -> dict:
    s = np.ascontiguousarray(x, np.float64).ravel()
    R = autocorr(s)
    N = s.size
    acf = np.zeros_like(R)
    if R[0] > 0:
        for k in range(min(MON_LAGS, N - 1) + 1):
            acf[k] = (R[k] / (N - k)) / (R[0] / N)
    out = {"acf": acf, "segments": 0, "peak_bin": 0, "center_freq": float("nan"),
           "peak_db": float("nan"), "floor_db": float("nan"), "snr_db": float("nan"),
           "stride": 0, "sign": 0, "gain_db": float("nan")}
    if s.size < PSD_L:
        return out
    P = welch_psd(s)
    b = 1 + int(np.argmax(P))                 # first largest bin
    rank = PSD_L // 4
    fl = float(np.partition(P, rank - 1)[rank - 1])
    k, sg = monitor_stride(b)
    e_in = float(np.dot(s[k:], s[k:]))
    e_out = float(np.sum((s[k:] - sg * s[:N - k]) ** 2))
    out.update(segments=1 + (s.size - PSD_L) // (PSD_L // 2), peak_bin=b, center_freq=b / PSD_L,
               peak_db=_db(float(P[b - 1])), floor_db=_db(fl),
               snr_db=_db(float(P.mean())) - _db(fl), stride=k, sign=sg,
               gain_db=_db(e_in) - _db(e_out))
    return out
