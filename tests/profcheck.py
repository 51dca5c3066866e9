"""Comparison of a GPU profile result with the oracle's (Sec. 4 profiler):
decisions exact (bracket, code, stream mask, probe count, curve codes and
ratios), statistics within 1e-9 relative (signed sums relative to the sum of
their absolute terms)."""
import math

import numpy as np

from oracle import oracle as O


def check_metrics(mg, mo, x, y, tol=1e-9):
    xd, yd = x.astype(np.float64).ravel(), y.astype(np.float64).ravel()
    d = xd - yd
    for k in ("sxx", "syy", "sdd"):
        assert abs(mg[k] - mo[k]) <= tol * abs(mo[k]) + 1e-300, k
    for k, terms in (("sum_x", np.abs(xd)), ("sum_y", np.abs(yd)), ("sum_d", np.abs(d)),
                     ("sds", np.abs(d * (xd + yd)))):
        assert abs(mg[k] - mo[k]) <= tol * float(terms.sum()) + 1e-300, k
    assert abs(mg["one_minus_r"] - mo["one_minus_r"]) <= tol * abs(mo["one_minus_r"]) + 1e-15
    for k in ("std_x", "std_y", "std_d"):
        assert abs(mg[k] - mo[k]) <= tol * abs(mo[k]) + 1e-12 * math.sqrt(mo["sxx"] / max(1, mo["n"])), k
    assert mg["max_abs_d"] == mo["max_abs_d"]
    assert mg["enc_bytes"] == mo["enc_bytes"] and mg["n"] == mo["n"]
    if math.isfinite(mo["snr_db"]):
        assert abs(mg["snr_db"] - mo["snr_db"]) <= 1e-8


def check_profile(pg, po, x, y):
    near = (pg["flags"] | po["flags"]) & 1
    assert (pg["c_floor"], pg["c_cap"], pg["n_sub"]) == (po["c_floor"], po["c_cap"], po["n_sub"])
    if near and pg["code"] != po["code"]:
        return False  # both decisions are acceptable inside the tie band
    assert pg["code"] == po["code"]
    assert pg["stream_mask"] == po["stream_mask"]
    assert pg["n_probes"] == po["n_probes"]
    for a, b in zip(pg["curve"], po["curve"]):
        assert a[0] == b[0] and a[1] == b[1]
        assert abs((1 - a[2]) - (1 - b[2])) <= 1e-9 * abs(1 - b[2]) + 1e-15
    check_metrics(pg["metrics"], po["metrics"], x, y)
    return True


def decoded_at(x, params, prof):
    p = dict(params, code=prof["code"],
             stream_mask=prof["stream_mask"] & (0x7F if params["mode"] == "fixed_rate" else 0xFF))
    return p, O.decode(O.encode(x, p))
