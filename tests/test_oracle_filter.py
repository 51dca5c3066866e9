"""Pins of the oracle's filter stream (Sec. 5 / Sec. 6: the redundancy
remover's filtered versions of the series; the signal monitor's centre
frequency picks the correlated neighbour x[n - k] and the sign).

The forward filter is checked against its definition in numpy, the decoder's
inverse against the closed form a[p] = sum_i s^i v[p - i k] and by round
trips, the monitor's (stride, sign) against the tones they cancel, and the
encoder's use of the stream by lossless round trips, block headers and sizes
on modulated carriers."""
import numpy as np
import pytest

import brute
import synth
from oracle import oracle as O


def wrap(v, W):
    m = (1 << W) - 1
    u = np.asarray(v, np.int64) & m
    return np.where(u >> (W - 1), u - (1 << W), u)


@pytest.mark.parametrize("B,W,k,sign", [(64, 16, 1, -1), (256, 8, 2, -1), (1024, 32, 16, 1), (128, 16, 5, 1),
                                        (256, 32, 3, -1), (64, 16, 16, -1)])
def test_filter_matches_definition(B, W, k, sign):
    rng = np.random.default_rng(B + k)
    a = wrap(rng.integers(-(1 << 40), 1 << 40, B), W)
    v = O.stream_values_f(a, (B,), W, 3, k, sign)
    prev = np.concatenate([np.zeros(k, np.int64), a[:-k]])
    assert np.array_equal(v, wrap(a - sign * prev, W))
    # without a filter stream 3 of a 1-d brick is the y difference: the samples
    assert np.array_equal(O.stream_values_f(a, (B,), W, 3, 0, 1), a)


@pytest.mark.parametrize("B,W,k,sign", [(64, 16, 1, -1), (256, 32, 7, 1), (1024, 16, 16, -1), (512, 8, 2, 1)])
def test_inverse_is_strided_running_sum(B, W, k, sign):
    rng = np.random.default_rng(7 * B + k)
    v = wrap(rng.integers(-(1 << 30), 1 << 30, B), W)
    a = O.stream_inverse(v, (B,), W, 3, k, sign)
    # closed form: a[p] = sum_i sign^i v[p - i k]
    exp = np.zeros(B, np.int64)
    for p in range(B):
        acc, i = 0, 0
        while p - i * k >= 0:
            acc += (sign ** i) * int(v[p - i * k])
            i += 1
        exp[p] = acc
    assert np.array_equal(a, wrap(exp, W))
    # and a round trip of every 1-d stream
    x = wrap(rng.integers(-(1 << 30), 1 << 30, B), W)
    for s in (0, 1, 2, 3):
        vv = O.stream_values_f(x, (B,), W, s, k, sign)
        assert np.array_equal(O.stream_inverse(vv, (B,), W, s, k, sign), x), s


@pytest.mark.parametrize("b", [512, 256, 341, 171, 100, 64])
def test_monitor_stride_cancels_its_tone(b):
    """A pure tone at bin b: the filter with the monitor's (stride, sign)
    leaves a residual far below the tone (exactly zero at bins where b k is a
    multiple of 512)."""
    k, sign = O.monitor_stride(b)
    t = np.arange(4096)
    x = np.cos(2 * np.pi * b * t / 1024 + 0.3)
    r = x[k:] - sign * x[:-k]
    resid = np.abs(r).max()
    m = (b * k) % 512
    dist = min(m, 512 - m)
    assert resid <= 2 * np.sin(np.pi * dist / 1024) + 1e-9  # |1 - e^{i pi dist/512}| bound
    if dist == 0:
        assert resid < 1e-9


@pytest.mark.parametrize("dt,b,brick", [(np.int16, 512, (256,)), (np.int16, 341, (256,)), (np.int32, 256, (64,)),
                                         (np.int8, 200, (128,)), (np.int16, 100, (1024,))])
def test_lossless_filter_encode(dt, b, brick):
    """Modulated carriers coded losslessly with the monitor's filter: exact
    round trip; most blocks choose stream 3; smaller than without it."""
    x = synth.modulated(dt, 40000, 3, b, noise=0.002)
    k, sign = O.monitor_stride(b)
    with_f = O.encode(x, {"mode": "lossless", "brick": brick, "filter": (k, sign)})
    plain = O.encode(x, {"mode": "lossless", "brick": brick})
    assert np.array_equal(O.decode(with_f), x)
    st = brute.Stream(with_f)
    assert st.mask & 0x08 and (st.b[46], st.b[47]) == (k, 1 if sign < 0 else 0)
    streams = [int(st.block(j)[0]) & 7 for j in range(st.nblocks)]
    assert streams.count(3) >= st.nblocks // 2
    assert with_f.size < plain.size


def test_lossy_filter_encode_error_bound():
    x = synth.modulated(np.float32, 64 * 300, 4, 512, noise=0.001)
    k, sign = O.monitor_stride(512)
    p = {"mode": "fixed_quality", "brick": (64,), "code": 80, "filter": (k, sign)}
    buf = O.encode(x, p)
    y = O.decode(buf)
    st = brute.Stream(buf)
    assert any((int(st.block(j)[0]) & 7) == 3 for j in range(st.nblocks))
    assert np.abs(x.astype(np.float64) - y).max() <= 0.5 / O.gain(80) + 3 * np.abs(x).max() * 2.0 ** -24


def test_filter_validation_and_header():
    x = synth.modulated(np.int16, 5000, 1, 512)
    for bad in ((17, 1), (0, -1)):
        with pytest.raises(O.OracleError) as e:
            O.encode(x, {"mode": "lossless", "brick": (64,), "filter": bad})
        assert e.value.code == O.E_INVALID
    with pytest.raises(O.OracleError) as e:  # 1-d only
        O.encode(x.reshape(50, 100), {"mode": "lossless", "brick": (4, 16), "filter": (1, -1)})
    assert e.value.code == O.E_INVALID
    buf = O.encode(x, {"mode": "lossless", "brick": (64,), "filter": (3, -1)})
    p = O.stream_info(buf)
    assert p.flags == O.filter_flags(3, -1)
    bad = buf.copy()
    bad[46] = 17
    assert O.decode_rc(bad, np.zeros_like(x)) == O.E_CORRUPT
    bad = buf.copy()
    bad[46] = 0  # a sign without a stride
    assert O.decode_rc(bad, np.zeros_like(x)) == O.E_CORRUPT
