"""Pins of the oracle's sequential adaptive loop (Sec. 6: the attenuator's
per-block gain follows a feedback loop towards the desired packet size).

The loop is pinned from its outputs, not by re-running it: closed-form
trajectories when every block is smaller (larger) than the target, the update
rule replayed from the stream's own block lengths, every block equal to the
independent per-block encoder at the replayed code, the quantisation error
bound of each block's code on decode, and the loop's convergence to the
target on a stationary signal."""
import numpy as np
import pytest

import brute
from oracle import oracle as O


def block_codes(buf, isint):
    st = brute.Stream(buf)
    out = []
    for j in range(st.nblocks):
        w0 = int(st.block(j)[0])
        if isint:
            c = (w0 >> 8) & 0x3FF
            c = c - 0x400 if c & 0x200 else c
        else:
            c = (w0 >> 8) & 0xFFFF
            c = c - 0x10000 if c & 0x8000 else c
        out.append(c)
    return st, out


def window(c0, isint):
    cmin, cmax = (-512, 0) if isint else (-17120, 16383)
    return max(cmin, c0 - O.ADAPT_HALF), min(cmax, c0 + O.ADAPT_HALF - 1)


def smooth(dt, n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    v = np.sin(2 * np.pi * 0.004 * t) + 0.2 * np.sin(2 * np.pi * 0.05 * t) + 0.01 * rng.standard_normal(n)
    v = v * (1.0 + 0.8 * np.sin(2 * np.pi * t / n))  # slowly varying level: the loop has to track it
    if np.dtype(dt).kind == "i":
        return np.rint(v / np.abs(v).max() * 0.4 * np.iinfo(dt).max).astype(dt)
    return (v * 50.0).astype(dt)


def replay_and_check(x, params):
    """The update rule replayed from the stream's block lengths; each block
    equal to the per-block encoder (fixed quality) at the replayed code."""
    isint = x.dtype.kind == "i"
    buf = O.encode(x, params)
    st, codes = block_codes(buf, isint)
    assert st.mode == O.ADAPTIVE_RATE
    T = st.budget
    c0 = params["code"]
    lo, hi = window(c0, isint)
    state = c0
    fq = {k: v for k, v in params.items() if k not in ("rate",)}
    fq["mode"] = "fixed_quality"
    for j in range(st.nblocks):
        _, cf, cc = O.block_bracket(x, params, j)
        assert codes[j] == min(max(state, cf), cc), j
        words, _, cj, _ = O.encode_block(x, dict(fq, code=state), j)
        assert cj == codes[j]
        assert np.array_equal(st.block(j), words), j
        n = st.lens[j]
        state += 1 if n < T else (-1 if n > T else 0)
        state = min(max(state, lo), hi)
    return buf, st, codes


@pytest.mark.parametrize("dt,shape,brick,rate,code", [
    (np.float32, (64 * 40,), (64,), 4.0, 40),
    (np.float64, (30, 40), (8, 8), 6.0, 250),
    (np.int16, (4000,), (128,), 3.0, -2),
    (np.int32, (6, 10, 12), (2, 4, 8), 2.5, -30),
    (np.float32, (512 * 6 + 30,), (512,), 5.0, 60),
])
def test_update_rule_and_blocks(dt, shape, brick, rate, code):
    n = int(np.prod(shape))
    x = smooth(dt, n, 3).reshape(shape)
    params = {"mode": "adaptive_rate", "brick": brick, "rate": rate, "code": code}
    buf, st, codes = replay_and_check(x, params)
    # each block's reconstruction error stays within its code's quantisation bound
    y = O.decode(buf)
    if x.dtype.kind == "f":
        nb = st.nblocks
        assert nb == len(codes)
        err = np.abs(x.astype(np.float64) - y.astype(np.float64)).max()
        cmin = min(codes)
        bound = 0.5 / O.gain(cmin) + np.abs(x).max() * (2.0 ** -23 if x.dtype == np.float32 else 2.0 ** -52) * 2
        assert err <= bound


def test_closed_form_when_every_block_fits():
    # a target far above any block's size: the requested code climbs one step
    # per block from c0 to the window's top and stays there
    x = smooth(np.float32, 64 * 50, 4)
    c0 = 30
    params = {"mode": "adaptive_rate", "brick": (64,), "rate": 0.05, "code": c0}
    st, codes = block_codes(O.encode(x, params), False)
    assert st.budget == (64 * 8 * 4 * 20) // 32 and st.budget > max(st.lens)
    lo, hi = window(c0, False)
    for j in range(st.nblocks):
        _, cf, cc = O.block_bracket(x, params, j)
        assert codes[j] == min(max(min(c0 + j, hi), cf), cc)


def test_closed_form_when_no_block_fits():
    # a one-word target (every float block header alone takes 48 bits): the
    # requested code falls one step per block to the window's bottom
    x = smooth(np.float32, 64 * 50, 5)
    c0 = 100
    params = {"mode": "adaptive_rate", "brick": (64,), "rate": 64.0, "code": c0}
    st, codes = block_codes(O.encode(x, params), False)
    assert st.budget == 1
    lo, hi = window(c0, False)
    for j in range(st.nblocks):
        _, cf, cc = O.block_bracket(x, params, j)
        assert codes[j] == min(max(max(c0 - j, lo), cf), cc)


def test_window_clipped_at_code_range():
    x = smooth(np.int16, 64 * 30, 6)
    params = {"mode": "adaptive_rate", "brick": (64,), "rate": 0.2, "code": -10}
    st, codes = block_codes(O.encode(x, params), True)
    # integer codes stop at 0 (the attenuator never amplifies an integer)
    assert max(codes) == 0 and codes[-1] == 0


def test_converges_to_target_on_stationary_noise():
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(256 * 400) * 10.0).astype(np.float32)
    params = {"mode": "adaptive_rate", "brick": (256,), "rate": 4.0, "code": 40}
    st, codes = block_codes(O.encode(x, params), False)
    T = st.budget
    tail = np.array(st.lens[200:], np.float64)
    # the state hovers at the crossing (noise moves it a few steps either way)
    assert abs(tail.mean() - T) <= 0.05 * T
    assert max(codes[200:]) - min(codes[200:]) <= 8


def test_validation():
    x = smooth(np.float32, 1000, 1)
    with pytest.raises(O.OracleError) as e:  # target below one word
        O.encode(x, {"mode": "adaptive_rate", "brick": (64,), "rate": 100.0, "code": 0})
    assert e.value.code == O.E_INVALID
    with pytest.raises(O.OracleError) as e:
        O.encode(x, {"mode": "adaptive_rate", "brick": (64,), "rate": 4.0, "code": 16384})
    assert e.value.code == O.E_INVALID
    with pytest.raises(O.OracleError) as e:
        O.profile(x, {"mode": "adaptive_rate", "brick": (64,), "rate": 4.0})
    assert e.value.code == O.E_UNSUPPORTED
