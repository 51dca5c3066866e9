"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against what the paper or mathematics fixes:
hand-derived golden blocks, brute force on tiny inputs (widths by search, JEE
costs by dynamic programming over every parse, stream choice by trying every
stream), library routines (numpy.diff / numpy.cumsum / numpy.rint /
math.fsum), closed forms and invariants.  See tests/brute.py.
"""
import math
import os
import struct

import numpy as np
import pytest

import brute
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        out[k.strip()] = v.split()
    return out


# ---------------------------------------------------------------- gain grid

def test_gain_grid_exact_and_monotone():
    prev = None
    for c in list(range(-600, 600)) + [-17120, -17119, 16383, 16000, -16000]:
        g = O.gain(c)
        assert g == brute.gain(c), c  # exact binary64 value of (16+f) 2^(k-4)
        if prev is not None and c > prev[0]:
            assert g > prev[1]
        prev = (c, g)
    assert O.gain(0) == 1.0
    assert O.gain(16) == 2.0 and O.gain(-16) == 0.5
    for f in range(16):
        assert O.inv_gain_mantissa(f) == float(brute.Fraction(16, 16 + f))


def _largest(M, lim, cmin, cmax):
    # linear scan from the top: the definition itself, no bisection
    for c in range(cmax, cmin - 1, -1):
        if M * brute.gain(c) <= lim:
            return c
    raise AssertionError


@pytest.mark.parametrize("dt,vals", [
    (np.float32, [1e3, 3.0, 1e-30, 3.4e38, 0.0, 7.25, 2.0 ** -140]),
    (np.float64, [1.0, 1e300, 1e-300, 5e-324, 123456.789, 0.0]),
    (np.int16, [32767, -32768, 1, 0, 100]),
    (np.int32, [2 ** 31 - 1, -2 ** 31, 1, 0]),
    (np.int8, [127, -128, 3, 0]),
])
def test_block_bracket_bruteforce(dt, vals):
    isint = np.dtype(dt).kind == "i"
    cmin, cmax = (-512, 0) if isint else (-17120, 16383)
    for v in vals:
        x = np.zeros(64, dt)
        x[5] = v
        M, cf, cc = O.block_bracket(x, {"mode": "fixed_quality", "brick": (64,)}, 0)
        assert M == abs(float(x[5]))
        assert cf == _largest(M, 0.5, cmin, cmax)
        assert cc == (0 if isint else _largest(M, 2 ** 31 - 1, cmin, cmax))
        # at c_floor every sample quantizes to 0, one code above not (M > 0)
        assert np.rint(M * brute.gain(cf)) == 0
        if M > 0 and cf < cmax:
            assert np.rint(M * brute.gain(cf + 1)) != 0


# ---------------------------------------------------------------- streams

BRICKS = [(64,), (8, 8), (4, 16), (2, 4, 8), (4, 4, 4)]


@pytest.mark.parametrize("brick", BRICKS)
@pytest.mark.parametrize("W", [8, 16, 32])
def test_streams_match_numpy_diff_and_invert_by_cumsum(brick, W):
    rng = np.random.default_rng(W + len(brick))
    nd = len(brick)
    allowed = {1: [0, 1, 2], 2: [0, 1, 2, 3, 5], 3: [0, 1, 2, 3, 4, 5, 6]}[nd]
    b3 = (1,) * (3 - nd) + tuple(brick)
    for trial in range(4):
        a = rng.integers(-(1 << (W - 1)), 1 << (W - 1), size=b3, dtype=np.int64)
        if trial == 1:
            a = np.clip(a, -3, 3)
        for s in allowed:
            v = O.stream_values(a, b3, W, s).reshape(b3)
            assert np.array_equal(v, brute.stream_np(a, s, W)), (brick, W, s)
            assert np.array_equal(brute.unstream_np(v, s, W), brute.wrap(a, W)), (brick, W, s)


def test_stream_closed_forms():
    n = np.arange(256, dtype=np.int64)
    ramp = 7 + 3 * n
    v = O.stream_values(ramp, (1, 1, 256), 32, 2)
    # second difference of a ramp: only samples 0 and 1 survive (edge terms)
    assert v[0] == 7 and v[1] == 3 - 7 and np.all(v[2:] == 0)
    yy, xx = np.mgrid[0:16, 0:16]
    plane = 5 + 2 * xx + 3 * yy
    v = O.stream_values(plane, (1, 16, 16), 32, 5).reshape(16, 16)
    assert v[0, 0] == 5 and np.all(v[1:, 1:] == 0)
    assert np.all(v[0, 1:] == 2) and np.all(v[1:, 0] == 3)


# ---------------------------------------------------------------- exponents

def test_group_eps_bruteforce():
    rng = np.random.default_rng(3)
    cases = [[0, 0, 0, 0], [-1, 0, 0, 0], [1, 0, 0, 0], [-2, 1, 0, 0], [2, 0, 0, 0],
             [-2 ** 31, 0, 0, 0], [2 ** 31 - 1, 0, 0, 0], [2 ** 30, -2 ** 30, 0, 0],
             [-32768, 32767, 0, 1], [127, -128, 0, 0]]
    for sh in range(0, 32):
        cases += [list(rng.integers(-(1 << sh), 1 << sh, 4)) for _ in range(6)]
    for W in (8, 16, 32):
        for c in cases:
            cw = [int(brute.wrap(t, W)) for t in c]
            e = O.group_eps(np.array(cw, np.int64), W)
            assert int(e[0]) == brute.eps_of(cw), (cw, W)


# ---------------------------------------------------------------- JEE

def _eps_cases():
    rng = np.random.default_rng(11)
    cases = []
    for G in (2, 3, 4, 5, 8, 16, 17):
        for _ in range(60):
            e = [int(rng.integers(0, 32))]
            for _ in range(G - 1):
                e.append(int(np.clip(e[-1] + rng.choice([-5, -3, -2, -1, 0, 0, 0, 1, 1, 2, 3, 7]),
                                     0, 31)))
            cases.append(e)
    # exhaustive over a small alphabet
    import itertools
    for e in itertools.product([0, 1, 2, 4], repeat=5):
        cases.append(list(e))
    return cases


def test_jee_greedy_is_minimal_and_decodes():
    for eps in _eps_cases():
        nib = O.jee_tokens(eps)
        assert 4 * len(nib) == brute.jee_min_bits(eps), eps
        dec, used = brute.token_decode(nib, eps[0], len(eps))
        assert dec == eps and used == len(nib)
        assert all(0 <= t <= 15 for t in nib)


def test_token_alphabet_counts():
    # nine 4-bit tokens for two differences in [-1,1]; five for one in [-2,2]
    pair_codes, single_codes = set(), set()
    for da in (-1, 0, 1):
        for db in (-1, 0, 1):
            nib = O.jee_tokens([10, 10 + da, 10 + da + db])
            assert len(nib) == 1
            pair_codes.add(nib[0])
    for d in (-2, -1, 0, 1, 2):
        nib = O.jee_tokens([10, 10 + d])  # one difference, nothing to pair with
        assert len(nib) == 1
        single_codes.add(nib[0])
    assert len(pair_codes) == 9 and len(single_codes) == 5
    assert not (pair_codes & single_codes)
    assert all(t < 14 for t in pair_codes | single_codes)
    # any other difference costs an 8-bit token carrying the exponent
    assert O.jee_tokens([10, 13]) == [14, 13] and O.jee_tokens([0, 31]) == [15, 15]


# ---------------------------------------------------------------- golden

def _block_words_of(x, params):
    s = O.encode(x, params)
    st = brute.Stream(s)
    assert st.nblocks == 1
    return [int(w) for w in st.block(0)], s


def test_golden_zero_block():
    g = read_golden("zero_i16_b64.txt")
    words, s = _block_words_of(np.zeros(64, np.int16), {"mode": "lossless", "brick": (64,)})
    assert words == [int(w, 16) for w in g["block_words"]]
    assert bytes(s).hex() == "".join(g["stream_hex"])


def test_golden_constant_block():
    g = read_golden("const5_i16_b64.txt")
    words, _ = _block_words_of(np.full(64, 5, np.int16), {"mode": "lossless", "brick": (64,)})
    assert words == [int(w, 16) for w in g["block_words"]]


def test_golden_float_impulse():
    g = read_golden("impulse_f32_b64.txt")
    x = np.zeros(64, np.float32)
    x[0] = 3.0
    words, _ = _block_words_of(x, {"mode": "fixed_quality", "brick": (64,), "code": 0})
    assert words == [int(w, 16) for w in g["block_words"]]


def test_closed_form_all_zero_and_constant_sizes():
    # all-zero block at G = 64: H + 4 * ceil(63/2) = 32 + 128 bits = 5 words
    s = O.encode(np.zeros(256 * 3, np.int16), {"mode": "lossless", "brick": (256,)})
    assert brute.Stream(s).lens == [5, 5, 5]
    # constant alpha under dx: H + 132 + 4 w(alpha) bits (w > 2)
    for alpha in (5, 100, -7000, 32767):
        s = O.encode(np.full(256, alpha, np.int16), {"mode": "lossless", "brick": (256,)})
        st = brute.Stream(s)
        w = brute.width_brute([alpha])
        assert st.lens[0] == (32 + 132 + 4 * w + 31) // 32, alpha
        assert brute.parse_block(st.block(0), True, 64, 16)[0] == 1


# ---------------------------------------------------------------- whole-block pins

def _quantized_block(x3, cj, isint, lossless):
    if lossless:
        return x3.astype(np.int64)
    return np.rint(x3.astype(np.float64) * brute.gain(cj)).astype(np.int64)


def _blocks_of(x, brick):
    """(j, brick array padded with 0, valid mask) in the container's block order."""
    nd = x.ndim
    b3 = (1,) * (3 - nd) + tuple(brick)
    x3 = x.reshape((1,) * (3 - nd) + x.shape)
    nz, ny, nx = x3.shape
    j = 0
    for bz in range(0, nz, b3[0]):
        for by in range(0, ny, b3[1]):
            for bx in range(0, nx, b3[2]):
                blk = np.zeros(b3, x.dtype)
                val = np.zeros(b3, bool)
                sub = x3[bz:bz + b3[0], by:by + b3[1], bx:bx + b3[2]]
                blk[:sub.shape[0], :sub.shape[1], :sub.shape[2]] = sub
                val[:sub.shape[0], :sub.shape[1], :sub.shape[2]] = True
                yield j, blk, val
                j += 1


W_OF = {np.dtype(np.int8): 8, np.dtype(np.int16): 16, np.dtype(np.int32): 32,
        np.dtype(np.float32): 32, np.dtype(np.float64): 32}


def _check_blocks(x, params, s):
    """Every block: chosen stream is the brute-force argmin (ties -> lowest),
    the used bits equal the size model, the payload equals the stream values
    recomputed with numpy.diff, and the block decodes independently."""
    st = brute.Stream(s)
    isint = x.dtype.kind == "i"
    W, H = W_OF[x.dtype], (32 if isint else 48)
    lossless = params["mode"] == "lossless"
    mask = st.mask
    brick = params["brick"]
    n = params.get("group", 4)
    G = int(np.prod(brick)) // n
    for j, blk, val in _blocks_of(x, brick):
        words = st.block(j)
        sid, eps0, code, eps, nib, vals, used = brute.parse_block(words, isint, G, W, n)
        a = np.where(val, _quantized_block(blk, code, isint, lossless), 0)
        sizes = {s_: brute.size_model(a, s_, W, H, val, n) for s_ in range(8) if mask >> s_ & 1}
        if params["mode"] != "fixed_rate":
            best = min(sizes.values())
            assert sid == min(k for k, v in sizes.items() if v == best), (j, sizes, sid)
        assert used == sizes[sid], (j, used, sizes)
        if sid == 7:
            assert vals == list(brute.wrap(a, W).ravel())
        else:
            v = np.where(val, brute.stream_np(a, sid, W), 0).ravel()
            assert vals == list(v), j
        # padding
        if params["mode"] == "fixed_rate":
            assert len(words) == st.budget and used <= 32 * st.budget
        else:
            assert len(words) == (used + 31) // 32
    return st


CASES = [
    (np.int16, (1000,), {"mode": "lossless", "brick": (64,)}),
    (np.int16, (700,), {"mode": "lossless", "brick": (256,)}),
    (np.int8, (20, 30), {"mode": "lossless", "brick": (8, 8)}),
    (np.int32, (5, 9, 13), {"mode": "lossless", "brick": (2, 4, 8)}),
    (np.float32, (33, 40), {"mode": "fixed_quality", "brick": (4, 16), "code": 40}),
    (np.float64, (3, 10, 17), {"mode": "fixed_quality", "brick": (2, 4, 8), "code": 200}),
    (np.float32, (600,), {"mode": "fixed_rate", "brick": (128,), "rate": 4.0, "code": 60}),
    (np.float64, (20, 24), {"mode": "fixed_rate", "brick": (8, 8), "rate": 6.0, "code": 300}),
    (np.int16, (900,), {"mode": "fixed_rate", "brick": (64,), "rate": 3.0, "code": 0}),
    (np.int32, (12, 12), {"mode": "fixed_quality", "brick": (4, 16), "code": -40}),
    # groups of 8 samples per exponent (Sec. 6 "groups of 4 or 8")
    (np.int16, (1000,), {"mode": "lossless", "brick": (64,), "group": 8}),
    (np.int32, (5, 9, 16), {"mode": "lossless", "brick": (2, 4, 8), "group": 8}),
    (np.float32, (33, 40), {"mode": "fixed_quality", "brick": (4, 16), "code": 40, "group": 8}),
    (np.float64, (20, 24), {"mode": "fixed_rate", "brick": (8, 8), "rate": 6.0, "code": 300, "group": 8}),
    (np.int8, (700,), {"mode": "fixed_rate", "brick": (128,), "rate": 2.0, "code": 0, "group": 8}),
]


def _tiny_input(dt, shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    t = np.arange(n)
    base = np.sin(2 * np.pi * 0.013 * t) * 0.9 + 0.05 * rng.standard_normal(n)
    base = base.reshape(shape).cumsum(axis=-1) / 4
    dt = np.dtype(dt)
    if dt.kind == "i":
        return np.rint(base / np.abs(base).max() * 0.45 * np.iinfo(dt).max).astype(dt)
    return (base * 1e2).astype(dt)


def test_incompressible_blocks_go_verbatim():
    # full-scale white noise: every BFPE stream costs more than B*W + H
    rng = np.random.default_rng(12)
    for dt, W in ((np.int16, 16), (np.int8, 8), (np.int32, 32)):
        info = np.iinfo(dt)
        x = rng.integers(info.min, info.max, 700, endpoint=True).astype(dt)
        # verbatim stays allowed even when the caller's mask leaves it out
        params = {"mode": "lossless", "brick": (256,), "stream_mask": 0x07}
        s = O.encode(x, params)
        st = _check_blocks(x, params, s)
        sids = [brute.parse_block(st.block(j), True, 64, W)[0] for j in range(st.nblocks)]
        assert 7 in sids, sids
        assert np.array_equal(O.decode(s), x)


@pytest.mark.parametrize("dt,shape,params", CASES)
def test_blocks_against_bruteforce(dt, shape, params):
    x = _tiny_input(dt, shape, 5)
    s = O.encode(x, params)
    st = _check_blocks(x, params, s)
    # index: offsets are the exclusive prefix sum of the lengths; superblock
    # offsets sit at every 64th block
    for k, off in enumerate(st.sbo):
        assert off == st.offsets[64 * k]
    assert st.total_words == st.payload_words
    assert len(s) == st.area + 4 * st.payload_words
    # each block equals the oracle's stand-alone block encoder
    p = dict(params)
    for j in range(0, st.nblocks, max(1, st.nblocks // 7)):
        w, sid, cj, ub = O.encode_block(x, p, j)
        assert np.array_equal(w, st.block(j))


@pytest.mark.parametrize("dt,shape,params", CASES)
def test_decode_is_dq_of_q_and_error_bound(dt, shape, params):
    x = _tiny_input(dt, shape, 6)
    s = O.encode(x, params)
    y = O.decode(s)
    assert y.dtype == x.dtype and y.shape == x.shape
    st = brute.Stream(s)
    isint = x.dtype.kind == "i"
    if params["mode"] == "lossless":
        assert np.array_equal(x, y)
        return
    n = params.get("group", 4)
    G = int(np.prod(params["brick"])) // n
    W = W_OF[x.dtype]
    for (j, blk, val), (_, yblk, _) in zip(_blocks_of(x, params["brick"]),
                                          _blocks_of(y, params["brick"])):
        code = brute.parse_block(st.block(j), isint, G, W, n)[2]
        a = _quantized_block(blk, code, isint, False)
        yd = brute.dequant_np(a, code)
        if x.dtype == np.float32:
            exp = yd.astype(np.float32)
        elif x.dtype == np.float64:
            exp = yd
        else:
            info = np.iinfo(x.dtype)
            exp = np.clip(np.rint(yd), info.min, info.max).astype(x.dtype)
        assert np.array_equal(exp[val], yblk[val]), j
        # reconstruction error bound implied by the attenuation
        g = brute.gain(code)
        bound = 0.5 / g * (1 + 2.0 ** -50)
        err = np.abs(blk.astype(np.float64) - yblk.astype(np.float64))[val]
        extra = np.abs(yblk.astype(np.float64))[val] * (2.0 ** -23 if x.dtype == np.float32 else 0)
        if isint:
            extra = extra + 0.5 + 1.0  # rint of the dequantized value, and clamping at the top
        assert np.all(err <= bound + extra), j


# ---------------------------------------------------------------- fixed rate

def _py_bracket(M, isint):
    cmin, cmax = (-512, 0) if isint else (-17120, 16383)

    def largest(lim):
        if M * brute.gain(cmax) <= lim:
            return cmax
        lo, hi = cmin, cmax
        while hi - lo > 1:
            mid = lo + ((hi - lo) >> 1)
            if M * brute.gain(mid) <= lim:
                lo = mid
            else:
                hi = mid
        return lo
    return largest(0.5), (0 if isint else largest(2 ** 31 - 1))


def _py_fixed_rate(blk, val, cp, mask, budget_bits, W, H, isint, n=4):
    M = float(np.abs(blk.astype(np.float64))[val].max()) if val.any() else 0.0
    cf, cc = _py_bracket(M, isint)
    c = min(max(cp, cf), cc)

    def size(s_, c_):
        a = np.where(val, np.rint(blk.astype(np.float64) * brute.gain(c_)).astype(np.int64), 0)
        return brute.size_model(a, s_, W, H, val, n)
    sizes = {s_: size(s_, c) for s_ in range(7) if mask >> s_ & 1}
    best = min(sizes.values())
    s_star = min(k for k, v in sizes.items() if v == best)
    if best <= budget_bits:
        return c, s_star
    hi = c
    while True:
        c = max(c - 16, cf)
        if size(s_star, c) <= budget_bits:
            break
        hi = c
    lo = c
    while hi - lo > 1:
        mid = lo + ((hi - lo) >> 1)
        if size(s_star, mid) <= budget_bits:
            lo = mid
        else:
            hi = mid
    return lo, s_star


@pytest.mark.parametrize("dt,shape,params", [c for c in CASES if c[2]["mode"] == "fixed_rate"])
def test_fixed_rate_search_replicated(dt, shape, params):
    x = _tiny_input(dt, shape, 7)
    s = O.encode(x, params)
    st = brute.Stream(s)
    isint = x.dtype.kind == "i"
    W, H = W_OF[x.dtype], (32 if isint else 48)
    n = params.get("group", 4)
    G = int(np.prod(params["brick"])) // n
    bpb = 8 * x.dtype.itemsize * int(np.prod(params["brick"]))
    assert st.budget == math.floor(bpb / (params["rate"] * 32))
    for j, blk, val in _blocks_of(x, params["brick"]):
        assert len(st.block(j)) == st.budget
        sid, _, code, *_ = brute.parse_block(st.block(j), isint, G, W, n)
        exp_c, exp_s = _py_fixed_rate(blk, val, params["code"], st.mask, 32 * st.budget, W, H,
                                      isint, n)
        assert (code, sid) == (exp_c, exp_s), j


def test_fixed_rate_search_non_monotone_blocks():
    """Noisy blocks started at the top of their bracket: every block descends.
    Size vs. code is not monotone near the budget, so for some blocks the
    procedure's result is not the largest fitting code: the result is pinned
    by replaying the procedure, not by an optimum."""
    rng = np.random.default_rng(0)
    n = 64 * 200
    x = (np.cumsum(rng.standard_normal(n)) + rng.standard_normal(n)).astype(np.float32)
    params = {"mode": "fixed_rate", "brick": (64,), "rate": 5.0, "code": 16383}
    s = O.encode(x, params)
    st = brute.Stream(s)
    W, H, isint = 32, 48, False
    not_largest = 0
    for j, blk, val in _blocks_of(x, (64,)):
        sid, _, code, *_ = brute.parse_block(st.block(j), isint, 16, W)
        exp_c, exp_s = _py_fixed_rate(blk, val, params["code"], st.mask, 32 * st.budget, W, H,
                                      isint)
        assert (code, sid) == (exp_c, exp_s), j
        for c in range(code + 1, code + 17):
            a = np.rint(blk.astype(np.float64) * brute.gain(c)).astype(np.int64)
            if brute.size_model(a, sid, W, H, val) <= 32 * st.budget:
                not_largest += 1
                break
    assert not_largest > 0


# ---------------------------------------------------------------- statistics

def test_stats_against_fsum_and_closed_forms():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(1000) * 10
    y = x + rng.standard_normal(1000) * 1e-3
    m = O.stats(x, y)
    d = x - y
    assert m["sxx"] == math.fsum(x * x)
    assert m["sdd"] == math.fsum(d * d)
    assert abs(m["sds"] - math.fsum(d * (x + y))) <= 1e-15 * math.fsum(abs(d * (x + y)))
    r_printed = math.fsum(x * y) / math.sqrt(math.fsum(x * x) * math.fsum(y * y))
    assert abs(m["r"] - r_printed) < 1e-14
    assert abs(m["snr_db"] - 10 * math.log10(math.fsum(x * x) / math.fsum(d * d))) < 1e-12
    assert abs(m["rms_db"] - 20 * math.log10(m["rms_pct"] / 100)) < 1e-12
    assert abs(m["std_x"] - np.std(x)) < 1e-12 * np.std(x)
    # y = alpha x -> r = 1
    assert abs(O.stats(x, 3.0 * x)["r"] - 1.0) < 1e-15
    # residual orthogonal to x: r = |x| / sqrt(|x|^2 + |d|^2)
    dd = rng.standard_normal(1000)
    dd -= x * (math.fsum(x * dd) / math.fsum(x * x))
    yy = x - dd
    exp = math.sqrt(math.fsum(x * x)) / math.sqrt(math.fsum(x * x) + math.fsum(dd * dd))
    assert abs(O.stats(x, yy)["r"] - exp) < 1e-12
    # all-zero decode: r reported as 0
    assert O.stats(x, np.zeros_like(x))["r"] == 0.0


# ---------------------------------------------------------------- profiler

def _py_r(x, params, c):
    isint = x.dtype.kind == "i"
    xs, ys = [], []
    for j, blk, val in _blocks_of(x, params["brick"]):
        M = float(np.abs(blk.astype(np.float64))[val].max()) if val.any() else 0.0
        cf, cc = _py_bracket(M, isint)
        cj = min(max(c, cf), cc)
        a = np.rint(blk.astype(np.float64) * brute.gain(cj))
        yd = brute.dequant_np(a, cj)
        if x.dtype == np.float32:
            yd = yd.astype(np.float32).astype(np.float64)
        xs.append(blk.astype(np.float64)[val])
        ys.append(yd[val])
    xv, yv = np.concatenate(xs), np.concatenate(ys)
    sxy, sxx, syy = math.fsum(xv * yv), math.fsum(xv * xv), math.fsum(yv * yv)
    return 0.0 if syy == 0 else sxy / math.sqrt(sxx * syy)


def test_profile_fixed_quality_bruteforce():
    x = _tiny_input(np.float32, (24, 32), 21)
    params = {"mode": "fixed_quality", "brick": (8, 8), "target_corr": 0.9999}
    r = O.profile_dict(O.profile(x, params))
    cf, cc = _py_bracket(float(np.abs(x).max()), False)
    assert (r["c_floor"], r["c_cap"]) == (cf, cc)
    # replay the bisection on brute-force r(c)
    lo, hi = cf, cc
    assert _py_r(x, params, hi) >= params["target_corr"]
    while hi - lo > 1:
        mid = lo + ((hi - lo) >> 1)
        if _py_r(x, params, mid) >= params["target_corr"]:
            hi = mid
        else:
            lo = mid
    assert r["code"] == hi
    assert r["metrics"]["r"] >= params["target_corr"]
    assert abs(r["metrics"]["r"] - _py_r(x, params, hi)) < 1e-13
    assert [c for c, _, _ in r["curve"]] == [hi + 4 * (t - 8) for t in range(17)]
    # encoded size at the chosen code matches the reported ratio
    s = O.encode(x, dict(params, code=r["code"], stream_mask=r["stream_mask"]))
    assert r["metrics"]["enc_bytes"] == len(s)
    assert abs(r["metrics"]["ratio"] - x.nbytes / len(s)) < 1e-12


def test_profile_fixed_rate_bruteforce():
    x = _tiny_input(np.float32, (640,), 22)
    params = {"mode": "fixed_rate", "brick": (64,), "rate": 4.0}
    r = O.profile_dict(O.profile(x, params))
    isint = False
    W, H = 32, 48
    budget = math.floor(64 * 32 / (4.0 * 32))
    blocks = list(_blocks_of(x, (64,)))
    need = math.ceil(0.9 * len(blocks))

    def fits(c):
        n = 0
        for j, blk, val in blocks:
            M = float(np.abs(blk.astype(np.float64))[val].max())
            cf, cc = _py_bracket(M, isint)
            a = np.where(val, np.rint(blk.astype(np.float64) * brute.gain(min(max(c, cf), cc))), 0)
            a = a.astype(np.int64)
            if min(brute.size_model(a, s_, W, H, val) for s_ in (0, 1, 2)) <= 32 * budget:
                n += 1
        return n >= need
    cf, cc = _py_bracket(float(np.abs(x).max()), False)
    assert not fits(cc)
    lo, hi = cf, cc
    while hi - lo > 1:
        mid = lo + ((hi - lo) >> 1)
        if fits(mid):
            lo = mid
        else:
            hi = mid
    assert r["code"] == lo
    # final metrics are those of an encode at the recommended point
    s = O.encode(x, dict(params, code=r["code"], stream_mask=r["stream_mask"] & 0x7F))
    y = O.decode(s)
    m = O.stats(x.astype(np.float64), y.astype(np.float64))
    assert abs(m["r"] - r["metrics"]["r"]) < 1e-14
    assert r["metrics"]["enc_bytes"] == len(s)


def test_profile_lossless_and_mask():
    x = _tiny_input(np.int16, (4096,), 23)
    r = O.profile_dict(O.profile(x, {"mode": "lossless", "brick": (256,)}))
    assert r["code"] == 0 and r["metrics"]["r"] == 1.0 and r["metrics"]["sdd"] == 0.0
    s = O.encode(x, {"mode": "lossless", "brick": (256,), "stream_mask": r["stream_mask"]})
    assert r["metrics"]["enc_bytes"] == len(s)
    st = brute.Stream(s)
    used = {brute.parse_block(st.block(j), True, 64, 16)[0] for j in range(st.nblocks)}
    assert used <= {s_ for s_ in range(8) if r["stream_mask"] >> s_ & 1}
    assert r["stream_mask"] & 0x81 == 0x81


# ---------------------------------------------------------------- validation / errors

def test_validation_block_size_rules():
    # Sec. 6: block size between 64 and 16384, any multiple of 4
    for B, ok in [(60, False), (64, True), (68, True), (66, False), (16384, True),
                  (16388, False)]:
        try:
            O.encode_bound(np.int16, (1000,), {"mode": "lossless", "brick": (B,)})
            assert ok, B
        except O.OracleError as e:
            assert not ok and e.code == O.E_INVALID, B
    with pytest.raises(O.OracleError) as e:
        O.encode_bound(np.float32, (1000,), {"mode": "lossless", "brick": (64,)})
    assert e.value.code == O.E_UNSUPPORTED
    with pytest.raises(O.OracleError):  # budget below an all-zero block
        O.encode_bound(np.float32, (1000,), {"mode": "fixed_rate", "brick": (64,), "rate": 40})
    with pytest.raises(O.OracleError):  # x extent not a multiple of 4
        O.encode_bound(np.int16, (64, 64), {"mode": "lossless", "brick": (32, 2)})


def test_nonfinite_rejected():
    x = np.ones(100, np.float32)
    x[50] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.encode(x, {"mode": "fixed_quality", "brick": (64,), "code": 0})
    assert e.value.code == O.E_NONFINITE


def test_corrupt_streams_detected():
    x = _tiny_input(np.int16, (2000,), 31)
    s = O.encode(x, {"mode": "lossless", "brick": (64,)})
    y = np.zeros_like(x)
    assert O.decode_rc(s, y) == 0
    bad = s.copy()
    bad[0] ^= 1
    assert O.decode_rc(bad, y) == O.E_CORRUPT
    assert O.decode_rc(s[:-4], y) == O.E_CORRUPT
    st = brute.Stream(s)
    bad = s.copy()
    bad[st.area + 3] |= 0x80  # reserved header bit of block 0
    assert O.decode_rc(bad, y) == O.E_CORRUPT
    bad = s.copy()
    struct.pack_into("<H", bad, 64, st.lens[0] + 1)  # index length disagrees
    assert O.decode_rc(bad, y) == O.E_CORRUPT
    assert O.decode_rc(s, np.zeros(10, np.int16)) == O.E_CAPACITY


def test_empty_array():
    s = O.encode(np.zeros(0, np.int16), {"mode": "lossless", "brick": (64,)})
    st = brute.Stream(s)
    assert st.nblocks == 0 and len(s) == st.area
    assert O.decode(s).size == 0


# ------------------------------------------------ Sec. 4 Window 4: 2-sigma S2R margin
def test_s2r_margin_constructed_ranks():
    # ratios 1..n by construction (x = i, y = i - 1): the nearest-rank 4.5th
    # percentile is the ceil(0.045 n)-th smallest
    for n, k in ((1000, 45), (100, 5), (200, 9), (1, 1), (23, 2)):
        x = np.arange(1, n + 1, dtype=np.float64)
        perm = np.random.default_rng(n).permutation(n)
        ratio, db = O.s2r_margin_xy(x[perm], x[perm] - 1)
        assert ratio == float(k)
        assert db == 20.0 * math.log10(k)


def test_s2r_margin_infinities():
    x = np.linspace(1, 2, 100)
    assert O.s2r_margin_xy(x, x) == (float("inf"), float("inf"))  # exact: d = 0
    x0 = np.concatenate([np.zeros(5), np.linspace(1, 2, 95)])
    y0 = x0 - 0.25                                                  # d != 0 everywhere
    assert O.s2r_margin_xy(x0, y0) == (0.0, float("-inf"))          # 5 of 100 zeros reach rank 5
    x1 = np.concatenate([np.zeros(4), np.linspace(1, 2, 96)])
    ratio, _ = O.s2r_margin_xy(x1, x1 - 0.25)
    assert ratio == 4.0                                             # rank 5: the smallest nonzero, 1 / 0.25


def test_s2r_margin_respects_the_attenuation_error_bound():
    # fixed quality at code c: |d| <= 1/(2 g(c)) plus the output rounding, so
    # every ratio is at least 2 g(c) |x| (to 1 %), hence so is the percentile
    rng = np.random.default_rng(5)
    x = (np.cumsum(rng.standard_normal(4096)) * 10 + 50).astype(np.float64)
    for c in (40, 200, 300):
        params = {"mode": "fixed_quality", "brick": (256,), "code": c}
        ratio, _ = O.s2r_margin(x, params)
        ax = np.sort(np.abs(x))
        bound = 2 * O.gain(c) * ax[math.ceil(0.045 * x.size) - 1]
        assert ratio >= 0.99 * bound, (c, ratio, bound)


# ------------------------------------------------ Sec. 4 Windows 3-4: Welch spectra
def test_psd_tone_peak_closed_form():
    # a cosine of amplitude A at bin f0 (integer cycles per segment): the
    # Hann-windowed DFT has |X_f0| = A * sum(w) / 2 = A L / 4, at every segment
    L = O.PSD_L
    for f0, A in ((37, 3.0), (200, 0.5), (511, 10.0)):
        i = np.arange(4 * L)
        x = A * np.cos(2 * np.pi * f0 * i / L)
        P = O.welch_psd(x)
        assert int(np.argmax(P)) + 1 == f0
        assert abs(P.max() / (A * L / 4) ** 2 - 1) < 1e-12
        m = O.spectral_metrics(x, x)
        assert abs(m["peak_x"] - 20 * math.log10(A * L / 4)) < 1e-9
        assert m["resid_mean"] == float("-inf") and m["srr"] == float("inf")  # d = 0


def test_psd_white_noise_level():
    # white noise of variance s2: E P[f] = s2 * sum(w^2) = s2 * 3L/8 for the Hann window
    L = O.PSD_L
    rng = np.random.default_rng(11)
    s = 2.0
    x = rng.standard_normal(1 << 17) * s
    P = O.welch_psd(x)
    assert abs(P.mean() / (s * s * 3 * L / 8) - 1) < 0.03


def test_psd_segments_and_scaling():
    L = O.PSD_L
    for n, K in ((L, 1), (L + L // 2 - 1, 1), (L + L // 2, 2), (3 * L, 5)):
        assert O.spectral_metrics(np.ones(n), np.zeros(n))["segments"] == K
    assert math.isnan(O.spectral_metrics(np.ones(L - 1), np.zeros(L - 1))["peak_x"])
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.standard_normal(8 * L))
    m = O.spectral_metrics(x, x / 2)            # d = x / 2: every P_d = P_x / 4
    assert abs(m["peak_d"] - (m["peak_x"] - 20 * math.log10(2))) < 1e-9
    assert abs(m["floor_d"] - (m["floor_x"] - 20 * math.log10(2))) < 1e-9
    assert abs(m["srr"] - (m["peak_x"] - m["resid_mean"])) < 1e-12
    assert abs(m["dr"] - (m["peak_x"] - m["floor_x"])) < 1e-12


# ------------------------------------------------ lagged stream choice (lossless)
@pytest.mark.parametrize("dt,shape,brick", [(np.int16, (5000,), (64,)), (np.int32, (40, 48), (8, 8)),
                                            (np.int8, (6, 10, 16), (2, 4, 8))])
def test_lagged_stream_is_the_previous_blocks_best(dt, shape, brick):
    rng = np.random.default_rng(4)
    n = int(np.prod(shape))
    base = np.cumsum(rng.standard_normal(n)) * (3 if dt == np.int8 else 25)
    x = np.clip(base, np.iinfo(dt).min, np.iinfo(dt).max).astype(dt).reshape(shape)
    p = {"mode": "lossless", "brick": brick}
    std = brute.Stream(O.encode(x, p))
    lag_buf = O.encode(x, dict(p, lagged=True))
    lag = brute.Stream(lag_buf)
    assert np.array_equal(O.decode(lag_buf), x)                     # still exact
    verbatim_words = (32 + int(np.prod(brick)) * np.dtype(dt).itemsize * 8 + 31) // 32
    if dt == np.int32:
        verbatim_words = (32 + int(np.prod(brick)) * 32 + 31) // 32
    for j in range(std.nblocks):
        own_prev = int(std.block(j - 1)[0] & 7) if j > 0 else 0    # best stream of block j-1
        st = int(lag.block(j)[0] & 7)
        # the previous block's best, or verbatim where that would be larger
        assert st == own_prev or (st == 7 and lag.lens[j] == verbatim_words), j
        assert std.lens[j] <= lag.lens[j] <= verbatim_words        # never below the best, never above verbatim


def test_lagged_noise_falls_back_to_verbatim():
    # white noise: derivative streams are larger than verbatim, so a lagged
    # derivative choice must give way to verbatim
    rng = np.random.default_rng(9)
    x = rng.integers(-32768, 32767, 4096, endpoint=True).astype(np.int16)
    x[:512] = np.arange(512, dtype=np.int16)          # smooth start: derivative is best there
    p = {"mode": "lossless", "brick": (64,)}
    buf = O.encode(x, dict(p, lagged=True))
    s = brute.Stream(buf)
    assert np.array_equal(O.decode(buf), x)
    assert max(s.lens) <= (32 + 64 * 16 + 31) // 32
    assert int(s.block(8)[0] & 7) == 7                 # first noise block: lagged choice was a derivative


def test_lagged_needs_lossless():
    x = np.linspace(0, 1, 1000).astype(np.float32)
    with pytest.raises(O.OracleError):
        O.encode(x, {"mode": "fixed_rate", "brick": (64,), "rate": 4.0, "code": 100, "lagged": True})


# ------------------------------------------------ Sec. 6 signal monitor
def test_autocorr_brute_force_and_wiener_khinchin():
    rng = np.random.default_rng(21)
    x = rng.integers(-50, 50, 40).astype(np.int32)
    R = O.autocorr(x)
    for k in range(O.MON_LAGS + 1):              # the definition, term by term
        want = 0
        for n in range(k, x.size):
            want += int(x[n]) * int(x[n - k])
        assert R[k] == want, k
    # the inverse transform of the zero-padded power spectrum is the same sum
    y = rng.standard_normal(3001)
    F = np.fft.fft(y, 2 * y.size)
    r = np.fft.ifft(np.abs(F) ** 2).real
    assert np.allclose(O.autocorr(y), r[:O.MON_LAGS + 1], rtol=0, atol=1e-9 * r[0])
    short = O.autocorr(np.array([2.0, 3.0, 5.0]))  # lags beyond the array sum nothing
    assert list(short[:3]) == [38.0, 21.0, 10.0] and not short[3:].any()


def test_monitor_stride_matches_tone_cancellation():
    # for a tone at bin b, x[n] - s x[n - k] keeps 2 (1 - s cos(2 pi b k / L)) of
    # its power: the chosen (k, s) reaches the least of it over k = 1..16 (s
    # of the same sign as the cosine), and no smaller lag does as well
    L = O.PSD_L
    assert O.monitor_stride(0) == (0, 0)
    for b in range(1, L // 2 + 1):
        k, s = O.monitor_stride(b)
        res = [1 - abs(math.cos(2 * math.pi * b * j / L)) for j in range(1, 17)]
        assert res[k - 1] <= min(res) + 1e-12, (b, k)
        assert all(res[j - 1] > res[k - 1] + 1e-12 for j in range(1, k)), (b, k)
        c = math.cos(2 * math.pi * b * k / L)
        assert s * c >= -1e-12, (b, k, s)
    assert O.monitor_stride(1) == (1, 1)         # oversampled low-pass: first difference
    assert O.monitor_stride(512) == (1, -1)      # Nyquist tone: x[n] + x[n - 1]
    assert O.monitor_stride(256) == (2, -1)      # quarter rate: x[n] + x[n - 2]


def test_monitor_tone_center_and_gain():
    L = O.PSD_L
    rng = np.random.default_rng(22)
    n = 1 << 16
    i = np.arange(n)
    for b, A in ((3, 5.0), (102, 1.0), (341, 2.0), (500, 0.25)):
        x = A * np.cos(2 * np.pi * b * i / L + 0.3) + 0.001 * rng.standard_normal(n)
        m = O.signal_monitor(x)
        assert m["peak_bin"] == b and m["center_freq"] == b / L
        assert abs(m["peak_db"] - 20 * math.log10(A * L / 4)) < 0.01
        k, s = O.monitor_stride(b)
        assert (m["stride"], m["sign"]) == (k, s)
        # tone A plus white noise sg: the filter keeps 2 (1 - s cos) of the
        # tone's power A^2 / 2 and doubles the noise power sg^2
        th = 2 * math.pi * b * k / L
        want = (A * A / 2 + 1e-6) / (A * A * (1 - s * math.cos(th)) + 2e-6)
        assert abs(m["gain_db"] - 10 * math.log10(want)) < 0.1, (b, m["gain_db"], 10 * math.log10(want))
        # the autocorrelation of a tone is the cosine of its lag phase
        for j in range(1, 17):
            assert abs(m["acf"][j] - math.cos(2 * math.pi * b * j / L)) < 2e-3


def test_monitor_white_noise_and_edges():
    rng = np.random.default_rng(23)
    m = O.signal_monitor(rng.standard_normal(1 << 17))
    assert abs(m["snr_db"]) < 0.3              # flat spectrum: mean over median about 1
    assert np.all(np.abs(m["acf"][1:]) < 0.02) and m["acf"][0] == 1.0
    assert abs(m["gain_db"] + 10 * math.log10(2)) < 0.05  # a filter of white noise doubles it
    short = O.signal_monitor(np.arange(1023, dtype=np.float64))
    assert short["peak_bin"] == 0 and short["stride"] == 0 and math.isnan(short["snr_db"])
    assert short["segments"] == 0 and short["acf"][0] == 1.0
    zero = O.signal_monitor(np.zeros(4096))
    assert not zero["acf"].any() and zero["peak_bin"] == 1 and math.isnan(zero["snr_db"])


# ---------------------------------------------------------------- profile outputs: curve, mask, tie, stats

def _curve_point_bruteforce(x, params, ct, mask):
    """(ratio, r) of Window 1's curve point at code ct: every (subsample)
    block at clamp(ct) to its own bracket, coded with the cheapest allowed
    stream (verbatim allowed), whole 32-bit words per block; r by fsum."""
    isint = x.dtype.kind == "i"
    W, H = (32, 48) if not isint else (8 * x.dtype.itemsize, 32)
    in_bits = out_bits = 0
    for j, blk, val in _blocks_of(x, params["brick"]):
        M = float(np.abs(blk.astype(np.float64))[val].max()) if val.any() else 0.0
        cf, cc = _py_bracket(M, isint)
        cj = min(max(ct, cf), cc)
        a = np.where(val, _quantized_block(blk, cj, isint, False), 0)
        bits = min(brute.size_model(a, s_, W, H, val) for s_ in range(8) if (mask | 0x81) >> s_ & 1)
        in_bits += int(val.sum()) * 8 * x.dtype.itemsize
        out_bits += 32 * ((bits + 31) // 32)
    return in_bits / out_bits, _py_r(x, params, ct)


@pytest.mark.parametrize("dt,shape,params", [
    (np.float32, (24, 32), {"mode": "fixed_quality", "brick": (8, 8), "target_corr": 0.9999}),
    (np.float32, (640,), {"mode": "fixed_rate", "brick": (64,), "rate": 4.0}),
])
def test_profile_curve_ratio_and_r_bruteforce(dt, shape, params):
    """Every point of the rate-correlation curve (Window 1): its ratio from
    an independent size model and its r from exactly rounded sums, at each of
    the 17 quarter-octave codes around the recommended one."""
    x = _tiny_input(dt, shape, 31)
    r = O.profile_dict(O.profile(x, params))
    codes = [min(max(r["code"] + 4 * (t - 8), -17120), 16383) for t in range(17)]
    assert [c for c, _, _ in r["curve"]] == codes
    for c, ratio, rr in r["curve"]:
        er, err = _curve_point_bruteforce(x, params, c, r["stream_mask"])
        assert ratio == er, (c, ratio, er)
        assert abs(rr - err) <= 1e-13, (c, rr, err)


def test_profile_mask_threshold_is_one_percent_rounded_up():
    """Stream mask = {0, 7} and the streams that at least ceil(n_sub / 100)
    subsample blocks choose: 250 blocks (all in the subsample) need 3; three
    ramp blocks (stream 2) get in, two constant blocks (stream 1) do not."""
    B = 64
    blocks = [np.zeros(B, np.int64) for _ in range(250)]
    n = np.arange(B)
    for k in (10, 90, 170):
        blocks[k] = 5 + 300 * n                     # a ramp: only the second difference vanishes
    for k in (40, 200):
        blocks[k] = np.full(B, 9000)                # a constant: the first difference vanishes
    x = np.concatenate(blocks).astype(np.int16)
    params = {"mode": "lossless", "brick": (B,)}
    # each block's cheapest stream, by the independent size model
    chosen = []
    for blk in blocks:
        sizes = {s_: brute.size_model(blk.reshape(1, 1, B), s_, 16, 32) for s_ in (0, 1, 2, 7)}
        best = min(sizes.values())
        chosen.append(min(s_ for s_, v in sizes.items() if v == best))
    assert chosen.count(2) == 3 and chosen.count(1) == 2 and chosen.count(0) == 245
    r = O.profile_dict(O.profile(x, params))
    assert r["n_sub"] == 250
    assert r["stream_mask"] == 0x85, hex(r["stream_mask"])
    # one more constant block makes stream 1 reach the threshold
    blocks[120] = np.full(B, -700)
    r = O.profile_dict(O.profile(np.concatenate(blocks).astype(np.int16), params))
    assert r["stream_mask"] == 0x87, hex(r["stream_mask"])


def _fq_probes(x, params, target):
    """The fixed-quality bisection replayed on exactly rounded r: every
    probe's (code, r) and the resulting code."""
    cf, cc = _py_bracket(float(np.abs(x).max()), False)
    probes = [(cc, _py_r(x, params, cc))]
    if probes[0][1] < target:
        return probes, cc
    lo, hi = cf, cc
    while hi - lo > 1:
        mid = lo + ((hi - lo) >> 1)
        r = _py_r(x, params, mid)
        probes.append((mid, r))
        if r >= target:
            hi = mid
        else:
            lo = mid
    return probes, hi


def test_profile_near_tie_flag():
    """NEAR_TIE is set exactly when some bisection probe's r lies within
    1e-11 of the target: targets placed 0.9e-11 and 1.1e-11 from the r of
    the first inner probe, on both sides, each checked against a replay of
    every probe."""
    x = _tiny_input(np.float32, (24, 32), 21)
    params = {"mode": "fixed_quality", "brick": (8, 8)}
    cf, cc = _py_bracket(float(np.abs(x).max()), False)
    r_mid = _py_r(x, params, cf + ((cc - cf) >> 1))
    seen = set()
    for off in (-1.1e-11, -0.9e-11, 0.9e-11, 1.1e-11, -3e-9):
        t = r_mid + off
        probes, code = _fq_probes(x, params, t)
        dist = min(abs(r - t) for _, r in probes)
        assert abs(dist - 1e-11) > 5e-14            # no probe sits on the threshold itself
        expect = dist < 1e-11
        got = O.profile_dict(O.profile(x, dict(params, target_corr=t)))
        assert bool(got["flags"] & O.NEAR_TIE) == expect, (off, dist, probes)
        assert got["code"] == code and got["n_probes"] == len(probes)
        seen.add(expect)
    assert seen == {True, False}


@pytest.mark.parametrize("dt,shape,params", [
    (np.float32, (24, 32), {"mode": "fixed_quality", "brick": (8, 8), "target_corr": 0.9999}),
    (np.float64, (6, 8, 16), {"mode": "fixed_quality", "brick": (2, 4, 8), "target_corr": 0.99999}),
    (np.float32, (640,), {"mode": "fixed_rate", "brick": (64,), "rate": 4.0}),
    (np.int16, (3000,), {"mode": "fixed_rate", "brick": (64,), "rate": 3.0}),
])
def test_profile_means_stds_maxd_against_decoded_array(dt, shape, params):
    """The profile's own metrics pass (means, population standard deviations
    by two passes, max |d|) equals numpy and exactly rounded sums over the
    array the oracle decodes at the recommended point."""
    x = _tiny_input(dt, shape, 41)
    r = O.profile_dict(O.profile(x, params))
    enc = dict(params, code=r["code"], stream_mask=r["stream_mask"] & (0x7F if params["mode"] == "fixed_rate" else 0xFF))
    y = O.decode(O.encode(x, enc)).astype(np.float64)
    xv = x.astype(np.float64).ravel()
    yv = y.ravel()
    d = xv - yv
    m = r["metrics"]
    nn = xv.size
    for name, v in (("x", xv), ("y", yv), ("d", d)):
        mean = math.fsum(v) / nn
        std = math.sqrt(math.fsum((v - mean) ** 2) / nn)
        assert abs(m[f"mean_{name}"] - mean) <= 1e-13 * max(1.0, abs(mean)), (name, m[f"mean_{name}"], mean)
        assert abs(m[f"std_{name}"] - std) <= 1e-12 * max(1e-300, std), (name, m[f"std_{name}"], std)
    assert m["max_abs_d"] == float(np.abs(d).max())


def test_spectral_floor_is_the_256th_smallest_bin():
    """Tones at bins 1..511 with seeded amplitudes and phases over exactly one
    segment.  The periodic Hann window sin^2(pi n / N) = 1/2 - cos(2 pi n / N) / 2
    turns each bin's DFT X[k] = (N / 2) A_k e^{i phi_k} into
    X[k] / 2 - X[k - 1] / 4 - X[k + 1] / 4, so the whole spectrum is known in
    closed form: the floor is its 256th smallest bin (its neighbours in rank
    differ from it), the peak its largest."""
    N = 1024
    rng = np.random.default_rng(77)
    A = rng.uniform(0.1, 2.0, 513)
    ph = rng.uniform(0, 2 * np.pi, 513)
    A[0] = A[512] = 0.0
    t = np.arange(N)
    x = np.zeros(N)
    for b in range(1, 512):
        x += A[b] * np.cos(2 * np.pi * b * t / N + ph[b])
    X = np.zeros(515, complex)
    X[1:514] = (N / 2) * A * np.exp(1j * ph)     # X[1 + k] holds bin k, zero padding either side
    P = np.abs(X[1:514] / 2 - X[0:513] / 4 - X[2:515] / 4) ** 2
    # Nyquist: its upper neighbour is bin 513 = the conjugate of bin 511
    P[512] = abs(-(X[512] + np.conj(X[512])) / 4) ** 2
    levels = np.sort(P[1:513])
    assert levels[254] < levels[255] < levels[256]
    s = O.spectral_metrics(x, np.zeros_like(x))
    assert abs(s["floor_x"] - 10 * math.log10(levels[255])) < 1e-9
    assert abs(s["peak_x"] - 10 * math.log10(levels[-1])) < 1e-9
    mon = O.signal_monitor(x)
    assert abs(mon["floor_db"] - 10 * math.log10(levels[255])) < 1e-9
