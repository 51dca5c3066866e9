"""Pins of the oracle's groups of 8 (Sec. 6: one exponent per group of N = 4
or 8 samples).  The per-block brute-force checks of test_oracle_pins.py run
on group-8 cases as well (size model, payload, stream choice, fixed-rate
search, decode = DQ(Q(x))); here: exponents over 8 samples against their
definition, the header bit, the size relation between N = 4 and N = 8 on
constant-width data, and the refusals."""
import numpy as np
import pytest

import brute
from oracle import oracle as O


def test_group_eps_over_eight_samples():
    rng = np.random.default_rng(1)
    v = rng.integers(-(1 << 20), 1 << 20, 64) >> rng.integers(0, 21, 64)
    import ctypes as C
    out = np.zeros(8, np.int32)
    vv = np.ascontiguousarray(v, np.int64)
    assert O.lib().orc_group_eps_n(vv.ctypes.data_as(C.c_void_p), 8, 8, out.ctypes.data_as(C.c_void_p)) == 0
    for i in range(8):
        assert out[i] == min(31, max(brute.width_brute([x]) for x in v[8 * i:8 * i + 8]))


def test_header_bit_and_refusals():
    x = (np.arange(4096) % 97).astype(np.int16)
    s = O.encode(x, {"mode": "lossless", "brick": (64,), "group": 8})
    assert s[8] == 0x11  # ndim 1, bit 4: groups of 8
    assert O.stream_info(s).flags & 0x4000
    assert np.array_equal(O.decode(s), x)
    bad = s.copy()
    bad[8] = 0x21
    assert O.decode_rc(bad, np.zeros_like(x)) == O.E_CORRUPT
    for brick, shape in (((68,), (4096,)), ((2, 36), (64, 64))):
        with pytest.raises(O.OracleError) as e:
            O.encode(x.reshape(shape), {"mode": "lossless", "brick": brick, "group": 8})
        assert e.value.code == O.E_INVALID


def test_constant_width_blocks_save_half_the_exponents():
    # every sample of width 9 (values 128..255): N = 8 halves the groups; all
    # exponent differences are 0, so tokens are ceil((G-1)/2) pair nibbles;
    # payloads are equal, so the difference is exactly the token nibbles saved
    x = (128 + (np.arange(256 * 8) % 100)).astype(np.int16)
    p = {"mode": "lossless", "brick": (256,), "stream_mask": 0x01}
    s4 = brute.Stream(O.encode(x, p))
    s8 = brute.Stream(O.encode(x, dict(p, group=8)))
    for j in range(s4.nblocks):
        b4 = brute.parse_block(s4.block(j), True, 64, 16, 4)
        b8 = brute.parse_block(s8.block(j), True, 32, 16, 8)
        assert b4[0] == b8[0] == 0
        assert b4[6] - b8[6] == 4 * ((64 - 1 + 1) // 2 - (32 - 1 + 1) // 2)
