"""CPU checks of the C-ABI library: it loads, exports every symbol the public
header declares, and its host-side logic (validation, bounds, stream-header
parsing) agrees with the oracle.  No GPU call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_1303_4994_amd import apax
    return apax


def declared_functions():
    src = open(os.path.join(ROOT, "include", "apax.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apax_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(A):
    names = declared_functions()
    assert {"apax_profile", "apax_encode", "apax_decode"} <= set(names)
    lib = C.CDLL(A.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


VALIDATION = [
    (np.int16, (1000,), {"mode": "lossless", "brick": (64,)}),
    (np.int16, (1000,), {"mode": "lossless", "brick": (60,)}),
    (np.int16, (1000,), {"mode": "lossless", "brick": (66,)}),
    (np.float32, (1000,), {"mode": "lossless", "brick": (64,)}),
    (np.float32, (64, 64), {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}),
    (np.float32, (64, 64), {"mode": "fixed_rate", "brick": (16, 16), "rate": 100.0}),
    (np.float32, (64, 64), {"mode": "fixed_rate", "brick": (16, 16), "rate": 0.0}),
    (np.float64, (8, 8, 8), {"mode": "fixed_quality", "brick": (4, 4, 8), "code": 16384}),
    (np.float64, (8, 8, 8), {"mode": "fixed_quality", "brick": (4, 4, 8), "code": 16383}),
    (np.int32, (8, 8, 8), {"mode": "fixed_quality", "brick": (4, 4, 8), "code": 1}),
    (np.int32, (8, 8, 8), {"mode": "fixed_quality", "brick": (4, 4, 8), "code": -512}),
    (np.int8, (8, 64), {"mode": "lossless", "brick": (2, 32), "stream_mask": 0x10}),
    (np.int8, (8, 64), {"mode": "lossless", "brick": (2, 32), "stream_mask": 0x28}),
    (np.int8, (8, 64), {"mode": "lossless", "brick": (32, 2)}),
    # blocks above 256 samples, up to 16384 (Sec. 6)
    (np.int16, (100000,), {"mode": "lossless", "brick": (16384,)}),
    (np.int16, (100000,), {"mode": "lossless", "brick": (16388,)}),
    (np.float32, (300, 300), {"mode": "fixed_rate", "brick": (128, 128), "rate": 4.0}),
    (np.float64, (8, 64, 64), {"mode": "fixed_quality", "brick": (16, 32, 32), "code": 0}),
    (np.int8, (8, 64, 64), {"mode": "fixed_rate", "brick": (4, 16, 16), "rate": 2.0, "code": 0}),
    # adaptive rate (Sec. 6 feedback loop): target words from the rate
    (np.float32, (64, 64), {"mode": "adaptive_rate", "brick": (16, 16), "rate": 4.0, "code": 20}),
    (np.float32, (64, 64), {"mode": "adaptive_rate", "brick": (16, 16), "rate": 400.0, "code": 20}),
    (np.float64, (64, 64), {"mode": "adaptive_rate", "brick": (16, 16), "rate": 4.0, "code": 16384}),
    (np.int16, (5000,), {"mode": "adaptive_rate", "brick": (64,), "rate": 2.0, "code": -600}),
    (np.int16, (5000,), {"mode": "adaptive_rate", "brick": (64,), "rate": 2.0, "code": -6}),
    # groups of 8 samples per exponent (Sec. 6)
    (np.int16, (5000,), {"mode": "lossless", "brick": (64,), "group": 8}),
    (np.int16, (5000,), {"mode": "lossless", "brick": (68,), "group": 8}),
    (np.float32, (64, 64), {"mode": "fixed_rate", "brick": (4, 16), "rate": 4.0, "group": 8}),
    (np.float32, (64, 64), {"mode": "fixed_rate", "brick": (4, 12), "rate": 4.0, "group": 8}),
    (np.int8, (64, 64), {"mode": "fixed_rate", "brick": (8, 8), "rate": 7.9, "group": 8}),
    # block and sample counts that would wrap 64-bit products are refused
    (np.float32, (1099509530628, 67108992, 16), {"mode": "fixed_quality", "brick": (2, 2, 16), "code": 0}),
    (np.int16, (1 << 40, 1 << 40, 1 << 40), {"mode": "lossless", "brick": (1, 1, 64)}),
    (np.int16, (1 << 30, 1 << 30), {"mode": "lossless", "brick": (1, 64)}),
]


@pytest.mark.parametrize("dt,shape,params", VALIDATION)
def test_validation_and_bound_match_oracle(A, dt, shape, params):
    import torch
    tdt = {np.int8: torch.int8, np.int16: torch.int16, np.int32: torch.int32,
           np.float32: torch.float32, np.float64: torch.float64}[dt]
    try:
        ob = O.encode_bound(dt, shape, params)
        oe = 0
    except O.OracleError as e:
        oe = e.code
    try:
        gb = A.apax_encode_bound(tdt, shape, params)
        ge = 0
    except A.ApaxError as e:
        ge = e.code
    assert ge == oe
    if oe == 0:
        assert gb == ob


def test_stream_info_parses_oracle_streams(A):
    x = np.arange(3000, dtype=np.int16).reshape(30, 100) // 3
    for params in ({"mode": "lossless", "brick": (4, 16)},
                   {"mode": "fixed_rate", "brick": (4, 16), "rate": 3.0, "code": -20},
                   {"mode": "adaptive_rate", "brick": (4, 16), "rate": 3.0, "code": -20},
                   {"mode": "lossless", "brick": (4, 16), "group": 8}):
        s = O.encode(x, params)
        info = A.apax_stream_info(bytes(s[:64]))
        assert info["shape"] == x.shape and info["brick"] == params["brick"]
        assert info["mode"] == params["mode"]
        assert A.stream_nbytes(bytes(s[:64])) == len(s)
    bad = bytearray(s[:64])
    bad[0] ^= 1
    with pytest.raises(A.ApaxError):
        A.apax_stream_info(bytes(bad))


def test_stream_header_with_wrapping_counts_is_corrupt(A):
    """A 64-byte header whose dims make the block count wrap in 64 bits (to a
    small number that it then also claims) is refused by the host, before any
    kernel could index past the buffers."""
    import struct
    x = np.zeros((4, 4, 32), np.float32)
    s = bytearray(O.encode(x, {"mode": "fixed_quality", "brick": (2, 2, 16), "code": 0})[:64])
    struct.pack_into("<QQQ", s, 16, 1099509530628, 67108992, 16)
    struct.pack_into("<Q", s, 48, 128)          # the wrapped block count
    with pytest.raises(A.ApaxError) as ei:
        A.apax_stream_info(bytes(s))
    assert ei.value.code == A.E_CORRUPT
    with pytest.raises(A.ApaxError) as ei:
        A.stream_nbytes(bytes(s))
    assert ei.value.code == A.E_CORRUPT


def test_stream_size_rejects_oversized_payload(A):
    """apax_stream_size: the payload-word field may not exceed the largest
    encoding of the blocks (and must equal nblocks * budget in fixed rate)."""
    import struct
    x = (np.arange(5000) % 77).astype(np.int16)
    for params in ({"mode": "lossless", "brick": (64,)},
                   {"mode": "fixed_rate", "brick": (64,), "rate": 2.0, "code": 0}):
        s = bytearray(O.encode(x, params)[:64])
        assert A.stream_nbytes(bytes(s)) == len(O.encode(x, params))
        struct.pack_into("<Q", s, 56, 1 << 60)
        with pytest.raises(A.ApaxError) as ei:
            A.stream_nbytes(bytes(s))
        assert ei.value.code == A.E_CORRUPT


def test_noalloc_encode_refuses_arrays_beyond_its_scratch(A):
    """apax_encode_noalloc refuses, on the host and before anything is
    enqueued, an array whose scratch (8 bytes per tile of look-back state)
    would exceed the library's 8 MiB array; no GPU call is made."""
    lib = C.CDLL(A.LIB_PATH)
    lib.apax_encode_noalloc.argtypes = [C.c_void_p, C.POINTER(A.Params), C.c_void_p, C.c_uint64,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
    import torch
    # 2^32 int16 samples in 256-sample blocks: 2^24 blocks, 16 MiB of chosen streams
    p = A.make_params(torch.int16, (1 << 32,), {"mode": "lossless", "brick": (256,)})
    fake = C.c_void_p(1 << 20)  # never dereferenced: the call returns first
    rc = lib.apax_encode_noalloc(fake, C.byref(p), fake, C.c_uint64(2 ** 64 - 1), fake, None, None)
    assert rc == A.E_CAPACITY
    # the profiled operating point is refused too (no profile writes the scratch)
    q = A.make_params(torch.int16, (1000,), {"mode": "lossless", "brick": (256,), "code": A.CODE_PROFILED})
    rc = lib.apax_encode_noalloc(fake, C.byref(q), fake, C.c_uint64(1 << 20), fake, None, None)
    assert rc == A.E_INVALID
