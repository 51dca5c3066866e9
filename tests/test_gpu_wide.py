"""GPU parity for blocks of more than 256 samples (Sec. 6 allows 64 to 16384;
the library runs them with one workgroup per block): bitstreams and decodes
byte-identical to the CPU oracle for every dtype, 1-/2-/3-d bricks, every
mode, ragged array edges, blocks of 260 (the first size above one wave's 64
groups), 512, 1024, 4096 and 16384 samples, fixed-rate budgets above any
encoding, the lagged choice, the decode-on-read consumer, and corrupt blocks
flagged exactly where the oracle's decoder refuses them.
"""
import numpy as np
import pytest

import brute
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_4994_amd import apax
    return apax


def field(dt, shape, seed, kind="smooth"):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    dt = np.dtype(dt)
    if kind == "noise":
        if dt.kind == "i":
            info = np.iinfo(dt)
            return rng.integers(info.min, info.max, n, endpoint=True).astype(dt).reshape(shape)
        return rng.standard_normal(n).astype(dt).reshape(shape)
    t = np.arange(n)
    base = (np.sin(2 * np.pi * 0.0021 * t) + 0.3 * np.sin(2 * np.pi * 0.037 * t)
            + 0.02 * rng.standard_normal(n)).reshape(shape)
    for ax in range(len(shape)):
        base = base.cumsum(axis=ax) / 8
    if dt.kind == "i":
        return np.rint(base / np.abs(base).max() * 0.45 * np.iinfo(dt).max).astype(dt)
    return (base * 1e2).astype(dt)


CASES = [
    ("i16-1d-B512-lossless", np.int16, (512 * 40 + 100,), {"mode": "lossless", "brick": (512,)}, "smooth"),
    ("i16-1d-B16384-lossless", np.int16, (16384 * 5 + 1000,), {"mode": "lossless", "brick": (16384,)}, "smooth"),
    ("i32-1d-B4096-noise", np.int32, (4096 * 5 + 12,), {"mode": "lossless", "brick": (4096,)}, "noise"),
    ("i8-2d-32x32-lossless", np.int8, (100, 70), {"mode": "lossless", "brick": (32, 32)}, "smooth"),
    ("i32-3d-8x8x16-lossless", np.int32, (20, 17, 40), {"mode": "lossless", "brick": (8, 8, 16)}, "smooth"),
    ("f32-2d-64x64-fr", np.float32, (300, 260), {"mode": "fixed_rate", "brick": (64, 64), "rate": 4.0, "code": 60},
     "smooth"),
    ("f64-3d-16x32x32-fq", np.float64, (40, 70, 80), {"mode": "fixed_quality", "brick": (16, 32, 32), "code": 200},
     "smooth"),
    ("f32-1d-B16384-fr-top", np.float32, (16384 * 4 + 500,),
     {"mode": "fixed_rate", "brick": (16384,), "rate": 5.0, "code": 16383}, "noise"),
    ("f64-2d-128x128-fr", np.float64, (300, 280), {"mode": "fixed_rate", "brick": (128, 128), "rate": 6.0, "code": 300},
     "smooth"),
    ("f32-1d-B260-fq", np.float32, (5000,), {"mode": "fixed_quality", "brick": (260,), "code": 100}, "smooth"),
    ("i16-2d-16x32-fr", np.int16, (90, 100), {"mode": "fixed_rate", "brick": (16, 32), "rate": 3.0, "code": 0},
     "smooth"),
    ("f32-1d-B1024-fr-bigbudget", np.float32, (10000,),
     {"mode": "fixed_rate", "brick": (1024,), "rate": 0.5, "code": 300}, "noise"),
    ("i8-3d-4x16x16-fr", np.int8, (9, 33, 50), {"mode": "fixed_rate", "brick": (4, 16, 16), "rate": 2.0, "code": 0},
     "smooth"),
    ("i32-2d-64x16-fq", np.int32, (130, 70), {"mode": "fixed_quality", "brick": (64, 16), "code": -40}, "smooth"),
    ("f64-1d-B2048-fq-noise", np.float64, (2048 * 3 + 4,), {"mode": "fixed_quality", "brick": (2048,), "code": 50},
     "noise"),
]


def gpu_roundtrip(A, x, params):
    xg = torch.from_numpy(x).to(DEV)
    ws = A.workspace(xg.dtype, tuple(x.shape), params, DEV)
    buf, nb = A.apax_encode(xg, params, ws=ws)
    assert A.apax_status(ws) == 0
    n = int(nb.item())
    got = buf[:n].cpu().numpy()
    y = A.apax_decode(buf, n, ws=ws)
    assert A.apax_status(ws) == 0
    return got, y.cpu().numpy()


def first_block_diff(got, exp):
    sg, se = brute.Stream(got), brute.Stream(exp)
    for j in range(se.nblocks):
        if not np.array_equal(sg.block(j), se.block(j)):
            return j, [hex(int(w)) for w in sg.block(j)[:8]], [hex(int(w)) for w in se.block(j)[:8]]
    return None


@pytest.mark.parametrize("name,dt,shape,params,kind", CASES, ids=[c[0] for c in CASES])
def test_wide_bitexact(A, name, dt, shape, params, kind):
    print(f"case {name}", flush=True)
    x = field(dt, shape, 5, kind)
    exp = O.encode(x, params)
    got, y = gpu_roundtrip(A, x, params)
    assert got.size == exp.size
    if not np.array_equal(got, exp):
        pytest.fail(f"bitstream differs, first block {first_block_diff(got, exp)}")
    yo = O.decode(exp)
    assert np.array_equal(y.view(np.uint8), yo.view(np.uint8))
    if params["mode"] == "lossless":
        assert np.array_equal(y, x)


LAG = [c for c in CASES if c[3]["mode"] == "lossless"]


@pytest.mark.parametrize("name,dt,shape,params,kind", LAG, ids=[c[0] for c in LAG])
def test_wide_lagged(A, name, dt, shape, params, kind):
    print(f"case {name} lagged", flush=True)
    x = field(dt, shape, 8, kind)
    p = dict(params, lagged=True)
    exp = O.encode(x, p)
    got, y = gpu_roundtrip(A, x, p)
    assert np.array_equal(got, exp)
    assert np.array_equal(y, x)


@pytest.mark.parametrize("name,dt,shape,params,kind", [c for c in CASES if c[0] in (
    "i16-1d-B16384-lossless", "f32-2d-64x64-fr", "f64-3d-16x32x32-fq", "i8-3d-4x16x16-fr")],
    ids=lambda v: v if isinstance(v, str) else None)
def test_wide_decode_dot(A, name, dt, shape, params, kind):
    print(f"case {name} dot", flush=True)
    x = field(dt, shape, 9, kind)
    w = field(dt, shape, 10, "noise")
    xg, wg = torch.from_numpy(x).to(DEV), torch.from_numpy(w).to(DEV)
    buf, nb = A.apax_encode(xg, params)
    n = int(nb.item())
    hdr = bytes(buf[:64].cpu().numpy().tobytes())
    ws = A.workspace(xg.dtype, tuple(x.shape), params, DEV)
    got = float(A.apax_decode_dot(buf, n, hdr, wg, ws=ws).item())
    assert A.apax_status(ws) == 0
    y = O.decode(O.encode(x, params)).astype(np.float64).ravel()
    wd = w.astype(np.float64).ravel()
    assert abs(got - float(np.dot(y, wd))) <= 1e-12 * float(np.abs(y * wd).sum()) + 1e-300


def test_wide_corrupt_blocks_flagged_as_the_oracle(A):
    """Single-bit flips in the words of wide blocks (headers, tokens, payload,
    padding): the GPU decoder reports E_CORRUPT exactly when the oracle's
    decoder refuses the stream, and otherwise decodes what the oracle does."""
    x = field(np.int16, (512 * 12 + 40,), 3)
    params = {"mode": "lossless", "brick": (512,)}
    exp = O.encode(x, params)
    st = brute.Stream(exp)
    ws = A.workspace(torch.int16, x.shape, params, DEV)

    def decode(buf):
        g = torch.from_numpy(buf).to(DEV)
        A.apax_status_clear(ws)
        y = A.apax_decode(g, buf.size, hdr=bytes(exp[:64]), ws=ws)
        return A.apax_status(ws), y.cpu().numpy()

    rc, y = decode(exp.copy())
    assert rc == 0 and np.array_equal(y, x)
    rng = np.random.default_rng(11)
    nflag = 0
    for t in range(40):
        bad = exp.copy()
        j = int(rng.integers(0, st.nblocks))
        w = int(rng.integers(0, st.lens[j]))
        bit = int(rng.integers(0, 32))
        pos = st.area + 4 * (st.offsets[j] + w) + bit // 8
        bad[pos] ^= np.uint8(1 << (bit % 8))
        yo = np.zeros_like(x)
        orc = O.decode_rc(bad, yo)
        print(f"flip block {j} word {w} bit {bit}: oracle rc {orc}", flush=True)
        rc, y = decode(bad)
        if orc == O.E_CORRUPT:
            assert rc == A.E_CORRUPT, (j, w, bit)
            nflag += 1
        else:
            assert orc == 0 and rc == 0, (j, w, bit, orc, rc)
            assert np.array_equal(y, yo), (j, w, bit)
    assert nflag > 0
