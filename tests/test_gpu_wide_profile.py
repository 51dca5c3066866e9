"""GPU parity of the profiler (Sec. 4) for blocks of more than 256 samples and
for groups of 8 samples per exponent (Sec. 6), which its passes run with one
workgroup per block: bracket, operating point, probe count, stream mask, curve
and metrics equal the oracle's (statistics within 1e-9 relative) in every
mode, 1-/2-/3-d, blocks of 260 to 16384 samples, a subsampled profile (1024
blocks and more), the filter stream; the 2-sigma S2R margin at the profiled
point equals the oracle's exactly; the profile-then-encode call gives the same
profile and stream bytes as the two separate calls."""
import numpy as np
import pytest

from oracle import oracle as O
from profcheck import check_profile, decoded_at

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_4994_amd import apax
    return apax


def field(dt, shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    dt = np.dtype(dt)
    t = np.arange(n)
    base = (np.sin(2 * np.pi * 0.0021 * t) + 0.3 * np.sin(2 * np.pi * 0.037 * t)
            + 0.02 * rng.standard_normal(n)).reshape(shape)
    for ax in range(len(shape)):
        base = base.cumsum(axis=ax) / 8
    if dt.kind == "i":
        return np.rint(base / np.abs(base).max() * 0.45 * np.iinfo(dt).max).astype(dt)
    return (base * 1e2).astype(dt)


CASES = [
    ("f32-1d-B512-fr", np.float32, (512 * 40 + 100,), {"mode": "fixed_rate", "brick": (512,), "rate": 4.0}),
    ("f32-1d-B260-fr-sub", np.float32, (260 * 1100 + 36,), {"mode": "fixed_rate", "brick": (260,), "rate": 3.0}),
    ("i16-1d-B1024-lossless", np.int16, (1024 * 30 + 7,), {"mode": "lossless", "brick": (1024,)}),
    ("i32-2d-32x32-fq", np.int32, (100, 70), {"mode": "fixed_quality", "brick": (32, 32)}),
    ("f64-3d-8x8x16-fq", np.float64, (20, 17, 40), {"mode": "fixed_quality", "brick": (8, 8, 16)}),
    ("f32-2d-64x64-fr", np.float32, (300, 260), {"mode": "fixed_rate", "brick": (64, 64), "rate": 4.0}),
    ("f64-1d-B16384-fr", np.float64, (16384 * 3 + 500,), {"mode": "fixed_rate", "brick": (16384,), "rate": 5.0}),
    ("i8-1d-B4096-fq", np.int8, (4096 * 6 + 12,), {"mode": "fixed_quality", "brick": (4096,)}),
    ("f32-1d-g8-B64-fr", np.float32, (64 * 300 + 20,), {"mode": "fixed_rate", "brick": (64,), "rate": 4.0,
                                                         "group": 8}),
    ("i16-2d-g8-8x16-lossless", np.int16, (90, 70), {"mode": "lossless", "brick": (8, 16), "group": 8}),
    ("f64-3d-g8-4x4x8-fq", np.float64, (12, 20, 33), {"mode": "fixed_quality", "brick": (4, 4, 8), "group": 8}),
    ("f32-1d-g8-B2048-fr", np.float32, (2048 * 12 + 40,), {"mode": "fixed_rate", "brick": (2048,), "rate": 4.0,
                                                            "group": 8}),
    ("i16-1d-B512-filter-lossless", np.int16, (512 * 50,), {"mode": "lossless", "brick": (512,),
                                                            "filter": (2, -1)}),
]


@pytest.mark.parametrize("name,dt,shape,params", CASES, ids=[c[0] for c in CASES])
def test_wide_profile_equals_oracle(A, name, dt, shape, params):
    print(f"case {name}", flush=True)
    x = field(dt, shape, 8)
    pp = dict(params, target_corr=0.9999)
    pg = A.apax_profile(torch.from_numpy(x).to(DEV), pp)
    po = O.profile_dict(O.profile(x, pp))
    _, y = decoded_at(x, pp, po)
    check_profile(pg, po, x, y)


S2R_CASES = [c for c in CASES if c[0] in ("f32-1d-B512-fr", "i32-2d-32x32-fq", "f64-3d-8x8x16-fq",
                                         "i16-1d-B1024-lossless", "f32-1d-g8-B64-fr", "f64-3d-g8-4x4x8-fq")]


@pytest.mark.parametrize("name,dt,shape,params", S2R_CASES, ids=[c[0] for c in S2R_CASES])
def test_wide_s2r_margin(A, name, dt, shape, params):
    print(f"case {name}", flush=True)
    x = field(dt, shape, 8)
    pp = dict(params, target_corr=0.9999)
    xg = torch.from_numpy(x).to(DEV)
    ws = A.workspace(xg.dtype, tuple(x.shape), pp, DEV)
    pg = A.apax_profile(xg, pp, ws=ws)
    ratio, db = A.apax_s2r_margin(xg, pp, ws)
    p_at = dict(pp, code=pg["code"],
                stream_mask=pg["stream_mask"] & (0x7F if pp["mode"] == "fixed_rate" else 0xFF))
    r_o, db_o = O.s2r_margin(x, p_at)
    assert ratio == r_o and db == db_o, (ratio, r_o, db, db_o)


@pytest.mark.parametrize("name", ["f32-1d-B512-fr", "f64-3d-g8-4x4x8-fq", "i16-1d-B1024-lossless"])
def test_wide_profile_encode(A, name):
    """apax_profile_encode_async runs the profile, then the plain encode at
    its point: the same profile and bytes as the separate calls, and the
    oracle's stream at that point."""
    _, dt, shape, params = next(c for c in CASES if c[0] == name)
    x = field(dt, shape, 5)
    pp = dict(params, target_corr=0.9999)
    xg = torch.from_numpy(x).to(DEV)
    ws = A.workspace(xg.dtype, tuple(x.shape), pp, DEV)
    A.apax_status_clear(ws)
    A.apax_profile_async(xg, pp, ws)
    ref, nref = A.apax_encode(xg, dict(pp, code=A.CODE_PROFILED), ws=ws, clear_status=False)
    torch.cuda.synchronize()
    pref = A.apax_profile_read(xg, pp, ws)
    ref = ref[: int(nref.item())].cpu().numpy()
    ws2 = A.workspace(xg.dtype, tuple(x.shape), pp, DEV)
    A.apax_status_clear(ws2)
    buf, nb = A.apax_profile_encode_async(xg, pp, ws2)
    torch.cuda.synchronize()
    assert A.apax_status(ws2) == 0
    assert A.apax_profile_read(xg, pp, ws2) == pref
    got = buf[: int(nb.item())].cpu().numpy()
    assert np.array_equal(got, ref)
    p_at, _ = decoded_at(x, pp, pref)
    assert np.array_equal(got, O.encode(x, p_at))
