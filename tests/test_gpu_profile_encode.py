"""apax_profile_encode_async (the profiler feeding the encoder, Sec. 4 -> Sec. 6,
in fixed rate the metrics pass writing the stream's blocks itself) against the
separate calls: the same profile result and the same stream bytes as
apax_profile_async followed by apax_encode with APAX_CODE_PROFILED, in every
mode, 1-/2-/3-d, the lagged choice, an empty array and the 4096^2 fp32 field;
and the stream decodes to the oracle's decode of the oracle's encode at the
profiled point."""
import numpy as np
import pytest

import synth
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


def field(dt, shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    t = np.arange(n)
    base = (np.sin(2 * np.pi * 0.013 * t) * 0.9 + 0.05 * rng.standard_normal(n)).reshape(shape)
    base = base.cumsum(axis=-1) / 4
    if np.dtype(dt).kind == "i":
        return np.rint(base / np.abs(base).max() * 0.45 * np.iinfo(dt).max).astype(dt)
    return (base * 1e2).astype(dt)


CASES = [
    ("f32-2d-16x16-fr", np.float32, (300, 260), {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}),
    ("f32-1d-B128-fr", np.float32, (6000,), {"mode": "fixed_rate", "brick": (128,), "rate": 4.0}),
    ("i8-1d-B64-fr", np.int8, (7000,), {"mode": "fixed_rate", "brick": (64,), "rate": 2.0}),
    ("f64-3d-4x4x8-fq", np.float64, (9, 33, 40), {"mode": "fixed_quality", "brick": (4, 4, 8)}),
    ("f32-2d-4x16-fq", np.float32, (70, 64), {"mode": "fixed_quality", "brick": (4, 16)}),
    ("i16-1d-B256-lossless", np.int16, (50000 + 37,), {"mode": "lossless", "brick": (256,)}),
    ("i32-3d-2x4x8-lossless", np.int32, (7, 20, 24), {"mode": "lossless", "brick": (2, 4, 8)}),
    ("i16-1d-lagged", np.int16, (20000,), {"mode": "lossless", "brick": (64,), "lagged": True}),
    ("f32-1d-filter-fr", np.float32, (64 * 300,), {"mode": "fixed_rate", "brick": (64,), "rate": 4.0,
                                                    "filter": (1, -1)}),
    ("f64-3d-4x4x8-fr", np.float64, (9, 33, 40), {"mode": "fixed_rate", "brick": (4, 4, 8), "rate": 3.0}),
    ("i16-2d-8x8-fr", np.int16, (90, 70), {"mode": "fixed_rate", "brick": (8, 8), "rate": 2.5}),
]


def separate(A, xg, params):
    ws = A.workspace(xg.dtype, tuple(xg.shape), params, DEV)
    A.apax_status_clear(ws)
    A.apax_profile_async(xg, params, ws)
    buf, nb = A.apax_encode(xg, dict(params, code=A.CODE_PROFILED), ws=ws, clear_status=False)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    return buf[: int(nb.item())].cpu().numpy(), A.apax_profile_read(xg, params, ws)


def fused(A, xg, params, side=False):
    """side: the profile's last passes on a second stream, joined before the
    profile is read."""
    ws = A.workspace(xg.dtype, tuple(xg.shape), params, DEV)
    A.apax_status_clear(ws)
    ev = torch.cuda.Event()
    main = torch.cuda.current_stream()
    if side:
        s2, fk = torch.cuda.Stream(), torch.cuda.Event()
        buf, nb = A.apax_profile_encode_async(xg, params, ws, encoded=ev, stream=main, side=s2, forked=fk)
        main.wait_stream(s2)
    else:
        buf, nb = A.apax_profile_encode_async(xg, params, ws, encoded=ev)
    ev.synchronize()
    n = int(nb.item())
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    return buf, n, A.apax_profile_read(xg, params, ws)


@pytest.mark.parametrize("side", [False, True], ids=["one-stream", "side-stream"])
@pytest.mark.parametrize("name,dt,shape,params", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_separate(A, name, dt, shape, params, side):
    print(f"case {name} side {side}", flush=True)
    params = dict(params, target_corr=0.9999)
    x = field(dt, shape, 3)
    xg = torch.from_numpy(x).to(DEV)
    ref, pref = separate(A, xg, params)
    buf, n, pf = fused(A, xg, params, side)
    got = buf[:n].cpu().numpy()
    assert pf == pref
    assert got.size == ref.size and np.array_equal(got, ref)
    # the oracle at the same operating point decodes to the same values
    mode = params["mode"]
    p = {k: v for k, v in params.items() if k != "lagged" or mode == "lossless"}
    p = dict(p, code=pf["code"], stream_mask=pf["stream_mask"] & (0x7F if mode == "fixed_rate" else 0xFF))
    y = A.apax_decode(buf, n).cpu().numpy()
    assert np.array_equal(y.view(np.uint8), O.decode(O.encode(x, p)).view(np.uint8))


def test_fused_empty(A):
    xg = torch.zeros((0,), dtype=torch.float32, device=DEV)
    p = {"mode": "fixed_rate", "brick": (64,), "rate": 4.0}
    buf, n, pf = fused(A, xg, p)
    ref, pref = separate(A, xg, p)
    assert np.array_equal(buf[:n].cpu().numpy(), ref) and pf == pref


@pytest.mark.timeout(600)
def test_fused_full_field(A):
    x = synth.grf2d(4096, 4096)
    xg = torch.from_numpy(x).to(DEV)
    p = {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}
    ref, pref = separate(A, xg, p)
    # the side stream runs the curve beside the metrics pass (each with its
    # own partial records) and the centred pass beside the encode: repeated,
    # so an overlap of the two streams' records or state write-backs shows
    for side in (False, True, True, True):
        buf, n, pf = fused(A, xg, p, side)
        assert pf == pref
        assert n == ref.size and torch.equal(buf[:n].cpu(), torch.from_numpy(ref))


def test_side_stream_back_to_back(A):
    """Six fused profile-encodes of the 4096^2 fp32 field enqueued back to
    back with the side stream (no host synchronisation between them), as a
    pipeline runs them: every stream equals the separate encode's and the
    profile left in the workspace equals the separate profile."""
    x = synth.grf2d(4096, 4096)
    xg = torch.from_numpy(x).to(DEV)
    p = {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}
    ref, pref = separate(A, xg, p)
    ws = A.workspace(xg.dtype, tuple(xg.shape), p, DEV)
    A.apax_status_clear(ws)
    main, s2, fk = torch.cuda.current_stream(), torch.cuda.Stream(), torch.cuda.Event()
    outs = []
    torch.cuda.synchronize()
    for _ in range(6):
        buf, nb = A.apax_profile_encode_async(xg, p, ws, stream=main, side=s2, forked=fk)
        main.wait_stream(s2)
        outs.append((buf, nb))
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    assert A.apax_profile_read(xg, p, ws) == pref
    for buf, nb in outs:
        n = int(nb.item())
        assert n == ref.size and torch.equal(buf[:n].cpu(), torch.from_numpy(ref))


def test_side_stream_graph_replays(A):
    """The forked sequence (profile, encode and a decode on one stream, the
    last profile passes on a second) captured as one hipGraph and replayed
    three times, eager work and synchronizations between the replays: every
    replay gives the eager profile, stream and decode."""
    x = synth.grf2d(512, 768, seed=synth.seed_of(1, 5))
    xg = torch.from_numpy(x).to(DEV)
    p = {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0}
    ref, pref = separate(A, xg, p)
    ws = A.workspace(xg.dtype, tuple(xg.shape), p, DEV)
    ws_dec = A.workspace(xg.dtype, tuple(xg.shape), p, DEV)
    out = torch.empty(ref.size + 64, dtype=torch.uint8, device=DEV)
    nb = torch.empty(1, dtype=torch.int64, device=DEV)
    y = torch.empty_like(xg)
    s2, fk = torch.cuda.Stream(), torch.cuda.Event()
    A.apax_status_clear(ws)
    A.apax_status_clear(ws_dec)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream()
        A.apax_profile_encode_async(xg, p, ws, out=out, nbytes=nb, stream=cap, side=s2, forked=fk)
        A.apax_decode(out, ref.size, hdr=bytes(ref[:64]), y=y, ws=ws_dec, stream=cap, clear_status=False)
        cap.wait_stream(s2)
    y_ref = O.decode(ref)
    for rep in range(3):
        out.fill_(0xAB)
        y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert A.apax_status(ws) == 0 and A.apax_status(ws_dec) == 0
        assert int(nb.item()) == ref.size
        assert np.array_equal(out[: ref.size].cpu().numpy(), ref), rep
        assert np.array_equal(y.cpu().numpy().view(np.uint8), y_ref.view(np.uint8)), rep
        assert A.apax_profile_read(xg, p, ws) == pref, rep


def test_side_stream_refused_when_malformed(A):
    xg = torch.zeros(4096, dtype=torch.float32, device=DEV)
    p = {"mode": "fixed_rate", "brick": (64,), "rate": 4.0}
    ws = A.workspace(xg.dtype, tuple(xg.shape), p, DEV)
    main = torch.cuda.Stream()  # not the null stream, which reads as "no side stream"
    for side, fk in ((main, torch.cuda.Event()), (torch.cuda.Stream(), None)):
        with pytest.raises(A.ApaxError) as e:
            A.apax_profile_encode_async(xg, p, ws, stream=main, side=side, forked=fk)
        assert e.value.code == A.E_INVALID


@pytest.mark.parametrize("name", ["f32-2d-16x16-fr", "i8-1d-B64-fr", "f64-3d-4x4x8-fq", "i16-1d-B256-lossless"])
def test_profile_encode_timed(A, name):
    """The instrumented sequence (events around every pass kernel, one
    stream) writes the same profile and bytes as the separate calls; in fixed
    rate the metrics pass, which writes the blocks, is the timed kernel."""
    print(f"case {name}", flush=True)
    _, dt, shape, params = next(c for c in CASES if c[0] == name)
    params = dict(params, target_corr=0.9999)
    x = field(dt, shape, 3)
    xg = torch.from_numpy(x).to(DEV)
    ref, pref = separate(A, xg, params)
    ws = A.workspace(xg.dtype, tuple(xg.shape), params, DEV)
    A.apax_status_clear(ws)
    prof, ms, buf, nb = A.apax_profile_encode_timed(xg, params, ws)
    torch.cuda.synchronize()
    assert A.apax_status(ws) == 0
    assert prof == pref
    assert np.array_equal(buf[: int(nb.item())].cpu().numpy(), ref)
    assert ms["metrics"] > 0 and ms["max"] > 0


def test_profile_encode_timed_refuses_wide(A):
    xg = torch.zeros((4096,), dtype=torch.float32, device=DEV)
    p = {"mode": "fixed_rate", "brick": (1024,), "rate": 4.0}
    ws = A.workspace(xg.dtype, tuple(xg.shape), p, DEV)
    with pytest.raises(A.ApaxError) as ei:
        A.apax_profile_encode_timed(xg, p, ws)
    assert ei.value.code == A.E_UNSUPPORTED
