"""Batches and the server with the items their shared launch does not take
(blocks of more than 256 samples, groups of 8 samples per exponent, the
lagged choice, adaptive rate): they run as single-array calls inside the same
batch run (and its hipGraph) or as single calls on the server's slot stream.
Every encoded stream equals the oracle's, every decode the oracle's decode,
beside ordinary items of the same batch; a replayed graph gives the same
bytes; per-item status is kept."""
import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def S(A):
    from paper_1303_4994_amd import serve
    return serve


def field(dt, n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    base = np.sin(2 * np.pi * 0.0021 * t) + 0.3 * np.sin(2 * np.pi * 0.037 * t) + 0.02 * rng.standard_normal(n)
    base = base.cumsum() / 8
    dt = np.dtype(dt)
    if dt.kind == "i":
        return np.rint(base / np.abs(base).max() * 0.45 * np.iinfo(dt).max).astype(dt)
    return (base * 1e2).astype(dt)


ITEMS = [
    ("plain-f32-B256-fr", np.float32, 40000, {"mode": "fixed_rate", "brick": (256,), "rate": 4.0, "code": 60}),
    ("wide-i16-B1024-lossless", np.int16, 1024 * 20 + 9, {"mode": "lossless", "brick": (1024,)}),
    ("wide-f32-B4096-fr", np.float32, 4096 * 6 + 100, {"mode": "fixed_rate", "brick": (4096,), "rate": 4.0,
                                                      "code": 50}),
    ("plain-i32-B64-lossless", np.int32, 9000, {"mode": "lossless", "brick": (64,)}),
    ("g8-f64-B64-fq", np.float64, 64 * 90 + 8, {"mode": "fixed_quality", "brick": (64,), "code": 300,
                                                "group": 8}),
    ("lagged-i16-B64", np.int16, 12000, {"mode": "lossless", "brick": (64,), "lagged": True}),
    ("adaptive-f32-B256", np.float32, 256 * 60, {"mode": "adaptive_rate", "brick": (256,), "rate": 4.0,
                                                 "code": 60}),
    ("wide-g8-f32-B512-fq", np.float32, 512 * 11 + 40, {"mode": "fixed_quality", "brick": (512,), "code": 70,
                                                        "group": 8}),
]


@pytest.fixture(scope="module")
def data():
    xs = [field(dt, n, 11 + k) for k, (_, dt, n, _) in enumerate(ITEMS)]
    exp = [O.encode(x, p) for x, (_, _, _, p) in zip(xs, ITEMS)]
    return xs, exp


def test_batch_encode_decode_alone_items(A, data):
    xs, exp = data
    xg = [torch.from_numpy(x).to(DEV) for x in xs]
    b = A.Batch.encode([(x, p) for x, (_, _, _, p) in zip(xg, ITEMS)])
    for rep in range(3):  # plain run, then two graph replays
        print(f"batch encode pass {rep}", flush=True)
        for o in b.outs:
            o.fill_(0xEE)
        b.nbytes.fill_(-1)
        torch.cuda.synchronize()
        if rep == 0:
            b.run()
        else:
            if rep == 1:
                b.capture()
            b.launch()
        torch.cuda.synchronize()
        assert b.status() == 0
        nb = b.nbytes.cpu().numpy()
        for i, (name, *_rest) in enumerate(ITEMS):
            got = b.outs[i][: int(nb[i])].cpu().numpy()
            assert np.array_equal(got, exp[i]), (rep, name)
    streams = [(b.outs[i], int(b.nbytes[i].item()), bytes(exp[i][:64])) for i in range(len(ITEMS))]
    d = A.Batch.decode(streams)
    for rep in range(2):
        print(f"batch decode pass {rep}", flush=True)
        for y in d.outs:
            y.zero_()
        torch.cuda.synchronize()
        if rep == 0:
            d.run()
        else:
            d.capture()
            d.launch()
        torch.cuda.synchronize()
        assert d.status() == 0
        for i, (name, *_rest) in enumerate(ITEMS):
            y = d.outs[i].cpu().numpy()
            assert np.array_equal(y.view(np.uint8), O.decode(exp[i]).view(np.uint8)), (rep, name)
    d.close()
    b.close()


def test_batch_alone_item_status(A):
    """A non-finite sample in an item that runs alone is reported by the
    batch's status like any other item's."""
    x = field(np.float32, 1024 * 8, 3)
    x[5000] = np.nan
    xg = torch.from_numpy(x).to(DEV)
    ok = torch.from_numpy(field(np.float32, 4096, 4)).to(DEV)
    b = A.Batch.encode([(ok, {"mode": "fixed_rate", "brick": (256,), "rate": 4.0, "code": 40}),
                        (xg, {"mode": "fixed_rate", "brick": (1024,), "rate": 4.0, "code": 40})])
    b.run()
    torch.cuda.synchronize()
    assert b.status() == A.E_NONFINITE
    b.close()


def test_server_alone_requests(A, S, data):
    xs, exp = data
    srv = S.Server(budget_bytes=256 << 20, slots=2, max_group=4, ws_bytes=8 << 20)
    outs, ids = [], []
    for k, (x, (name, _, _, p)) in enumerate(zip(xs, ITEMS)):
        xg = torch.from_numpy(x).to(DEV)
        bound = A.apax_encode_bound(xg.dtype, tuple(x.shape), p)
        out = torch.empty(max(bound, 64), dtype=torch.uint8, device=DEV)
        nb = torch.zeros(1, dtype=torch.int64, device=DEV)
        torch.cuda.synchronize()
        outs.append((xg, out, nb))
        ids.append(srv.submit_encode(xg, p, out, nb, tag=k))
    ys = []
    for k, x in enumerate(xs):
        buf = torch.from_numpy(exp[k]).to(DEV)
        y = torch.empty(x.shape, dtype=outs[k][0].dtype, device=DEV)
        torch.cuda.synchronize()
        ys.append((buf, y))
        ids.append(srv.submit_decode(buf, exp[k].size, bytes(exp[k][:64]), y, tag=100 + k))
    seen = {}
    import time
    t0 = time.time()
    while len(seen) < len(ids) and time.time() - t0 < 60:
        for c in srv.poll():
            seen[c["tag"]] = c["status"]
    srv.close()
    torch.cuda.synchronize()
    assert len(seen) == len(ids)
    assert all(v == 0 for v in seen.values()), seen
    for k, (name, *_rest) in enumerate(ITEMS):
        _, out, nb = outs[k]
        assert np.array_equal(out[: int(nb.item())].cpu().numpy(), exp[k]), name
        assert np.array_equal(ys[k][1].cpu().numpy().view(np.uint8), O.decode(exp[k]).view(np.uint8)), name
