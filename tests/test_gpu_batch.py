"""Batched encode/decode (one persistent launch per block-shape class, hipGraph
replay): every item's output equals a separate apax_encode / apax_decode
call byte for byte, for every launch geometry the autotuner may pick, and
matches the CPU oracle on a sample of items."""
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


@pytest.fixture(scope="module")
def items():
    """~120 mixed items: sizes log-uniform 4 KB..1 MB, int16/int32/fp32/fp64,
    lossless or fixed rate, plus N-d items, other block sizes and an empty one."""
    pools = synth.Pools(n=1 << 20, seed=99)
    out = []
    for i in range(110):
        spec = synth.item_spec(i, seed=1234, hi_bytes=1 << 20)
        x = pools.item(spec)
        if spec["mode"] == "lossless":
            params = {"mode": "lossless", "brick": (256,)}
        else:
            isint = x.dtype.kind == "i"
            # start codes: the cap for half of them (every block searches), a
            # mid-range code for the rest
            code = 0 if isint else (16383 if i % 2 else 200)
            params = {"mode": "fixed_rate", "brick": (256,), "rate": spec["rate"], "code": code}
        out.append((x, params))
    rng = np.random.default_rng(5)
    f2 = synth.grf2d(96, 80, seed=7)
    out.append((f2, {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0, "code": 120}))
    out.append((f2, {"mode": "fixed_quality", "brick": (8, 8), "code": 150}))
    f3 = synth.blobs3d(8, 24, 40, seed=8)
    out.append((f3, {"mode": "fixed_quality", "brick": (4, 4, 8), "code": 400}))
    i16 = synth.sinusoids(5000, seed=9)
    out.append((i16, {"mode": "lossless", "brick": (64,)}))
    out.append((rng.integers(-100, 100, 3000).astype(np.int8), {"mode": "lossless", "brick": (128,)}))
    out.append((np.zeros(0, np.float32), {"mode": "fixed_rate", "brick": (256,), "rate": 4.0, "code": 10}))
    out.append((np.zeros(0, np.int16), {"mode": "lossless", "brick": (256,)}))
    return out


def individual(A, arrays):
    res = []
    for x, params in arrays:
        xg = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        buf, nb = A.apax_encode(xg, params)
        n = int(nb.item())
        res.append(buf[:n].cpu().numpy())
    return res


def batch_outputs(b):
    torch.cuda.synchronize()
    nb = b.nbytes.cpu().numpy()
    return [o[: int(nb[i])].cpu().numpy() for i, o in enumerate(b.outs)]


@pytest.mark.parametrize("tune", [None, {"waves_per_wg": 2, "wgs_per_cu": 2, "tiles_per_ticket": 4},
                                  {"waves_per_wg": 8, "wgs_per_cu": 16, "tiles_per_ticket": 1}])
def test_batch_encode_equals_separate_calls(A, items, tune):
    print(f"tune {tune}", flush=True)
    arrays = [(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), p) for x, p in items]
    ref = individual(A, items)
    b = A.Batch.encode(arrays, tune=tune)
    b.run()
    assert b.status() == 0
    got = batch_outputs(b)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert np.array_equal(g, r), (i, items[i][1], g.size, r.size)
    b.close()


def test_batch_matches_oracle_sample(A, items):
    arrays = [(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), p) for x, p in items]
    b = A.Batch.encode(arrays)
    b.run()
    got = batch_outputs(b)
    for i in list(range(0, len(items), 9)) + list(range(len(items) - 7, len(items))):
        x, p = items[i]
        assert np.array_equal(got[i], O.encode(x, p)), (i, p)
    b.close()


def test_batch_graph_replay_and_decode(A, items):
    arrays = [(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), p) for x, p in items]
    ref = individual(A, items)
    b = A.Batch.encode(arrays)
    b.capture()
    for rep in range(3):
        for o in b.outs:  # eager work between replays
            o.zero_()
        b.nbytes.fill_(-1)
        b.launch()
        torch.cuda.synchronize()
        got = batch_outputs(b)
        for i, (g, r) in enumerate(zip(got, ref)):
            assert np.array_equal(g, r), (rep, i)
    # batched decode of the batch's streams, also replayed from a graph
    streams = [(b.outs[i], int(b.nbytes[i].item()), bytes(ref[i][:64])) for i in range(len(items))]
    d = A.Batch.decode(streams)
    d.capture()
    for rep in range(2):
        for y in d.outs:
            y.zero_()
        d.launch()
        torch.cuda.synchronize()
        assert d.status() == 0
        for i, (x, p) in enumerate(items):
            y = d.outs[i].cpu().numpy()
            single = A.apax_decode(b.outs[i], int(b.nbytes[i].item())).cpu().numpy()
            assert np.array_equal(y.view(np.uint8), single.view(np.uint8)), (rep, i)
            if p["mode"] == "lossless":
                assert np.array_equal(y, x)
    b.close()
    d.close()


def test_tuner_picks_a_candidate(A, items, tmp_path, monkeypatch):
    from paper_1303_4994_amd import tune as T
    monkeypatch.setenv("APAX_TUNE_CACHE", str(tmp_path / "tune.json"))
    arrays = [(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), p) for x, p in items[:40]]
    cands = [{"waves_per_wg": 4, "wgs_per_cu": 8, "tiles_per_ticket": 1},
             {"waves_per_wg": 2, "wgs_per_cu": 4, "tiles_per_ticket": 2}]
    best = T.tune(A.OP_ENCODE, arrays, candidates=cands, reps=1)
    assert best in cands
    assert T.tune(A.OP_ENCODE, arrays, candidates=cands, reps=1) == best  # cached


def test_batch_large_items_match_oracle(A):
    """Items of 16-64 MB (one per dtype, from the C0-C2 generators; lossless
    and fixed rate), batched with small ones: encodes equal the oracle's
    streams and decodes the oracle's decoded arrays, byte for byte."""
    pools = synth.Pools(n=1 << 24, seed=77)
    big = []
    for i, (dt, gen, mode, nbytes) in enumerate([(np.int16, 0, "lossless", 16 << 20),
                                                 (np.int32, 1, "fixed_rate", 24 << 20),
                                                 (np.float32, 1, "fixed_rate", 64 << 20),
                                                 (np.float64, 2, "fixed_rate", 40 << 20)]):
        spec = {"dtype": np.dtype(dt), "gen": gen, "n": nbytes // np.dtype(dt).itemsize,
                "offset": 12345 * (i + 1), "mode": mode, "rate": 3.0 + 2.5 * i}
        x = pools.item(spec)
        if mode == "lossless":
            p = {"mode": "lossless", "brick": (256,)}
        else:
            p = {"mode": "fixed_rate", "brick": (256,), "rate": spec["rate"], "code": 0 if dt == np.int32 else 180}
        big.append((x, p))
    small = [(synth.sinusoids(3000, seed=11), {"mode": "lossless", "brick": (256,)}),
             (synth.grf2d(64, 64, seed=12).ravel(), {"mode": "fixed_rate", "brick": (256,), "rate": 5.0,
                                                    "code": 100})]
    items = big + small
    print("large batch items", [(x.dtype.name, x.nbytes) for x, _ in items], flush=True)
    arrays = [(torch.from_numpy(np.ascontiguousarray(x)).to(DEV), p) for x, p in items]
    b = A.Batch.encode(arrays)
    b.run()
    assert b.status() == 0
    got = batch_outputs(b)
    exps = []
    for i, (x, p) in enumerate(items):
        exps.append(O.encode(x, p))
        assert np.array_equal(got[i], exps[i]), (i, x.dtype, p)
    # the batched decode of the same streams equals the oracle's decode
    streams = [(torch.from_numpy(g).to(DEV), g.size, bytes(g[:64])) for g in got]
    d = A.Batch.decode(streams)
    d.run()
    assert d.status() == 0
    torch.cuda.synchronize()
    for i in range(len(items)):
        yo = O.decode(exps[i])
        assert np.array_equal(d.outs[i].cpu().numpy().view(np.uint8), yo.view(np.uint8)), i
    b.close()
    d.close()
