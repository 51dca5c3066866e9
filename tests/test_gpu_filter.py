"""GPU parity of the filter stream (Sec. 5 / Sec. 6: the redundancy remover's
filtered series x[n] - s x[n-k], with the stride and sign the signal monitor
picks for a modulated carrier): streams and decodes byte-identical to the
oracle in every mode, blocks of 64..1024 samples (one wave holding one, two or
four blocks, and the one-workgroup-per-block path), strides 1..16 with both
signs, the lagged choice, the profiler's decisions, and batches."""
import numpy as np
import pytest

import brute
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


CASES = [
    ("i16-b512-B256", np.int16, 50000 + 37, 512, (256,), {"mode": "lossless"}),
    ("i16-b341-B64", np.int16, 20000, 341, (64,), {"mode": "lossless"}),
    ("i32-b256-B128", np.int32, 30000 + 5, 256, (128,), {"mode": "lossless"}),
    ("i8-b200-B256", np.int8, 9000, 200, (256,), {"mode": "lossless"}),
    ("i16-b100-B1024-wide", np.int16, 40000 + 100, 100, (1024,), {"mode": "lossless"}),
    ("f32-b512-fr", np.float32, 64 * 500, 512, (64,), {"mode": "fixed_rate", "rate": 4.0, "code": 60}),
    ("f64-b171-fq", np.float64, 25000, 171, (256,), {"mode": "fixed_quality", "code": 300}),
    ("f32-b64-fq-B512-wide", np.float32, 512 * 30 + 8, 64, (512,), {"mode": "fixed_quality", "code": 90}),
    ("f32-b300-adaptive", np.float32, 256 * 200, 300, (256,), {"mode": "adaptive_rate", "rate": 4.0, "code": 60}),
]


def roundtrip(A, x, params):
    xg = torch.from_numpy(x).to(DEV)
    ws = A.workspace(xg.dtype, tuple(x.shape), params, DEV)
    buf, nb = A.apax_encode(xg, params, ws=ws)
    assert A.apax_status(ws) == 0
    n = int(nb.item())
    got = buf[:n].cpu().numpy()
    y = A.apax_decode(buf, n, ws=ws)
    assert A.apax_status(ws) == 0
    return got, y.cpu().numpy()


def check(A, x, params):
    exp = O.encode(x, params)
    got, y = roundtrip(A, x, params)
    if got.size != exp.size or not np.array_equal(got, exp):
        sg, se = brute.Stream(got), brute.Stream(exp)
        j = next((j for j in range(se.nblocks) if not np.array_equal(sg.block(j), se.block(j))), None)
        pytest.fail(f"stream differs ({got.size} vs {exp.size} bytes), first block {j}")
    assert np.array_equal(y.view(np.uint8), O.decode(exp).view(np.uint8))
    return exp


@pytest.mark.parametrize("name,dt,n,b,brick,params", CASES, ids=[c[0] for c in CASES])
def test_filter_stream_equals_oracle(A, name, dt, n, b, brick, params):
    """The monitor (GPU) picks the stride and sign; the encode with that
    filter equals the oracle's and the filter stream is chosen."""
    print(f"case {name}", flush=True)
    x = synth.modulated(dt, n, 3, b, noise=0.002)
    mon = A.apax_signal_monitor(torch.from_numpy(x).to(DEV))
    k, s = O.monitor_stride(b)
    assert (mon["stride"], mon["sign"]) == (k, s)
    p = dict(params, brick=brick, filter=(k, s))
    exp = check(A, x, p)
    st = brute.Stream(exp)
    assert sum((int(st.block(j)[0]) & 7) == 3 for j in range(st.nblocks)) >= st.nblocks // 3
    if params["mode"] == "lossless":
        assert exp.size < O.encode(x, dict(params, brick=brick)).size


@pytest.mark.parametrize("k,sign", [(1, 1), (2, -1), (3, 1), (4, -1), (5, -1), (7, 1), (8, 1), (13, -1), (16, -1),
                                    (16, 1)])
def test_every_stride(A, k, sign):
    """Every stride class (inside one lane, across one to four lanes) with a
    carrier the filter cancels, blocks of 64 and 256 samples."""
    print(f"stride {k} sign {sign}", flush=True)
    # a tone that x[n] - sign x[n-k] cancels: b k / 1024 a multiple of 1/2 (sign -1) or 1 (sign +1)
    b = (512 // k) if sign < 0 else (1024 // k) % 512
    x = synth.modulated(np.int16, 12000 + 3 * k, k, b if b else 1, noise=0.01)
    for brick in ((64,), (256,)):
        check(A, x, {"mode": "lossless", "brick": brick, "filter": (k, sign)})


def test_filter_lagged_profile_and_batch(A):
    x = synth.modulated(np.int16, 40000, 9, 512, noise=0.003)
    k, s = O.monitor_stride(512)
    check(A, x, {"mode": "lossless", "brick": (256,), "filter": (k, s), "lagged": True})
    # the profiler sees the filter stream like any other (its mask may keep it)
    xf = synth.modulated(np.float32, 64 * 400, 4, 512, noise=0.001)
    pp = {"mode": "fixed_quality", "brick": (64,), "target_corr": 0.99999, "filter": (k, s)}
    pg = A.apax_profile(torch.from_numpy(xf).to(DEV), pp)
    po = O.profile_dict(O.profile(xf, pp))
    if not ((pg["flags"] | po["flags"]) & 1):
        assert (pg["code"], pg["stream_mask"], pg["n_probes"]) == (po["code"], po["stream_mask"], po["n_probes"])
        assert pg["stream_mask"] & 0x08
    # batch items with and without the filter
    items = [(x, {"mode": "lossless", "brick": (256,), "filter": (k, s)}),
             (x[:7000].copy(), {"mode": "lossless", "brick": (64,), "filter": (3, -1)}),
             (x[:5000].copy(), {"mode": "lossless", "brick": (256,)})]
    b = A.Batch.encode([(torch.from_numpy(xi).to(DEV), p) for xi, p in items])
    b.run()
    assert b.status() == 0
    torch.cuda.synchronize()
    nb = b.nbytes.cpu().numpy()
    for i, (xi, p) in enumerate(items):
        assert np.array_equal(b.outs[i][: int(nb[i])].cpu().numpy(), O.encode(xi, p)), i
    b.close()


def test_filter_refused_outside_1d(A):
    x = torch.zeros((64, 64), dtype=torch.int16, device=DEV)
    with pytest.raises(A.ApaxError) as e:
        A.apax_encode(x, {"mode": "lossless", "brick": (8, 8), "filter": (1, -1)})
    assert e.value.code == A.E_INVALID
