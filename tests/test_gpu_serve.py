"""Serving loop (continuous batching over slots with resident codec state):
every served result equals the CPU oracle's and the same request run alone,
whatever group and slot it landed in; admission never exceeds the HBM
budget; per-request status; requests above the budget are refused at
submit."""
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
def S(A):
    from paper_1303_4994_amd import serve
    return serve


def make_requests(A, n=96, seed=4242):
    """Mixed encode/decode requests, 4 KB..2 MB, all four batch dtypes."""
    pools = synth.Pools(n=1 << 20, seed=seed)
    reqs = []
    for i in range(n):
        spec = synth.item_spec(i, seed=seed, lo_bytes=4 << 10, hi_bytes=2 << 20)
        x = pools.item_device(spec, DEV)
        if spec["mode"] == "lossless":
            params = {"mode": "lossless", "brick": (256,)}
        else:
            code = 0 if x.dtype in (torch.int16, torch.int32) else 150
            params = {"mode": "fixed_rate", "brick": (256,), "rate": spec["rate"], "code": code}
        kind = "encode" if i % 2 == 0 else "decode"
        r = {"kind": kind, "x": x, "params": params}
        buf, nb = A.apax_encode(x, params)            # the standalone result
        n_ = int(nb.item())
        r["ref_stream"] = buf[:n_].cpu().numpy()
        # the oracle's stream and decode of the same bytes
        r["orc_stream"] = O.encode(x.cpu().numpy(), params)
        if kind == "decode":
            r["stream"], r["nbytes"] = buf, n_
            r["hdr"] = bytes(r["ref_stream"][:64])
            r["ref_y"] = A.apax_decode(buf, n_).cpu().numpy()
            r["orc_y"] = O.decode(r["orc_stream"])
        reqs.append(r)
    torch.cuda.synchronize()
    return reqs


def test_served_results_equal_standalone(A, S):
    reqs = make_requests(A)
    slots, ws = 3, 1 << 20
    budget = 2 * slots * ws + (12 << 20)       # forces admission waits
    srv = S.Server(budget_bytes=budget, slots=slots, max_group=8, ws_bytes=ws)
    rng = np.random.default_rng(17)
    arrivals = np.cumsum(rng.exponential(2e-4, len(reqs)))
    outs = [None] * len(reqs)
    peak = [0]

    def job(k):
        r = reqs[k]
        if r["kind"] == "encode":
            bound = A.apax_encode_bound(r["x"].dtype, tuple(r["x"].shape), r["params"])
            out = torch.empty(max(bound, 64), dtype=torch.uint8, device=DEV)
            nb = torch.full((1,), -1, dtype=torch.int64, device=DEV)
            outs[k] = (out, nb)
            return srv.submit_encode(r["x"], r["params"], out, nb, tag=k), r["x"].numel() * r["x"].element_size()
        y = torch.empty_like(r["x"])
        outs[k] = y
        return srv.submit_decode(r["stream"], r["nbytes"], r["hdr"], y, tag=k), y.numel() * y.element_size()

    def done(k, c):
        assert c["tag"] == k
        peak[0] = max(peak[0], srv.stats()["in_flight_bytes"])

    st = S.drive(srv, [lambda k=k: job(k) for k in range(len(reqs))], list(arrivals), on_done=done,
                 deadline_s=60.0)
    print(st, flush=True)
    assert st["requests"] == len(reqs) and st["groups"] > 1
    assert peak[0] <= budget - 2 * slots * ws
    torch.cuda.synchronize()
    for k, r in enumerate(reqs):
        if r["kind"] == "encode":
            out, nb = outs[k]
            n_ = int(nb.item())
            got = out[:n_].cpu().numpy()
            assert np.array_equal(got, r["orc_stream"]), ("served != oracle", k)
            assert np.array_equal(got, r["ref_stream"]), ("served != alone", k)
        else:
            got = outs[k].cpu().numpy()
            assert np.array_equal(got.view(np.uint8), r["orc_y"].view(np.uint8)), ("served != oracle", k)
            assert np.array_equal(got.view(np.uint8), r["ref_y"].view(np.uint8)), ("served != alone", k)
    srv.close()


def test_per_request_status_and_budget_refusal(A, S):
    srv = S.Server(budget_bytes=(4 << 20) + (1 << 20), slots=2, max_group=4, ws_bytes=1 << 20)
    good = torch.linspace(-5, 5, 4096, device=DEV, dtype=torch.float32)
    bad = good.clone()
    bad[1000] = float("nan")
    p = {"mode": "fixed_rate", "brick": (256,), "rate": 4.0, "code": 100}
    bound = A.apax_encode_bound(torch.float32, (4096,), p)
    res = {}
    ids = {}
    for name, x in (("good0", good), ("bad", bad), ("good1", good)):
        out = torch.empty(bound, dtype=torch.uint8, device=DEV)
        nb = torch.zeros(1, dtype=torch.int64, device=DEV)
        res[name] = (out, nb)
        ids[srv.submit_encode(x, p, out, nb)] = name
    torch.cuda.synchronize()
    got = {}
    for _ in range(200000):
        for c in srv.poll():
            got[ids[c["id"]]] = c["status"]
        if len(got) == 3:
            break
    assert got == {"good0": 0, "bad": A.E_NONFINITE, "good1": 0}
    ref, nref = A.apax_encode(good, p)
    n0 = int(nref.item())
    for name in ("good0", "good1"):
        out, nb = res[name]
        assert int(nb.item()) == n0
        assert torch.equal(out[:n0], ref[:n0])
    big = torch.zeros(1 << 20, dtype=torch.float32, device=DEV)   # 4 MB in + bound out > budget
    out = torch.empty(A.apax_encode_bound(torch.float32, (1 << 20,), p), dtype=torch.uint8, device=DEV)
    with pytest.raises(A.ApaxError) as ei:
        srv.submit_encode(big, p, out, torch.zeros(1, dtype=torch.int64, device=DEV))
    assert ei.value.code == A.E_CAPACITY
    srv.close()


def test_large_requests_run_alone_with_their_status(A, S):
    """Requests of 16 MB and more run as single calls inside their group: the
    results equal the standalone ones, and a non-finite large request fails
    alone (the small and large requests around it succeed)."""
    seed = 515
    pools = synth.Pools(n=1 << 24, seed=seed)
    srv = S.Server(budget_bytes=8 << 30, slots=2, max_group=6, ws_bytes=64 << 20)
    jobs, refs, outs = [], [], []
    planted = False
    for i in range(12):
        lo, hi = ((16 << 20), (40 << 20)) if i % 3 != 2 else ((4 << 10), (1 << 20))
        spec = synth.item_spec(i, seed=seed, lo_bytes=lo, hi_bytes=hi)
        x = pools.item_device(spec, DEV)
        if x.dtype in (torch.float32, torch.float64):
            params = {"mode": "fixed_rate", "brick": (256,), "rate": spec.get("rate", 4.0), "code": 150}
        else:
            params = {"mode": "lossless", "brick": (256,)}
        if not planted and i % 3 != 2 and x.dtype in (torch.float32, torch.float64):
            x = x.clone()  # one large request fails alone
            x[x.numel() // 2] = float("inf")
            planted = True
        buf, nb = A.apax_encode(x, params, ws=A.workspace(x.dtype, tuple(x.shape), params, DEV))
        n_ = int(nb.item())
        refs.append(buf[:n_].clone())
        out = torch.empty_like(buf)
        nbo = torch.zeros(1, dtype=torch.int64, device=DEV)
        outs.append((out, nbo))
        jobs.append((x, params, out, nbo))
    torch.cuda.synchronize()
    ids = {srv.submit_encode(x, p, o, nb, tag=k): k for k, (x, p, o, nb) in enumerate(jobs)}
    status = {}
    for _ in range(2000000):
        for c in srv.poll():
            status[ids[c["id"]]] = c["status"]
        if len(status) == len(jobs):
            break
    assert len(status) == len(jobs) and planted
    torch.cuda.synchronize()
    for k, (x, p, o, nb) in enumerate(jobs):
        nonfinite = not bool(torch.isfinite(x).all()) if x.is_floating_point() else False
        assert status[k] == (A.E_NONFINITE if nonfinite else 0), (k, status[k])
        if not nonfinite:
            n_ = int(nb.item())
            assert n_ == refs[k].numel() and torch.equal(o[:n_], refs[k]), k
            if k < 4:  # the first large ones (16-40 MB) also against the oracle
                assert np.array_equal(o[:n_].cpu().numpy(), O.encode(x.cpu().numpy(), p)), k
    srv.close()
