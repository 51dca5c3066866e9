"""apax_encode_noalloc (the encode for callers that cannot allocate) against
apax_encode: byte-identical streams and byte counts, on two calls in a row
through the C ABI, the second with a smaller input than the first, so any
state the first call left in the library's scratch would show."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_4994_amd import apax
    return apax


def _ref(A, xg, params):
    buf, nb = A.apax_encode(xg, params)
    n = int(nb.item())
    return buf[:n].cpu().numpy()


def _noalloc(A, xg, params):
    bound = A.apax_encode_bound(xg.dtype, tuple(xg.shape), params)
    out = torch.full((bound,), 0xA5, dtype=torch.uint8, device=DEV)
    nb = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    st = torch.full((1,), 12345, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()  # the fills above are on torch's stream; the encode is on it too
    A.apax_encode_noalloc(xg, params, out, nb, st)
    torch.cuda.synchronize()
    n = int(nb.item())
    return out[:n].cpu().numpy(), int(st.item())


CASES = [
    # variable size (ticket + look-back states in the scratch)
    ("i16-1d-lossless", lambda s: synth.sinusoids(s, seed=synth.seed_of(0, 7)),
     [1 << 18, 5000 + 37], {"mode": "lossless", "brick": (256,)}),
    # lagged choice (per-block best streams in the scratch)
    ("i16-1d-lossless-lagged", lambda s: synth.sinusoids(s, seed=synth.seed_of(0, 8)),
     [1 << 17, 3000 + 5], {"mode": "lossless", "brick": (256,), "lagged": True}),
    # fixed rate (status word only)
    ("f32-2d-fixed-rate", lambda s: synth.grf2d(s[0], s[1], seed=synth.seed_of(1, 7)),
     [(512, 512), (96, 80)], {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0, "code": 40}),
    # fixed quality, 3-d
    ("f64-3d-fixed-quality", lambda s: synth.blobs3d(*s, seed=synth.seed_of(2, 7)),
     [(32, 64, 64), (9, 17, 30)], {"mode": "fixed_quality", "brick": (4, 4, 8), "code": 300}),
]


@pytest.mark.parametrize("name,gen,sizes,params", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_encode_twice_second_smaller(A, name, gen, sizes, params):
    for size in sizes:  # the second input is the smaller one
        x = gen(size)
        print(f"noalloc case {name} shape {x.shape}", flush=True)
        xg = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        ref = _ref(A, xg, params)
        got, st = _noalloc(A, xg, params)
        assert st == 0
        assert got.shape == ref.shape and np.array_equal(got, ref), name


def test_noalloc_nonfinite_status_and_refusals(A):
    x = synth.grf2d(64, 64, seed=synth.seed_of(1, 8))
    x[3, 5] = np.nan
    xg = torch.from_numpy(x).to(DEV)
    params = {"mode": "fixed_rate", "brick": (16, 16), "rate": 4.0, "code": 40}
    _, st = _noalloc(A, xg, params)
    assert st == -5  # APAX_E_NONFINITE
    # a clean call afterwards reports OK again (the status word is cleared per call)
    x[3, 5] = 0.0
    _, st = _noalloc(A, torch.from_numpy(x).to(DEV), params)
    assert st == 0
    # the profiled operating point needs a workspace: refused on the host
    with pytest.raises(A.ApaxError):
        A.apax_encode_noalloc(xg, dict(params, code=A.CODE_PROFILED),
                              torch.empty(1 << 16, dtype=torch.uint8, device=DEV),
                              torch.empty(1, dtype=torch.int64, device=DEV))
