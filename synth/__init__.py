"""Seeded synthetic inputs shaped like the paper's datasets (Table 2 types:
int time series, fp32 climate/geology-like fields, fp64 simulation fields).

This module holds input generation only -- none of the codec's arithmetic --
and is the one module that both the GPU tests/benchmark and the CPU oracle
use.  Everything is host numpy with numpy.random.default_rng(seed).
"""
from __future__ import annotations

import math

import numpy as np

SEED0 = 13034994


def seed_of(config: int, item: int = 0) -> int:
    return SEED0 + 1000 * config + item


# --------------------------------------------------------------------------
# time series: three sinusoids + Gaussian noise, int16 (sensor-like, Sec. 5
# oversampling and ADC noise)

def sinusoids(n: int = 1 << 20, seed: int | None = None, amp_total: float = 12000.0,
              noise: float = 40.0) -> np.ndarray:
    rng = np.random.default_rng(seed_of(0) if seed is None else seed)
    f = rng.uniform(0.001, 0.1, 3)
    ph = rng.uniform(0.0, 2 * math.pi, 3)
    w = rng.uniform(0.0, 1.0, 3)
    amp = amp_total * w / w.sum()
    t = np.arange(n, dtype=np.float64)
    s = np.zeros(n)
    for k in range(3):
        s += amp[k] * np.sin(2 * math.pi * f[k] * t + ph[k])
    s += rng.normal(0.0, noise, n)
    return np.clip(np.rint(s), -32768, 32767).astype(np.int16)


# --------------------------------------------------------------------------
# 2-D Gaussian random field with power spectrum k^-3, scaled to [-1e3, 1e3]
# plus white noise (climate / geology-like fp32 field)

def grf2d(ny: int = 4096, nx: int = 4096, seed: int | None = None, lo: float = -1e3,
          hi: float = 1e3, noise: float = 1e-2) -> np.ndarray:
    rng = np.random.default_rng(seed_of(1) if seed is None else seed)
    w = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    k = np.sqrt(ky * ky + kx * kx)
    k[0, 0] = 1.0
    amp = k ** -1.5
    amp[0, 0] = 0.0
    w *= amp
    f = np.fft.ifft2(w).real
    del w
    fmin, fmax = f.min(), f.max()
    f = lo + (f - fmin) * ((hi - lo) / (fmax - fmin))
    f += rng.normal(0.0, noise, f.shape)
    return f.astype(np.float32)


# --------------------------------------------------------------------------
# 3-D simulation-like field: 32 separable Gaussian blobs + linear gradient +
# tiny white noise (fp64)

def blobs3d(nz: int = 256, ny: int = 512, nx: int = 512, seed: int | None = None,
            nblobs: int = 32, noise_rel: float = 1e-6) -> np.ndarray:
    rng = np.random.default_rng(seed_of(2) if seed is None else seed)
    cz = rng.uniform(0, nz, nblobs)
    cy = rng.uniform(0, ny, nblobs)
    cx = rng.uniform(0, nx, nblobs)
    sig = rng.uniform(8.0, 48.0, nblobs)
    A = rng.uniform(-1.0, 1.0, nblobs)
    a, b, c = rng.uniform(-0.5, 0.5, 3)
    z = np.arange(nz, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    x = np.arange(nx, dtype=np.float64)
    gz = A[:, None] * np.exp(-0.5 * ((z[None, :] - cz[:, None]) / sig[:, None]) ** 2)
    gy = np.exp(-0.5 * ((y[None, :] - cy[:, None]) / sig[:, None]) ** 2)
    gx = np.exp(-0.5 * ((x[None, :] - cx[:, None]) / sig[:, None]) ** 2)
    gyx = (gy[:, :, None] * gx[:, None, :]).reshape(nblobs, ny * nx)
    f = (gz.T @ gyx).reshape(nz, ny, nx)
    del gyx
    f += (a * z / nz)[:, None, None]
    f += (b * y / ny)[None, :, None]
    f += (c * x / nx)[None, None, :]
    rngv = float(f.max() - f.min())
    f += rng.normal(0.0, noise_rel * rngv, f.shape)
    return f


# --------------------------------------------------------------------------
# batched items (mixed sizes / dtypes / generators)

BATCH_DTYPES = (np.int16, np.int32, np.float32, np.float64)


def item_spec(i: int, seed: int | None = None, lo_bytes: int = 4 << 10,
              hi_bytes: int = 64 << 20) -> dict:
    """Parameters of batched item i: dtype, length, generator, mode, rate."""
    rng = np.random.default_rng((seed_of(3) if seed is None else seed) + 7919 * i)
    nbytes = int(math.floor(math.exp(rng.uniform(math.log(lo_bytes), math.log(hi_bytes)))))
    dt = np.dtype(BATCH_DTYPES[int(rng.integers(0, 4))])
    n = max(1, nbytes // dt.itemsize)
    gen = int(rng.integers(0, 3))
    offset = int(rng.integers(0, 1 << 30))
    if dt.kind == "i":
        mode = "lossless" if rng.uniform() < 0.5 else "fixed_rate"
    else:
        mode = "fixed_rate"
    rate = float(rng.uniform(3.0, 10.0))
    return {"index": i, "dtype": dt, "n": n, "gen": gen, "offset": offset, "mode": mode,
            "rate": rate}


class Pools:
    """Three float64 sample pools (one per generator), flattened to 1-D.

    A batched item is a window of one pool, cast to its dtype.  Ints scale the
    pool peak to 0.366 of the dtype maximum and round (the 12000/32767
    headroom of the int16 time series)."""

    def __init__(self, n: int = 1 << 26, seed: int | None = None):
        s = seed_of(3) if seed is None else seed
        self.n = n
        ts = sinusoids(n, seed=s + 1).astype(np.float64)
        side = int(math.isqrt(n))
        while n % side:
            side -= 1
        f2 = grf2d(n // side, side, seed=s + 2).astype(np.float64).ravel()
        nz = max(1, n // (256 * 256))
        f3 = blobs3d(nz, 256, 256, seed=s + 3).ravel()
        if f3.size < n:
            f3 = np.resize(f3, n)
        self.pool = [ts[:n], f2[:n], f3[:n]]
        self.peak = [float(np.abs(p).max()) or 1.0 for p in self.pool]

    def item(self, spec: dict) -> np.ndarray:
        p = self.pool[spec["gen"]]
        n = spec["n"]
        start = spec["offset"] % max(1, self.n - n) if n < self.n else 0
        w = p[start:start + n]
        if w.size < n:
            w = np.resize(w, n)
        dt = spec["dtype"]
        if dt.kind == "i":
            scale = 0.366 * np.iinfo(dt).max / self.peak[spec["gen"]]
            return np.rint(w * scale).astype(dt)
        return w.astype(dt)

    def item_device(self, spec: dict, device):
        """The same window as item(), cut and cast on the device from a
        device-resident copy of the pool (identical values: the product and
        the half-to-even rounding are the same binary64 operations)."""
        import torch
        if not hasattr(self, "_dev"):
            self._dev = {}
        key = (str(device), spec["gen"])
        if key not in self._dev:
            self._dev[key] = torch.from_numpy(self.pool[spec["gen"]]).to(device)
        p = self._dev[key]
        n = spec["n"]
        start = spec["offset"] % max(1, self.n - n) if n < self.n else 0
        w = p[start:start + n]
        if w.numel() < n:
            w = w.repeat((n + w.numel() - 1) // w.numel())[:n]
        dt = spec["dtype"]
        tdt = {np.dtype(np.int16): torch.int16, np.dtype(np.int32): torch.int32,
               np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64,
               np.dtype(np.int8): torch.int8}[np.dtype(dt)]
        if dt.kind == "i":
            scale = 0.366 * np.iinfo(dt).max / self.peak[spec["gen"]]
            return torch.round(w * scale).to(tdt)
        return w.to(tdt).contiguous()


# --------------------------------------------------------------------------
# served request stream

def requests(n: int, seed: int | None = None, lo_bytes: int = 64 << 10,
             hi_bytes: int = 256 << 20) -> list:
    """Request list: Poisson arrival gaps are drawn later (they depend on the
    measured plain throughput); here: payload size, dtype, generator, kind."""
    out = []
    base = seed_of(4) if seed is None else seed
    for i in range(n):
        spec = item_spec(i, seed=base, lo_bytes=lo_bytes, hi_bytes=hi_bytes)
        rng = np.random.default_rng(base + 104729 * i + 1)
        spec["kind"] = "encode" if rng.uniform() < 0.5 else "decode"
        spec["gap_u"] = float(rng.uniform())
        out.append(spec)
    return out


def modulated(dt, n: int, seed: int, b: int, noise: float = 0.01) -> np.ndarray:
    """A carrier at bin b of 1024 (b / 1024 cycles per sample) under a slow
    envelope, plus white noise; integers scaled to 90 % of the dtype's range."""
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    env = 1.0 + 0.3 * np.sin(2 * np.pi * t / 5000.0)
    s = env * np.cos(2 * np.pi * b * t / 1024 + 0.7) + noise * rng.standard_normal(n)
    dt = np.dtype(dt)
    if dt.kind == "i":
        return np.rint(s / np.abs(s).max() * 0.9 * np.iinfo(dt).max).astype(dt)
    return (s * 3.0).astype(dt)
