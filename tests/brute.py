"""Independent pure-Python checkers for tiny inputs.

Nothing here is shared with the CPU oracle or the GPU library: widths are
found by search, JEE costs by dynamic programming over every valid parse,
derivative streams with numpy.diff, their inverses with numpy.cumsum, and the
container is parsed from the byte layout.  These are the pins the oracle is
checked against.
"""
from __future__ import annotations

import struct
from fractions import Fraction

import numpy as np

MAGIC = 0x58415041


# ---------------------------------------------------------------- widths

def width_brute(vals) -> int:
    """Smallest w >= 0 such that every value is a w-bit two's-complement
    number (w = 0 only for all-zero groups)."""
    vals = [int(v) for v in vals]
    if all(v == 0 for v in vals):
        return 0
    w = 1
    while not all(-(1 << (w - 1)) <= v <= (1 << (w - 1)) - 1 for v in vals):
        w += 1
    return w


def eps_of(vals) -> int:
    return min(width_brute(vals), 31)


def pw_of(eps: int, W: int) -> int:
    return 32 if (W == 32 and eps == 31) else eps


# ---------------------------------------------------------------- JEE

def jee_min_bits(eps) -> int:
    """Minimum token bits over every valid JEE parse of eps[1:] (pairs of
    differences in [-1, 1] as one 4-bit token, single differences in
    [-2, 2] as a 4-bit token, anything as an 8-bit absolute token)."""
    G = len(eps)
    f = [0] * (G + 2)
    for i in range(G - 1, 0, -1):
        d = eps[i] - eps[i - 1]
        best = 8 + f[i + 1]
        if abs(d) <= 2:
            best = min(best, 4 + f[i + 1])
        if i + 1 <= G - 1 and abs(d) <= 1 and abs(eps[i + 1] - eps[i]) <= 1:
            best = min(best, 4 + f[i + 2])
        f[i] = best
    return f[1] if G > 1 else 0


def token_decode(nibbles, eps0: int, G: int):
    """Decode a JEE nibble sequence back to the exponent sequence.
    Codes: 0..8 two differences (3(da+1) + (db+1)); 9..13 one difference
    (code - 11); 14/15 escape, exponent = 16 (code - 14) + next nibble."""
    eps = [eps0]
    k = 0
    while len(eps) < G:
        t = nibbles[k]
        k += 1
        if t <= 8:
            eps.append(eps[-1] + t // 3 - 1)
            eps.append(eps[-1] + t % 3 - 1)
        elif t <= 13:
            eps.append(eps[-1] + t - 11)
        else:
            eps.append(16 * (t - 14) + nibbles[k])
            k += 1
    assert len(eps) == G
    return eps, k


# ---------------------------------------------------------------- streams

DERIV_AXES = {0: (), 1: (2,), 2: (2, 2), 3: (1,), 4: (0,), 5: (1, 2), 6: (0, 1, 2)}


def wrap(v, W):
    v = np.asarray(v, np.int64)
    m = (1 << W) - 1
    u = v & m
    return np.where(u >> (W - 1) & 1, u - (1 << W), u).astype(np.int64)


def stream_np(a3, s: int, W: int):
    """Stream s of a (bz, by, bx) brick via numpy.diff (neighbour outside the
    brick = 0)."""
    v = np.asarray(a3, np.int64)
    for ax in DERIV_AXES[s]:
        v = np.diff(v, axis=ax, prepend=0)
    return wrap(v, W)


def unstream_np(v3, s: int, W: int):
    v = np.asarray(v3, np.int64)
    for ax in DERIV_AXES[s]:
        v = np.cumsum(v, axis=ax)
    return wrap(v, W)


def size_model(a3, s: int, W: int, H: int, valid3=None, n: int = 4) -> int:
    """Bits of a block coded with stream s: header + minimal JEE tokens +
    BFPE payload (n samples per exponent)."""
    B = a3.size
    if s == 7:
        return H + B * W
    v = stream_np(a3, s, W).ravel()
    if valid3 is not None:
        v = np.where(np.asarray(valid3).ravel(), v, 0)
    eps = [eps_of(v[n * i:n * i + n]) for i in range(B // n)]
    return H + jee_min_bits(eps) + sum(n * pw_of(e, W) for e in eps)


# ---------------------------------------------------------------- gain grid

def gain_exact(c: int) -> Fraction:
    k, f = divmod(c, 16)
    return Fraction(16 + f) * (Fraction(2) ** (k - 4))


def gain(c: int) -> float:
    return float(gain_exact(c))


def dequant_np(a, c: int):
    k, f = divmod(c, 16)
    R = float(Fraction(16, 16 + f))
    return np.ldexp(np.asarray(a, np.float64) * R, -k)


# ---------------------------------------------------------------- container

class Stream:
    def __init__(self, buf):
        b = bytes(np.asarray(buf, np.uint8))
        self.b = b
        (self.magic, self.version, self.dtype, self.mode, self.ndim, self.mask,
         self.budget, self.code) = struct.unpack_from("<IHBBBBHi", b, 0)
        self.dims = struct.unpack_from("<3Q", b, 16)[: self.ndim]
        self.brick = struct.unpack_from("<3H", b, 40)[: self.ndim]
        self.nblocks, self.payload_words = struct.unpack_from("<QQ", b, 48)
        nb = self.nblocks
        if self.mode == 1:
            self.area = 64
            self.lens = [self.budget] * nb
            self.sbo = []
        else:
            self.lens = list(struct.unpack_from(f"<{nb}H", b, 64)) if nb else []
            off = 64 + (2 * nb + 7) // 8 * 8
            nsb = (nb + 63) // 64
            self.sbo = list(struct.unpack_from(f"<{nsb}Q", b, off)) if nsb else []
            self.area = (off + 8 * nsb + 15) // 16 * 16
        self.offsets = [0] * nb
        acc = 0
        for j in range(nb):
            self.offsets[j] = acc
            acc += self.lens[j]
        self.total_words = acc

    def block(self, j):
        o = self.area + 4 * self.offsets[j]
        return np.frombuffer(self.b[o:o + 4 * self.lens[j]], np.uint32)


class BitReader:
    def __init__(self, words):
        self.v = 0
        for i, w in enumerate(words):
            self.v |= int(w) << (32 * i)
        self.n = 32 * len(words)
        self.pos = 0

    def get(self, n):
        r = (self.v >> self.pos) & ((1 << n) - 1)
        self.pos += n
        return r

    def sget(self, n):
        r = self.get(n)
        if n and r >> (n - 1):
            r -= 1 << n
        return r


def parse_block(words, isint: bool, G: int, W: int, n: int = 4):
    """Return (stream, eps0, code, eps list, nibbles, payload values, bits used)
    of a block of G exponent groups of n samples."""
    br = BitReader(words)
    s = br.get(3)
    eps0 = br.get(5)
    code = br.sget(10 if isint else 16)
    rsv = br.get(14 if isint else 24)
    assert rsv == 0
    if s == 7:
        vals = [br.sget(W) for _ in range(n * G)]
        return s, eps0, code, None, [], vals, br.pos
    nib = []
    eps = [eps0]
    while len(eps) < G:
        t = br.get(4)
        nib.append(t)
        if t <= 8:
            eps += [eps[-1] + t // 3 - 1]
            eps += [eps[-1] + t % 3 - 1]
        elif t <= 13:
            eps.append(eps[-1] + t - 11)
        else:
            lo = br.get(4)
            nib.append(lo)
            eps.append(16 * (t - 14) + lo)
    vals = []
    for e in eps:
        p = pw_of(e, W)
        vals += [br.sget(p) for _ in range(n)]
    return s, eps0, code, eps, nib, vals, br.pos
