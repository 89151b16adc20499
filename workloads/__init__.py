"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the hashing or sketching arithmetic: only random
streams and the distributions the workloads draw from.  Everything is
counter-based, so element ``i`` of a stream depends only on ``(seed, stream, i)``
and the same code runs on CPU tensors and on GPU tensors (torch, int64 bit
patterns standing for uint64).

Generators
  * SplitMix64 (Steele, Lea, Flood 2014) as a counter-based stream: output i of
    a stream is the SplitMix64 finaliser applied to ``key + (i+1)*0x9E3779B97F4A7C15``.
  * uniform keys, bounded integers by rejection, log-uniform integers,
  * Zipf(s) over ranks 1..N by rejection-inversion (Hormann and Derflinger,
    "Rejection-inversion to generate variates from monotone discrete
    distributions", 1996), key = rank - 1,
  * uniform values in [0, p^2) for the quotient/remainder workload, by
    rejection on random bits.
"""
from __future__ import annotations

import math

import torch

GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_STREAM_MUL = 0xD1B54A32D192ED03


def _s64(v: int) -> int:
    """Python int (mod 2^64) -> the signed int64 with the same bits."""
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >> 63 else v


def _shr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _shr(z, 30)) * _s64(_M1)
    z = (z ^ _shr(z, 27)) * _s64(_M2)
    return z ^ _shr(z, 31)


def _mix_int(z: int) -> int:
    z &= 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * _M1) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * _M2) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return _mix_int((seed & 0xFFFFFFFFFFFFFFFF) ^ ((stream * _STREAM_MUL) & 0xFFFFFFFFFFFFFFFF))


def raw64(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """64 random bits per counter value in ``idx`` (int64 tensor), as int64."""
    key = stream_key(seed, stream)
    z = (idx + 1) * _s64(GOLDEN) + _s64(key)
    return _mix(z)


def _arange(n: int, device) -> torch.Tensor:
    return torch.arange(n, dtype=torch.int64, device=device)


def uniform01(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """Doubles uniform in (0, 1) from the top 53 bits."""
    r = _shr(raw64(seed, stream, idx), 11)
    return (r.to(torch.float64) + 0.5) * (2.0 ** -53)


def uniform_u32(seed: int, n: int, device="cpu", stream: int = 1) -> torch.Tensor:
    """n keys uniform in [0, 2^32), as int64 (values fit in uint32)."""
    return _shr(raw64(seed, stream, _arange(n, device)), 32)


def uniform_u64(seed: int, n: int, device="cpu", stream: int = 1) -> torch.Tensor:
    """n keys uniform in [0, 2^64), int64 bit patterns."""
    return raw64(seed, stream, _arange(n, device))


def bounded_int(seed: int, n: int, lo: int, hi: int, device="cpu", stream: int = 2) -> torch.Tensor:
    """n integers uniform in [lo, hi] (inclusive) by rejection on the top bits."""
    span = hi - lo + 1
    if span <= 0 or span > (1 << 62):
        raise ValueError("bad range")
    bits = max(1, (span - 1).bit_length())
    idx = _arange(n, device)
    out = torch.empty(n, dtype=torch.int64, device=device)
    pending = idx
    attempt = 0
    while pending.numel():
        v = _shr(raw64(seed, stream, pending + (attempt << 40)), 64 - bits)
        ok = v < span
        out[pending[ok]] = v[ok] + lo
        pending = pending[~ok]
        attempt += 1
    return out


def loguniform_int(seed: int, n: int, lo_exp: float, hi_exp: float, device="cpu", stream: int = 3) -> torch.Tensor:
    """floor(2^U) with U uniform in [lo_exp, hi_exp)."""
    u = uniform01(seed, stream, _arange(n, device))
    return torch.floor(torch.exp2(lo_exp + (hi_exp - lo_exp) * u)).to(torch.int64)


class _ZipfConst:
    def __init__(self, s: float, N: int):
        self.s, self.N = s, N
        self.hx1 = self.H(1.5) - 1.0
        self.hN = self.H(N + 0.5)
        self.sconst = 2.0 - self.Hinv(self.H(2.5) - self.h(2.0))

    def H(self, x: float) -> float:
        return (x ** (1.0 - self.s) - 1.0) / (1.0 - self.s)

    def Hinv(self, y: float) -> float:
        return (1.0 + y * (1.0 - self.s)) ** (1.0 / (1.0 - self.s))

    def h(self, x: float) -> float:
        return x ** (-self.s)


def zipf(seed: int, n: int, s: float, N: int, device="cpu", stream: int = 4) -> torch.Tensor:
    """n keys = rank - 1, rank ~ Zipf(s) on {1..N} (s > 0, s != 1), by rejection-inversion."""
    if s <= 0 or s == 1.0:
        raise ValueError("s must be positive and != 1")
    c = _ZipfConst(s, N)
    one_minus_s = 1.0 - s
    idx = _arange(n, device)
    out = torch.empty(n, dtype=torch.int64, device=device)
    pending = idx
    attempt = 0
    while pending.numel():
        u01 = uniform01(seed, stream, pending + (attempt << 40))
        u = c.hN + u01 * (c.hx1 - c.hN)
        x = torch.pow(1.0 + u * one_minus_s, 1.0 / one_minus_s)
        k = torch.floor(x + 0.5).clamp_(1.0, float(N))
        hk = (torch.pow(k + 0.5, one_minus_s) - 1.0) / one_minus_s - torch.pow(k, -s)
        ok = ((k - x) <= c.sconst) | (u >= hk)
        out[pending[ok]] = k[ok].to(torch.int64) - 1
        pending = pending[~ok]
        attempt += 1
    return out


def _ult(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Unsigned < on int64 bit patterns."""
    bias = -(1 << 63)
    return (a ^ bias) < (b ^ bias)


def below_limbs(bound: int, nlimbs: int, seed: int, n: int, device="cpu", stream: int = 5) -> torch.Tensor:
    """n values uniform in [0, bound) as little-endian int64 limbs, shape (n, nlimbs),
    by rejection on bound.bit_length() random bits."""
    bits = bound.bit_length()
    if bits > 64 * nlimbs:
        raise ValueError("bound does not fit")
    bl = [_s64(bound >> (64 * j)) for j in range(nlimbs)]
    out = torch.empty((n, nlimbs), dtype=torch.int64, device=device)
    pending = _arange(n, device)
    attempt = 0
    while pending.numel():
        limbs = []
        for j in range(nlimbs):
            rb = min(64, max(0, bits - 64 * j))
            r = raw64(seed, stream * 16 + j, pending + (attempt << 40))
            limbs.append(torch.zeros_like(r) if rb == 0 else _shr(r, 64 - rb) if rb < 64 else r)
        # lexicographic unsigned compare from the top limb
        lt = torch.zeros_like(pending, dtype=torch.bool)
        eq = torch.ones_like(pending, dtype=torch.bool)
        for j in reversed(range(nlimbs)):
            b = torch.full_like(limbs[j], bl[j])
            lt = lt | (eq & _ult(limbs[j], b))
            eq = eq & (limbs[j] == b)
        ok = lt
        out[pending[ok]] = torch.stack([l[ok] for l in limbs], dim=1)
        pending = pending[~ok]
        attempt += 1
    return out


def as_uint64_numpy(t: torch.Tensor):
    """CPU numpy uint64 view of an int64 tensor's bits."""
    return t.detach().cpu().numpy().view("uint64")


# ----------------------------------------------------------------------------
# Workload recipes (seeds, sizes and distributions), one per named workload.
# ----------------------------------------------------------------------------
DATA_SEED = 0x2008086540


def stream_small_u32(n: int = 1 << 16, device="cpu", seed: int = DATA_SEED + 0):
    """Single stream: n uint32 keys uniform, weights int64 = 1."""
    keys = uniform_u32(seed, n, device)
    w = torch.ones(n, dtype=torch.int64, device=device)
    return keys, w


def stream_zipf_u64(n: int = 1 << 28, s: float = 1.1, device="cpu", seed: int = DATA_SEED + 1):
    """Single stream at scale: uint64 keys Zipf(s) over [2^32], int32 weights in [-100, 100]."""
    keys = zipf(seed, n, s, 1 << 32, device)
    w = bounded_int(seed, n, -100, 100, device).to(torch.int32)
    return keys, w


def stream_uniform_u64(n: int = 1 << 26, device="cpu", seed: int = DATA_SEED + 2):
    """uint64 keys uniform over [2^64], weights int64 = 1 (89-bit prime sketch)."""
    keys = uniform_u64(seed, n, device)
    w = torch.ones(n, dtype=torch.int64, device=device)
    return keys, w


def served_tenants(count: int = 1024, seed: int = DATA_SEED + 5):
    """Served workload tenants: log2 of the bucket count uniform in {12..18} (7 rows each)."""
    return bounded_int(seed, count, 12, 18, stream=6)


def served_requests(n: int, tenants: int, seed: int = DATA_SEED + 5, f2_frac: float = 0.1):
    """Served workload requests: tenant uniform, F2 query with probability f2_frac, otherwise an
    update of floor(2^U(10, 20)) keys.  Returns (tenant, is_f2, size) CPU int64 tensors (size 0
    for F2)."""
    tenant = bounded_int(seed, n, 0, tenants - 1, stream=7)
    is_f2 = (uniform01(seed, 8, _arange(n, "cpu")) < f2_frac).to(torch.int64)
    size = loguniform_int(seed, n, 10.0, 20.0, stream=9) * (1 - is_f2)
    return tenant, is_f2, size


def poisson_arrivals(n: int, rate: float, seed: int = DATA_SEED + 5, stream: int = 10):
    """Arrival times (seconds, float64, CPU) of a Poisson process of the given rate."""
    u = uniform01(seed, stream, _arange(n, "cpu"))
    return torch.cumsum(-torch.log1p(-u) / rate, 0)


def log2_ceil(v: int) -> int:
    return max(0, (v - 1).bit_length())


def fact_zipf_top_mass(s: float, N: int, top: int) -> float:
    """Probability mass of the `top` most likely ranks of Zipf(s) on {1..N} (for docs/tests)."""
    # mass ~ sum_{k<=top} k^-s / sum_{k<=N} k^-s, tail by the integral approximation
    head = sum(k ** (-s) for k in range(1, top + 1))
    def tail(a, b):
        return (b ** (1 - s) - a ** (1 - s)) / (1 - s)
    total = sum(k ** (-s) for k in range(1, 10001)) + tail(10000.5, N + 0.5)
    return head / total


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "torch", "annotations")]
