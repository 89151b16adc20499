"""Oracle: a plain CPU statement of what the GPU library computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library and never imports or links it.

The arithmetic lives in ``oracle.c`` (unsigned __int128 with the compiler's
``%`` and ``/``; textbook base-2^32 long division for the 89-bit prime).  This
module compiles it with gcc on first use (or via :func:`build`) and wraps it with
ctypes over numpy arrays.

Conventions (Section 1.2 of the paper): a polynomial's coefficients are
``a_0 .. a_{k-1}``; coefficient arrays are row-major (row, polynomial, a_i); an
89-bit value is two little-endian uint64 limbs; tables are int64[rows][m].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

P61 = (1 << 61) - 1
P89 = (1 << 89) - 1
P64_59 = (1 << 64) - 59

PRIME_P61, PRIME_P89, PRIME_P64_59 = 1, 2, 3
TWO_FOR_ONE, TWO_FOR_ONE_MSB, TWO_POLY, ARB_R = 0, 1, 2, 3

OK, EINVAL, EDOMAIN, EOVERFLOW = 0, -1, -3, -4


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} returned status {status}")
        self.status = status


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP for the row loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            u64, i64, u32, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
            P = ctypes.c_void_p
            lib.orc_splitmix64.restype = u64
            lib.orc_splitmix64.argtypes = [P]
            lib.orc_coeffs_p61.argtypes = [u64, u64, P]
            lib.orc_coeffs_p89.argtypes = [u64, u64, P]
            lib.orc_hash_small.restype = u64
            lib.orc_hash_small.argtypes = [u64, P, u32, u64]
            lib.orc_hash_p89.argtypes = [P, u32, u64, P]
            for name in ("orc_cs_update_small",):
                getattr(lib, name).argtypes = [u64, u32, u32, i32, u32, u64, P, P, P, u64, P]
            lib.orc_cs_update_small_keypar.argtypes = [u64, u32, u32, i32, u32, u64, P, P, P, u64, P, i32]
            lib.orc_cs_update_p89.argtypes = [u32, i32, u32, u64, P, P, P, u64, P]
            lib.orc_bucket_sign_small.argtypes = [u64, u32, u32, i32, u64, P, u32, u64, P, P]
            lib.orc_bucket_sign_p89.argtypes = [u32, i32, u64, P, u32, u64, P, P]
            lib.orc_cs_estimate.argtypes = [P, u32, u64, P, P]
            lib.orc_exact_f2.argtypes = [P, P, u64, P]
            lib.orc_divmod.argtypes = [i32, P, u64, P, P]
            lib.orc_enum_hash.argtypes = [u64, u32, P, u32, P]
            lib.orc_enum_bucket_sign.argtypes = [u64, u32, u32, i32, u64, P, u32, P, P]
            lib.orc_enum_estimate_moments.argtypes = [u64, u32, u32, i32, u64, P, P, u64, P, P]
            lib.orc_bucket_map_exact.argtypes = [u64, u64, P, u64, u64, P]
            lib.orc_bucket_map_mersenne.argtypes = [u32, P, u64, u64, P]
            for f in (lib.orc_cs_update_small, lib.orc_cs_update_small_keypar, lib.orc_cs_update_p89,
                      lib.orc_bucket_sign_small, lib.orc_bucket_sign_p89, lib.orc_cs_estimate,
                      lib.orc_exact_f2, lib.orc_divmod, lib.orc_enum_hash, lib.orc_enum_bucket_sign,
                      lib.orc_enum_estimate_moments, lib.orc_bucket_map_exact, lib.orc_bucket_map_mersenne):
                f.restype = i32
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _u64(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.uint64:
        a = a.astype(np.int64).view(np.uint64) if a.dtype.kind == "i" else a.astype(np.uint64)
    return np.ascontiguousarray(a)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a).astype(np.int64))


def _check(status: int, what: str):
    if status != OK:
        raise OracleError(status, what)


def prime_bits(prime: int) -> int:
    return {PRIME_P61: 61, PRIME_P89: 89}[prime]


# --------------------------------------------------------------------------
# seed expansion and coefficients
# --------------------------------------------------------------------------
def splitmix64_stream(seed: int, count: int) -> list[int]:
    lib = _load()
    st = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return [int(lib.orc_splitmix64(ctypes.byref(st))) for _ in range(count)]


def npoly(mode: int) -> int:
    return 2 if mode == TWO_POLY else 1


def coeffs_from_seed(prime: int, rows: int, mode: int, seed: int, k: int = 4) -> np.ndarray:
    """Coefficients uniform in [p] expanded from ``seed``: shape (rows*npoly*k,)
    for p61, (rows*npoly*k, 2) for p89, in row / polynomial / a_i order."""
    lib = _load()
    count = rows * npoly(mode) * k
    if prime == PRIME_P61:
        out = np.zeros(count, dtype=np.uint64)
        lib.orc_coeffs_p61(seed & 0xFFFFFFFFFFFFFFFF, count, _ptr(out))
    elif prime == PRIME_P89:
        out = np.zeros((count, 2), dtype=np.uint64)
        lib.orc_coeffs_p89(seed & 0xFFFFFFFFFFFFFFFF, count, _ptr(out))
    else:
        raise ValueError("sketch primes are p61 and p89")
    return out


# --------------------------------------------------------------------------
# hashing
# --------------------------------------------------------------------------
def hash_small(p: int, a, x: int) -> int:
    a = _u64(a)
    return int(_load().orc_hash_small(p, _ptr(a), len(a), x & 0xFFFFFFFFFFFFFFFF))


def hash_p89(a, x: int) -> int:
    """a: (k, 2) limbs.  Returns the hash as a Python int."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, 2))
    out = np.zeros(2, dtype=np.uint64)
    _load().orc_hash_p89(_ptr(a), a.shape[0], x & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return int(out[0]) | (int(out[1]) << 64)


def bucket_sign(prime: int, mode: int, m: int, coeffs, row: int, x: int, k: int = 4,
                p: int | None = None, b: int | None = None) -> tuple[int, int]:
    lib = _load()
    bk = ctypes.c_uint64(0)
    sg = ctypes.c_int(0)
    if prime == PRIME_P89:
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint64).reshape(-1, 2))
        _check(lib.orc_bucket_sign_p89(k, mode, m, _ptr(c), row, x, ctypes.byref(bk), ctypes.byref(sg)), "bucket_sign")
    else:
        c = _u64(coeffs).reshape(-1)
        pp = P61 if p is None else p
        bb = 61 if b is None else b
        _check(lib.orc_bucket_sign_small(pp, bb, k, mode, m, _ptr(c), row, x, ctypes.byref(bk), ctypes.byref(sg)), "bucket_sign")
    return int(bk.value), int(sg.value)


# --------------------------------------------------------------------------
# Count Sketch
# --------------------------------------------------------------------------
def cs_update(prime: int, mode: int, rows: int, m: int, coeffs, keys, weights, table=None,
              k: int = 4, p: int | None = None, b: int | None = None, threads: int | None = None) -> np.ndarray:
    """Process every (key, weight) into ``table`` (int64[rows][m]; new zero table if None).

    ``p``/``b`` override the modulus for the tiny-prime checks (Mersenne p = 2^b - 1).
    ``threads`` selects the key-parallel variant with that many private tables."""
    lib = _load()
    keys = _u64(keys).reshape(-1)
    weights = _i64(weights).reshape(-1)
    if keys.shape != weights.shape:
        raise ValueError("keys and weights differ in length")
    if table is None:
        table = np.zeros((rows, m), dtype=np.int64)
    if table.dtype != np.int64 or not table.flags.c_contiguous or table.size != rows * m:
        raise ValueError("table must be a C-contiguous int64 array of rows*m entries")
    n = keys.shape[0]
    if prime == PRIME_P89:
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint64).reshape(-1, 2))
        st = lib.orc_cs_update_p89(k, mode, rows, m, _ptr(c), _ptr(keys), _ptr(weights), n, _ptr(table))
    else:
        c = _u64(coeffs).reshape(-1)
        pp = P61 if p is None else p
        bb = 61 if b is None else b
        if threads:
            st = lib.orc_cs_update_small_keypar(pp, bb, k, mode, rows, m, _ptr(c), _ptr(keys), _ptr(weights),
                                                n, _ptr(table), int(threads))
        else:
            st = lib.orc_cs_update_small(pp, bb, k, mode, rows, m, _ptr(c), _ptr(keys), _ptr(weights), n,
                                         _ptr(table))
    _check(st, "cs_update")
    return table


def cs_estimate(table) -> tuple[int, np.ndarray]:
    """Median-of-rows F2 estimate and the per-row estimates X_j = sum_i C[j][i]^2."""
    table = np.ascontiguousarray(np.asarray(table, dtype=np.int64))
    rows, m = table.shape
    rows_out = np.zeros(rows, dtype=np.int64)
    med = ctypes.c_int64(0)
    _check(_load().orc_cs_estimate(_ptr(table), rows, m, _ptr(rows_out), ctypes.byref(med)), "cs_estimate")
    return int(med.value), rows_out


def cs_estimate_status(table) -> tuple[int, int, np.ndarray]:
    """(status, median, per-row X_j) without raising; an X_j that does not fit
    in int64 reads INT64_MAX and the status is EOVERFLOW."""
    table = np.ascontiguousarray(np.asarray(table, dtype=np.int64))
    rows, m = table.shape
    rows_out = np.zeros(rows, dtype=np.int64)
    med = ctypes.c_int64(0)
    st = _load().orc_cs_estimate(_ptr(table), rows, m, _ptr(rows_out), ctypes.byref(med))
    return int(st), int(med.value), rows_out


def exact_f2(keys, weights) -> int:
    keys = _u64(keys).reshape(-1)
    weights = _i64(weights).reshape(-1)
    out = np.zeros(2, dtype=np.uint64)
    _check(_load().orc_exact_f2(_ptr(keys), _ptr(weights), keys.shape[0], _ptr(out)), "exact_f2")
    v = int(out[0]) | (int(out[1]) << 64)
    return v - (1 << 128) if v >> 127 else v


# --------------------------------------------------------------------------
# quotient and remainder
# --------------------------------------------------------------------------
def divmod_batch(prime: int, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """x: uint64 limbs, shape (n, 2) for p61 / p64-59, (n, 3) for p89.
    Returns (q, r) with shape (n,) each, or (n, 2) each for p89."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    n = x.shape[0]
    w = 2 if prime == PRIME_P89 else 1
    q = np.zeros((n, w), dtype=np.uint64)
    r = np.zeros((n, w), dtype=np.uint64)
    _check(_load().orc_divmod(prime, _ptr(x), n, _ptr(q), _ptr(r)), "divmod")
    if w == 1:
        return q.reshape(-1), r.reshape(-1)
    return q, r


# --------------------------------------------------------------------------
# maps of hash values in [p] to [r] buckets (Sections 1.4 and 1.5)
# --------------------------------------------------------------------------
def _limbs2(v) -> np.ndarray:
    """Values below 2^128 (Python ints or a uint64 array) as an (n, 2) uint64 limb array."""
    a = np.asarray(v)
    if a.ndim == 2:
        return np.ascontiguousarray(a.astype(np.uint64))
    if a.dtype == np.uint64 or (a.dtype.kind in "iu" and a.dtype.itemsize <= 8):
        out = np.zeros((a.shape[0], 2), dtype=np.uint64)
        out[:, 0] = _u64(a)
        return out
    out = np.zeros((len(v), 2), dtype=np.uint64)
    for i, x in enumerate(v):
        out[i, 0], out[i, 1] = int(x) & 0xFFFFFFFFFFFFFFFF, int(x) >> 64
    return out


def bucket_map_exact(p: int, v, r: int) -> np.ndarray:
    """floor(v * r / p) for each v in [p] (p < 2^89), as uint32."""
    x = _limbs2(v)
    out = np.zeros(x.shape[0], dtype=np.uint32)
    _check(_load().orc_bucket_map_exact(p & 0xFFFFFFFFFFFFFFFF, p >> 64, _ptr(x), x.shape[0], r, _ptr(out)),
           "bucket_map_exact")
    return out


def bucket_map_mersenne(b: int, v, r: int) -> np.ndarray:
    """floor((v + 1) * r / 2^b) for each v in [2^b - 1], as uint32."""
    x = _limbs2(v)
    out = np.zeros(x.shape[0], dtype=np.uint32)
    _check(_load().orc_bucket_map_mersenne(b, _ptr(x), x.shape[0], r, _ptr(out)), "bucket_map_mersenne")
    return out


# --------------------------------------------------------------------------
# wide quotient and remainder (Section 4's experiment): x of 2b bits divided by
# p = 2^b - c, b a multiple of 32.  Values are "limb planes": a uint32 array of
# shape (limbs, n) whose row j holds limb j (bits 32j..32j+31) of every value.
# The oracle is the plain definition, Python's integer divmod per value.
# --------------------------------------------------------------------------
def planes_to_ints(planes) -> list[int]:
    planes = np.asarray(planes, dtype=np.uint32)
    out = [0] * planes.shape[1]
    for j in range(planes.shape[0] - 1, -1, -1):
        row = planes[j].tolist()
        out = [(o << 32) | v for o, v in zip(out, row)]
    return out


def ints_to_planes(vals, limbs: int) -> np.ndarray:
    out = np.zeros((limbs, len(vals)), dtype=np.uint32)
    for i, v in enumerate(vals):
        if v < 0 or v >> (32 * limbs):
            raise ValueError("value does not fit the limbs")
        for j in range(limbs):
            out[j, i] = (v >> (32 * j)) & 0xFFFFFFFF
    return out


def divmod_wide(b: int, c: int, x_planes) -> tuple[np.ndarray, np.ndarray]:
    """floor(x / p) and x mod p for p = 2^b - c and every 2b-bit x (planes of 2b/32 limbs).
    Returns (quotient planes with b/32 + 1 limbs, remainder planes with b/32 limbs)."""
    if b % 32 or b <= 0 or not 0 < c < (1 << b) - 1:
        raise ValueError("b must be a positive multiple of 32 and 0 < c < 2^b - 1")
    w = b // 32
    x_planes = np.asarray(x_planes, dtype=np.uint32)
    if x_planes.shape[0] != 2 * w:
        raise ValueError("x needs 2b/32 limbs")
    p = (1 << b) - c
    qs, rs = [], []
    for x in planes_to_ints(x_planes):
        q, r = divmod(x, p)
        qs.append(q)
        rs.append(r)
    return ints_to_planes(qs, w + 1), ints_to_planes(rs, w)


# --------------------------------------------------------------------------
# exhaustive enumeration over Z_p^k (tiny primes)
# --------------------------------------------------------------------------
def enum_hash(p: int, k: int, keys) -> np.ndarray:
    keys = _u64(keys).reshape(-1)
    out = np.zeros((p ** k, keys.shape[0]), dtype=np.uint64)
    _check(_load().orc_enum_hash(p, k, _ptr(keys), keys.shape[0], _ptr(out)), "enum_hash")
    return out


def enum_bucket_sign(p: int, b: int, k: int, mode: int, m: int, keys) -> tuple[np.ndarray, np.ndarray]:
    keys = _u64(keys).reshape(-1)
    bk = np.zeros((p ** k, keys.shape[0]), dtype=np.uint64)
    sg = np.zeros((p ** k, keys.shape[0]), dtype=np.int32)
    _check(_load().orc_enum_bucket_sign(p, b, k, mode, m, _ptr(keys), keys.shape[0], _ptr(bk), _ptr(sg)),
           "enum_bucket_sign")
    return bk, sg


def enum_estimate_moments(p: int, b: int, k: int, mode: int, m: int, keys, weights) -> tuple[int, int]:
    keys = _u64(keys).reshape(-1)
    weights = _i64(weights).reshape(-1)
    s1 = np.zeros(2, dtype=np.uint64)
    s2 = np.zeros(2, dtype=np.uint64)
    _check(_load().orc_enum_estimate_moments(p, b, k, mode, m, _ptr(keys), _ptr(weights), keys.shape[0],
                                             _ptr(s1), _ptr(s2)), "enum_estimate_moments")
    return int(s1[0]) | (int(s1[1]) << 64), int(s2[0]) | (int(s2[1]) << 64)
