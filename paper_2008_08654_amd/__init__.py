"""Python binding of libmcs.so (include/mcs.h) -- argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module converts
torch tensors to device pointers and HIP streams to handles, calls the C ABI
through ctypes and turns non-zero statuses into exceptions.  There is no
fallback: if libmcs.so is missing, importing the binding functions raises.

Build the library first with ``python -m paper_2008_08654_amd.build`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcs.so")

# enums mirrored from include/mcs.h
CS_OK, CS_EINVAL, CS_ENOMEM, CS_EDOMAIN, CS_EOVERFLOW, CS_EDEVICE, CS_EBUSY = 0, -1, -2, -3, -4, -5, -6
CS_P61, CS_P89, CS_P64_59 = 1, 2, 3
CS_TWO_FOR_ONE, CS_TWO_FOR_ONE_MSB, CS_TWO_POLY, CS_ARB_R = 0, 1, 2, 3
CS_MAP_EXACT, CS_MAP_MERSENNE = 0, 1
CS_WIDE_ALG5, CS_WIDE_CCH = 0, 1
CS_U32, CS_U64, CS_I32, CS_I64 = 0, 1, 2, 3
CS_PATH_AUTO, CS_PATH_LDS, CS_PATH_GLOBAL, CS_PATH_BINNED, CS_PATH_BINNED_NOCOMBINE, CS_PATH_ROWS = 0, 1, 2, 3, 4, 5

_STATUS_NAMES = {0: "CS_OK", -1: "CS_EINVAL", -2: "CS_ENOMEM", -3: "CS_EDOMAIN", -4: "CS_EOVERFLOW",
                 -5: "CS_EDEVICE", -6: "CS_EBUSY"}

_lib = None


class MCSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libmcs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2008_08654_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "cs_create": [u32, u64, i32, u64, P],
            "cs_create_ex": [u32, u64, i32, u64, i32, u32, P],
            "cs_create_with_coeffs": [u32, u64, i32, i32, u32, P, P],
            "cs_update": [P, P, i32, P, i32, u64, P],
            "cs_estimate_f2": [P, P, P, P],
            "cs_query": [P, P, i32, u64, P, P],
            "cs_read_counters": [P, P, P],
            "cs_table_device": [P, P],
            "cs_read_coeffs": [P, P],
            "cs_info": [P, P, P, P, P, P],
            "cs_reset": [P, P],
            "cs_merge": [P, P, P],
            "cs_sync": [P, P],
            "cs_set_update_path": [P, i32],
            "mersenne_divmod": [i32, P, u64, P, P, P],
            "mersenne_div": [i32, P, u64, P, P],
            "mersenne_mod": [i32, P, u64, P, P],
            "mersenne_divmod_naive": [i32, P, u64, P, P, P],
            "mersenne_status": [P],
            "mersenne_bucket_map": [i32, i32, P, u64, u64, P, P],
            "mersenne_divmod_wide": [u32, u32, i32, P, u64, P, P, P],
            "cs_batch_create": [P, u32, i32, i32, P, P],
            "cs_batch_update": [P, P],
            "cs_batch_autotune": [P, P, P],
            "cs_batch_get_options": [P, P],
            "cs_batch_classes": [P, P, P, P, P],
            "cs_server_create": [i32, i32, u32, i32, i32, P, P],
            "cs_server_admit": [P, u32, u64, u64, P],
            "cs_server_evict": [P, u32],
            "cs_server_submit_update": [P, u32, P, P, u64, P],
            "cs_server_submit_f2": [P, u32, P],
            "cs_server_wait": [P, u64, P],
            "cs_server_drain": [P],
            "cs_server_read_counters": [P, u32, P],
            "cs_server_get_stats": [P, P],
            "cs_server_replay": [P, P, u32, P, P],
            "cs_status_from_hip_error": [i32],
            "cs_reserve": [P, u64],
            "cs_ceiling_run": [i32, P, u64, u32, P, P],
            "cs_update_noalloc": [P, P, i32, P, i32, u64, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.cs_destroy.argtypes = [P]
        L.cs_destroy.restype = None
        L.cs_batch_destroy.argtypes = [P]
        L.cs_batch_destroy.restype = None
        L.cs_server_destroy.argtypes = [P]
        L.cs_server_destroy.restype = None
        L.cs_last_error.restype = ctypes.c_char_p
        L.cs_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != CS_OK:
        raise MCSError(st, lib().cs_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    """HIP stream handle: None -> torch's current stream on the current device."""
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _key_dtype(t) -> int:
    import torch
    if t.dtype in (torch.int32, torch.uint32):
        return CS_U32
    if t.dtype in (torch.int64, torch.uint64):
        return CS_U64
    raise ValueError(f"unsupported key dtype {t.dtype}")


def _weight_dtype(t) -> int:
    import torch
    if t.dtype == torch.int32:
        return CS_I32
    if t.dtype == torch.int64:
        return CS_I64
    raise ValueError(f"unsupported weight dtype {t.dtype}")


def npoly(mode: int) -> int:
    return 2 if mode == CS_TWO_POLY else 1


class Sketch:
    """Owning handle of a cs_sketch (rows x buckets int64 counters on the current device)."""

    def __init__(self, rows: int, buckets: int, prime: int = CS_P61, seed: int = 0, mode: int = CS_TWO_FOR_ONE,
                 k: int = 4, coeffs: np.ndarray | None = None):
        self._h = ctypes.c_void_p()
        if coeffs is None:
            _check(lib().cs_create_ex(rows, buckets, prime, seed & 0xFFFFFFFFFFFFFFFF, mode, k, ctypes.byref(self._h)))
        else:
            c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint64))
            _check(lib().cs_create_with_coeffs(rows, buckets, prime, mode, k, c.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(self._h)))
        self.rows, self.buckets, self.prime, self.mode, self.k = rows, buckets, prime, mode, k

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self):
        if self._h:
            lib().cs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # Algorithm 2, Process over a batch
    def update(self, keys, weights, stream=None, n: int | None = None):
        n = keys.numel() if n is None else n
        if weights.numel() < n or keys.numel() < n:
            raise ValueError("keys/weights shorter than n")
        _check(lib().cs_update(self._h, _dev_ptr(keys), _key_dtype(keys), _dev_ptr(weights), _weight_dtype(weights),
                               n, _stream(stream)))

    def update_noalloc(self, keys, weights, stream=None, n: int | None = None):
        """cs_update_noalloc: the same update, no allocation (include/mcs_noalloc.h)."""
        n = keys.numel() if n is None else n
        if weights.numel() < n or keys.numel() < n:
            raise ValueError("keys/weights shorter than n")
        _check(lib().cs_update_noalloc(self._h, _dev_ptr(keys), _key_dtype(keys), _dev_ptr(weights),
                                       _weight_dtype(weights), n, _stream(stream)))

    # Algorithm 2, Output + median over rows
    def estimate_f2(self, stream=None) -> tuple[int, np.ndarray]:
        f2 = ctypes.c_int64()
        rows = np.zeros(self.rows, dtype=np.int64)
        _check(lib().cs_estimate_f2(self._h, ctypes.byref(f2), rows.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return int(f2.value), rows

    def estimate_f2_status(self, stream=None) -> tuple[int, int, np.ndarray]:
        """Like estimate_f2 but returns the status instead of raising."""
        f2 = ctypes.c_int64()
        rows = np.zeros(self.rows, dtype=np.int64)
        st = lib().cs_estimate_f2(self._h, ctypes.byref(f2), rows.ctypes.data_as(ctypes.c_void_p), _stream(stream))
        return st, int(f2.value), rows

    def query(self, keys, out, stream=None):
        _check(lib().cs_query(self._h, _dev_ptr(keys), _key_dtype(keys), keys.numel(), _dev_ptr(out), _stream(stream)))

    def counters(self, stream=None) -> np.ndarray:
        out = np.zeros((self.rows, self.buckets), dtype=np.int64)
        _check(lib().cs_read_counters(self._h, out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return out

    def table_ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(lib().cs_table_device(self._h, ctypes.byref(p)))
        return p.value

    def coeffs(self) -> np.ndarray:
        count = self.rows * npoly(self.mode) * self.k
        out = np.zeros(count * (2 if self.prime == CS_P89 else 1), dtype=np.uint64)
        _check(lib().cs_read_coeffs(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(count, 2) if self.prime == CS_P89 else out

    def set_update_path(self, path: int):
        _check(lib().cs_set_update_path(self._h, path))

    def reserve(self, keys: int):
        """Workspace for two-pass rounds of `keys` keys (see cs_reserve)."""
        _check(lib().cs_reserve(self._h, keys))

    def reset(self, stream=None):
        _check(lib().cs_reset(self._h, _stream(stream)))

    def merge(self, other: "Sketch", stream=None):
        _check(lib().cs_merge(self._h, other._h, _stream(stream)))

    def sync(self, stream=None):
        _check(lib().cs_sync(self._h, _stream(stream)))


class _BatchItem(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_void_p), ("keys", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("n", ctypes.c_uint64)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("lds_table_max", ctypes.c_uint32), ("lds_chunk_keys", ctypes.c_uint32),
                ("combine", ctypes.c_int), ("use_graph", ctypes.c_int), ("direct_fraction", ctypes.c_double),
                ("keys_per_thread", ctypes.c_uint32), ("row_resident", ctypes.c_int)]


class Batch:
    """Owning handle of a cs_batch over (sketch, keys, weights) members (include/mcs_batch.h)."""

    def __init__(self, members, options: BatchOptions | None = None):
        if not members:
            raise ValueError("empty batch")
        items = (_BatchItem * len(members))()
        kt = wt = None
        self._keep = []
        for i, (sk, keys, weights) in enumerate(members):
            if keys.numel() != weights.numel():
                raise ValueError("keys and weights differ in length")
            k_dt = _key_dtype(keys) if keys.numel() else (kt if kt is not None else CS_U64)
            w_dt = _weight_dtype(weights) if weights.numel() else (wt if wt is not None else CS_I64)
            if kt is None:
                kt, wt = k_dt, w_dt
            elif keys.numel() and (k_dt != kt or w_dt != wt):
                raise ValueError("all members must share key and weight dtypes")
            items[i].sketch = sk.handle.value
            items[i].keys = keys.data_ptr() if keys.numel() else None
            items[i].weights = weights.data_ptr() if weights.numel() else None
            items[i].n = keys.numel()
            self._keep.append((sk, keys, weights))
        self._h = ctypes.c_void_p()
        _check(lib().cs_batch_create(items, len(members), kt, wt,
                                     ctypes.byref(options) if options is not None else None, ctypes.byref(self._h)))

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def update(self, stream=None):
        _check(lib().cs_batch_update(self._h, _stream(stream)))

    def autotune(self, stream=None) -> BatchOptions:
        out = BatchOptions()
        _check(lib().cs_batch_autotune(self._h, _stream(stream), ctypes.byref(out)))
        return out

    def options(self) -> BatchOptions:
        out = BatchOptions()
        _check(lib().cs_batch_get_options(self._h, ctypes.byref(out)))
        return out

    def classes(self) -> tuple[int, int, int, int]:
        """Members per class: (direct atomics, LDS, row-resident, two-pass)."""
        a, b, c, d = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().cs_batch_classes(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def close(self):
        if self._h:
            lib().cs_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CS_REQ_UPDATE, CS_REQ_F2 = 0, 1


class PreparedRequests:
    """Requests marshalled once for Server.replay (see Server.prepare)."""

    def __init__(self, array, n, keep):
        self.array, self.n, self._keep = array, n, keep

    def __len__(self):
        return self.n


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("step_keys", ctypes.c_uint64), ("work_bytes", ctypes.c_uint64),
                ("direct_fraction", ctypes.c_double)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("f2", ctypes.c_int64), ("arrival_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("step", ctypes.c_uint64)]


class ServerRequest(ctypes.Structure):
    _fields_ = [("tenant", ctypes.c_uint32), ("kind", ctypes.c_uint32), ("keys", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("requests", ctypes.c_uint64), ("keys", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64), ("tenants", ctypes.c_uint32)]


class Server:
    """Owning handle of a cs_server (include/mcs_serve.h): tenants, queued update/F2
    requests and continuous batching on a worker thread of the library."""

    def __init__(self, prime: int = CS_P61, mode: int = CS_TWO_FOR_ONE, k: int = 4, key_type: int = CS_U64,
                 weight_type: int = CS_I32, hbm_budget: int = 0, step_keys: int = 0, work_bytes: int = 0,
                 direct_fraction: float = 0.0):
        opts = ServerOptions(hbm_budget, step_keys, work_bytes, direct_fraction)
        self._h = ctypes.c_void_p()
        self._kt, self._wt = key_type, weight_type
        self._keep = {}  # ticket -> tensors that must stay alive until the update completes
        self._untracked = []  # tensors of updates without a ticket, released by drain()
        _check(lib().cs_server_create(prime, mode, k, key_type, weight_type, ctypes.byref(opts),
                                      ctypes.byref(self._h)))

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def admit(self, rows: int, buckets: int, seed: int) -> int:
        t = ctypes.c_uint32()
        _check(lib().cs_server_admit(self._h, rows, buckets, seed, ctypes.byref(t)))
        return t.value

    def evict(self, tenant: int):
        _check(lib().cs_server_evict(self._h, tenant))

    def submit_update(self, tenant: int, keys, weights, ticket: bool = False):
        """Queue an update; keys/weights stay referenced until wait(ticket) (ticket=True)
        or drain().  Returns the ticket, or None."""
        if keys.numel() != weights.numel():
            raise ValueError("keys and weights differ in length")
        if keys.numel() and (_key_dtype(keys) != self._kt or _weight_dtype(weights) != self._wt):
            raise ValueError("key or weight dtype differs from the server's")
        t = ctypes.c_uint64()
        _check(lib().cs_server_submit_update(self._h, tenant, _dev_ptr(keys) if keys.numel() else None,
                                             _dev_ptr(weights) if weights.numel() else None, keys.numel(),
                                             ctypes.byref(t) if ticket else None))
        if ticket:
            self._keep[t.value] = (keys, weights)
            return t.value
        self._untracked.append((keys, weights))
        return None

    def submit_f2(self, tenant: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().cs_server_submit_f2(self._h, tenant, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int) -> ServerResult:
        out = ServerResult()
        _check(lib().cs_server_wait(self._h, ticket, ctypes.byref(out)))
        self._keep.pop(ticket, None)
        return out

    def drain(self):
        _check(lib().cs_server_drain(self._h))
        self._untracked.clear()

    def counters(self, tenant: int, rows: int, buckets: int) -> np.ndarray:
        out = np.empty((rows, buckets), dtype=np.int64)
        _check(lib().cs_server_read_counters(self._h, tenant, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def stats(self) -> ServerStats:
        out = ServerStats()
        _check(lib().cs_server_get_stats(self._h, ctypes.byref(out)))
        return out

    def prepare(self, requests) -> "PreparedRequests":
        """Marshals requests, a list of (tenant, kind, keys, weights) with device tensors
        (None for F2), into the C array cs_server_replay takes; replay() then skips this
        work.  The tensors are referenced until the returned object is dropped."""
        n = len(requests)
        reqs = (ServerRequest * n)()
        keep = []
        for i, (tenant, kind, keys, weights) in enumerate(requests):
            reqs[i].tenant, reqs[i].kind = tenant, kind
            if kind == CS_REQ_UPDATE and keys is not None and keys.numel():
                if _key_dtype(keys) != self._kt or _weight_dtype(weights) != self._wt:
                    raise ValueError("key or weight dtype differs from the server's")
                reqs[i].keys, reqs[i].weights, reqs[i].n = keys.data_ptr(), weights.data_ptr(), keys.numel()
                keep.append((keys, weights))
        return PreparedRequests(reqs, n, keep)

    def replay(self, requests, arrival_s):
        """requests: a list as for prepare(), or its result; arrival_s: non-decreasing seconds
        after the call starts (a sequence or a float64 array).  Returns one ServerResult per
        request (a ctypes array)."""
        if not isinstance(requests, PreparedRequests):
            requests = self.prepare(requests)
        n = requests.n
        arr = np.ascontiguousarray(np.asarray(arrival_s, dtype=np.float64))
        if arr.shape != (n,):
            raise ValueError("one arrival time per request")
        res = (ServerResult * n)()
        _check(lib().cs_server_replay(self._h, requests.array, n,
                                      arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), res))
        return res

    def close(self):
        if self._h:
            lib().cs_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()
            self._untracked.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mersenne_divmod(prime: int, x, quot=None, rem=None, stream=None, naive: bool = False):
    """Quotient/remainder of x (uint64 limbs as int64 tensor, shape (n, 2) or (n, 3)) by the prime."""
    n = x.shape[0]
    fn = lib().mersenne_divmod_naive if naive else lib().mersenne_divmod
    _check(fn(prime, _dev_ptr(x), n, _dev_ptr(quot) if quot is not None else None,
              _dev_ptr(rem) if rem is not None else None, _stream(stream)))


def mersenne_div(prime: int, x, quot, stream=None):
    _check(lib().mersenne_div(prime, _dev_ptr(x), x.shape[0], _dev_ptr(quot), _stream(stream)))


def mersenne_mod(prime: int, x, rem, stream=None):
    _check(lib().mersenne_mod(prime, _dev_ptr(x), x.shape[0], _dev_ptr(rem), _stream(stream)))


def mersenne_bucket_map(prime: int, v, r: int, out, method: int = CS_MAP_EXACT, stream=None):
    """Buckets in [r] of hash values v < p (uint64 tensor of shape (n,), or (n, 2) limbs for
    2^89 - 1) into out (int32 tensor of n uint32 bit patterns)."""
    _check(lib().mersenne_bucket_map(prime, method, _dev_ptr(v), v.shape[0], r, _dev_ptr(out), _stream(stream)))


def mersenne_divmod_wide(b: int, c: int, x, quot=None, rem=None, method: int = CS_WIDE_ALG5, stream=None):
    """Quotient and remainder of 2b-bit values by 2^b - c.  x: int32 tensor of limb planes,
    shape (2b/32, n); quot: (b/32 + 1, n); rem: (b/32, n) (uint32 bit patterns)."""
    w = b // 32
    if x.shape[0] != 2 * w or (quot is not None and quot.shape[0] != w + 1) or (rem is not None and rem.shape[0] != w):
        raise ValueError("limb-plane shapes do not match b")
    _check(lib().mersenne_divmod_wide(b, c, method, _dev_ptr(x), x.shape[1], _dev_ptr(quot) if quot is not None else None,
                                      _dev_ptr(rem) if rem is not None else None, _stream(stream)))


def mersenne_status(stream=None):
    _check(lib().mersenne_status(_stream(stream)))


def version() -> str:
    return lib().cs_version().decode()
