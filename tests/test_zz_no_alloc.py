"""cs_update_noalloc (include/mcs_noalloc.h) against cs_update, through the C ABI.

The entry point is for callers that cannot allocate: its two-pass workspace is the
library's fixed scratch array.  Two calls in a row, the second with fewer keys, must
leave the same counters as cs_update on a sketch with the same coefficients, counter
by counter; both results are also checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

try:
    import paper_2008_08654_amd as M
except Exception:  # pragma: no cover
    M = None

DEV = "cuda:0"


def _oracle(prime, mode, rows, m, seed, keys, w, table=None):
    p = O.PRIME_P61 if prime == M.CS_P61 else O.PRIME_P89
    c = O.coeffs_from_seed(p, rows, mode, seed=seed)
    k = keys.cpu().numpy().view(np.uint64)
    return O.cs_update(p, mode, rows, m, c, k, w.cpu().numpy().astype(np.int64), table=table)


@pytest.mark.parametrize("rows,log2m,prime,mode,path,n1,n2", [
    # forced two-pass path on the headline shape: 3M keys take two scratch rounds
    (9, 16, 1, 0, 3, 3_000_000 + 77, 200_003),
    # automatic two-pass path with block tiles and the combining probe (2^20 buckets)
    (5, 20, 2, 0, 0, 2_500_000 + 11, 70_001),
    # a path without scratch (LDS table)
    (5, 10, 1, 2, 0, 100_000, 9_999),
])
def test_noalloc_matches_cs_update(rows, log2m, prime, mode, path, n1, n2):
    print(f"noalloc parity: rows {rows}, m 2^{log2m}, prime {prime}, mode {mode}, path {path}, n {n1} then {n2}",
          flush=True)
    keys = W.zipf(7000 + log2m, n1, 1.1, 1 << 32).to(DEV)
    w = W.bounded_int(7000 + log2m, n1, -100, 100).to(torch.int32).to(DEV)
    seed = 900 + log2m
    a = M.Sketch(rows, 1 << log2m, prime=prime, seed=seed, mode=mode)
    b = M.Sketch(rows, 1 << log2m, prime=prime, seed=seed, mode=mode)
    if path:
        a.set_update_path(path)
        b.set_update_path(path)
    a.update(keys, w)
    b.update_noalloc(keys, w)
    torch.cuda.synchronize()
    want = _oracle(prime, mode, rows, 1 << log2m, seed, keys, w)
    got_a, got_b = a.counters(), b.counters()
    assert np.array_equal(got_a, want)
    assert np.array_equal(got_b, got_a), f"{int((got_b != got_a).sum())} counters differ after the first call"
    # second call, fewer keys: the scratch array still holds the first call's records
    k2, w2 = keys[:n2].contiguous(), w[:n2].contiguous()
    a.update(k2, w2)
    b.update_noalloc(k2, w2)
    torch.cuda.synchronize()
    _oracle(prime, mode, rows, 1 << log2m, seed, k2, w2, table=want)
    got_a, got_b = a.counters(), b.counters()
    assert np.array_equal(got_a, want)
    assert np.array_equal(got_b, got_a), f"{int((got_b != got_a).sum())} counters differ after the second call"
    fa, _ = a.estimate_f2()
    fb, _ = b.estimate_f2()
    assert fa == fb
    a.close()
    b.close()


def test_noalloc_rejects_bad_arguments():
    sk = M.Sketch(3, 1 << 12, prime=M.CS_P61, seed=1)
    L = M.lib()
    assert L.cs_update_noalloc(sk.handle, None, M.CS_U64, None, M.CS_I32, 10, None) == M.CS_EINVAL
    assert L.cs_update_noalloc(None, None, M.CS_U64, None, M.CS_I32, 10, None) == M.CS_EINVAL
    keys = torch.zeros(4, dtype=torch.int64, device=DEV)
    w = torch.zeros(4, dtype=torch.int32, device=DEV)
    assert L.cs_update_noalloc(sk.handle, M._dev_ptr(keys), 7, M._dev_ptr(w), M.CS_I32, 4, None) == M.CS_EINVAL
    assert L.cs_update_noalloc(sk.handle, M._dev_ptr(keys), M.CS_U64, M._dev_ptr(w), M.CS_I32, 0, None) == M.CS_OK
    sk.close()
