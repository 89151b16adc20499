"""GPU parity for the wide quotient and remainder (the b-sweep of the paper's division
experiment): Algorithm 5 + 6 and the Crandall-Chung-Hasan comparator against the oracle's
plain integer division, for b = 32 .. 1024 and several c, bit-exact."""
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


def _inputs(b, c, n, seed):
    limbs = 2 * b // 32
    x = W.uniform_u32(seed, limbs * n).reshape(limbs, n).numpy().astype(np.uint32)
    p = (1 << b) - c
    edges = [0, 1, p - 1, p, p + 1, 2 * p - 1, 2 * p, p * p - 1, p * p, (1 << (2 * b)) - 1, (1 << b) - 1,
             1 << b, (1 << b) + 1, 12345 * p + 6789, (p - 1) * p + (p - 1)]
    edges = [e for e in edges if 0 <= e < 1 << (2 * b)]
    return np.concatenate([x, O.ints_to_planes(edges, limbs)], axis=1)


def _run(b, c, xh, method):
    w = b // 32
    n = xh.shape[1]
    x = torch.from_numpy(xh.view(np.int32)).to(DEV)
    q = torch.empty((w + 1, n), dtype=torch.int32, device=DEV)
    r = torch.empty((w, n), dtype=torch.int32, device=DEV)
    M.mersenne_divmod_wide(b, c, x, q, r, method=method)
    torch.cuda.synchronize()
    return q.cpu().numpy().view(np.uint32), r.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("b", [32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("c", [1, 3, 59, 65521])
@pytest.mark.parametrize("method", [0, 1])
def test_wide_divmod_matches_oracle(b, c, method):
    if 2 * (c - 1).bit_length() >= b:
        pytest.skip("the library takes c with 2 ceil(log2 c) < b")
    n = 3000 if b >= 512 else 9000
    xh = _inputs(b, c, n, seed=b * 7 + c + method)
    q, r = _run(b, c, xh, method)
    wq, wr = O.divmod_wide(b, c, xh)
    assert np.array_equal(r, wr), "remainders differ"
    assert np.array_equal(q, wq), "quotients differ"


def test_wide_divmod_one_output_and_arguments():
    b, c = 128, 1
    xh = _inputs(b, c, 1000, seed=5)
    x = torch.from_numpy(xh.view(np.int32)).to(DEV)
    wq, wr = O.divmod_wide(b, c, xh)
    q = torch.empty((5, xh.shape[1]), dtype=torch.int32, device=DEV)
    r = torch.empty((4, xh.shape[1]), dtype=torch.int32, device=DEV)
    M.mersenne_divmod_wide(b, c, x, quot=q)
    M.mersenne_divmod_wide(b, c, x, rem=r, method=M.CS_WIDE_CCH)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy().view(np.uint32), wq)
    assert np.array_equal(r.cpu().numpy().view(np.uint32), wr)
    for bb, cc, meth in ((48, 1, 0), (64, 0, 0), (64, 1 << 31, 0), (32, 1 << 16, 0), (64, 1, 2)):
        xx = torch.zeros((2 * max(bb, 32) // 32, 4), dtype=torch.int32, device=DEV)
        qq = torch.zeros((max(bb, 32) // 32 + 1, 4), dtype=torch.int32, device=DEV)
        with pytest.raises((M.MCSError, ValueError)):
            M.mersenne_divmod_wide(bb, cc, xx, quot=qq, method=meth)
