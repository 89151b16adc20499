"""Batched update (include/mcs_batch.h): every member sketch ends with exactly the
oracle's table for its own stream, whatever update class it falls in, across HIP
graph replays, with the graph off, and after autotuning."""
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

# (rows, log2 buckets, keys): direct-atomic members (n < m/8), LDS members, two-pass members,
# an empty stream, ragged tails
SHAPES = [(5, 8, 300), (5, 10, 5000), (3, 12, 70000), (5, 13, 12345), (5, 16, 4000), (5, 16, 150000),
          (4, 14, 2049), (5, 11, 0), (5, 9, 1), (2, 17, 40000), (5, 15, 99999), (1, 18, 3 * 512 + 7)]


def _members(seed0=100):
    members, specs = [], []
    stream_keys = W.zipf(W.DATA_SEED + 3, 400000, 1.1, 1 << 32)
    stream_w = W.bounded_int(W.DATA_SEED + 3, 400000, -100, 100).to(torch.int32)
    off = 0
    for i, (rows, lm, n) in enumerate(SHAPES):
        k = stream_keys[off: off + n].contiguous().to(DEV)
        w = stream_w[off: off + n].contiguous().to(DEV)
        off += n
        sk = M.Sketch(rows, 1 << lm, prime=M.CS_P61, seed=seed0 + i)
        members.append((sk, k, w))
        specs.append((rows, lm, seed0 + i))
    return members, specs


def _oracle(spec, k, w, times=1):
    rows, lm, seed = spec
    coeffs = O.coeffs_from_seed(O.PRIME_P61, rows, O.TWO_FOR_ONE, seed)
    t = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, rows, 1 << lm, coeffs, k.cpu().numpy().view(np.uint64),
                    w.cpu().numpy().astype(np.int64))
    return t * times


def test_batch_all_classes_and_graph_replays():
    members, specs = _members()
    b = M.Batch([(sk, k, w) for sk, k, w in members])
    ng, nl, nt = b.classes()
    assert ng >= 2 and nl >= 2 and nt >= 3, (ng, nl, nt)
    want = [_oracle(sp, k, w) for sp, (sk, k, w) in zip(specs, members)]
    for replay in range(1, 4):
        b.update()
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.arange(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        for (sk, k, w), t in zip(members, want):
            got = sk.counters()
            assert np.array_equal(got, t * replay), (replay, sk.rows, sk.buckets, k.numel())
    assert int(junk) > 0


def test_batch_without_graph_and_vs_plain_updates():
    members, specs = _members(seed0=300)
    opts = M.BatchOptions(0, 0, -1, -1)  # no combining, no graph
    b = M.Batch([(sk, k, w) for sk, k, w in members], opts)
    b.update()
    plain = [M.Sketch(sp[0], 1 << sp[1], prime=M.CS_P61, seed=sp[2]) for sp in specs]
    for p, (sk, k, w) in zip(plain, members):
        p.update(k, w)
    torch.cuda.synchronize()
    for p, (sk, k, w), sp in zip(plain, members, specs):
        assert np.array_equal(sk.counters(), p.counters())
        assert np.array_equal(sk.counters(), _oracle(sp, k, w))


def test_batch_autotune_zeroes_then_exact():
    members, specs = _members(seed0=500)
    b = M.Batch([(sk, k, w) for sk, k, w in members])
    chosen = b.autotune()
    assert chosen.lds_table_max in (8, 20480, 40960, 65536, 163840)
    assert chosen.direct_fraction in (1.0 / 128, 0.125, 1.0)
    for sk, k, w in members:
        assert not sk.counters().any()
    b.update()
    torch.cuda.synchronize()
    for (sk, k, w), sp in zip(members, specs):
        assert np.array_equal(sk.counters(), _oracle(sp, k, w))


def test_batch_two_pass_members_with_narrow_counter_blocks():
    """Two-pass members whose per-wave counter block (rows * ranges * 4 bytes) is
    not a multiple of 16: the per-wave LDS regions stay aligned; plain updates of
    the same members agree."""
    stream_keys = W.zipf(W.DATA_SEED + 5, 200000, 1.1, 1 << 32)
    stream_w = W.bounded_int(W.DATA_SEED + 5, 200000, -100, 100).to(torch.int32)
    shapes = [(5, 11, 70001), (5, 12, 30000), (7, 11, 5000), (3, 12, 9000), (1, 11, 2048 * 5)]
    members, specs, off = [], [], 0
    for i, (rows, lm, n) in enumerate(shapes):
        k = stream_keys[off: off + n].contiguous().to(DEV)
        w = stream_w[off: off + n].contiguous().to(DEV)
        off += n
        members.append((M.Sketch(rows, 1 << lm, prime=M.CS_P61, seed=700 + i), k, w))
        specs.append((rows, lm, 700 + i))
    b = M.Batch(members, M.BatchOptions(16384, 0, 0, 0))
    assert b.classes()[2] >= 4
    b.update()
    plain = [M.Sketch(sp[0], 1 << sp[1], prime=M.CS_P61, seed=sp[2]) for sp in specs]
    for p, (sk, k, w) in zip(plain, members):
        p.update(k, w)
    torch.cuda.synchronize()
    for p, (sk, k, w), sp in zip(plain, members, specs):
        want = _oracle(sp, k, w)
        assert np.array_equal(sk.counters(), want), sp
        assert np.array_equal(p.counters(), want), sp


def test_batch_rejects_mixed_members():
    a = M.Sketch(3, 64, prime=M.CS_P61, seed=1)
    c = M.Sketch(3, 64, prime=M.CS_P89, seed=1)
    k = torch.ones(4, dtype=torch.int64, device=DEV)
    with pytest.raises(M.MCSError):
        M.Batch([(a, k, k), (c, k, k)])
