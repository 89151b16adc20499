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


@pytest.mark.parametrize("row_resident,lds_table_max,classes", [
    (0, 0, (3, 0, 7, 1)),        # default: one persistent launch for every table of up to 2^16 buckets
    (1, 65536, (3, 2, 5, 1)),    # small tables in the LDS class beside it
    (-1, 0, (3, 2, 0, 6)),       # no row-resident class: LDS and two-pass classes
])
def test_batch_all_classes_and_graph_replays(row_resident, lds_table_max, classes):
    members, specs = _members()
    opts = M.BatchOptions()
    opts.row_resident = row_resident
    opts.lds_table_max = lds_table_max
    b = M.Batch([(sk, k, w) for sk, k, w in members], opts)
    assert b.classes() == classes
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


def test_batch_autotune_keeps_counters_then_exact():
    """Autotuning runs its trials on the members' own tables and puts back what they
    held: counters from an earlier update survive it unchanged, and the next update
    adds exactly one more stream's worth."""
    members, specs = _members(seed0=500)
    b = M.Batch([(sk, k, w) for sk, k, w in members])
    b.update()
    torch.cuda.synchronize()
    want = [_oracle(sp, k, w) for sp, (sk, k, w) in zip(specs, members)]
    for (sk, k, w), t in zip(members, want):
        assert np.array_equal(sk.counters(), t)
    chosen = b.autotune()
    assert chosen.lds_table_max in (8, 20480, 40960, 65536, 163840)
    assert chosen.direct_fraction in (1.0 / 128, 0.125, 1.0)
    assert chosen.keys_per_thread in (0, 2, 4, 8) and chosen.row_resident in (1, -1)
    assert b.options().lds_table_max == chosen.lds_table_max
    for (sk, k, w), t in zip(members, want):
        assert np.array_equal(sk.counters(), t), (sk.rows, sk.buckets, k.numel())
        assert sk.estimate_f2_status()[0] == M.CS_OK
    b.update()
    torch.cuda.synchronize()
    for (sk, k, w), t in zip(members, want):
        assert np.array_equal(sk.counters(), 2 * t)


# (rows, buckets, keys) of a row-resident batch: one row group per block (2^16, 2^15
# buckets), whole sketches per block, ragged tails, a stream shorter than one wave tile,
# direct members, a member with no keys
ROW_SHAPES = [(5, 1 << 16, 70001), (5, 1 << 15, 40000), (5, 1 << 12, 33333), (7, 1 << 13, 9000),
              (3, 1 << 14, 300), (5, 1 << 16, 2000), (4, 1 << 10, 100000), (5, 1 << 8, 7), (2, 1 << 11, 0)]


def _row_batch_members(prime, mode, kt, wt, seed0, arb=False):
    members, specs, off = [], [], 0
    total = sum(n for _, _, n in ROW_SHAPES)
    keys = W.zipf(seed0, total, 1.1, 1 << 32)
    keys[::5] |= W.uniform_u64(seed0, keys[::5].numel()) & (((1 << 60) - 1) ^ 0xFFFFFFFF)
    w = W.bounded_int(seed0, total, -100, 100)
    w[1::61] = (1 << 15) - 1
    w[2::61] = -(1 << 15) + 1
    w[3::61] = 1 << 15
    w[4::61] = -(1 << 15)
    w[5::61] = (1 << 31) - 1 if wt == "i32" else (1 << 62) + 3
    w[6::61] = -(1 << 31) if wt == "i32" else -(1 << 62) - 5
    keys = keys.to(torch.int32) if kt == "u32" else keys
    w = w.to(torch.int32) if wt == "i32" else w
    for i, (rows, m, n) in enumerate(ROW_SHAPES):
        buckets = m - 3 * i - 1 if arb else m
        seed = seed0 + i
        sk = M.Sketch(rows, buckets, prime=prime, seed=seed, mode=mode)
        members.append((sk, keys[off: off + n].contiguous().to(DEV), w[off: off + n].contiguous().to(DEV)))
        specs.append((rows, buckets, seed))
        off += n
    return members, specs


def _row_oracle(prime, mode, spec, k, w):
    rows, buckets, seed = spec
    p = O.PRIME_P61 if prime == M.CS_P61 else O.PRIME_P89
    a = k.cpu().numpy()
    a = a.view(np.uint32).astype(np.uint64) if a.dtype == np.int32 else a.view(np.uint64)
    return O.cs_update(p, mode, rows, buckets, O.coeffs_from_seed(p, rows, mode, seed=seed), a,
                       w.cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("prime,mode,kt,wt,kpt", [
    (1, 0, "u64", "i32", 8),   # the batched workload's types
    (1, 0, "u64", "i32", 4),
    (1, 2, "u32", "i64", 8),   # two polynomials
    (2, 1, "u64", "i64", 4),   # 2^89 - 1, Algorithm 3's bit layout
    (1, 3, "u64", "i32", 8),   # any bucket count
    (1, 0, "u32", "i32", 2),   # two keys per lane
])
def test_batch_row_resident_matches_oracle(prime, mode, kt, wt, kpt):
    """Every member in the one persistent row-resident launch (no LDS class: table limit
    8 bytes): each sketch ends with the oracle's counters, with weights at and beyond
    the 16-bit fields' edge, keys past 2^32 and ragged tails, on two updates."""
    members, specs = _row_batch_members(prime, mode, kt, wt, 900 + 10 * mode + prime, arb=(mode == 3))
    opts = M.BatchOptions()
    opts.lds_table_max = 8
    opts.keys_per_thread = kpt
    b = M.Batch(members, opts)
    ng, nl, nr, nt = b.classes()
    assert (ng, nl, nr, nt) == (3, 0, 5, 0), (ng, nl, nr, nt)
    b.update()
    b.update()
    torch.cuda.synchronize()
    for (sk, k, w), sp in zip(members, specs):
        want = 2 * _row_oracle(prime, mode, sp, k, w)
        got = sk.counters()
        assert np.array_equal(got, want), (sp, int((got != want).sum()))


def test_batch_rejects_bad_keys_per_thread():
    sk = M.Sketch(3, 1 << 12, prime=M.CS_P61, seed=1)
    k = torch.ones(4096, dtype=torch.int64, device=DEV)
    opts = M.BatchOptions()
    opts.keys_per_thread = 6
    with pytest.raises(M.MCSError):
        M.Batch([(sk, k, k)], opts)


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
    opts = M.BatchOptions(16384, 0, 0, 0)
    opts.row_resident = -1
    b = M.Batch(members, opts)
    assert b.classes()[3] >= 4
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
