"""GPU parity: the HIP path through the C ABI against the oracle, bit-exact.

Inputs come from ``workloads`` (seeded, synthetic); expected values from
``oracle`` only.  Sizes span several 1024-key tiles plus a ragged tail.
"""
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

PRIMES = {M.CS_P61 if M else 1: O.PRIME_P61, M.CS_P89 if M else 2: O.PRIME_P89}


def _u64(t: torch.Tensor) -> np.ndarray:
    """Host uint64 values of a key tensor (int32 tensors hold uint32 bit patterns)."""
    a = t.detach().cpu().numpy()
    if a.dtype == np.int32:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64)


def _oracle_table(sk, keys, weights):
    coeffs = O.coeffs_from_seed(PRIMES[sk.prime], sk.rows, sk.mode, seed=sk._seed, k=sk.k) \
        if getattr(sk, "_seed", None) is not None else sk._coeffs
    return O.cs_update(PRIMES[sk.prime], sk.mode, sk.rows, sk.buckets, coeffs, _u64(keys),
                       weights.detach().cpu().numpy().astype(np.int64), k=sk.k)


def _make(rows, m, prime, seed, mode=0, k=4):
    sk = M.Sketch(rows, m, prime=prime, seed=seed, mode=mode, k=k)
    sk._seed = seed
    return sk


def _check_sketch(sk, keys, weights, table=None):
    torch.cuda.synchronize()
    got = sk.counters()
    want = _oracle_table(sk, keys, weights) if table is None else table
    assert np.array_equal(got, want), f"{int((got != want).sum())} counters differ"
    st, f2, rows = sk.estimate_f2_status()
    wst, wmed, wrows = O.cs_estimate_status(want)
    assert st == {O.OK: M.CS_OK, O.EOVERFLOW: M.CS_EOVERFLOW}[wst]
    assert list(rows) == list(wrows) and f2 == wmed
    return want


def test_coefficients_match_oracle():
    for prime in (M.CS_P61, M.CS_P89):
        for mode in (0, 1, 2):
            sk = M.Sketch(7, 64, prime=prime, seed=123456789, mode=mode, k=4)
            want = O.coeffs_from_seed(PRIMES[prime], 7, mode, seed=123456789)
            assert np.array_equal(sk.coeffs(), want)


def test_single_stream_u32_workload_bit_exact():
    """n = 2^16 uint32 keys uniform, weights int64 = 1, p = 2^61-1, t = 5, m = 2^10."""
    keys, w = W.stream_small_u32(1 << 16)
    keys = keys.to(torch.int32).to(DEV)  # uint32 bit patterns
    w = w.to(DEV)
    sk = _make(5, 1 << 10, M.CS_P61, seed=1001)
    sk.update(keys, w)
    table = _check_sketch(sk, keys, w)
    exact = O.exact_f2(_u64(keys), w.cpu().numpy())
    f2, _ = sk.estimate_f2()
    assert abs(f2 - exact) / exact < 0.25
    assert int(np.abs(table).sum()) > 0


@pytest.mark.parametrize("prime", [1, 2])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("kt,wt", [("u32", "i32"), ("u32", "i64"), ("u64", "i32"), ("u64", "i64")])
def test_modes_primes_dtypes(prime, mode, kt, wt):
    n = 5 * 1024 + 77
    g = torch.Generator().manual_seed(prime * 100 + mode * 10 + len(kt + wt))
    if kt == "u32":
        keys = W.uniform_u32(7 + mode, n).to(torch.int32)
    else:
        keys = W.uniform_u64(7 + mode, n)
        if prime == M.CS_P61:
            keys = keys & ((1 << 60) - 1)
            keys[: 3 * 1024] &= 0xFFFFFFFF  # first waves take the one-limb path
    if wt == "i32":
        w = torch.randint(-(1 << 31), (1 << 31) - 1, (n,), generator=g, dtype=torch.int64).to(torch.int32)
    else:
        w = torch.randint(-(1 << 62), 1 << 62, (n,), generator=g, dtype=torch.int64)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(3, 256, prime, seed=40 + prime, mode=mode)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


def test_large_table_zipf_two_for_one_and_two_poly():
    """t = 9, m = 2^16 (4.5 MiB table) on 2^17 Zipf(1.1) keys with int32 weights in [-100, 100]."""
    keys, w = W.stream_zipf_u64(1 << 17)
    keys, w = keys.to(DEV), w.to(DEV)
    for mode in (M.CS_TWO_FOR_ONE, M.CS_TWO_POLY):
        sk = _make(9, 1 << 16, M.CS_P61, seed=1002, mode=mode)
        sk.update(keys, w)
        _check_sketch(sk, keys, w)


@pytest.mark.parametrize("mode", [0, 2])
def test_full_size_zipf_beyond_one_round(mode):
    """t = 9, m = 2^16 on 2^27 + 4099 Zipf(1.1) keys with int32 weights in [-100, 100]:
    the workload's shape at half its key count, past the 2^27 keys of one two-pass round,
    so the round loop and its ragged last round meet the oracle (the sketch is linear,
    Section 1.3.1, so rounds add up to the same table).  The automatic path and the
    forced two-pass path are both compared, counter by counter."""
    n = (1 << 27) + 4099
    keys, w = W.stream_zipf_u64(n, device=DEV)
    torch.cuda.synchronize()
    print(f"full-size parity: mode {mode}, n = {n}", flush=True)
    auto = _make(9, 1 << 16, M.CS_P61, seed=1002, mode=mode)
    auto.update(keys, w)
    binned = _make(9, 1 << 16, M.CS_P61, seed=1002, mode=mode)
    binned.set_update_path(M.CS_PATH_BINNED)
    binned.update(keys, w)
    want = _oracle_table(auto, keys, w)
    _check_sketch(auto, keys, w, table=want)
    _check_sketch(binned, keys, w, table=want)
    auto.close()
    binned.close()


@pytest.mark.parametrize("path", [2, 3, 4, 5])
@pytest.mark.parametrize("rows,log2m,prime,mode", [
    (9, 16, 1, 0), (9, 16, 1, 2), (5, 20, 2, 0), (64, 10, 1, 1), (3, 15, 2, 2), (2, 22, 1, 0),
    # one or two bucket ranges per row, where rows * ranges * 4 bytes of
    # per-wave counters is not a multiple of 16 (per-wave LDS regions must stay aligned)
    (5, 11, 1, 0), (5, 12, 1, 0), (7, 11, 2, 1), (3, 12, 1, 2), (1, 11, 1, 0)])
def test_forced_paths_match_oracle(path, rows, log2m, prime, mode):
    """The global-atomic and the two-pass (binned) update give the oracle's counters,
    including ragged tiles, bucket ranges smaller than one partition, and weights too
    large for a record (they take the direct atomic)."""
    n = 3 * 2048 + 555
    keys = W.zipf(31 + log2m, n, 1.1, 1 << 32)
    w = W.bounded_int(31 + log2m, n, -100, 100)
    w[::97] = torch.randint(-(1 << 62), 1 << 62, w[::97].shape, generator=torch.Generator().manual_seed(1))
    w[1::89] = 1 << 17
    w[2::89] = -(1 << 17)
    w[3::89] = (1 << 17) - 1
    w[4::89] = -(1 << 17) + 1
    w[5::89] = 1 << 20
    w[6::89] = -(1 << 20)
    w[7::89] = (1 << 20) - 1
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(rows, 1 << log2m, prime, seed=500 + log2m, mode=mode)
    sk.set_update_path(path)
    sk.update(keys, w)
    sk.update(keys[: n // 3].contiguous(), w[: n // 3].contiguous())
    want = _oracle_table(sk, keys, w)
    _oracle_add = O.cs_update(PRIMES[prime], mode, rows, 1 << log2m,
                              O.coeffs_from_seed(PRIMES[prime], rows, mode, seed=500 + log2m),
                              _u64(keys[: n // 3]), w[: n // 3].cpu().numpy(), table=want)
    _check_sketch(sk, keys, w, table=want)


@pytest.mark.parametrize("rows,buckets,prime,mode,k,kt,wt", [
    (9, 1 << 16, 1, 0, 4, "u64", "i32"),    # the workload's shape: one row per block
    (9, 1 << 16, 1, 2, 4, "u64", "i32"),    # two polynomials
    (9, 1 << 12, 1, 0, 4, "u32", "i64"),    # all nine rows in one block
    (6, 1 << 15, 2, 1, 4, "u64", "i64"),    # two rows per block, 2^89 - 1, Algorithm 3's bit layout
    (8, 1 << 14, 1, 0, 8, "u64", "i32"),    # four rows per block, k = 8
    (7, 12345, 1, 3, 2, "u64", "i32"),      # any bucket count, odd r (the padding bucket shares r - 1's word)
    (3, 65535, 2, 3, 4, "u32", "i32"),      # any bucket count, 2^16 - 1 buckets
    (1, 1 << 16, 1, 0, 4, "u64", "i64"),    # one row
    (5, 2, 1, 0, 4, "u64", "i32"),          # two buckets: one word per row
])
def test_rows_path_matches_oracle(rows, buckets, prime, mode, k, kt, wt):
    """The row-resident update (16-bit fields in LDS, wraps carried into the int64
    counters) gives the oracle's counters: ragged tiles, keys past 2^32 (the two-limb
    hash), and weights at the edge of the fields (+-(2^15 - 1) stay in LDS, +-2^15 and
    beyond go to the counters directly)."""
    n = 3 * 8192 + 1234
    seed = 800 + rows + (buckets & 0xFFFF)
    keys = W.zipf(seed, n, 1.1, 1 << 32)
    if kt == "u64":
        keys[::5] |= W.uniform_u64(seed, keys[::5].numel()) & (((1 << 60) - 1) ^ 0xFFFFFFFF)
    w = W.bounded_int(seed, n, -100, 100)
    w[1::61] = (1 << 15) - 1
    w[2::61] = -(1 << 15) + 1
    w[3::61] = 1 << 15
    w[4::61] = -(1 << 15)
    w[5::61] = (1 << 31) - 1 if wt == "i32" else (1 << 62) + 3
    w[6::61] = -(1 << 31) if wt == "i32" else -(1 << 62) - 5
    keys = keys.to(torch.int32) if kt == "u32" else keys
    w = w.to(torch.int32) if wt == "i32" else w
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(rows, buckets, prime, seed=seed, mode=mode, k=k)
    sk.set_update_path(M.CS_PATH_ROWS)
    sk.update(keys, w)
    sk.update(keys[: n // 3].contiguous(), w[: n // 3].contiguous())
    want = _oracle_table(sk, keys, w)
    O.cs_update(PRIMES[prime], mode, rows, buckets, O.coeffs_from_seed(PRIMES[prime], rows, mode, seed=seed, k=k),
                _u64(keys[: n // 3]), w[: n // 3].cpu().numpy().astype(np.int64), table=want, k=k)
    _check_sketch(sk, keys, w, table=want)


@pytest.mark.parametrize("mode", [0, 2])
def test_rows_path_field_wraps(mode):
    """Few keys with weights +-(2^15 - 1): every field drifts past its 16-bit range many
    times in both directions (low and high halves, carries out of the word), and each
    wrap must reach the int64 counters exactly."""
    n = 1 << 20
    keys = (W.uniform_u64(11, n) & 63) * 0x9E3779B97F4A7C15 & ((1 << 60) - 1)
    w = torch.full((n,), (1 << 15) - 1, dtype=torch.int64)
    w[(n * 3) // 5:] = -(1 << 15) + 1
    w[::3] = W.bounded_int(12, w[::3].numel(), -(1 << 15) + 1, (1 << 15) - 1)
    keys, w = keys.to(DEV), w.to(torch.int32).to(DEV)
    sk = _make(9, 1 << 16, M.CS_P61, seed=1002, mode=mode)
    sk.set_update_path(M.CS_PATH_ROWS)
    sk.update(keys, w)
    table = _check_sketch(sk, keys, w)
    assert int(np.abs(table).max()) > 1 << 20  # the counters went far beyond 16 bits


@pytest.mark.parametrize("path", [3, 4])
def test_combining_repeated_keys_exact(path):
    """Heavy repetition inside tiles, weights that cancel to zero, and combined weights
    too large for a record: the two-pass update stays exact."""
    n = 5 * 2048 + 17
    keys = W.uniform_u64(3, n) & ((1 << 60) - 1)
    keys[::3] = 12345            # one key on a third of the stream
    keys[1::7] = (1 << 59) + 1   # another on a seventh
    w = W.bounded_int(3, n, -100, 100)
    w[::3] = torch.tensor([5, -5]).repeat(n)[: w[::3].numel()]  # cancels in pairs
    w[1::7] = 1 << 19            # sums far beyond the record field
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(7, 1 << 17, M.CS_P61, seed=71)
    sk.set_update_path(path)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


@pytest.mark.parametrize("log2m,prime", [(16, 1), (20, 2)])  # wave tiles, block tiles
@pytest.mark.parametrize("kind", ["uniform", "zipf", "one_key"])
@pytest.mark.parametrize("n", [100, 5 * 2048 + 77])
def test_automatic_combining_choice_matches_oracle(log2m, prime, kind, n):
    """The automatic path probes the keys and runs pass 1 with or without combining
    (uniform keys: without; repeated keys: with); the counters are the oracle's either way."""
    if kind == "uniform":
        keys = W.uniform_u64(70, n)
        if prime == 1:
            keys = keys & ((1 << 60) - 1)
    elif kind == "zipf":
        keys = W.zipf(71, n, 1.1, 1 << 32)
    else:
        keys = torch.full((n,), 123456789, dtype=torch.int64)
    w = W.bounded_int(72, n, -100, 100)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(4, 1 << log2m, prime, 73)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


def test_lds_path_forced_on_small_table():
    keys, w = W.stream_zipf_u64(10000, seed=3)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(4, 1 << 11, M.CS_P61, seed=9)
    sk.set_update_path(M.CS_PATH_LDS)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


def test_p89_large_table_uniform_u64():
    """p = 2^89-1, t = 5, m = 2^20 (40 MiB table), uniform uint64 keys, int64 weights = 1."""
    keys, w = W.stream_uniform_u64(1 << 15)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(5, 1 << 20, M.CS_P89, seed=1003)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


@pytest.mark.parametrize("k", [2, 8])
@pytest.mark.parametrize("prime", [1, 2])
def test_polynomial_degrees(k, prime):
    keys = W.uniform_u64(5, 3000)
    if prime == M.CS_P61:
        keys = keys & ((1 << 60) - 1)
    w = W.bounded_int(5, 3000, -50, 50)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = _make(4, 512, prime, seed=77, k=k)
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


def test_empty_stream_and_edge_keys():
    sk = _make(5, 1024, M.CS_P61, seed=3)
    empty = torch.empty(0, dtype=torch.int64, device=DEV)
    sk.update(empty, empty)
    f2, rows = sk.estimate_f2()
    assert f2 == 0 and not rows.any() and not sk.counters().any()
    edge = torch.tensor([0, 1, 2, (1 << 32) - 1, 1 << 32, (1 << 59), (1 << 60) - 1, (1 << 60) - 2], device=DEV)
    w = torch.tensor([1, -1, 5, 7, -9, 11, 13, -(1 << 40)], device=DEV)
    sk.update(edge, w)
    _check_sketch(sk, edge, w)
    sk89 = _make(3, 1 << 12, M.CS_P89, seed=4, mode=M.CS_TWO_FOR_ONE_MSB)
    e89 = torch.tensor([0, 1, -1, -2, -(1 << 63), (1 << 63) - 1, 1 << 32], device=DEV)  # -1 = 2^64-1
    w89 = torch.ones(7, dtype=torch.int64, device=DEV)
    sk89.update(e89, w89)
    _check_sketch(sk89, e89, w89)


def test_domain_error_is_sticky_and_reset_clears_it():
    sk = _make(2, 64, M.CS_P61, seed=5)
    bad = torch.tensor([1, 1 << 60, 3], device=DEV)
    sk.update(bad, torch.ones(3, dtype=torch.int64, device=DEV))
    st, _, _ = sk.estimate_f2_status()
    assert st == M.CS_EDOMAIN
    with pytest.raises(M.MCSError):
        sk.sync()
    sk.reset()
    sk.sync()
    assert not sk.counters().any()


def test_estimate_overflow():
    sk = _make(3, 64, M.CS_P61, seed=6)
    keys = torch.tensor([5], device=DEV)
    sk.update(keys, torch.tensor([1 << 32], device=DEV))
    st, f2, rows = sk.estimate_f2_status()
    assert st == M.CS_EOVERFLOW and f2 == np.iinfo(np.int64).max
    with pytest.raises(O.OracleError):
        O.cs_estimate(sk.counters())  # the counters stay readable
    # overflow concerns that estimate only: after cancelling the key it fits again
    sk.update(keys, torch.tensor([-(1 << 32) + 3], device=DEV))
    f2, rows = sk.estimate_f2()
    assert f2 == 9 and list(rows) == [9, 9, 9]


def test_point_query_matches_oracle():
    keys, w = W.stream_zipf_u64(20000, seed=99)
    keys, w = keys.to(DEV), w.to(DEV)
    for prime in (M.CS_P61, M.CS_P89):
        sk = _make(5, 1 << 10, prime, seed=8)
        sk.update(keys, w)
        table = sk.counters()
        q = keys[:500].contiguous()
        out = torch.empty(500, dtype=torch.int64, device=DEV)
        sk.query(q, out)
        torch.cuda.synchronize()
        coeffs = O.coeffs_from_seed(PRIMES[prime], 5, 0, seed=8)
        want = []
        for x in _u64(q):
            vals = []
            for r in range(5):
                b, s = O.bucket_sign(PRIMES[prime], 0, 1 << 10, coeffs, r, int(x))
                vals.append(s * int(table[r, b]))
            want.append(sorted(vals)[2])
        assert out.cpu().tolist() == want


def test_linearity_merge_and_split_updates():
    keys, w = W.stream_zipf_u64(50000, seed=5)
    keys, w = keys.to(DEV), w.to(DEV)
    for m in (1 << 8, 1 << 16):
        a = _make(5, m, M.CS_P61, seed=10)
        b = _make(5, m, M.CS_P61, seed=10)
        whole = _make(5, m, M.CS_P61, seed=10)
        a.update(keys[:20000].contiguous(), w[:20000].contiguous())
        b.update(keys[20000:].contiguous(), w[20000:].contiguous())
        whole.update(keys, w)
        a.merge(b)
        assert np.array_equal(a.counters(), whole.counters())
        whole.update(keys, -w)
        assert not whole.counters().any()


# ---------------------------------------------------------------------------
# quotient and remainder
# ---------------------------------------------------------------------------
def _divmod_inputs(prime, n, seed):
    p = {M.CS_P61: O.P61, M.CS_P89: O.P89, M.CS_P64_59: O.P64_59}[prime]
    nl = 3 if prime == M.CS_P89 else 2
    x = W.below_limbs(p * p, nl, seed, n)
    extra = [0, 1, p - 1, p, p + 1, 2 * p - 1, 2 * p, p * p - 1, 12345 * p, 12345 * p - 1, (2 ** 64 - 1),
             2 ** 64, 2 ** 64 + 1]
    if prime == M.CS_P61:
        extra += [2 ** 122 - 1, 2 ** 122 - 2, p * p, (2 ** 61 + 1) * p - 1]  # Mersenne domain beyond p^2
    elif prime == M.CS_P89:
        extra += [2 ** 178 - 1, 2 ** 178 - 2, p * p, 2 ** 128 - 1, 2 ** 128, 2 ** 128 + 1]
    else:
        extra += [p * 2 ** 64 - 1, 2 ** 127, (2 ** 64 - 60) * p + (p - 1)]
    ex = torch.tensor([[((v >> (64 * j)) & (2 ** 64 - 1)) - (2 ** 64 if (v >> (64 * j + 63)) & 1 else 0)
                        for j in range(nl)] for v in extra], dtype=torch.int64)
    return torch.cat([x, ex]).contiguous()


@pytest.mark.parametrize("prime", [1, 2, 3])
@pytest.mark.parametrize("naive", [False, True])
def test_divmod_matches_oracle(prime, naive):
    x = _divmod_inputs(prime, 100003, seed=prime)
    n = x.shape[0]
    qw = 2 if prime == M.CS_P89 else 1
    xd = x.to(DEV)
    q = torch.empty((n, qw), dtype=torch.int64, device=DEV)
    r = torch.empty((n, qw), dtype=torch.int64, device=DEV)
    M.mersenne_divmod(prime, xd, q, r, naive=naive)
    M.mersenne_status()
    oprime = {1: O.PRIME_P61, 2: O.PRIME_P89, 3: O.PRIME_P64_59}[prime]
    wq, wr = O.divmod_batch(oprime, x.numpy().view(np.uint64))
    assert np.array_equal(q.cpu().numpy().view(np.uint64).reshape(wq.shape), wq)
    assert np.array_equal(r.cpu().numpy().view(np.uint64).reshape(wr.shape), wr)


@pytest.mark.parametrize("prime", [1, 2, 3])
def test_div_and_mod_alone(prime):
    x = _divmod_inputs(prime, 4097, seed=10 + prime)
    n = x.shape[0]
    qw = 2 if prime == M.CS_P89 else 1
    xd = x.to(DEV)
    q = torch.empty((n, qw), dtype=torch.int64, device=DEV)
    r = torch.empty((n, qw), dtype=torch.int64, device=DEV)
    M.mersenne_div(prime, xd, q)
    M.mersenne_mod(prime, xd, r)
    M.mersenne_status()
    oprime = {1: O.PRIME_P61, 2: O.PRIME_P89, 3: O.PRIME_P64_59}[prime]
    wq, wr = O.divmod_batch(oprime, x.numpy().view(np.uint64))
    assert np.array_equal(q.cpu().numpy().view(np.uint64).reshape(wq.shape), wq)
    assert np.array_equal(r.cpu().numpy().view(np.uint64).reshape(wr.shape), wr)


def test_divmod_domain_flag():
    x = torch.tensor([[5, 0], [0, 1 << 58]], dtype=torch.int64, device=DEV)  # second value = 2^122
    q = torch.empty(2, dtype=torch.int64, device=DEV)
    M.mersenne_divmod(M.CS_P61, x, q, None)
    with pytest.raises(M.MCSError) as e:
        M.mersenne_status()
    assert e.value.status == M.CS_EDOMAIN
    M.mersenne_status()  # cleared


def _lazy_fold_carries(y: int, x: int, a: int) -> bool:
    """Whether folding P = y*x + a at bit 64 (P mod 2^64 + 8 (P >> 64)) carries out
    of 64 bits: the case in which the library's faster Horner steps are inexact and
    the wave recomputes its keys with the exact ones."""
    p_ = y * x + a
    return (p_ % (1 << 64)) + 8 * (p_ >> 64) >= 1 << 64


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("path", ["auto", "rows", "lds", "global", "binned"])
def test_lazy_fold_carry_path(path, mode, k):
    """Keys and coefficients chosen so that the first Horner step's fold at bit 64
    carries: a_{k-1} = 2^33 + 2, a_{k-2} = 0 and key 2^32 - 1 give P = 2^65 - 2.
    Waves holding such a key must recompute with the exact steps; every counter
    must equal the oracle's."""
    top, x_bad = (1 << 33) + 2, (1 << 32) - 1
    assert _lazy_fold_carries(top, x_bad, 0) and top < O.P61
    rows, m = 3, 1 << 12
    npoly = 2 if mode == 2 else 1
    rng = np.random.default_rng(4242 + k)
    coeffs = rng.integers(0, O.P61, size=(rows, npoly, k), dtype=np.uint64)
    coeffs[0, :, k - 1] = top
    coeffs[0, :, k - 2] = 0
    coeffs[1, 0, k - 1] = top
    n = 5 * 4096 + 77
    keys = W.uniform_u32(31 + k, n).to(torch.int64)
    keys[::97] = x_bad
    keys[n - 1] = x_bad
    w = W.bounded_int(31 + k, n, -100, 100)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = M.Sketch(rows, m, prime=M.CS_P61, mode=mode, k=k, coeffs=coeffs.reshape(-1))
    sk._coeffs = coeffs.reshape(-1)
    if path != "auto":
        sk.set_update_path({"rows": M.CS_PATH_ROWS, "lds": M.CS_PATH_LDS, "global": M.CS_PATH_GLOBAL,
                            "binned": M.CS_PATH_BINNED}[path])
    sk.update(keys, w)
    _check_sketch(sk, keys, w)
    # point queries hash the same keys (the first is 2^32 - 1)
    qk = keys[:200].contiguous()
    q = torch.empty(200, dtype=torch.int64, device=DEV)
    sk.query(qk, q)
    torch.cuda.synchronize()
    table = sk.counters()
    want_q = []
    for x in _u64(qk):
        vals = []
        for r in range(rows):
            b, s = O.bucket_sign(O.PRIME_P61, mode, m, sk._coeffs, r, int(x), k=k)
            vals.append(s * int(table[r, b]))
        want_q.append(sorted(vals)[rows // 2])
    assert q.cpu().tolist() == want_q


@pytest.mark.parametrize("k", [2, 4, 8])
@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("path", ["auto", "rows", "lds", "global", "binned"])
def test_last_step_guard_path(path, mode, k):
    """Coefficients chosen so that the last Horner step of key 2^32 - 1 reaches
    P = y*x + a_0 = p exactly (a_1 = 2^29, a_0 = 2^29 - 1, higher ones 0, so y = 2^29):
    bits 32..60 of P are all ones and the unfolded low word lo32(P) + lo32(P >> 61)
    would be 2^32 - 1 where h = 0.  Waves holding such a key must recompute with the
    exact steps; every counter must equal the oracle's."""
    x_bad = (1 << 32) - 1
    assert (1 << 29) * x_bad + (1 << 29) - 1 == O.P61
    rows, m = 3, 1 << 12
    npoly = 2 if mode == 2 else 1
    rng = np.random.default_rng(2929 + k)
    coeffs = rng.integers(0, O.P61, size=(rows, npoly, k), dtype=np.uint64)
    for r, a0 in ((0, (1 << 29) - 1), (1, (1 << 29) - 2)):
        coeffs[r, :, 2:] = 0
        coeffs[r, :, 1] = 1 << 29
        coeffs[r, :, 0] = a0
    n = 5 * 4096 + 77
    keys = W.uniform_u32(53 + k, n).to(torch.int64)
    keys[::97] = x_bad
    keys[n - 1] = x_bad
    w = W.bounded_int(53 + k, n, -100, 100)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = M.Sketch(rows, m, prime=M.CS_P61, mode=mode, k=k, coeffs=coeffs.reshape(-1))
    sk._coeffs = coeffs.reshape(-1)
    if path != "auto":
        sk.set_update_path({"rows": M.CS_PATH_ROWS, "lds": M.CS_PATH_LDS, "global": M.CS_PATH_GLOBAL,
                            "binned": M.CS_PATH_BINNED}[path])
    sk.update(keys, w)
    _check_sketch(sk, keys, w)


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("path,log2m", [("auto", 12), ("rows", 12), ("lds", 12), ("global", 12), ("binned", 12),
                                        ("binned", 18)])
def test_last_step_guard_path_p89(path, log2m, mode):
    """p = 2^89 - 1, k = 4: a_3 = a_2 = 0, a_1 = 2^25 and a_0 = 2^25 - 1 give key
    2^64 - 1 the last step P = p: bits 64..88 of P are all ones and the unfolded low
    word would be 2^32 - 1 where h = 0.  Waves holding such a key must take that step
    with the fold; every counter must equal the oracle's."""
    x_bad = (1 << 64) - 1
    assert (1 << 25) * x_bad + (1 << 25) - 1 == O.P89
    rows, m, k = 3, 1 << log2m, 4  # 2^18 buckets: more than 16 ranges, block tiles
    npoly = 2 if mode == 2 else 1
    rng = np.random.default_rng(8989)
    vals = [[[int(rng.integers(0, 1 << 62)) * (1 << 27) % O.P89 for _ in range(k)] for _ in range(npoly)]
            for _ in range(rows)]
    for r, a0 in ((0, (1 << 25) - 1), (1, (1 << 25) - 2)):
        for q in range(npoly):
            vals[r][q] = [a0, 1 << 25, 0, 0]
    coeffs = np.array([[v & ((1 << 64) - 1), v >> 64] for row in vals for poly in row for v in poly],
                      dtype=np.uint64)
    n = 5 * 4096 + 77
    keys = W.uniform_u64(71, n)
    keys[::97] = -1  # 2^64 - 1
    keys[n - 1] = -1
    w = W.bounded_int(71, n, -100, 100)
    keys, w = keys.to(DEV), w.to(DEV)
    sk = M.Sketch(rows, m, prime=M.CS_P89, mode=mode, k=k, coeffs=coeffs.reshape(-1))
    sk._coeffs = coeffs
    assert np.array_equal(sk.coeffs(), coeffs)
    if path != "auto":
        sk.set_update_path({"rows": M.CS_PATH_ROWS, "lds": M.CS_PATH_LDS, "global": M.CS_PATH_GLOBAL,
                            "binned": M.CS_PATH_BINNED}[path])
    sk.update(keys, w)
    _check_sketch(sk, keys, w)
