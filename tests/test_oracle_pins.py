"""Pins of the oracle to facts the paper and elementary number theory fix.

Each test checks the oracle (``oracle/``) against something other than itself:
closed forms, exact identities the paper proves, exhaustive enumeration on tiny
Mersenne primes, invariants, or brute force.  They run on the CPU only.
"""
import os
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# seed expansion
# ---------------------------------------------------------------------------
def test_splitmix64_known_answers():
    """Published SplitMix64 outputs (golden/splitmix64.txt)."""
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            seed, vals = line.split(":")
            want = [int(v) for v in vals.split()]
            assert O.splitmix64_stream(int(seed), len(want)) == want


def test_coefficients_in_field_and_rejection():
    c61 = O.coeffs_from_seed(O.PRIME_P61, rows=64, mode=O.TWO_POLY, seed=7)
    assert c61.shape == (64 * 2 * 4,)
    assert int(c61.max()) < O.P61
    # low 61 bits of consecutive SplitMix64 outputs (no draw equals p here)
    raw = O.splitmix64_stream(7, 512)
    assert [int(v) for v in c61] == [r & O.P61 for r in raw]
    c89 = O.coeffs_from_seed(O.PRIME_P89, rows=16, mode=O.TWO_FOR_ONE, seed=3)
    vals = [int(lo) | (int(hi) << 64) for lo, hi in c89]
    assert all(v < O.P89 for v in vals)
    raw = O.splitmix64_stream(3, 128)
    assert vals == [raw[2 * i] | ((raw[2 * i + 1] & ((1 << 25) - 1)) << 64) for i in range(64)]
    # top bits are used: some coefficient of a big sample exceeds 2^88 and 2^60
    assert max(vals) >= 1 << 88
    assert int(c61.max()) >= 1 << 60


# ---------------------------------------------------------------------------
# hash h_a(x) = sum a_i x^i mod p   (Section 1.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("x", [0, 1, 2, 3, 12345, (1 << 32) - 1, (1 << 59) + 17, (1 << 60) - 1])
def test_hash_p61_coefficient_positions(x):
    p = O.P61
    c = 987654321987654321 % p
    assert O.hash_small(p, [c, 0, 0, 0], x) == c
    assert O.hash_small(p, [0, 1, 0, 0], x) == x % p
    # a_2 multiplies x^2 and a_3 multiplies x^3, checked on powers of two below


@pytest.mark.parametrize("e", [0, 1, 20, 31, 32, 45, 59])
def test_hash_p61_powers_of_two(e):
    """2^61 = 1 mod p, so (2^e)^i = 2^(i*e mod 61)."""
    p, x = O.P61, 1 << e
    assert O.hash_small(p, [0, 0, 1, 0], x) == 1 << (2 * e % 61)
    assert O.hash_small(p, [0, 0, 0, 1], x) == 1 << (3 * e % 61)
    assert O.hash_small(p, [0, 0, 0, 5], x) == (5 << (3 * e % 61)) % p


def test_hash_p61_largest_key_binomial():
    """(2^60 - 1)^3 = 2^180 - 3*2^120 + 3*2^60 - 1 = 2^58 - 3*2^59 + 3*2^60 - 1 (mod 2^61 - 1)."""
    p = O.P61
    want = (2 ** 58 - 3 * 2 ** 59 + 3 * 2 ** 60 - 1) % p
    assert O.hash_small(p, [0, 0, 0, 1], (1 << 60) - 1) == want
    # (2^60 - 1)^2 = 2^120 - 2^61 + 1 = 2^59 - 1 + 1 (mod p)
    assert O.hash_small(p, [0, 0, 1, 0], (1 << 60) - 1) == (2 ** 59 - 1 + 1) % p


def _limbs(v):
    return [v & (2 ** 64 - 1), v >> 64]


@pytest.mark.parametrize("e", [0, 1, 31, 32, 44, 63])
def test_hash_p89_powers_of_two(e):
    """2^89 = 1 mod p: (2^e)^i = 2^(i*e mod 89)."""
    x = 1 << e
    z = [0, 0]
    one = [1, 0]
    assert O.hash_p89([z, one, z, z], x) == x
    assert O.hash_p89([z, z, one, z], x) == 1 << (2 * e % 89)
    assert O.hash_p89([z, z, z, one], x) == 1 << (3 * e % 89)


def test_hash_p89_all_ones_key():
    """(2^64 - 1)^3 = 2^192 - 3*2^128 + 3*2^64 - 1 = 2^14 - 3*2^39 + 3*2^64 - 1 (mod 2^89 - 1)."""
    p = O.P89
    z, one = [0, 0], [1, 0]
    x = 2 ** 64 - 1
    assert O.hash_p89([z, z, z, one], x) == (2 ** 14 - 3 * 2 ** 39 + 3 * 2 ** 64 - 1) % p
    assert O.hash_p89([z, z, one, z], x) == (2 ** 39 - 2 * 2 ** 64 + 1) % p
    big = p - 1  # -1 mod p: h = -(x^3 + x^2 + x + 1)
    h = O.hash_p89([_limbs(big)] * 4, x)
    assert h == (-(2 ** 14 - 3 * 2 ** 39 + 3 * 2 ** 64 - 1) - (2 ** 39 - 2 * 2 ** 64 + 1) - x - 1) % p


def test_hash_linear_in_coefficients():
    """h_{a+a'}(x) = h_a(x) + h_{a'}(x) mod p (the family is linear in a)."""
    rng = np.random.default_rng(5)
    for p, keymax in ((O.P61, 1 << 60),):
        for _ in range(50):
            a = [int(v) % p for v in rng.integers(0, 2 ** 63, 4, dtype=np.uint64)]
            b = [int(v) % p for v in rng.integers(0, 2 ** 63, 4, dtype=np.uint64)]
            x = int(rng.integers(0, keymax, dtype=np.uint64))
            s = [(u + v) % p for u, v in zip(a, b)]
            assert O.hash_small(p, s, x) == (O.hash_small(p, a, x) + O.hash_small(p, b, x)) % p
    p = O.P89
    for _ in range(50):
        a = [int.from_bytes(rng.bytes(12), "little") % p for _ in range(4)]
        b = [int.from_bytes(rng.bytes(12), "little") % p for _ in range(4)]
        x = int(rng.integers(0, 2 ** 63, dtype=np.uint64)) * 2 + 1
        s = [(u + v) % p for u, v in zip(a, b)]
        assert O.hash_p89([_limbs(v) for v in s], x) == \
            (O.hash_p89([_limbs(v) for v in a], x) + O.hash_p89([_limbs(v) for v in b], x)) % p


def test_hash_matches_power_sum_bigint():
    """Cross-check (not a pin by itself): Horner with % equals sum a_i * pow(x, i, p)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        a = [int.from_bytes(rng.bytes(8), "little") % O.P61 for _ in range(4)]
        x = int.from_bytes(rng.bytes(8), "little") >> 4
        assert O.hash_small(O.P61, a, x) == sum(ai * pow(x, i, O.P61) for i, ai in enumerate(a)) % O.P61
        a = [int.from_bytes(rng.bytes(12), "little") % O.P89 for _ in range(4)]
        x = int.from_bytes(rng.bytes(8), "little")
        assert O.hash_p89([_limbs(v) for v in a], x) == sum(ai * pow(x, i, O.P89) for i, ai in enumerate(a)) % O.P89


# ---------------------------------------------------------------------------
# k-universality on tiny Mersenne primes (Definition in Section 1.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("keys", [[0, 1, 2, 3], [5, 11, 17, 30], [1, 8, 9, 27]])
def test_four_wise_independence_p31(keys):
    """For 4 distinct keys, a -> (h_a(x_0..x_3)) is a bijection of Z_31^4 (Vandermonde)."""
    p = 31
    h = O.enum_hash(p, 4, keys).astype(np.int64)
    code = ((h[:, 0] * p + h[:, 1]) * p + h[:, 2]) * p + h[:, 3]
    assert np.array_equal(np.sort(code), np.arange(p ** 4))


def test_two_wise_independence_p127():
    p = 127
    for keys in ([0, 1], [3, 126], [64, 65]):
        h = O.enum_hash(p, 2, keys).astype(np.int64)
        assert np.array_equal(np.sort(h[:, 0] * p + h[:, 1]), np.arange(p * p))


def test_per_key_uniformity_p127_k4_sampled():
    """Each key's hash takes every value in [p] equally often over a_0 (shift by a_0)."""
    p = 127
    rng = np.random.default_rng(2)
    for _ in range(20):
        a1, a2, a3 = (int(v) for v in rng.integers(0, p, 3))
        x = int(rng.integers(0, p))
        vals = sorted(O.hash_small(p, [a0, a1, a2, a3], x) for a0 in range(p))
        assert vals == list(range(p))


# ---------------------------------------------------------------------------
# bucket / sign selection (Section 1.2.1, Algorithm 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB])
@pytest.mark.parametrize("m", [2, 4, 8])
def test_bucket_probabilities_p31(mode, m):
    """eq. coll-ell<r-1 / coll-ell=r-1: (p+1)/r values per bucket, one fewer for bucket r-1;
    the special value p (all ones) lands in bucket r-1 with sign -1."""
    p, b = 31, 5
    bk, sg = O.enum_bucket_sign(p, b, 4, mode, m, [7])
    counts = np.bincount(bk[:, 0].astype(np.int64), minlength=m)
    per_value = p ** 3  # each hash value occurs p^3 times over Z_p^4
    want = np.full(m, (p + 1) // m * per_value)
    want[m - 1] -= per_value
    assert np.array_equal(counts, want)
    # sign bit: value p has a = 1, so a = 1 has (p+1)/2 - 1 values
    assert int((sg[:, 0] == -1).sum()) == ((p + 1) // 2 - 1) * per_value


@pytest.mark.parametrize("mode", [O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB])
@pytest.mark.parametrize("m", [2, 4, 8])
def test_collision_probability_p31(mode, m):
    """eq. coll: Pr[i(x) = i(y)] = (1 + (r-1)/p^2)/r for distinct keys."""
    p, b = 31, 5
    bk, _ = O.enum_bucket_sign(p, b, 4, mode, m, [3, 20])
    coll = int((bk[:, 0] == bk[:, 1]).sum())
    assert Fraction(coll, p ** 4) == Fraction(1, m) * (1 + Fraction(m - 1, p * p))


def _lemma_check(bk, sg, p, m, A):
    """E[s(x0) A] == E[A | i(x0) = m-1] / p, exactly, over all coefficient tuples."""
    i = bk.astype(np.int64)
    s = sg.astype(np.int64)
    a_vals = A(i, s)
    lhs = Fraction(int((s[:, 0] * a_vals).sum()), p ** 4)
    cond = i[:, 0] == m - 1
    rhs = Fraction(int(a_vals[cond].sum()), int(cond.sum())) / p
    return lhs, rhs


@pytest.mark.parametrize("mode", [O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB])
def test_lemma_remove_si_p31(mode):
    """Lemma remove-si (Section 1.3.3) exactly, for several A depending on i(x0..x3), s(x1..x3)."""
    p, b, m = 31, 5, 4
    bk, sg = O.enum_bucket_sign(p, b, 4, mode, m, [2, 9, 13, 30])
    As = [
        lambda i, s: (i[:, 0] == i[:, 1]) * s[:, 1],
        lambda i, s: i[:, 0] * s[:, 1] * s[:, 2] * s[:, 3] + i[:, 3],
        lambda i, s: (i[:, 0] == m - 1) + 2 * (i[:, 1] == i[:, 2]) * s[:, 3] + i[:, 0] * i[:, 0],
    ]
    for A in As:
        lhs, rhs = _lemma_check(bk, sg, p, m, A)
        assert lhs == rhs
    # the classical cancellation E[s(x0) A] = 0 does NOT hold (the 1/p term is real)
    lhs, _ = _lemma_check(bk, sg, p, m, As[2])
    assert lhs != 0


# ---------------------------------------------------------------------------
# Count Sketch estimator: Theorem h-and-s-p (exact mean, variance bound)
# ---------------------------------------------------------------------------
def _moments(keys, weights):
    f = {}
    for k, w in zip(keys, weights):
        f[k] = f.get(k, 0) + w
    F1 = sum(f.values())
    F2 = sum(v * v for v in f.values())
    n = sum(1 for v in f.values() if v != 0)
    return F1, F2, n


STREAMS = [
    ([0, 1, 2, 3, 5], [3, -1, 2, 2, -4]),
    ([4, 4, 7, 9, 9, 9, 15], [5, -2, 1, 1, 1, -7, 3]),
    ([1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15], [1] * 15),
    ([6, 6, 11], [4, -4, 9]),  # key 6 cancels to f = 0
]


@pytest.mark.parametrize("mode", [O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB])
@pytest.mark.parametrize("m", [2, 4, 8])
@pytest.mark.parametrize("stream", STREAMS)
def test_theorem_exact_mean_and_variance_p31(mode, m, stream):
    """Sum over all a in Z_31^4 of X = p^4 F2 + p^2 (F1^2 - F2)  (eq. E-F2-p), and Var[X] < 2 F2^2 / r."""
    p, b = 31, 5
    keys, weights = stream
    F1, F2, n = _moments(keys, weights)
    s1, s2 = O.enum_estimate_moments(p, b, 4, mode, m, keys, weights)
    N = p ** 4
    assert s1 == N * F2 + p * p * (F1 * F1 - F2)
    # |E[X] - F2| <= F2 (n-1)/p^2   (eq. E-F2-p-com)
    assert abs(Fraction(s1, N) - F2) <= Fraction(F2 * (n - 1), p * p)
    var = Fraction(s2, N) - Fraction(s1, N) ** 2
    assert var < Fraction(2 * F2 * F2, m)


@pytest.mark.parametrize("m", [2, 4])
@pytest.mark.parametrize("stream", [([0, 1, 2, 3], [2, -1, 3, 1]), ([1, 1, 2, 5], [1, 2, -3, 4])])
def test_two_polynomial_exact_mean_p7(m, stream):
    """Independent bucket and sign polynomials (two 4-universal hashes, Section 1.3.1):
    E[X] = F2 + (F1^2 - F2) * E[s_x s_y] * Pr[i_x = i_y] with E[s_x s_y] = 1/p^2 and
    Pr[i_x = i_y] = (1 + (r-1)/p^2)/r, over all of Z_7^8."""
    p, b = 7, 3
    keys, weights = stream
    F1, F2, _ = _moments(keys, weights)
    s1, _ = O.enum_estimate_moments(p, b, 4, O.TWO_POLY, m, keys, weights)
    N = p ** 8
    want = Fraction(F2) + (F1 * F1 - F2) * Fraction(1, p * p) * Fraction(1, m) * (1 + Fraction(m - 1, p * p))
    assert Fraction(s1, N) == want


# ---------------------------------------------------------------------------
# update / estimate mechanics
# ---------------------------------------------------------------------------
def test_identity_polynomial_table_by_hand():
    """a = (0,1,0,0) makes h(x) = x: bucket and sign follow from the key's bits."""
    rows, m = 3, 16
    keys = [0, 1, 2, 3, 31, 32, 33, 100, 1000001]
    weights = [5, -3, 7, 1, 2, -9, 4, 6, -1]
    for prime in (O.PRIME_P61, O.PRIME_P89):
        if prime == O.PRIME_P61:
            coeffs = np.array([0, 1, 0, 0] * rows, dtype=np.uint64)
        else:
            coeffs = np.array([[0, 0], [1, 0], [0, 0], [0, 0]] * rows, dtype=np.uint64)
        for mode in (O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB):
            t = O.cs_update(prime, mode, rows, m, coeffs, keys, weights)
            want = np.zeros((rows, m), dtype=np.int64)
            for x, w in zip(keys, weights):
                if mode == O.TWO_FOR_ONE:
                    bucket, a = (x >> 1) % m, x & 1
                else:
                    bucket, a = x % m, 0  # key < 2^(b-1): top bit clear
                want[:, bucket] += (1 - 2 * a) * w
            assert np.array_equal(t, want), (prime, mode)


def test_constant_polynomial_estimate_is_F1_squared():
    """a = (c,0,0,0): every key hits one bucket with one sign, so X = F1^2 in every row."""
    keys = [3, 3, 8, 1, 77]
    weights = [2, 5, -1, 4, 10]
    coeffs = np.array([12345, 0, 0, 0, 999, 0, 0, 0], dtype=np.uint64)
    t = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 2, 64, coeffs, keys, weights)
    med, rows = O.cs_estimate(t)
    assert list(rows) == [sum(weights) ** 2] * 2 and med == sum(weights) ** 2


def test_linearity_and_cancellation():
    """The sketch is linear (Section 1.3.1): split and permuted streams give the same table;
    adding the negated stream gives the zero table."""
    rng = np.random.default_rng(9)
    n, rows, m = 3000, 5, 256
    keys = rng.integers(0, 1 << 60, n, dtype=np.uint64)
    weights = rng.integers(-1000, 1000, n)
    for prime in (O.PRIME_P61, O.PRIME_P89):
        for mode in (O.TWO_FOR_ONE, O.TWO_FOR_ONE_MSB, O.TWO_POLY):
            coeffs = O.coeffs_from_seed(prime, rows, mode, seed=21)
            full = O.cs_update(prime, mode, rows, m, coeffs, keys, weights)
            part = O.cs_update(prime, mode, rows, m, coeffs, keys[:1234], weights[:1234])
            O.cs_update(prime, mode, rows, m, coeffs, keys[1234:], weights[1234:], table=part)
            assert np.array_equal(full, part)
            perm = rng.permutation(n)
            assert np.array_equal(full, O.cs_update(prime, mode, rows, m, coeffs, keys[perm], weights[perm]))
            O.cs_update(prime, mode, rows, m, coeffs, keys, -weights, table=full)
            assert not full.any()


def test_key_parallel_variant_equals_row_parallel():
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 1 << 32, 20000, dtype=np.uint64)
    weights = rng.integers(-100, 101, 20000)
    coeffs = O.coeffs_from_seed(O.PRIME_P61, 9, O.TWO_FOR_ONE, seed=1001)
    a = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 9, 1024, coeffs, keys, weights)
    b = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 9, 1024, coeffs, keys, weights, threads=4)
    assert np.array_equal(a, b)


def test_estimate_by_hand_and_median():
    t = np.array([[1, -2, 3], [0, 0, 10], [4, 4, 4], [-1, 0, 0], [7, 0, -7]], dtype=np.int64)
    med, rows = O.cs_estimate(t)
    assert list(rows) == [14, 100, 48, 1, 98]
    assert med == 48  # sorted 1, 14, 48, 98, 100
    med, rows = O.cs_estimate(t[:4])  # even count: lower median of 1, 14, 48, 100
    assert med == 14


def test_estimate_overflow_detected():
    t = np.array([[1 << 31, 1 << 31], [3, 4]], dtype=np.int64)  # 2^62 + 2^62 = 2^63 does not fit
    with pytest.raises(O.OracleError) as e:
        O.cs_estimate(t)
    assert e.value.status == O.EOVERFLOW
    t = np.array([[-(1 << 63)]], dtype=np.int64)
    with pytest.raises(O.OracleError):
        O.cs_estimate(t)


def test_exact_f2_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(20):
        keys = rng.integers(0, 30, 200, dtype=np.uint64)
        weights = rng.integers(-50, 50, 200)
        f = {}
        for k, w in zip(keys.tolist(), weights.tolist()):
            f[k] = f.get(k, 0) + w
        assert O.exact_f2(keys, weights) == sum(v * v for v in f.values())


def test_domain_error_p61():
    coeffs = O.coeffs_from_seed(O.PRIME_P61, 1, O.TWO_FOR_ONE, seed=1)
    O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 1, 8, coeffs, [(1 << 60) - 1], [1])
    with pytest.raises(O.OracleError) as e:
        O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 1, 8, coeffs, [1 << 60], [1])
    assert e.value.status == O.EDOMAIN


def test_invalid_bucket_counts():
    coeffs = O.coeffs_from_seed(O.PRIME_P61, 1, O.TWO_FOR_ONE, seed=1)
    for m in (0, 3, 6):
        with pytest.raises(O.OracleError):
            O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 1, m, coeffs, [1], [1])
    # sign bit and bucket bits must be distinct: l <= b - 1 (Lemma remove-si's premise)
    small = [1, 2, 3, 4]
    O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 1, 16, small, [1], [1], p=31, b=5)
    with pytest.raises(O.OracleError):
        O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 1, 32, small, [1], [1], p=31, b=5)
    O.cs_update(O.PRIME_P61, O.TWO_POLY, 1, 32, small * 2, [1], [1], p=31, b=5)


# ---------------------------------------------------------------------------
# quotient and remainder (Section 1.5, Section 4): x = q p + r, 0 <= r < p
# ---------------------------------------------------------------------------
def _to_limbs(vals, n):
    return np.array([[(v >> (64 * j)) & (2 ** 64 - 1) for j in range(n)] for v in vals], dtype=np.uint64)


def _edge_values(p, top):
    vals = {0, 1, p - 1, p, p + 1, 2 * p - 1, 2 * p, 2 * p + 1, p * p - 1, p * p, top - 1,
            2 ** 64 - 1, 2 ** 64, 2 ** 64 + 1, 2 ** 128 - 1 if top > 2 ** 128 else top - 2}
    for k in (3, 5, 2 ** 20 + 7, p - 2, p - 1, p):
        for d in (-1, 0, 1):
            vals.add(k * p + d)
    return sorted(v for v in vals if 0 <= v < top)


@pytest.mark.parametrize("prime,p,top,nl", [
    (O.PRIME_P61, O.P61, 2 ** 122, 2),
    (O.PRIME_P64_59, O.P64_59, O.P64_59 * 2 ** 64, 2),
    (O.PRIME_P89, O.P89, 2 ** 178, 3),
])
def test_divmod_defining_property(prime, p, top, nl):
    rng = np.random.default_rng(prime)
    vals = _edge_values(p, top) + [int.from_bytes(rng.bytes(32), "little") % top for _ in range(3000)]
    q, r = O.divmod_batch(prime, _to_limbs(vals, nl))
    for i, v in enumerate(vals):
        qi = int(q[i]) if q.ndim == 1 else int(q[i, 0]) | (int(q[i, 1]) << 64)
        ri = int(r[i]) if r.ndim == 1 else int(r[i, 0]) | (int(r[i, 1]) << 64)
        assert 0 <= ri < p and qi * p + ri == v, v


@pytest.mark.parametrize("prime,bad", [
    (O.PRIME_P61, 2 ** 122), (O.PRIME_P64_59, O.P64_59 * 2 ** 64), (O.PRIME_P89, 2 ** 178)])
def test_divmod_domain(prime, bad):
    nl = 3 if prime == O.PRIME_P89 else 2
    with pytest.raises(O.OracleError) as e:
        O.divmod_batch(prime, _to_limbs([5, bad], nl))
    assert e.value.status == O.EDOMAIN


def test_oracle_is_independent_of_the_library():
    """The oracle neither imports nor links the GPU package."""
    here = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle")
    for name in os.listdir(here):
        if name.endswith((".py", ".c", ".h")):
            with open(os.path.join(here, name)) as f:
                src = f.read()
            assert "paper_2008_08654_amd" not in src and "libmcs" not in src and "mcs.h" not in src, name


# ---------------------------------------------------------------------------
# arbitrary numbers of buckets: most uniform maps (Section 1.4, Lemma
# most-uniform; Section 1.5 on pseudo-Mersenne primes) and Algorithm 8
# (Section 3.3, eq. prix0 / prixneq0, Lemma ix-r-dist, Lemma
# remove-si-r-dist, Theorem h-and-s-p-arb-r)
# ---------------------------------------------------------------------------
def _most_uniform(counts, q, r):
    lo, hi = q // r, -(-q // r)
    return len(counts) == r and all(c in (lo, hi) for c in counts) and sum(counts) == q


@pytest.mark.parametrize("b", [5, 7, 13])
@pytest.mark.parametrize("r", [2, 3, 5, 6, 7, 10, 12, 16, 31])
def test_mersenne_map_is_most_uniform(b, r):
    """Lemma most-uniform (iii): v -> ((v+1) r) >> b is most uniform from [2^b - 1] to [r]."""
    if r > (1 << b) - 1:
        pytest.skip("more buckets than values")
    q = (1 << b) - 1
    out = O.bucket_map_mersenne(b, list(range(q)), r)
    assert _most_uniform(np.bincount(out, minlength=r).tolist(), q, r)
    assert (np.diff(out.astype(np.int64)) >= 0).all()


def test_plus_c_trick_fails_for_pseudo_mersenne():
    """Section 1.4: for q = 2^b - c with c >= 2, v -> ((v+c) r) >> b leaves bucket 0 with
    ceil(2^b / r) - c values, so it is not most uniform in general (negative control on
    the counting used by the pins above)."""
    b, c, r = 8, 5, 7           # q = 251
    q = (1 << b) - c
    counts = np.bincount([((v + c) * r) >> b for v in range(q)], minlength=r).tolist()
    assert counts[0] == -(-(1 << b) // r) - c
    assert not _most_uniform(counts, q, r)


@pytest.mark.parametrize("p", [31, 127, 251, 8191, 65521])
@pytest.mark.parametrize("r", [2, 3, 7, 10, 30])
def test_exact_map_is_most_uniform(p, r):
    """floor(v r / p) is most uniform from [p] to [r] for any p (Section 1.4), including the
    pseudo-Mersenne 251 = 2^8 - 5 and 65521 = 2^16 - 15 (Section 1.5)."""
    out = O.bucket_map_exact(p, list(range(p)), r)
    assert _most_uniform(np.bincount(out, minlength=r).tolist(), p, r)
    assert (np.diff(out.astype(np.int64)) >= 0).all()


def test_maps_at_the_large_primes_edges():
    """Edges of the three library primes: v = 0 lands in bucket 0 and v = p - 1 in bucket
    r - 1; v >= p is outside the domain."""
    for p, b in (((1 << 61) - 1, 61), ((1 << 89) - 1, 89), ((1 << 64) - 59, None)):
        for r in (1, 2, 1000, (1 << 32) - 1):
            e = O.bucket_map_exact(p, [0, p - 1], r)
            assert e.tolist() == [0, r - 1]
            if b is not None:
                f = O.bucket_map_mersenne(b, [0, p - 1], r)
                assert f.tolist() == [r >> b, r - 1]
        with pytest.raises(O.OracleError):
            O.bucket_map_exact(p, [p], 10)


def _arb_split_all_h(p, b, r):
    """(bucket, sign) of Algorithm 8 for every hash value h in [p]: with k = 1 the
    polynomial is the constant a_0, so enumerating a_0 enumerates h."""
    bk, sg = O.enum_bucket_sign(p, b, 1, O.ARB_R, r, [3])
    return bk[:, 0].astype(np.int64), sg[:, 0].astype(np.int64)


@pytest.mark.parametrize("p,b", [(31, 5), (127, 7), (8191, 13)])
@pytest.mark.parametrize("r", [2, 3, 5, 6, 7, 12, 15, 16])
def test_algorithm8_bucket_and_sign_counts(p, b, r):
    """eq. prix0 / prixneq0: over h in [p], bucket 0 gets 2 ceil(2^(b-1)/r) - 1 values and
    every other bucket 2 floor(2^(b-1)/r) or 2 ceil(2^(b-1)/r); the sign bit is 1 for
    2^(b-1) values; Lemma ix-r-dist's bounds hold."""
    if r > 1 << (b - 1):
        pytest.skip("r > 2^(b-1)")
    bk, sg = _arb_split_all_h(p, b, r)
    assert bk.min() >= 0 and bk.max() < r
    cnt = np.bincount(bk, minlength=r)
    half = 1 << (b - 1)
    lo, hi = half // r, -(-half // r)
    assert cnt[0] == 2 * hi - 1
    assert all(c in (2 * lo, 2 * hi) for c in cnt[1:])
    assert (sg == -1).sum() == half and (sg == 1).sum() == half - 1   # s = 1 - 2a, a = bit b-1 of h+1
    pr = Fraction(1, p)
    assert cnt[0] * pr <= (1 + Fraction(r, 1 << b)) / r                       # eq. ix=0
    assert sum(Fraction(int(c), p) ** 2 for c in cnt) <= (1 + Fraction(r, 1 << b) ** 2) / r   # eq. ix=iy


@pytest.mark.parametrize("p,b", [(31, 5), (127, 7)])
@pytest.mark.parametrize("r", [3, 5, 6])
def test_algorithm8_sign_surplus_only_in_bucket_zero(p, b, r):
    """Lemma remove-si-r-dist with A = [i_x = i]: summed over h in [p], s_x [i_x = i] is 0
    for every bucket i != 0, and bucket 0 keeps a surplus of -1 (h + 1 = 2^(b-1) has sign
    bit 1 and j = 0, with no partner h + 1 = 0).  So E[s_x [i_x = 0]] = -1/p: the lemma's
    E[A | i_x = 0]/p up to the global sign of its opposite convention s = 2a - 1."""
    bk, sg = _arb_split_all_h(p, b, r)
    for i in range(r):
        assert sg[bk == i].sum() == (-1 if i == 0 else 0)


@pytest.mark.parametrize("r", [3, 5, 6, 7])
@pytest.mark.parametrize("stream", STREAMS)
def test_theorem_arb_r_exact_mean_and_variance_p31(r, stream):
    """Theorem h-and-s-p-arb-r over all of Z_31^4 (u = 16 keys, 1 < r <= u/2,
    p = 31 > u): E[X] = F2 + (F1^2 - F2)/p^2 exactly, |E[X] - F2| <= F2 (n-1)/p^2 and
    Var[X] < 2 (1 + (r/2^b)^2) F2^2 / r."""
    p, b = 31, 5
    keys, weights = stream
    F1, F2, n = _moments(keys, weights)
    s1, s2 = O.enum_estimate_moments(p, b, 4, O.ARB_R, r, keys, weights)
    N = p ** 4
    assert s1 == N * F2 + p * p * (F1 * F1 - F2)
    assert abs(Fraction(s1, N) - F2) <= Fraction(F2 * (n - 1), p * p)
    var = Fraction(s2, N) - Fraction(s1, N) ** 2
    assert var < 2 * (1 + Fraction(r, 1 << b) ** 2) * F2 * F2 / r


def test_algorithm8_with_power_of_two_r_selects_bits():
    """For r = 2^l, floor(r j / 2^(b-1)) is the top l bits of the low b-1 bits of h + 1: a
    plain bit selection of the hash value, checked against the independent hash functions
    for p = 2^61 - 1 and 2^89 - 1 (identity polynomial h(x) = x and random polynomials)."""
    keys = [0, 1, 5, (1 << 59) + 12345, (1 << 60) - 1]
    for l in (1, 4, 10):
        r = 1 << l
        for prime, b in ((O.PRIME_P61, 61), (O.PRIME_P89, 89)):
            coeffs = O.coeffs_from_seed(prime, 2, O.ARB_R, seed=77)
            for row in range(2):
                for x in keys:
                    bk, s = O.bucket_sign(prime, O.ARB_R, r, coeffs, row, x)
                    if prime == O.PRIME_P61:
                        h = O.hash_small(O.P61, coeffs[row * 4:(row + 1) * 4], x)
                    else:
                        h = O.hash_p89(coeffs.reshape(-1, 2)[row * 4:(row + 1) * 4], x)
                    hx = h + 1
                    assert bk == (hx & ((1 << (b - 1)) - 1)) >> (b - 1 - l)
                    assert s == 1 - 2 * ((hx >> (b - 1)) & 1)


def test_arb_r_invalid_counts_and_linearity():
    small = [1, 2, 3, 4]
    for r in (0, 1, 17):          # r = 17 > 2^(b-1) for b = 5
        with pytest.raises(O.OracleError):
            O.cs_update(O.PRIME_P61, O.ARB_R, 1, r, small, [1], [1], p=31, b=5)
    coeffs = O.coeffs_from_seed(O.PRIME_P61, 3, O.ARB_R, seed=5)
    keys = list(range(1000, 1400))
    w = [(i * 37) % 201 - 100 for i in range(400)]
    whole = O.cs_update(O.PRIME_P61, O.ARB_R, 3, 1000, coeffs, keys, w)
    part = O.cs_update(O.PRIME_P61, O.ARB_R, 3, 1000, coeffs, keys[:150], w[:150])
    O.cs_update(O.PRIME_P61, O.ARB_R, 3, 1000, coeffs, keys[150:], w[150:], table=part)
    assert np.array_equal(whole, part)
    assert int(np.abs(whole).sum()) > 0


# ---------------------------------------------------------------------------
# wide quotient and remainder (the b-sweep of Section 5's division experiment)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b", [32, 64, 128, 256, 512, 1024])
def test_wide_divmod_closed_forms(b):
    """p = 2^b - 1: 2^(2b) - 1 = p (p + 2) gives q = p + 2 = 2^b + 1, r = 0; p^2 - 1 gives
    q = p - 1, r = p - 1; k p + j gives (k, j); 0 gives (0, 0)."""
    p = (1 << b) - 1
    vals = [(1 << (2 * b)) - 1, p * p - 1, 0, p, p - 1, 5 * p + 3, (p - 1) * p + (p - 1)]
    want = [(p + 2, 0), (p - 1, p - 1), (0, 0), (1, 0), (0, p - 1), (5, 3), (p - 1, p - 1)]
    q, r = O.divmod_wide(b, 1, O.ints_to_planes(vals, 2 * b // 32))
    got = list(zip(O.planes_to_ints(q), O.planes_to_ints(r)))
    assert got == want


def test_wide_divmod_matches_128_bit_oracle():
    """b = 64, c = 59 (p = 2^64 - 59): the same values through the C oracle's 128-bit
    division (an independent implementation)."""
    rng = np.random.default_rng(3)
    p = (1 << 64) - 59
    vals = [int(v) for v in rng.integers(0, 2 ** 63, 200, dtype=np.uint64)]
    vals = [(v * p + (v % p)) % (p << 64) for v in vals] + [0, p - 1, p, (p << 64) - 1]
    x = np.array([[v & (2 ** 64 - 1), v >> 64] for v in vals], dtype=np.uint64)
    q1, r1 = O.divmod_batch(O.PRIME_P64_59, x)
    q2, r2 = O.divmod_wide(64, 59, O.ints_to_planes(vals, 4))
    assert O.planes_to_ints(q2) == [int(v) for v in q1]
    assert O.planes_to_ints(r2) == [int(v) for v in r1]


def test_wide_planes_round_trip_and_arguments():
    vals = [0, 1, (1 << 256) - 1, 12345678901234567890123456789]
    assert O.planes_to_ints(O.ints_to_planes(vals, 8)) == vals
    with pytest.raises(ValueError):
        O.ints_to_planes([1 << 256], 8)
    with pytest.raises(ValueError):
        O.divmod_wide(48, 1, np.zeros((3, 1), dtype=np.uint32))
    with pytest.raises(ValueError):
        O.divmod_wide(64, 1, np.zeros((3, 1), dtype=np.uint32))
