"""CPU checks of the integer identities the update kernels use in place of the
textbook reduction steps (run without a GPU).  Each is stated from the
arithmetic of Z_p with p = 2^61 - 1 and checked on random and edge values
against Python's exact integers:

* a Horner step y*x + a with the fold at bit 64 (2^64 = 8 mod p) gives a value
  congruent to y*x + a unless the 64-bit sum carries, and then it is exactly
  8 short (the kernels detect that case and take the fold at bit 61);
* the fold at bit 61 of y*x + a_0 + 1 is r = h + 1 or h + 1 + p for
  h = (y*x + a_0) mod p, so the low word of h is lo32(r) + (r >> 61) - 1;
* for y < 2^64 the last step needs no fold at all: P = y*x + a_0 < 2^96, and
  unless bits 32..60 of P reach 2^29 - 8, (P mod 2^61) + (P >> 61) < p is h, so
  the low word of h is lo32(P) + lo32(P >> 61) (the kernels send the wave to the
  exact steps when a lane's bits reach that bound);
* the same for p = 2^89 - 1 with r >> 89, and its unfolded last step (y < 2p,
  bits 64..88 of P below 2^25 - 2);
* a 16-bit field's wrap test, taken in 32 bits, is exact for every 32-bit
  signed weight, and the carried multiples of 2^16 are floor((f + s*w) / 2^16).
"""
import random

P61 = (1 << 61) - 1
P89 = (1 << 89) - 1
M32, M64 = (1 << 32) - 1, (1 << 64) - 1


def fold61(v: int) -> int:
    return (v & P61) + (v >> 61)


def lazy_step(y: int, x: int, a: int) -> tuple[int, bool]:
    """The kernel's bit-64 step on 32-bit limbs: A = y0 x + a0 and B = y1 x + a1, the
    high word of A plus the low word of B with its carry into B's high word (the
    v_add_co_u32 / v_addc_co_u32 pair), then (mid:A_lo) + 8 top in 64 bits, with its
    carry-out."""
    y0, y1, a0, a1 = y & M32, y >> 32, a & M32, a >> 32
    A = y0 * x + a0
    B = y1 * x + a1
    assert A <= M64 and B <= M64
    mid = (A >> 32) + (B & M32)
    top = (B >> 32) + (mid >> 32)
    assert top <= M32  # B < 2^64 - 2^32, so its high word takes the carry
    low = ((mid & M32) << 32) | (A & M32)
    assert low + (top << 64) == y * x + a  # the pair is P mod 2^64 and P >> 64
    s = low + 8 * top
    return s & M64, s > M64


def exact_step(y: int, x: int, a_lo: int, a_hi: int) -> int:
    """The kernel's bit-61 step: returns (P mod 2^61) + (P >> 61) for P = y x + a."""
    y0, y1 = y & M32, y >> 32
    t = y0 * x + a_lo
    assert t <= M64
    u = y1 * x + (t >> 32) + a_hi
    assert u <= M64
    P = (u << 32) | (t & M32)
    return fold61(P)


def _values(rng, n):
    edge_y = [0, 1, P61 - 1, P61, 2 * P61 - 1, (1 << 62) - 1, M64, M64 - 1, 1 << 63]
    edge_x = [0, 1, M32, M32 - 1, 1 << 31]
    edge_a = [0, 1, P61 - 1]
    for y in edge_y:
        for x in edge_x:
            for a in edge_a:
                yield y, x, a
    for _ in range(n):
        yield rng.getrandbits(64), rng.getrandbits(32), rng.randrange(P61)


def test_lazy_fold_is_congruent_or_reports_a_carry():
    rng = random.Random(2008)
    carries = 0
    for i, (y, x, a) in enumerate(_values(rng, 20000)):
        s, c = lazy_step(y, x, a)
        want = (y * x + a) % P61
        if c:
            carries += i >= 135  # the edge values (first 135) carry often; random ones should not
            assert (s + 8) % P61 == want  # exactly 8 short: 2^64 = 8 (mod p)
        else:
            assert s % P61 == want
    # the constructed case of the GPU test carries, and random ones practically never
    s, c = lazy_step((1 << 33) + 2, M32, 0)
    assert c and (s + 8) % P61 == ((1 << 33) + 2) * M32 % P61
    assert carries <= 3


def test_last_step_with_a0_plus_one_gives_the_low_word():
    rng = random.Random(61)
    for y, x, a in _values(rng, 20000):
        h = (y * x + a) % P61
        r = exact_step(y, x, (a & M32) + 1, a >> 32)
        assert 1 <= r < 2 * P61 + 1 and r in (h + 1, h + 1 + P61)
        assert ((r & M32) + (r >> 61) - 1) & M32 == h & M32
    # h = p - 1: r is p or 2p
    y, x = 1, P61 - 1
    r = exact_step(y, x, 1, 0)
    assert ((r & M32) + (r >> 61) - 1) & M32 == (P61 - 1) & M32


GUARD = (1 << 29) - 8


def last_lo(y: int, x: int, a: int) -> tuple[int, int]:
    """The kernel's unfolded last step on 32-bit limbs: (lo32(t) + lo32(u >> 29)) mod
    2^32 and bits 32..60 of P, for t = y0 x + a0, u = y1 x + t_hi + a1 = P >> 32."""
    y0, y1, a0, a1 = y & M32, y >> 32, a & M32, a >> 32
    t = y0 * x + a0
    assert t <= M64
    u = y1 * x + (t >> 32) + a1
    assert u <= M64
    return ((t & M32) + ((u >> 29) & M32)) & M32, u & ((1 << 29) - 1)


def test_unfolded_last_step_gives_the_low_word_below_the_guard():
    rng = random.Random(96)
    guarded = 0
    cases = list(_values(rng, 20000))
    # values of P just below, at and above the bound, and P = p, 2p (where the
    # unfolded sum is not yet reduced)
    for P in (P61, 2 * P61, P61 - 1, (GUARD << 32) - 1, GUARD << 32, (GUARD << 32) + M32, (1 << 61) + 5):
        cases += [(1, x, P - x) for x in (0, 1, 12345) if 0 <= P - x < P61]
    for i, (y, x, a) in enumerate(cases):
        h = (y * x + a) % P61
        lo, bits = last_lo(y, x, a)
        assert bits == ((y * x + a) >> 32) & ((1 << 29) - 1)
        if bits >= GUARD:
            guarded += 135 <= i < 20135  # the random values, not the edge or constructed ones
            continue
        assert lo == h & M32
    # the bound is needed: P = p (bits 32..60 all ones) has h = 0 but lo32(P) = 2^32 - 1
    lo, bits = last_lo(1, 0, P61)
    assert bits >= GUARD and lo != 0
    # a random lane reaches the bound about once in 2^26
    assert guarded <= 2


def test_last_step_p89_low_word():
    rng = random.Random(89)
    for _ in range(5000):
        y, x, a = rng.randrange(2 * P89), rng.getrandbits(64), rng.randrange(P89)
        h = (y * x + a) % P89
        P = y * x + a + 1
        r = (P & P89) + (P >> 89)
        assert r < 2 * P89 + 1
        assert ((r & M32) + (r >> 89) - 1) & M32 == h & M32


def test_unfolded_last_step_p89():
    rng = random.Random(8989)
    guard = (1 << 25) - 2
    hits = 0
    cases = [(rng.randrange(2 * P89), rng.getrandbits(64), rng.randrange(P89)) for _ in range(20000)]
    cases += [(1 << 25, M64, (1 << 25) - 1), (1 << 25, M64, (1 << 25) - 2), (2 * P89 - 1, M64, P89 - 1)]
    for i, (y, x, a) in enumerate(cases):
        P = y * x + a
        assert P >> 89 < 1 << 65
        if (P >> 64) & ((1 << 25) - 1) >= guard:
            hits += i < 20000
            continue
        assert ((P & M32) + ((P >> 89) & M32)) & M32 == (P % P89) & M32
    # the constructed case of the GPU test: P = p, h = 0, the unfolded word 2^32 - 1
    P = (1 << 25) * M64 + (1 << 25) - 1
    assert P == P89 and (P >> 64) & ((1 << 25) - 1) >= guard and (P & M32) + ((P >> 89) & M32) == M32
    assert hits <= 2


def test_field_wrap_test_is_exact_for_32_bit_weights():
    rng = random.Random(16)
    weights = [0, 1, -1, (1 << 15) - 1, -(1 << 15), 1 << 15, (1 << 31) - 1, -(1 << 31), 1 << 30, -(1 << 30)]
    weights += [rng.randrange(-(1 << 31), 1 << 31) for _ in range(3000)]
    for w in weights:
        for a in (0, 1):
            sw_true = -w if a else w
            sw32 = ((w ^ -a) + a) & M32  # (w ^ -a) + a in 32 bits
            sw32 = sw32 - (1 << 32) if sw32 >> 31 else sw32
            for f in (0, 1, 0x7FFF, 0x8000, 0xFFFE, 0xFFFF, rng.randrange(1 << 16)):
                t32 = (f + sw32) & M32
                wrapped_32 = t32 > 0xFFFF
                t = f + sw_true
                assert wrapped_32 == (not 0 <= t < 1 << 16)
                if wrapped_32:
                    # the kernel's 64-bit recomputation of s*w from the 32-bit one
                    swl = (1 << 31) if (a and sw32 == -(1 << 31)) else sw32
                    assert swl == sw_true
                    cw = (f + swl) >> 16  # floor division
                    assert (f + swl) - cw * (1 << 16) == (f + sw_true) % (1 << 16)
