"""GPU parity for any number of buckets: Algorithm 8 sketches (CS_ARB_R) on every update
path, point queries, merge and the unpadded counter read, in single sketches, batches and
the server; and the most uniform bucket maps for the three primes.  Expected values come
from the oracle only; comparisons are bit-exact."""
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
PRIMES = {1: O.PRIME_P61, 2: O.PRIME_P89}


def _u64(t):
    a = t.detach().cpu().numpy()
    return a.view(np.uint32).astype(np.uint64) if a.dtype == np.int32 else a.view(np.uint64)


def _oracle(prime, rows, r, seed, keys, w, k=4):
    c = O.coeffs_from_seed(PRIMES[prime], rows, O.ARB_R, seed=seed, k=k)
    return O.cs_update(PRIMES[prime], O.ARB_R, rows, r, c, _u64(keys), w.cpu().numpy().astype(np.int64), k=k)


def _check(sk, want):
    torch.cuda.synchronize()
    got = sk.counters()
    assert got.shape == want.shape
    assert np.array_equal(got, want), f"{int((got != want).sum())} counters differ"
    st, f2, rows = sk.estimate_f2_status()
    wst, wmed, wrows = O.cs_estimate_status(want)
    assert st == {O.OK: M.CS_OK, O.EOVERFLOW: M.CS_EOVERFLOW}[wst]
    assert list(rows) == list(wrows) and f2 == wmed


# (rows, r): in LDS, two-pass wave tiles, two-pass block tiles; r just above and below
# powers of two, primes, r = 2, the maximum 2^30 is covered by the shape test below
SHAPES = [(5, 3), (5, 1000), (3, 2049), (9, 50000), (7, 65535), (4, 65537), (2, 1000003), (1, 2)]


@pytest.mark.parametrize("prime", [1, 2])
@pytest.mark.parametrize("rows,r", SHAPES)
@pytest.mark.parametrize("path", [0, 2, 3])
def test_arb_r_all_paths_match_oracle(prime, rows, r, path):
    n = 3 * 2048 + 333
    keys = W.zipf(40 + rows, n, 1.1, 1 << 32)
    if prime == 2:
        keys[::5] = W.uniform_u64(41, keys[::5].numel())  # full 64-bit keys for 2^89 - 1
    w = W.bounded_int(40 + rows, n, -100, 100)
    w[::101] = 1 << 40  # too wide for a record: direct atomics
    keys, w = keys.to(DEV), w.to(DEV)
    sk = M.Sketch(rows, r, prime=prime, seed=600 + rows, mode=M.CS_ARB_R)
    if path:
        sk.set_update_path(path)
    sk.update(keys, w)
    _check(sk, _oracle(prime, rows, r, 600 + rows, keys, w))


def test_arb_r_k2_k8_u32_keys_and_lds_table():
    keys = W.uniform_u32(9, 5000).to(torch.int32).to(DEV)
    w = torch.ones(5000, dtype=torch.int64, device=DEV)
    for k in (2, 8):
        sk = M.Sketch(3, 777, prime=M.CS_P61, seed=31, mode=M.CS_ARB_R, k=k)
        sk.set_update_path(M.CS_PATH_LDS)
        sk.update(keys, w)
        _check(sk, _oracle(1, 3, 777, 31, keys, w, k=k))


def test_arb_r_query_merge_and_info():
    keys, w = W.stream_zipf_u64(30000, seed=77)
    keys, w = keys.to(DEV), w.to(DEV)
    r = 12345
    for prime in (M.CS_P61, M.CS_P89):
        a = M.Sketch(5, r, prime=prime, seed=3, mode=M.CS_ARB_R)
        b = M.Sketch(5, r, prime=prime, seed=3, mode=M.CS_ARB_R)
        a.update(keys[:10000].contiguous(), w[:10000].contiguous())
        b.update(keys[10000:].contiguous(), w[10000:].contiguous())
        a.merge(b)
        want = _oracle(prime, 5, r, 3, keys, w)
        _check(a, want)
        q = keys[:300].contiguous()
        out = torch.empty(300, dtype=torch.int64, device=DEV)
        a.query(q, out)
        torch.cuda.synchronize()
        coeffs = O.coeffs_from_seed(PRIMES[prime], 5, O.ARB_R, seed=3)
        exp = []
        for x in _u64(q):
            vals = []
            for row in range(5):
                bk, s = O.bucket_sign(PRIMES[prime], O.ARB_R, r, coeffs, row, int(x))
                vals.append(s * int(want[row, bk]))
            exp.append(sorted(vals)[2])
        assert out.cpu().tolist() == exp
        c = M.Sketch(5, r + 1, prime=prime, seed=3, mode=M.CS_ARB_R)
        with pytest.raises(M.MCSError):
            a.merge(c)  # same padded width, different r


def test_arb_r_shape_limits():
    for bad in (0, 1, (1 << 30) + 1):
        with pytest.raises(M.MCSError):
            M.Sketch(2, bad, prime=M.CS_P61, seed=1, mode=M.CS_ARB_R)
    with pytest.raises(M.MCSError):
        M.Sketch(2, 1000, prime=M.CS_P61, seed=1)  # power-of-two modes still need 2^l


def test_arb_r_largest_count():
    """r = 2^30 (one 8 GiB row): point queries and F2 equal what the oracle's buckets give
    for the touched counters (every other counter is zero)."""
    r, n = 1 << 30, 4096
    big = M.Sketch(1, r, prime=M.CS_P61, seed=1, mode=M.CS_ARB_R)
    keys = W.uniform_u64(5, n) & ((1 << 60) - 1)
    w = W.bounded_int(5, n, -100, 100)
    big.update(keys.to(DEV), w.to(DEV))
    c = O.coeffs_from_seed(O.PRIME_P61, 1, O.ARB_R, seed=1)
    table, where = {}, []
    for x, wt in zip(_u64(keys), w.tolist()):
        bk, s = O.bucket_sign(O.PRIME_P61, O.ARB_R, r, c, 0, int(x))
        table[bk] = table.get(bk, 0) + s * wt
        where.append((bk, s))
    out = torch.empty(n, dtype=torch.int64, device=DEV)
    big.query(keys.to(DEV), out)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [s * table[bk] for bk, s in where]
    f2, _ = big.estimate_f2()
    assert f2 == sum(v * v for v in table.values())
    big.close()


def test_arb_r_batch_and_server():
    keys = W.zipf(W.DATA_SEED + 8, 200000, 1.2, 1 << 32).to(DEV)
    w = W.bounded_int(W.DATA_SEED + 8, 200000, -100, 100).to(torch.int32).to(DEV)
    shapes = [(7, 3000), (7, 100000), (5, 777), (3, 250000)]
    members, off = [], 0
    for i, (rows, r) in enumerate(shapes):
        n = [5000, 80000, 20000, 90000][i]
        members.append((M.Sketch(rows, r, prime=M.CS_P61, seed=900 + i, mode=M.CS_ARB_R),
                        keys[off:off + n], w[off:off + n], rows, r, 900 + i))
        off += n
    b = M.Batch([(sk, k, ww) for sk, k, ww, *_ in members])
    b.update()
    torch.cuda.synchronize()
    for sk, k, ww, rows, r, seed in members:
        assert np.array_equal(sk.counters(), _oracle(1, rows, r, seed, k, ww))
    srv = M.Server(mode=M.CS_ARB_R)
    ids = [srv.admit(rows, r, seed) for _, _, _, rows, r, seed in members if r <= 1 << 18]
    for t, (sk, k, ww, rows, r, seed) in zip(ids, members):
        srv.submit_update(t, k, ww)
    tk = [srv.submit_f2(t) for t in ids]
    res = [srv.wait(x) for x in tk]
    for t, res_t, (sk, k, ww, rows, r, seed) in zip(ids, res, members):
        want = _oracle(1, rows, r, seed, k, ww)
        assert np.array_equal(srv.counters(t, rows, r), want)
        assert res_t.f2 == O.cs_estimate_status(want)[1]
    srv.close()


# ---------------------------------------------------------------------------
# most uniform maps of hash values to [r]
# ---------------------------------------------------------------------------
P = {M.CS_P61 if M else 1: (1 << 61) - 1, M.CS_P89 if M else 2: (1 << 89) - 1, M.CS_P64_59 if M else 3: (1 << 64) - 59}


def _limb_rows(vals, nl):
    return torch.from_numpy(np.array([[(x >> (64 * j)) & ((1 << 64) - 1) for j in range(nl)] for x in vals],
                                     dtype=np.uint64).view(np.int64))


def _values(prime, n, seed):
    p = P[prime]
    nl = 2 if prime == M.CS_P89 else 1
    v = W.below_limbs(p, nl, seed, n).reshape(-1, nl)
    edges = [0, 1, 2, p - 2, p - 1, p // 2, p // 3, (1 << 32) - 1, 1 << 32]
    if prime == M.CS_P89:
        edges += [(1 << 64) - 1, 1 << 64, (1 << 88) - 1, 1 << 88]
    v = torch.cat([v, _limb_rows(edges, nl)]).contiguous()
    return (v.reshape(-1) if nl == 1 else v), nl


@pytest.mark.parametrize("prime", [1, 2, 3])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("r", [1, 2, 7, 1000, 65536, 1000003, (1 << 32) - 1])
def test_bucket_maps_match_oracle(prime, method, r):
    if method == M.CS_MAP_MERSENNE and prime == M.CS_P64_59:
        pytest.skip("the (v+1) r >> b map is for Mersenne primes")
    v, nl = _values(prime, 100003, 70 + prime)
    out = torch.empty(v.shape[0], dtype=torch.int32, device=DEV)
    vd = v.to(DEV)
    M.mersenne_bucket_map(prime, vd, r, out, method=method)
    M.mersenne_status()
    got = out.cpu().numpy().view(np.uint32)
    vh = v.numpy().view(np.uint64)
    if method == M.CS_MAP_EXACT:
        want = O.bucket_map_exact(P[prime], vh, r)
    else:
        want = O.bucket_map_mersenne({1: 61, 2: 89}[prime], vh, r)
    assert np.array_equal(got, want)


def test_bucket_map_domain_and_arguments():
    for prime in (1, 2, 3):
        nl = 2 if prime == M.CS_P89 else 1
        p = P[prime]
        bad = _limb_rows([p], nl)
        bad = (bad.reshape(-1) if nl == 1 else bad).contiguous().to(DEV)
        out = torch.empty(1, dtype=torch.int32, device=DEV)
        M.mersenne_bucket_map(prime, bad, 10, out)
        with pytest.raises(M.MCSError) as e:
            M.mersenne_status()
        assert e.value.status == M.CS_EDOMAIN
        M.mersenne_status()  # cleared
    v = torch.zeros(4, dtype=torch.int64, device=DEV)
    out = torch.empty(4, dtype=torch.int32, device=DEV)
    for prime, method, r in ((3, 1, 10), (1, 0, 0), (1, 0, 1 << 32), (1, 5, 10)):
        with pytest.raises(M.MCSError):
            M.mersenne_bucket_map(prime, v, r, out, method=method)
