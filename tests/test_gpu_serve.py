"""Serving runtime (include/mcs_serve.h) on the GPU: per-tenant counters and F2 answers
equal the oracle's, a tenant's results are identical alone and mixed with other
tenants' traffic, admission respects the device-memory budget, and the open-loop
replay answers every request."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_08654_amd as M
import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0") if torch.cuda.is_available() else None

# (rows, log2 buckets): LDS-sized, direct-atomic-prone and two-pass tables
TENANTS = [(7, 12), (7, 14), (7, 16), (7, 18), (3, 8), (5, 10), (1, 11), (16, 13)]


def _trace(n_req, seed, max_log2=15.0):
    tenant, is_f2, _ = W.served_requests(n_req, len(TENANTS), seed=seed)
    size = W.loguniform_int(seed, n_req, 0.0, max_log2, stream=9) * (1 - is_f2)
    size[3] = 0  # an empty update
    total = int(size.sum())
    keys = W.zipf(seed, total, 1.2, 1 << 32).to(DEV)
    w = W.bounded_int(seed, total, -100, 100).to(torch.int32).to(DEV)
    reqs, off = [], 0
    for t, f, n in zip(tenant.tolist(), is_f2.tolist(), size.tolist()):
        if f:
            reqs.append((t, M.CS_REQ_F2, None, None))
        else:
            reqs.append((t, M.CS_REQ_UPDATE, keys[off: off + n], w[off: off + n]))
            off += n
    return reqs


def _oracle_answers(reqs, seed0):
    """Oracle tables after the whole trace and the F2 status/answer of each F2 request."""
    tables = [np.zeros((r, 1 << l), dtype=np.int64) for r, l in TENANTS]
    coeffs = [O.coeffs_from_seed(O.PRIME_P61, r, O.TWO_FOR_ONE, seed0 + i) for i, (r, l) in enumerate(TENANTS)]
    answers = {}
    for i, (t, kind, k, w) in enumerate(reqs):
        r, l = TENANTS[t]
        if kind == M.CS_REQ_UPDATE:
            if k.numel():
                O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, r, 1 << l, coeffs[t], W.as_uint64_numpy(k),
                            w.cpu().numpy().astype(np.int64), table=tables[t])
        else:
            st, med, _ = O.cs_estimate_status(tables[t])
            answers[i] = (st, med)
    return tables, answers


def _admit_all(srv, seed0):
    return [srv.admit(r, 1 << l, seed0 + i) for i, (r, l) in enumerate(TENANTS)]


def test_served_mixed_and_alone_match_oracle():
    seed0 = 900
    reqs = _trace(160, W.DATA_SEED + 50)
    want_tables, want_f2 = _oracle_answers(reqs, seed0)

    # mixed: every tenant's requests interleaved, small steps and a 1 MiB workspace (many rounds)
    mixed = M.Server(step_keys=1 << 16, work_bytes=1 << 20)
    ids = _admit_all(mixed, seed0)
    tickets = []
    for t, kind, k, w in reqs:
        tickets.append(mixed.submit_f2(ids[t]) if kind == M.CS_REQ_F2 else mixed.submit_update(ids[t], k, w))
    got_mixed = {i: mixed.wait(tk) for i, tk in enumerate(tickets) if reqs[i][1] == M.CS_REQ_F2}
    mixed.drain()
    assert mixed.stats().steps > 1

    # alone: one tenant at a time, drained before the next tenant starts
    alone = M.Server()
    ids_a = _admit_all(alone, seed0)
    got_alone = {}
    for t in range(len(TENANTS)):
        mine = [(i, r) for i, r in enumerate(reqs) if r[0] == t]
        tk = {i: (alone.submit_f2(ids_a[t]) if kind == M.CS_REQ_F2 else alone.submit_update(ids_a[t], k, w))
              for i, (_, kind, k, w) in mine}
        for i, (_, kind, _, _) in mine:
            if kind == M.CS_REQ_F2:
                got_alone[i] = alone.wait(tk[i])
        alone.drain()

    for t, (r, l) in enumerate(TENANTS):
        cm = mixed.counters(ids[t], r, 1 << l)
        ca = alone.counters(ids_a[t], r, 1 << l)
        assert np.array_equal(cm, want_tables[t]), (t, r, l)
        assert np.array_equal(ca, cm), (t, r, l)
    assert len(want_f2) > 5
    for i, (st, med) in want_f2.items():
        for got in (got_mixed[i], got_alone[i]):
            assert got.status == st and (st != O.OK or got.f2 == med), (i, got.status, got.f2, st, med)
        assert got_mixed[i].done_ns >= got_mixed[i].arrival_ns
    mixed.close()
    alone.close()


def test_served_f2_sees_exactly_the_earlier_updates():
    """Update, F2, update, F2 on one tenant, queued at once (one step would hold them
    all if the ordering rule did not hold the second update back)."""
    srv = M.Server()
    t = srv.admit(5, 1 << 12, 77)
    keys = W.zipf(5, 30000, 1.2, 1 << 32).to(DEV)
    w = W.bounded_int(5, 30000, -100, 100).to(torch.int32).to(DEV)
    coeffs = O.coeffs_from_seed(O.PRIME_P61, 5, O.TWO_FOR_ONE, 77)
    tk = [srv.submit_update(t, keys[:10000], w[:10000], ticket=True), srv.submit_f2(t),
          srv.submit_update(t, keys[10000:], w[10000:], ticket=True), srv.submit_f2(t)]
    res = [srv.wait(x) for x in tk]
    table = np.zeros((5, 1 << 12), dtype=np.int64)
    for (lo, hi), i in (((0, 10000), 1), ((10000, 30000), 3)):
        O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 5, 1 << 12, coeffs, W.as_uint64_numpy(keys[lo:hi]),
                    w[lo:hi].cpu().numpy().astype(np.int64), table=table)
        st, med, _ = O.cs_estimate_status(table)
        assert res[i].status == st and res[i].f2 == med
    assert res[1].f2 != res[3].f2
    srv.close()


def test_served_admission_budget_and_eviction():
    work = 1 << 20
    own = work + 2 * ((4 << 20) + 32768 * 8)  # workspace plus the two steps' list and result buffers
    tenant_bytes = 4 * (1 << 14) * 8 + 200000  # table plus an upper bound for the small buffers
    srv = M.Server(hbm_budget=own + tenant_bytes + 1000, work_bytes=work)
    a = srv.admit(4, 1 << 14, 1)
    with pytest.raises(M.MCSError) as e:
        srv.admit(4, 1 << 14, 2)
    assert e.value.status == M.CS_EBUSY
    st = srv.stats()
    assert st.tenants == 1 and st.resident_bytes <= st.budget_bytes
    keys = W.zipf(9, 5000, 1.2, 1 << 32).to(DEV)
    w = W.bounded_int(9, 5000, -100, 100).to(torch.int32).to(DEV)
    srv.submit_update(a, keys, w)
    srv.evict(a)  # waits for the queued update, then frees
    with pytest.raises(M.MCSError):
        srv.submit_update(a, keys, w)
    b = srv.admit(4, 1 << 14, 2)
    srv.submit_update(b, keys, w)
    want = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 4, 1 << 14, O.coeffs_from_seed(O.PRIME_P61, 4, 0, 2),
                       W.as_uint64_numpy(keys), w.cpu().numpy().astype(np.int64))
    assert np.array_equal(srv.counters(b, 4, 1 << 14), want)
    with pytest.raises(M.MCSError):
        srv.admit(17, 1 << 10, 3)   # more rows than the batched update takes
    with pytest.raises(M.MCSError):
        srv.admit(4, 1 << 19, 3)    # more buckets than the batched update takes
    with pytest.raises(M.MCSError):
        M.Server(hbm_budget=own - 1, work_bytes=work)
    srv.close()


def test_held_back_tenant_does_not_close_the_step():
    """F2(a), update(a), update(b), F2(b), F2(a) queued at once: a's update waits for a
    later step (a's first F2 must not see it) and so does a's second F2, while b's
    requests still join the first step; every answer is the oracle's for exactly the
    updates submitted before it."""
    srv = M.Server(step_keys=1 << 22)
    a, b = srv.admit(3, 1 << 10, 41), srv.admit(4, 1 << 12, 42)
    keys = W.zipf(11, 20000, 1.2, 1 << 32).to(DEV)
    w = W.bounded_int(11, 20000, -100, 100).to(torch.int32).to(DEV)
    ka, wa, kb, wb = keys[:8000], w[:8000], keys[8000:], w[8000:]
    trace = [(a, M.CS_REQ_F2, None, None), (a, M.CS_REQ_UPDATE, ka, wa), (b, M.CS_REQ_UPDATE, kb, wb),
             (b, M.CS_REQ_F2, None, None), (a, M.CS_REQ_F2, None, None)]
    res = srv.replay(trace, np.zeros(len(trace)))
    assert all(r.status == M.CS_OK for r in res)

    def f2_after(rows, log2m, seed, k, ww):
        table = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, rows, 1 << log2m,
                            O.coeffs_from_seed(O.PRIME_P61, rows, O.TWO_FOR_ONE, seed), W.as_uint64_numpy(k),
                            ww.cpu().numpy().astype(np.int64))
        return O.cs_estimate_status(table)[1]

    assert res[0].f2 == 0  # nothing of a's was submitted before it
    assert res[3].f2 == f2_after(4, 12, 42, kb, wb)
    assert res[4].f2 == f2_after(3, 10, 41, ka, wa)
    assert res[2].step == res[3].step == res[0].step  # b joined the step a's update was held from
    assert res[1].step > res[0].step and res[4].step >= res[1].step
    srv.close()


@pytest.mark.parametrize("prepared", [False, True])
def test_served_open_loop_replay(prepared):
    seed0 = 950
    reqs = _trace(240, W.DATA_SEED + 51, max_log2=14.0)
    _, want_f2 = _oracle_answers(reqs, seed0)
    srv = M.Server(step_keys=1 << 15)
    ids = _admit_all(srv, seed0)
    arrivals = W.poisson_arrivals(len(reqs), 20000.0, seed=W.DATA_SEED + 51)
    mapped = [(ids[t], kind, k, w) for t, kind, k, w in reqs]
    if prepared:  # marshalled once, arrivals as a float64 array
        res = srv.replay(srv.prepare(mapped), arrivals.numpy())
    else:
        res = srv.replay(mapped, arrivals.tolist())
    assert len(res) == len(reqs)
    assert all(r.status == O.OK or i in want_f2 for i, r in enumerate(res))
    for i, (st, med) in want_f2.items():
        assert res[i].status == st and (st != O.OK or res[i].f2 == med), i
    lat = np.array([r.done_ns - r.arrival_ns for r in res], dtype=np.float64)
    assert (lat > 0).all()
    steps = {r.step for r in res}
    assert len(steps) > 1
    srv.close()
