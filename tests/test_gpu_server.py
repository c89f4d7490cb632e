"""J-Merge server (knng_server_*).  Every request must equal one
balanced-append J-Merge of the base with its rows (the oracle's, id for id)
whatever runs beside it, and the resident graph must equal the base lists
with every request's new entries folded in (top k of the union)."""
import threading

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import assert_same_graph, dev, host

pytestmark = pytest.mark.gpu

M64 = 2 ** 64 - 1


def _sets(nb, sizes, d, seed):
    g = synth.rng(seed)
    base = g.standard_normal((nb, d)).astype(np.float32)
    reqs = [(g.standard_normal((m, d)) + 0.3).astype(np.float32) for m in sizes]
    return base, reqs


def _seed(seed, req_id):
    return oracle.splitmix64((seed ^ oracle.splitmix64(req_id)) & M64)


def _alone(X, G, raw, k, metric, first, s, seed, req_id):
    """The oracle's J-Merge of the base with one request, ids renumbered to
    the server's (request rows from `first`)."""
    m = X.shape[0]
    oi, od, ost = oracle.jmerge(X, G, raw, k, metric, sample=s, seed=_seed(seed, req_id),
                                balanced=True)
    oi = np.where(oi >= m, oi - m + first, oi)
    return oi, od, ost


def _fold(G, results, m, k):
    """Base lists with every request's entries of request rows folded in,
    followed by the requests' own rows (in id order)."""
    ids, dist = [], []
    for u in range(m):
        cand = {int(a): float(b) for a, b in zip(G[0][u], G[1][u])}
        for oi, od, _, first, n in results:
            for a, b in zip(oi[u], od[u]):
                if a >= m:
                    cand[int(a)] = float(b)
        best = sorted(cand.items(), key=lambda e: (np.float32(e[1]), e[0]))[:k]
        ids.append([a for a, _ in best])
        dist.append([b for _, b in best])
    for oi, od, _, first, n in sorted(results, key=lambda r: r[3]):
        ids.extend(oi[m:m + n].tolist())
        dist.extend(od[m:m + n].tolist())
    return np.array(ids, np.int32), np.array(dist, np.float32)


def _server(hip, base, G, k, metric, **kw):
    return hip.Server(dev(base), (dev(G[0]), dev(G[1])), k, metric, **kw)


@pytest.mark.parametrize("metric", ["l2", "cos"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_each_request_is_the_oracles_merge_with_the_base(hip, metric, precision):
    # the BF16 path covers the bf16 copy and norms written at submission at
    # the request's store rows, the two-segment row view and the list-mode
    # join; its screen must not change a single result
    k, s, seed = 8, 6, 31
    base, reqs = _sets(1200, [37, 5, 60], 11, 120)
    m = base.shape[0]
    G = oracle.exact_graph(base, k, metric)
    srv = _server(hip, base, G, k, metric, capacity=1400, max_request=100, slots=0, sample=s,
                  seed=seed, precision=precision)
    try:
        rids = [101, 202, 303]
        tickets = [srv.submit(dev(r) if i % 2 else r, rid)
                   for i, (r, rid) in enumerate(zip(reqs, rids))]
        assert srv.step() and srv.step() and srv.step() and not srv.step()
        first, results = m, []
        for t, raw, rid in zip(tickets, reqs, rids):
            ids, dist, info = srv.wait(t, len(raw))
            oi, od, ost = _alone(base, G, raw, k, metric, first, s, seed, rid)
            assert info["first_id"] == first and info["rows"] == len(raw)
            assert info["rounds"] == ost["rounds"] and info["evals"] == ost["evals"]
            assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], f"request {rid}")
            results.append((oi, od, ost, first, len(raw)))
            first += len(raw)
        si, sd = srv.snapshot()
        ei, ed = _fold(G, results, m, k)
        assert_same_graph(host(si), host(sd), ei, ed, "resident graph")
        assert srv.status() == {"base": m, "committed": first - m, "pending": 0}
    finally:
        srv.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_results_are_the_same_in_a_mix(hip, precision):
    # ten requests from two threads on three slots: each result equals the
    # request merged alone, and the resident graph does not depend on the
    # order in which they finished
    k, s, seed = 10, 6, 5
    sizes = [int(v) for v in synth.rng(9).integers(1, 70, 10)]
    base, reqs = _sets(1500, sizes, 16, 121)
    m = base.shape[0]
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=m + sum(sizes), max_request=80, slots=3,
                  sample=s, seed=seed, precision=precision)
    assert srv.slots == 3
    tickets = {}
    lock = threading.Lock()

    def submitter(part):
        for i in part:
            t = srv.submit(dev(reqs[i]), 1000 + i)
            with lock:
                tickets[i] = t

    th = [threading.Thread(target=submitter, args=(range(j, len(reqs), 2),)) for j in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    got = {i: srv.wait(t, len(reqs[i])) for i, t in tickets.items()}
    si, sd = (host(a) for a in srv.snapshot())
    srv.close()
    results = []
    for i, (ids, dist, info) in got.items():
        oi, od, ost = _alone(base, G, reqs[i], k, "l2", info["first_id"], s, seed, 1000 + i)
        assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], f"request {i} in the mix")
        assert info["submit_us"] <= info["start_us"] <= info["done_us"]
        assert 0 <= info["slot"] < 3
        results.append((oi, od, ost, info["first_id"], len(reqs[i])))
    ei, ed = _fold(G, results, m, k)
    assert_same_graph(si, sd, ei, ed, "resident graph after the mix")


def test_batching_merges_queued_requests_as_one_raw_set(hip):
    k, s, seed = 8, 6, 11
    base, reqs = _sets(1000, [20, 7, 33], 10, 124)
    m = base.shape[0]
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=1100, max_request=64, slots=0,
                  batching=True, sample=s, seed=seed)
    try:
        tickets = [srv.submit(r, 50 + i) for i, r in enumerate(reqs)]
        assert srv.step() and not srv.step()   # 60 rows fit in one merge of at most 64
        raw = np.concatenate(reqs)
        oi, od, ost = _alone(base, G, raw, k, "l2", m, s, seed, 50)
        first = m
        for t, r in zip(tickets, reqs):
            ids, dist, info = srv.wait(t, len(r))
            assert info["merged_first"] == m and info["merged_rows"] == len(raw)
            assert info["rounds"] == ost["rounds"]
            lo = first - m
            assert_same_graph(ids.numpy(), dist.numpy(), oi[m + lo:m + lo + len(r)],
                              od[m + lo:m + lo + len(r)], "batched request")
            first += len(r)
        si, sd = srv.snapshot()
        ei, ed = _fold(G, [(oi, od, ost, m, len(raw))], m, k)
        assert_same_graph(host(si), host(sd), ei, ed, "resident graph after a batch")
    finally:
        srv.close()


def test_rebase_lets_later_requests_meet_earlier_rows(hip):
    k, s, seed = 8, 5, 77
    base, reqs = _sets(900, [40, 30], 9, 123)
    m = base.shape[0]
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=1000, max_request=64, slots=0, sample=s,
                  seed=seed)
    try:
        t0 = srv.submit(reqs[0], 7)
        assert srv.step()
        srv.wait(t0, 40)
        srv.rebase()
        si, sd = (host(a) for a in srv.snapshot())
        assert srv.status() == {"base": m + 40, "committed": 0, "pending": 0}
        t1 = srv.submit(reqs[1], 8)
        assert srv.step()
        ids, dist, info = srv.wait(t1, 30)
        X1 = np.concatenate([base, reqs[0]])
        oi, od, _ = _alone(X1, (si, sd), reqs[1], k, "l2", m + 40, s, seed, 8)
        assert_same_graph(ids.numpy(), dist.numpy(), oi[m + 40:], od[m + 40:], "after rebase")
    finally:
        srv.close()


def test_wide_base_lists_and_a_rebase(hip):
    # base lists longer than k: a request keeps the first k entries of an
    # unselected row and returns the rest as its rear part; after a rebase
    # the base lists are the resident top k
    k, s, seed = 6, 5, 41
    base, reqs = _sets(700, [25, 18], 8, 125)
    m = base.shape[0]
    G = oracle.exact_graph(base, k + 3)
    srv = _server(hip, base, G, k, "l2", capacity=760, max_request=32, slots=0, sample=s,
                  seed=seed)
    try:
        t0 = srv.submit(reqs[0], 70)
        assert srv.step()
        ids, dist, info = srv.wait(t0, 25)
        oi, od, _ = _alone(base, G, reqs[0], k, "l2", m, s, seed, 70)
        assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], "wide base")
        srv.rebase()
        si, sd = (host(a) for a in srv.snapshot())
        t1 = srv.submit(reqs[1], 71)
        assert srv.step()
        ids, dist, info = srv.wait(t1, 18)
        X1 = np.concatenate([base, reqs[0]])
        oi, od, _ = _alone(X1, (si, sd), reqs[1], k, "l2", m + 25, s, seed, 71)
        assert_same_graph(ids.numpy(), dist.numpy(), oi[m + 25:], od[m + 25:],
                          "after rebase of a wide base")
    finally:
        srv.close()


def test_server_errors(hip):
    from paper_1908_00814_amd.knng import KnngError
    k = 6
    base, reqs = _sets(300, [10, 50], 5, 122)
    G = oracle.exact_graph(base, k)
    need = hip.server_bytes(400, 40, 5, k, k, "l2", slots=1, sample=4)
    with pytest.raises(KnngError, match="ENOMEM"):
        _server(hip, base, G, k, "l2", capacity=400, max_request=40, hbm_budget=need // 2,
                sample=4)
    srv = _server(hip, base, G, k, "l2", capacity=330, max_request=40, hbm_budget=10 * need,
                  slots=0, sample=4)
    try:
        with pytest.raises(KnngError, match="EINVAL"):
            srv.submit(reqs[1], 1)                    # more rows than max_request
        bad = reqs[0].copy()
        bad[3, 2] = np.nan
        with pytest.raises(KnngError, match="EINVAL"):
            srv.submit(bad, 2)                        # rejected, nothing reserved
        t = srv.submit(reqs[0], 3)
        with pytest.raises(KnngError, match="EBUSY"):
            srv.wait(t, 10, timeout_us=0)             # no slots: not run yet
        with pytest.raises(KnngError, match="EBUSY"):
            srv.snapshot()                            # queued work on a server without slots
        t2 = srv.submit(reqs[0][:5], 4)
        t3 = srv.submit(reqs[0][:10], 5)
        with pytest.raises(KnngError, match="ENOMEM"):
            srv.submit(reqs[0][:10], 6)               # 300 + 25 + 10 > 330
        assert srv.status()["pending"] == 25
        while srv.step():
            pass
        ids, _, info = srv.wait(t, 10)
        assert info["first_id"] == 300 and info["rows"] == 10
        assert (ids.numpy() >= 0).all() and (ids.numpy() < 325).all()
        srv.wait(t2, 5)
        srv.wait(t3, 10)
        with pytest.raises(KnngError, match="EINVAL"):
            srv.wait(t3, 10)                          # already collected
    finally:
        srv.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_many_requests_on_one_slot_each_equal_the_oracle(hip, precision):
    # one slot keeps its merge state between requests (tags of earlier merges
    # read as "never", only rows they changed are restored): 25 requests in a
    # row, sizes from 1 to 60 rows, each must equal its merge on fresh state
    k, s, seed = 8, 6, 17
    sizes = [int(v) for v in synth.rng(140).integers(1, 61, 25)]
    base, reqs = _sets(900, sizes, 7, 141)
    m = base.shape[0]
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=m + sum(sizes), max_request=64, slots=0,
                  sample=s, seed=seed, precision=precision)
    try:
        first, results = m, []
        for i, r in enumerate(reqs):
            t = srv.submit(dev(r), 500 + i)
            assert srv.step()
            ids, dist, info = srv.wait(t, len(r))
            oi, od, ost = _alone(base, G, r, k, "l2", first, s, seed, 500 + i)
            assert info["rounds"] == ost["rounds"]
            assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], f"request {i}")
            results.append((oi, od, ost, first, len(r)))
            first += len(r)
        si, sd = srv.snapshot()
        ei, ed = _fold(G, results, m, k)
        assert_same_graph(host(si), host(sd), ei, ed, "resident graph after 25 requests")
    finally:
        srv.close()


@pytest.mark.parametrize("slots", [0, 2])
def test_a_failed_request_fails_alone(hip, slots):
    # a request made to fail before its commit (the test hook forces, from the
    # host, the path of a merge that reported an error) fails alone: the
    # other requests equal the oracle, the resident graph is the base with
    # only their entries folded in, the failed rows keep their ids with empty
    # lists, and the server goes on serving
    from paper_1908_00814_amd.knng import KnngError
    k, s, seed = 8, 6, 13
    sizes = [20, 15, 25, 6]
    base, reqs = _sets(800, sizes, 7, 126)
    m = base.shape[0]
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=m + sum(sizes), max_request=32, slots=slots,
                  sample=s, seed=seed)
    rids = [301, 302, 303, 304]
    try:
        srv.fail_request(302)
        tickets = [srv.submit(r, rid) for r, rid in zip(reqs[:3], rids[:3])]
        if slots == 0:
            while srv.step():
                pass
        results, first = [], m
        for t, r, rid in zip(tickets, reqs[:3], rids[:3]):
            if rid == 302:
                with pytest.raises(KnngError, match="EDEVICE"):
                    srv.wait(t, len(r))
                failed = (first, len(r))
            else:
                ids, dist, info = srv.wait(t, len(r))
                assert info["first_id"] == first
                oi, od, ost = _alone(base, G, r, k, "l2", first, s, seed, rid)
                assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], f"request {rid}")
                results.append((oi, od, ost, first, len(r)))
            first += len(r)
        # served after the failure
        t4 = srv.submit(reqs[3], 304)
        if slots == 0:
            assert srv.step()
        ids, dist, info = srv.wait(t4, len(reqs[3]))
        oi, od, ost = _alone(base, G, reqs[3], k, "l2", first, s, seed, 304)
        assert_same_graph(ids.numpy(), dist.numpy(), oi[m:], od[m:], "request after the failure")
        results.append((oi, od, ost, first, len(reqs[3])))
        st = srv.status()
        assert st["committed"] == sum(sizes) - sizes[1] and st["pending"] == 0
        si, sd = (host(a) for a in srv.snapshot())
        ei, ed = _fold(G, results, m, k)
        # expected: base rows, then request rows in id order with the failed
        # request's rows empty
        rows_i, rows_d = list(ei[:m]), list(ed[:m])
        done = {r[3]: r for r in results}
        cur = m
        for n_ in sizes:
            if cur == failed[0]:
                rows_i += [[-1] * k] * n_
                rows_d += [[np.inf] * k] * n_
            else:
                oi_, od_ = done[cur][0], done[cur][1]
                rows_i += list(oi_[m:m + n_])
                rows_d += list(od_[m:m + n_])
            cur += n_
        assert_same_graph(si, sd, np.array(rows_i, np.int32), np.array(rows_d, np.float32),
                          "resident graph around a failed request")
    finally:
        srv.close()


def test_graph_rounds_equal_host_rounds(hip):
    # the same requests through the slot's captured round graph and through
    # the host-driven loop: identical results and round counts
    k, s, seed = 10, 6, 23
    sizes = [1, 3, 40, 77, 9]
    base, reqs = _sets(1300, sizes, 12, 127)
    G = oracle.exact_graph(base, k)
    out = {}
    for host_rounds in (False, True):
        srv = _server(hip, base, G, k, "l2", capacity=1300 + sum(sizes), max_request=80,
                      slots=0, sample=s, seed=seed, precision="bf16", host_rounds=host_rounds)
        try:
            got = []
            for i, r in enumerate(reqs):
                t = srv.submit(dev(r), 900 + i)
                assert srv.step()
                ids, dist, info = srv.wait(t, len(r))
                got.append((ids.numpy(), dist.numpy(), info["rounds"], info["evals"]))
            out[host_rounds] = (got, [host(a) for a in srv.snapshot()])
        finally:
            srv.close()
    for (gi, gd, gr, ge), (hi, hd, hr, he) in zip(out[False][0], out[True][0]):
        assert_same_graph(gi, gd, hi, hd, "graph vs host rounds")
        assert gr == hr and ge == he
    assert_same_graph(*out[False][1], *out[True][1], "resident graph")
