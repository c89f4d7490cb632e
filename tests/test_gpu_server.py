"""J-Merge server (knng_server_*): batches of requests against a resident
graph.  Each batch must equal one balanced-append J-Merge of the resident set
with the batch's rows (the oracle's, id for id), and the resident graph must
equal the chain of those merges."""
import threading

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import assert_same_graph, dev, host

pytestmark = pytest.mark.gpu


def _sets(nb, sizes, d, seed, metric="l2"):
    g = synth.rng(seed)
    base = g.standard_normal((nb, d)).astype(np.float32)
    reqs = [(g.standard_normal((m, d)) + 0.3).astype(np.float32) for m in sizes]
    return base, reqs


def _server(hip, base, G, k, metric, **kw):
    return hip.Server(dev(base), (dev(G[0]), dev(G[1])), k, metric, **kw)


@pytest.mark.parametrize("metric", ["l2", "cos"])
def test_manual_batches_equal_the_oracle_chain(hip, metric):
    k, s, seed = 8, 6, 31
    base, reqs = _sets(1200, [37, 5, 60, 22, 9], 11, 120)
    G = oracle.exact_graph(base, k, metric)
    srv = _server(hip, base, G, k, metric, capacity=1400, max_batch=120, manual=True,
                  sample=s, seed=seed)
    try:
        # batch 0: the first three requests (102 rows); batch 1: the other two
        X, GX = base, G
        for b, group in enumerate(([0, 1, 2], [3, 4])):
            tickets = [srv.submit(dev(reqs[i]) if i % 2 else reqs[i]) for i in group]
            assert srv.step() and not srv.step()
            raw = np.concatenate([reqs[i] for i in group])
            oi, od, ost = oracle.jmerge(X, GX, raw, k, metric, sample=s, seed=seed + b,
                                        balanced=True)
            first = X.shape[0]
            for t, i in zip(tickets, group):
                ids, dist, info = srv.wait(t, len(reqs[i]))
                assert info["first_id"] == first and info["batch"] == b
                assert info["batch_rows"] == len(raw) and info["rounds"] == ost["rounds"]
                assert info["evals"] == ost["evals"]
                rows = slice(first, first + len(reqs[i]))
                assert_same_graph(ids.numpy(), dist.numpy(), oi[rows], od[rows],
                                  f"batch {b} request {i}")
                first += len(reqs[i])
            si, sd = srv.snapshot()
            assert_same_graph(host(si), host(sd), oi, od, f"snapshot after batch {b}")
            X, GX = np.concatenate([X, raw]), (oi, od)
        assert srv.status() == {"resident": X.shape[0], "pending": 0, "batches": 2}
    finally:
        srv.close()


def test_worker_batches_replay_as_expand_chain(hip):
    # requests submitted from two threads while the worker merges: whatever
    # batches formed, the resident graph is the chain of balanced J-Merges of
    # those batches, replayed here with knng_expand
    k, s, seed = 10, 6, 5
    base, reqs = _sets(3000, [int(v) for v in synth.rng(9).integers(1, 90, 24)], 16, 121)
    G = oracle.exact_graph(base, k)
    srv = _server(hip, base, G, k, "l2", capacity=3000 + sum(map(len, reqs)), max_batch=200,
                  sample=s, seed=seed)
    tickets = {}
    lock = threading.Lock()

    def submitter(part):
        for i in part:
            t = srv.submit(dev(reqs[i]))
            with lock:
                tickets[i] = t

    th = [threading.Thread(target=submitter, args=(range(j, len(reqs), 2),)) for j in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    infos = {}
    res = {}
    for i, t in tickets.items():
        ids, dist, info = srv.wait(t, len(reqs[i]))
        infos[i], res[i] = info, (ids.numpy(), dist.numpy())
    si, sd = (host(a) for a in srv.snapshot())
    srv.close()
    # rows in id order, grouped by batch
    order = sorted(infos, key=lambda i: infos[i]["first_id"])
    X = base
    Gi, Gd = dev(G[0]), dev(G[1])
    b_prev = -1
    groups = []
    for i in order:
        if infos[i]["batch"] != b_prev:
            groups.append([])
            b_prev = infos[i]["batch"]
        groups[-1].append(i)
    assert [infos[g[0]]["batch"] for g in groups] == list(range(len(groups)))
    for b, grp in enumerate(groups):
        raw = np.concatenate([reqs[i] for i in grp])
        assert all(infos[i]["batch_rows"] == len(raw) for i in grp)
        gi, gd, _ = hip.expand(dev(X), (Gi, Gd), dev(raw), k, "l2", sample=s, seed=seed + b,
                               balanced=True)
        for i in grp:
            lo = infos[i]["first_id"]
            np.testing.assert_array_equal(res[i][0], host(gi)[lo:lo + len(reqs[i])])
        X = np.concatenate([X, raw])
        Gi, Gd = gi, gd
    assert_same_graph(si, sd, host(Gi), host(Gd), "resident graph")
    # every request waited no longer than its batch ran after it arrived
    for i in infos:
        assert infos[i]["submit_us"] <= infos[i]["start_us"] <= infos[i]["done_us"]


def test_server_errors(hip):
    from paper_1908_00814_amd.knng import KnngError
    k = 6
    base, reqs = _sets(300, [10, 50], 5, 122)
    G = oracle.exact_graph(base, k)
    need = hip.server_bytes(400, 40, 5, k, k, "l2", sample=4)
    with pytest.raises(KnngError, match="ENOMEM"):
        _server(hip, base, G, k, "l2", capacity=400, max_batch=40, hbm_budget=need - 1,
                sample=4)
    srv = _server(hip, base, G, k, "l2", capacity=330, max_batch=40, hbm_budget=need,
                  manual=True, sample=4)
    try:
        with pytest.raises(KnngError, match="EINVAL"):
            srv.submit(reqs[1])                       # more rows than max_batch
        bad = reqs[0].copy()
        bad[3, 2] = np.nan
        with pytest.raises(KnngError, match="EINVAL"):
            srv.submit(bad)                           # rejected, nothing reserved
        t = srv.submit(reqs[0])
        with pytest.raises(KnngError, match="EBUSY"):
            srv.wait(t, 10, timeout_us=0)             # manual server: not run yet
        t2 = srv.submit(reqs[0][:5])
        t3 = srv.submit(reqs[0][:10])
        with pytest.raises(KnngError, match="ENOMEM"):
            srv.submit(reqs[0][:10])                  # 300 + 25 + 10 > 330
        assert srv.status()["pending"] == 25
        assert srv.step()
        ids, _, info = srv.wait(t, 10)
        assert info["first_id"] == 300 and info["batch_rows"] == 25
        assert (ids.numpy() >= 0).all() and (ids.numpy() < 325).all()
        srv.wait(t2, 5)
        srv.wait(t3, 10)
        with pytest.raises(KnngError, match="EINVAL"):
            srv.wait(t3, 10)                          # already collected
    finally:
        srv.close()
