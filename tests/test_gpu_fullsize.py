"""The benchmark workloads at full size: 2 x 500,000 x d128 byte-valued
clusters (l2) and 2 x 250,000 x d960 normalised rows (cosine), approximate k=20
inputs, merged to k=20, s=20, delta=0.001, in the
launch configuration bench.py times.  The oracle cannot run it whole, so the
checks are per-row values it computes one by one (canonical distances of
sampled rows, FP64 errors) and properties that hold at any size."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

N1 = N2 = 500_000
K = 20


@pytest.fixture(scope="module")
def w2(hip):
    import torch
    from synth.graphs import approximate_graph
    S1, S2 = synth.byte_cluster_sets(N1, N2, workload=2)
    G1 = approximate_graph(S1, K, 0.9, device="cuda", stream=6)
    G2 = approximate_graph(S2, K, 0.9, device="cuda", stream=7)
    d = lambda a: torch.from_numpy(a).cuda()
    args = (d(S1), (d(G1[0]), d(G1[1])), d(S2), (d(G2[0]), d(G2[1])), K, "l2")
    out = {}
    for prec in ("fp32", "bf16"):
        ids, dist, st = hip.merge(*args, sample=20, delta=0.001, seed=2004, precision=prec)
        out[prec] = (ids.cpu().numpy(), dist.cpu().numpy(), st)
    return np.concatenate([S1, S2]), G1, G2, out


def test_lists_are_sorted_self_free_and_duplicate_free(w2):
    X, _, _, out = w2
    ids, dist, _ = out["fp32"]
    n = X.shape[0]
    assert ids.shape == (n, K) and (ids >= 0).all() and (ids < n).all()
    assert not (ids == np.arange(n)[:, None]).any()
    s = np.sort(ids, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()
    key = dist.astype(np.float64) * 2.0 ** 31 + ids          # (distance, id) order
    assert (np.diff(dist, axis=1) >= 0).all()
    tie = np.diff(dist, axis=1) == 0
    assert (np.diff(ids, axis=1)[tie] > 0).all()
    assert np.isfinite(key).all()


def test_stored_distances_are_canonical_and_exact(w2):
    # every stored value equals the oracle's canonical FP32 distance bit for
    # bit; on integer rows it also equals the FP64 value (relative error 0,
    # within the 1e-5 bound)
    X, _, _, out = w2
    ids, dist, _ = out["fp32"]
    rows = synth.rng(31).choice(X.shape[0], 200, replace=False)
    worst_rel = 0.0
    for i in rows:
        for j in range(K):
            c = oracle.dist32("l2", X[i], X[ids[i, j]])
            assert np.float32(c).view(np.uint32) == dist[i, j].view(np.uint32), (i, j)
            e = oracle.dist64("l2", X[i], X[ids[i, j]])
            worst_rel = max(worst_rel, abs(float(dist[i, j]) - e) / max(e, 1e-30))
    assert worst_rel <= 1e-5


def test_bf16_screen_gives_the_fp32_graph(w2):
    _, _, _, out = w2
    assert np.array_equal(out["fp32"][0], out["bf16"][0])
    assert np.array_equal(out["fp32"][1].view(np.uint32), out["bf16"][1].view(np.uint32))
    assert out["bf16"][2]["screen_violations"] == 0


def test_lists_only_improve_and_same_set_ids_come_from_the_input(w2):
    # S-Merge never compares two points of one set, so a row's same-set
    # neighbours are members of its input list; the merged list is the top k
    # of a superset of the input list, so it is elementwise no worse
    X, G1, G2, out = w2
    ids, dist, _ = out["fp32"]
    rows = synth.rng(32).choice(X.shape[0], 2000, replace=False)
    for i in rows:
        own1 = i < N1
        gi = G1[0][i] if own1 else G2[0][i - N1] + N1
        gd = G1[1][i] if own1 else G2[1][i - N1]
        assert (dist[i] <= gd).all()
        same = ids[i][(ids[i] < N1) == own1]
        assert set(same.tolist()) <= set(gi.tolist())


def test_recall_at_10(w2):
    import torch
    X, _, _, out = w2
    ids, _, st = out["fp32"]
    rows = synth.rng(2008).choice(X.shape[0], 1000, replace=False)
    Xd = torch.from_numpy(X).cuda().double()
    sq = (Xd * Xd).sum(1)
    hits = 0
    for lo in range(0, len(rows), 100):
        r = torch.from_numpy(rows[lo:lo + 100]).cuda()
        D = sq[r, None] + sq[None, :] - 2.0 * (Xd[r] @ Xd.T)    # exact on integer rows
        D[torch.arange(len(r), device="cuda"), r] = float("inf")
        kth = torch.topk(D, 10, dim=1, largest=False)[0][:, 9]
        got = torch.from_numpy(ids[rows[lo:lo + 100], :10].astype(np.int64)).cuda()
        hits += (torch.gather(D, 1, got) <= kth[:, None]).sum().item()
    assert hits / (len(rows) * 10) >= 0.95
    assert st["rounds"] < 30


# ---------------------------------------------------------------- cosine, d960

@pytest.fixture(scope="module")
def w3(hip):
    # 2 x 250,000 x d960 L2-normalised nonnegative rows, approximate k=20
    # inputs given without distances (the library computes them)
    import torch
    from synth.graphs import approximate_graph
    S1, S2 = synth.cosine_sets()
    G1 = approximate_graph(S1, K, 0.9, device="cuda", workload=3, stream=6)[0]
    G2 = approximate_graph(S2, K, 0.9, device="cuda", workload=3, stream=7)[0]
    d = lambda a: torch.from_numpy(a).cuda()
    args = (d(S1), (d(G1), None), d(S2), (d(G2), None), K, "cos")
    out = {}
    for prec in ("fp32", "bf16"):
        ids, dist, st = hip.merge(*args, sample=20, delta=0.001, seed=2007, precision=prec)
        out[prec] = (ids.cpu().numpy(), dist.cpu().numpy(), st)
    return np.concatenate([S1, S2]), out


def test_cosine_d960_valid_canonical_and_close_to_fp64(w3):
    X, out = w3
    ids, dist, _ = out["fp32"]
    n = X.shape[0]
    assert (ids >= 0).all() and (ids < n).all()
    assert not (ids == np.arange(n)[:, None]).any()
    s = np.sort(ids, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()
    assert (np.diff(dist, axis=1) >= 0).all()
    rows = synth.rng(33).choice(n, 100, replace=False)
    rel = []
    for i in rows:
        for j in range(K):
            c = oracle.dist32("cos", X[i], X[ids[i, j]])
            assert np.float32(c).view(np.uint32) == dist[i, j].view(np.uint32), (i, j)
            e = oracle.dist64("cos", X[i], X[ids[i, j]])
            rel.append(abs(float(dist[i, j]) - e) / max(e, 1e-3))
    # canonical FP32 against FP64: relative above 1e-3, absolute (scaled by
    # 1e-3) below; the sequential sum of 960 terms stays well inside 1e-5
    assert max(rel) <= 1e-5


def test_cosine_d960_bf16_screen_gives_the_fp32_graph(w3):
    _, out = w3
    assert np.array_equal(out["fp32"][0], out["bf16"][0])
    assert np.array_equal(out["fp32"][1].view(np.uint32), out["bf16"][1].view(np.uint32))
    assert out["bf16"][2]["screen_violations"] == 0
    assert out["bf16"][2]["rescored"] > 0
