"""GPU parity of the hierarchy (H-Merge keeping its layers), graph
diversification (Algorithm 3) and the top-down search (Section 4) with the
oracle: identical ids, bit-identical distances."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import assert_same_graph, dev, host

pytestmark = pytest.mark.gpu


def _gauss(n, d, seed, shift=0.0):
    return (synth.rng(seed).standard_normal((n, d)) + shift).astype(np.float32)


@pytest.mark.parametrize("metric", ["l2", "l1", "cos"])
def test_diversify_identical_to_oracle(hip, metric):
    X = _gauss(1501, 13, 801)
    G = oracle.exact_graph(X, 10, metric)
    oi, od = oracle.diversify(X, G, 6, metric)
    gi, gd = hip.diversify(dev(X), (dev(G[0]), dev(G[1])), 6, metric)
    assert_same_graph(host(gi), host(gd), oi, od, f"diversify {metric}")


def test_diversify_hub_rows_and_padding(hip):
    # rows 0 and 1 sit in every list (in-degree ~n: many 64-candidate chunks of
    # reverse list), some lists are short (padded with -1), k = 24, cap 12
    X = _gauss(900, 9, 802)
    ids, dist = oracle.exact_graph(X, 24)
    ids, dist = ids.copy(), dist.copy()
    for a in range(2, len(X)):
        row = [(float(dist[a, j]), int(ids[a, j])) for j in range(24) if ids[a, j] not in (0, 1)]
        row = row[:20] + [(oracle.dist32("l2", X[a], X[h]), h) for h in (0, 1)]
        if a % 7 == 0:
            row = row[:9]
        row.sort(key=lambda e: (np.float32(e[0]), e[1]))
        ids[a] = [e[1] for e in row] + [-1] * (24 - len(row))
        dist[a] = [e[0] for e in row] + [np.inf] * (24 - len(row))
    oi, od = oracle.diversify(X, (ids, dist), 12)
    gi, gd = hip.diversify(dev(X), (dev(ids), dev(dist)), 12)
    assert_same_graph(host(gi), host(gd), oi, od, "diversify hubs")


@pytest.mark.parametrize("metric", ["l2", "cos"])
def test_hierarchy_identical_to_oracle(hip, metric):
    X = _gauss(2300, 11, 803)
    order, layers = oracle.hmerge_hierarchy(X, 12, 150, metric, sample=8, seed=21)
    perm, xp, glayers, _ = hip.hmerge_hierarchy(dev(X), 12, 150, metric, sample=8, seed=21)
    np.testing.assert_array_equal(host(perm), order)
    np.testing.assert_array_equal(host(xp), X[order])
    assert len(glayers) == len(layers)
    for l, ((oi, od), (gi, gd)) in enumerate(zip(layers, glayers)):
        assert_same_graph(host(gi), host(gd), oi, od, f"layer {l}")


@pytest.mark.parametrize("metric,ef,topk", [("l2", 16, 1), ("l2", 64, 10), ("cos", 32, 5),
                                            ("l1", 48, 3)])
def test_search_identical_to_oracle(hip, metric, ef, topk):
    X = _gauss(3000, 16, 804)
    Q = _gauss(400, 16, 805, 0.1)
    order, layers = oracle.hmerge_hierarchy(X, 16, 100, metric, sample=8, seed=5)
    Xp = X[order]
    div = [oracle.diversify(Xp[:L[0].shape[0]], L, 8, metric)[0] for L in layers]
    oi, od, oev = oracle.search(Xp, div, Q, topk, ef, seed=77, metric=metric)
    gi, gd, gev = hip.search(dev(Xp), [dev(a) for a in div], dev(Q), topk, ef, seed=77,
                             metric=metric)
    assert_same_graph(host(gi), host(gd), oi, od, f"search {metric}")
    assert gev == oev


def test_search_full_list_over_a_complete_graph_is_exact(hip):
    # ef = 256 (the kernel's largest list) over a complete bottom graph of 256
    # rows: the answer is the brute-force top k
    g = synth.rng(806)
    X = g.integers(0, 30, size=(256, 6)).astype(np.float32)
    Q = g.integers(0, 30, size=(70, 6)).astype(np.float32)
    full = oracle.exact_graph(X, 255)[0]
    top = oracle.diversify(X[:40], oracle.exact_graph(X[:40], 8), 6)[0]
    gi, gd, _ = hip.search(dev(X), [dev(top), dev(full)], dev(Q), 12, 256, seed=1)
    oi, od, _ = oracle.search(X, [top, full], Q, 12, 256, seed=1)
    assert_same_graph(host(gi), host(gd), oi, od, "complete graph")
    D = ((Q[:, None, :].astype(np.int64) - X[None].astype(np.int64)) ** 2).sum(-1)
    for i in range(len(Q)):
        assert host(gi)[i].tolist() == sorted(range(256), key=lambda j: (D[i, j], j))[:12]
