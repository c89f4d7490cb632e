"""Pins of the oracle's graph diversification (Algorithm 3, Section 4) and of
its top-down search over a graph hierarchy (Section 4), against facts fixed
outside the oracle: a case worked by hand from the algorithm's rule
(tests/golden/), the path structure that the rule leaves on points of a
line, and exact answers where the search must find them.  No GPU."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_diversify_six_points_worked_by_hand():
    g = json.load(open(os.path.join(GOLDEN, "diversify_six_points.json")))
    X = np.array(g["points"], np.float32)
    G = oracle.exact_graph(X, g["k"], g["metric"])
    for cap, exp in g["expected"].items():
        ids, dist = oracle.diversify(X, G, int(cap), g["metric"])
        np.testing.assert_array_equal(ids, np.array(exp["ids"], np.int32))
        want = np.array([[np.inf if v is None else v for v in row] for row in exp["dist"]],
                        np.float32)
        np.testing.assert_array_equal(dist, want)


def test_diversify_keeps_a_candidate_as_far_from_a_kept_one_as_from_the_owner():
    g = json.load(open(os.path.join(GOLDEN, "diversify_tie.json")))
    X = np.array(g["points"], np.float32)
    G = oracle.exact_graph(X, g["k"], g["metric"])
    ids, dist = oracle.diversify(X, G, g["cap"], g["metric"])
    r = g["row"]
    assert ids[r].tolist() == g["ids"]
    np.testing.assert_array_equal(dist[r], np.array(g["dist"], np.float32))


@pytest.mark.parametrize("k", [2, 3, 7, 15])
def test_diversified_graph_of_a_line_keeps_the_nearest_on_each_side(k):
    # On distinct points of a line, Algorithm 3 applied to any candidate set
    # keeps exactly the nearest candidate on each side of the owner: a
    # farther candidate on the same side is closer to that one than to the
    # owner (occluded), and a candidate on the other side is farther from
    # every kept point of the first side than from the owner (never
    # occluded).  So the diversified list is the union of the nearest left
    # and right members of the list and of the reverse list.
    g = synth.rng(700 + k)
    x = g.permutation(4000)[:300].astype(np.float32)   # distinct integers
    X = x[:, None]
    G = oracle.exact_graph(X, k)
    ids, dist = oracle.diversify(X, G, 4)

    def sides(i, cand):
        out = []
        for side in (-1, 1):
            c = [j for j in cand if (x[j] - x[i]) * side > 0]
            if c:
                out.append(min(c, key=lambda j: ((x[i] - x[j]) ** 2, j)))
        return out

    for i in range(len(x)):
        rev = np.nonzero((G[0] == i).any(1))[0].tolist()
        want = sorted(set(sides(i, G[0][i].tolist()) + sides(i, rev)),
                      key=lambda j: ((x[i] - x[j]) ** 2, j))
        got = [v for v in ids[i] if v >= 0]
        assert got == want, (i, got, want)
        np.testing.assert_array_equal(dist[i, :len(want)],
                                      np.array([(x[i] - x[j]) ** 2 for j in want], np.float32))


def test_diversified_list_is_a_subset_of_list_and_reverse_list():
    X = synth.rng(711).standard_normal((400, 6)).astype(np.float32)
    G = oracle.exact_graph(X, 10)
    ids, dist = oracle.diversify(X, G, 6)
    for a in range(len(X)):
        fwd = set(G[0][a].tolist())
        rev = set(np.nonzero((G[0] == a).any(1))[0].tolist())
        got = [v for v in ids[a] if v >= 0]
        assert got and set(got) <= fwd | rev
        assert G[0][a][0] in got          # the nearest neighbour is always kept
        d = dist[a][:len(got)]
        assert np.all(np.diff(d) >= 0)


def _line_hierarchy(x, sizes):
    """layer graphs over prefixes of the points of a line: each vertex linked
    to its immediate left and right neighbours among the layer's points (the
    path of the line), built here with a sort"""
    layers = []
    for m in sizes:
        order = np.argsort(x[:m], kind="stable")
        adj = np.full((m, 2), -1, np.int32)
        adj[order[1:], 0] = order[:-1]
        adj[order[:-1], 1] = order[1:]
        layers.append(adj)
    return layers


@pytest.mark.parametrize("topk,ef", [(1, 1), (1, 8), (5, 5), (5, 16)])
def test_search_on_a_line_finds_the_exact_neighbours(topk, ef):
    # On a path over points of a line the distance to a query is unimodal
    # along the path, so the greedy descent of the upper layers and the
    # best-first bottom search reach the nearest points; the topk nearest
    # of a line form an interval around the query, found with ef >= topk.
    g = synth.rng(720)
    x = g.permutation(100_000)[:2000].astype(np.float32)
    layers = _line_hierarchy(x, [40, 250, 2000])
    q = (g.random(300) * 100_000).astype(np.float32)
    ids, dist, ev = oracle.search(x[:, None], layers, q[:, None], topk, ef, seed=3)
    for i in range(len(q)):
        d2 = (x.astype(np.float64) - q[i]) ** 2
        want = sorted(range(len(x)), key=lambda j: (np.float32(d2[j]), j))[:topk]
        assert ids[i].tolist() == want, i
    assert ev > 0


def test_upper_layers_descend_to_the_nearest_vertex_of_the_last_upper_layer():
    # a bottom layer without edges: the bottom search expands only the vertex
    # the upper layers reached, so the answer is where the greedy descent on
    # the paths of the upper layers ends, the nearest point of the second
    # layer's 250 points (the distance is unimodal along a path)
    g = synth.rng(725)
    x = g.permutation(100_000)[:2000].astype(np.float32)
    layers = _line_hierarchy(x, [40, 250]) + [np.full((2000, 2), -1, np.int32)]
    q = (g.random(300) * 100_000).astype(np.float32)
    ids, dist, ev = oracle.search(x[:, None], layers, q[:, None], 1, 4, seed=9)
    for i in range(len(q)):
        d2 = (x[:250].astype(np.float64) - q[i]) ** 2
        want = min(range(250), key=lambda j: (np.float32(d2[j]), j))
        assert ids[i, 0] == want, i


def test_search_with_a_complete_bottom_graph_and_a_full_list_is_exact():
    # every vertex is a neighbour of every other and the ranked list holds
    # all of them: the answer is the brute-force top k by (distance, id)
    g = synth.rng(730)
    X = g.integers(0, 20, size=(120, 5)).astype(np.float32)
    Q = g.integers(0, 20, size=(40, 5)).astype(np.float32)
    full = oracle.exact_graph(X, 119)[0]
    top = oracle.diversify(X[:30], oracle.exact_graph(X[:30], 8), 4)[0]
    ids, dist, _ = oracle.search(X, [top, full], Q, 10, 120, seed=5)
    D = ((Q[:, None, :].astype(np.int64) - X[None, :, :].astype(np.int64)) ** 2).sum(-1)
    for i in range(len(Q)):
        want = sorted(range(len(X)), key=lambda j: (D[i, j], j))[:10]
        assert ids[i].tolist() == want
        np.testing.assert_array_equal(dist[i], D[i, want].astype(np.float32))


def test_search_start_depends_on_the_seed_and_the_answer_is_reproducible():
    g = synth.rng(740)
    X = g.standard_normal((500, 4)).astype(np.float32)
    Q = g.standard_normal((50, 4)).astype(np.float32)
    layers = [oracle.diversify(X[:m], oracle.exact_graph(X[:m], 8), 6)[0] for m in (60, 500)]
    a = oracle.search(X, layers, Q, 3, 12, seed=1)
    b = oracle.search(X, layers, Q, 3, 12, seed=1)
    c = oracle.search(X, layers, Q, 3, 12, seed=2)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[2] == b[2] and a[2] != c[2]


def test_hierarchy_layers_are_the_ones_hmerge_builds():
    # the kept layers are H-Merge's own: the bottom one, mapped back to row
    # numbers and sorted, is hmerge's answer; layer sizes follow the schedule
    X = synth.rng(750).standard_normal((700, 5)).astype(np.float32)
    order, layers = oracle.hmerge_hierarchy(X, 8, 60, sample=6, seed=4)
    sched = oracle.hmerge_layers(700, 60, 8)
    assert [(L[0].shape[0], L[0].shape[1]) for L in layers] == sched
    ids, dist, _ = oracle.hmerge(X, 8, 60, sample=6, seed=4)
    bi, bd = layers[-1]
    rid = order[bi]
    srt = np.lexsort((rid, bd), axis=1)
    got_i = np.empty_like(rid)
    got_d = np.empty_like(bd)
    got_i[order] = np.take_along_axis(rid, srt, axis=1)
    got_d[order] = np.take_along_axis(bd, srt, axis=1)
    np.testing.assert_array_equal(got_i, ids)
    np.testing.assert_array_equal(got_d, dist)
