"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

The merges are deterministic by construction (hash-priority sampling,
set-semantics inserts, canonical FP32 distances), so the bar here is
identity: the same ids in the same order and bit-identical distances, plus
the same per-round counters.  Sizes span several tiles/workgroups and ragged
tails (d not a multiple of 4, n not a multiple of 64)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def assert_same_graph(gi, gd, oi, od, what=""):
    if not np.array_equal(gi, oi):
        bad = np.argwhere(np.any(gi != oi, axis=1))[:, 0]
        r = bad[0]
        raise AssertionError(f"{what}: {len(bad)} rows differ in ids; first row {r}:\n"
                             f" gpu    {gi[r].tolist()}\n {gd[r].tolist()}\n"
                             f" oracle {oi[r].tolist()}\n {od[r].tolist()}")
    diff = gd.view(np.uint32) != od.view(np.uint32)
    if np.any(diff):
        r, c = np.argwhere(diff)[0]
        raise AssertionError(f"{what}: distances differ at ({r},{c}): {gd[r, c]!r} vs "
                             f"{od[r, c]!r}")


def ragged_sets(n1, n2, d, seed):
    g = synth.rng(seed)
    S1 = g.standard_normal((n1, d)).astype(np.float32)
    S2 = (g.standard_normal((n2, d)) + 0.3).astype(np.float32)
    return S1, S2


# ---------------------------------------------------------------- exact graph

@pytest.mark.parametrize("metric", ["l2", "l1", "cos"])
def test_exact_graph_bit_exact(hip, metric):
    X = synth.rng(101).standard_normal((333, 37)).astype(np.float32)
    oi, od = oracle.exact_graph(X, 7, metric)
    gi, gd = hip.exact_graph(dev(X), 7, metric)
    assert_same_graph(host(gi), host(gd), oi, od, f"exact {metric}")


def test_exact_graph_integer_ties(hip):
    # many equal distances: the order must follow ids exactly
    X = synth.rng(102).integers(0, 3, size=(257, 4)).astype(np.float32)
    oi, od = oracle.exact_graph(X, 12, "l2")
    gi, gd = hip.exact_graph(dev(X), 12, "l2")
    assert_same_graph(host(gi), host(gd), oi, od, "exact ties")


# ---------------------------------------------------------------- brute-force merge

@pytest.mark.parametrize("metric", ["l2", "l1", "cos"])
def test_bruteforce_merge_bit_exact(hip, metric):
    S1, S2 = ragged_sets(301, 190, 13, 103)
    G1 = oracle.exact_graph(S1, 9, metric)
    G2 = oracle.exact_graph(S2, 6, metric)
    oi, od = oracle.merge_bruteforce(S1, G1, S2, G2, 9, metric)
    gi, gd = hip.merge_bruteforce(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2),
                                  (dev(G2[0]), dev(G2[1])), 9, metric)
    assert_same_graph(host(gi), host(gd), oi, od, f"bruteforce {metric}")


def test_bruteforce_merge_workload1(hip):
    # two sets of 5,000 x 32 N(0,1), exact k=10 inputs, merged to k=10
    S1, S2 = synth.gaussian_sets(5000, 5000, 32)
    G1 = oracle.exact_graph(S1, 10)
    G2 = oracle.exact_graph(S2, 10)
    oi, od = oracle.merge_bruteforce(S1, G1, S2, G2, 10)
    gi, gd = hip.merge_bruteforce(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2),
                                  (dev(G2[0]), dev(G2[1])), 10)
    assert_same_graph(host(gi), host(gd), oi, od, "bruteforce W1")
    # and it equals the exact graph of the union (merging exact graphs)
    ei, ed = oracle.exact_graph(np.concatenate([S1, S2]), 10)
    assert_same_graph(host(gi), host(gd), ei, ed, "bruteforce W1 vs exact")


# ---------------------------------------------------------------- S-Merge

def _smerge_both(hip, S1, S2, G1, G2, k, metric, **kw):
    oi, od, ost = oracle.smerge(S1, G1, S2, G2, k, metric, **kw)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1[0]), None if G1[1] is None else dev(G1[1])),
                            dev(S2), (dev(G2[0]), None if G2[1] is None else dev(G2[1])), k,
                            metric, **kw)
    return (host(gi), host(gd), gst), (oi, od, ost)


def _same_stats(gst, ost):
    assert gst["rounds"] == ost["rounds"]
    assert gst["c"] == ost["c"], (gst["c"], ost["c"])
    assert gst["pairs"] == ost["pairs"]
    assert gst["evals"] == ost["evals"]


@pytest.mark.parametrize("metric", ["l2", "l1", "cos"])
def test_smerge_identical_to_oracle(hip, metric):
    S1, S2 = ragged_sets(700, 513, 19, 104)
    G1 = oracle.exact_graph(S1, 10, metric)
    G2 = oracle.exact_graph(S2, 10, metric)
    (gi, gd, gst), (oi, od, ost) = _smerge_both(hip, S1, S2, G1, G2, 10, metric, sample=8,
                                                seed=77)
    assert_same_graph(gi, gd, oi, od, f"smerge {metric}")
    _same_stats(gst, ost)


def test_smerge_recomputed_distances_and_unequal_k(hip):
    # input lists without distances (computed and sorted by the library),
    # G1 with more columns than G2, odd k and a non-default keep ratio
    S1, S2 = ragged_sets(420, 380, 11, 105)
    G1 = oracle.exact_graph(S1, 12)
    G2 = oracle.exact_graph(S2, 8)
    perm = synth.rng(5).permutation(12)
    G1n = (G1[0][:, perm], None)
    (gi, gd, gst), (oi, od, ost) = _smerge_both(hip, S1, S2, G1n, (G2[0], None), 9, "l2",
                                                sample=6, keep_ratio=0.34, seed=3)
    assert_same_graph(gi, gd, oi, od, "smerge recompute")
    _same_stats(gst, ost)


def test_smerge_workload1_full(hip):
    # the small benchmark workload: 2 x 5,000 x 32, exact k=10 inputs,
    # sample size 10, seed 1004
    S1, S2 = synth.gaussian_sets(5000, 5000, 32)
    G1 = oracle.exact_graph(S1, 10)
    G2 = oracle.exact_graph(S2, 10)
    (gi, gd, gst), (oi, od, ost) = _smerge_both(hip, S1, S2, G1, G2, 10, "l2", sample=10,
                                                seed=1004)
    assert_same_graph(gi, gd, oi, od, "smerge W1")
    _same_stats(gst, ost)


def test_smerge_delta_and_round_cap(hip):
    S1, S2 = ragged_sets(300, 300, 8, 106)
    G1 = oracle.exact_graph(S1, 8)
    G2 = oracle.exact_graph(S2, 8)
    for kw in ({"delta": 0.01}, {"max_rounds": 2}, {"max_rounds": 0}):
        (gi, gd, gst), (oi, od, ost) = _smerge_both(hip, S1, S2, G1, G2, 8, "l2", sample=5,
                                                    seed=9, **kw)
        assert_same_graph(gi, gd, oi, od, f"smerge {kw}")
        _same_stats(gst, ost)


# ---------------------------------------------------------------- J-Merge

def _jmerge_both(hip, Sb, G, Sr, k, metric, **kw):
    oi, od, ost = oracle.jmerge(Sb, G, Sr, k, metric, **kw)
    gG = None if G is None else (dev(G[0]), None if G[1] is None else dev(G[1]))
    gi, gd, gst = hip.expand(None if Sb is None else dev(Sb), gG, dev(Sr), k, metric, **kw)
    return (host(gi), host(gd), gst), (oi, od, ost)


@pytest.mark.parametrize("metric", ["l2", "cos", "l1"])
def test_jmerge_identical_to_oracle(hip, metric):
    Sb, Sr = ragged_sets(650, 277, 21, 107)
    G = oracle.exact_graph(Sb, 10, metric)
    (gi, gd, gst), (oi, od, ost) = _jmerge_both(hip, Sb, G, Sr, 10, metric, sample=7, seed=5)
    assert_same_graph(gi, gd, oi, od, f"jmerge {metric}")
    _same_stats(gst, ost)


def test_nn_descent_from_empty_base(hip):
    X = synth.rng(108).standard_normal((900, 9)).astype(np.float32)
    (gi, gd, gst), (oi, od, ost) = _jmerge_both(hip, None, None, X, 10, "l2", sample=10,
                                                seed=2)
    assert_same_graph(gi, gd, oi, od, "nn-descent")
    _same_stats(gst, ost)


def test_jmerge_tiny_raw_set(hip):
    # one raw point: each base list gets that point appended
    Sb, Sr = ragged_sets(200, 1, 6, 109)
    G = oracle.exact_graph(Sb, 8)
    (gi, gd, gst), (oi, od, ost) = _jmerge_both(hip, Sb, G, Sr, 8, "l2", sample=4, seed=1)
    assert_same_graph(gi, gd, oi, od, "jmerge tiny raw")


@pytest.mark.parametrize("metric", ["l2", "cos", "l1"])
def test_jmerge_balanced_identical_to_oracle(hip, metric):
    # a raw set far smaller than the base: only hash-selected base rows are
    # divided and appended to; rows that never see a NEW member are skipped
    Sb, Sr = ragged_sets(1500, 70, 13, 114)
    G = oracle.exact_graph(Sb, 10, metric)
    (gi, gd, gst), (oi, od, ost) = _jmerge_both(hip, Sb, G, Sr, 10, metric, sample=7, seed=6,
                                                balanced=True)
    assert_same_graph(gi, gd, oi, od, f"jmerge balanced {metric}")
    _same_stats(gst, ost)


def test_jmerge_balanced_wide_input_delta_and_bf16(hip):
    # input lists wider than k and without distances, a delta stop relative
    # to the rows that start with NEW entries, and the BF16 screen
    Sb, Sr = ragged_sets(900, 41, 20, 115)
    G = oracle.exact_graph(Sb, 12)
    G = (G[0][:, synth.rng(6).permutation(12)], None)
    for kw in ({"delta": 0.02}, {"precision": "bf16"}, {"max_rounds": 1}):
        okw = {a: b for a, b in kw.items() if a != "precision"}
        oi, od, ost = oracle.jmerge(Sb, G, Sr, 9, "l2", sample=5, seed=8, balanced=True, **okw)
        gi, gd, gst = hip.expand(dev(Sb), (dev(G[0]), None), dev(Sr), 9, "l2", sample=5, seed=8,
                                 balanced=True, **kw)
        assert_same_graph(host(gi), host(gd), oi, od, f"jmerge balanced {kw}")
        _same_stats(gst, ost)


# ---------------------------------------------------------------- behaviour

def test_deterministic_repeat(hip):
    S1, S2 = ragged_sets(900, 800, 16, 110)
    G1 = oracle.exact_graph(S1, 10)
    G2 = oracle.exact_graph(S2, 10)
    args = (dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2), (dev(G2[0]), dev(G2[1])), 10)
    a = hip.merge(*args, sample=6, seed=4)
    b = hip.merge(*args, sample=6, seed=4)
    assert np.array_equal(host(a[0]), host(b[0]))
    assert np.array_equal(host(a[1]).view(np.uint32), host(b[1]).view(np.uint32))


def test_invalid_inputs_raise(hip):
    import torch
    S1, S2 = ragged_sets(50, 40, 4, 111)
    G1 = oracle.exact_graph(S1, 6)
    G2 = oracle.exact_graph(S2, 6)
    bad = G1[0].copy()
    bad[3, 2] = bad[3, 1]
    with pytest.raises(hip.KnngError, match="EINVAL"):
        hip.merge(dev(S1), (dev(bad), None), dev(S2), (dev(G2[0]), None), 6)
    bad = G1[0].copy()
    bad[7, 0] = 7
    with pytest.raises(hip.KnngError, match="itself"):
        hip.merge(dev(S1), (dev(bad), None), dev(S2), (dev(G2[0]), None), 6)
    bad = G1[0].copy()
    bad[0, 0] = 50
    with pytest.raises(hip.KnngError, match="range"):
        hip.merge(dev(S1), (dev(bad), None), dev(S2), (dev(G2[0]), None), 6)
    d = G1[1].copy()
    d[1] = d[1][::-1]
    with pytest.raises(hip.KnngError, match="sorted"):
        hip.merge(dev(S1), (dev(G1[0]), dev(d)), dev(S2), (dev(G2[0]), dev(G2[1])), 6)
    Z = S1.copy()
    Z[4, 1] = np.nan
    with pytest.raises(hip.KnngError, match="finite"):
        hip.merge(dev(Z), (dev(G1[0]), None), dev(S2), (dev(G2[0]), None), 6)
    Z = S1.copy()
    Z[4] = 0
    with pytest.raises(hip.KnngError, match="zero norm"):
        hip.merge(dev(Z), (dev(G1[0]), None), dev(S2), (dev(G2[0]), None), 6, "cos")
    with pytest.raises(hip.KnngError, match="k ="):
        hip.merge(dev(S1), (dev(G1[0]), None), dev(S2), (dev(G2[0]), None), 100)
    with pytest.raises(hip.KnngError, match="device"):
        _host_pointer_call(hip, S1, G1, S2, G2)
    # after errors the library still works
    gi, gd, _ = hip.merge(dev(S1), (dev(G1[0]), None), dev(S2), (dev(G2[0]), None), 6)
    assert host(gi).shape == (90, 6)


def _host_pointer_call(hip, S1, G1, S2, G2):
    import ctypes
    lib = hip.load()
    s1 = hip.Set(S1.shape[0], S1.shape[1], S1.ctypes.data)  # host memory
    s2 = hip.Set(S2.shape[0], S2.shape[1], S2.ctypes.data)
    g = hip.Graph(0, 0, None, None)
    o = hip.opts()
    rc = lib.knng_merge(ctypes.byref(s1), ctypes.byref(g), ctypes.byref(s2), ctypes.byref(g), 6,
                        0, ctypes.byref(o), ctypes.byref(g), None, 0, None, None)
    hip._check(rc)


# ---------------------------------------------------------------- BF16-MFMA screen

@pytest.mark.parametrize("metric", ["l2", "cos"])
def test_bf16_smerge_identical_to_oracle(hip, metric):
    # MFMA screen + canonical FP32 rescore gives the FP32 path's result exactly
    S1, S2 = ragged_sets(700, 513, 19, 104)
    G1 = oracle.exact_graph(S1, 10, metric)
    G2 = oracle.exact_graph(S2, 10, metric)
    oi, od, ost = oracle.smerge(S1, G1, S2, G2, 10, metric, sample=8, seed=77)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2), (dev(G2[0]), dev(G2[1])),
                            10, metric, sample=8, seed=77, precision="bf16")
    assert_same_graph(host(gi), host(gd), oi, od, f"bf16 smerge {metric}")
    _same_stats(gst, ost)
    assert gst["screen_violations"] == 0
    assert 0 < gst["rescored"] < sum(gst["pairs"])


def test_bf16_integer_data_and_large_d(hip):
    # byte-valued rows (bf16-exact) at d = 128, the benchmark's value law
    X = synth.byte_cluster_points(1500, 128, 12, 20.0, workload=2)
    S1, S2 = X[:800], X[800:]
    G1 = oracle.exact_graph(S1, 12)
    G2 = oracle.exact_graph(S2, 12)
    oi, od, ost = oracle.smerge(S1, G1, S2, G2, 12, sample=6, seed=3)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2), (dev(G2[0]), dev(G2[1])),
                            12, sample=6, seed=3, precision="bf16")
    assert_same_graph(host(gi), host(gd), oi, od, "bf16 integer")
    _same_stats(gst, ost)
    assert gst["screen_violations"] == 0


@pytest.mark.parametrize("metric", ["l2", "cos"])
def test_bf16_jmerge_identical_to_oracle(hip, metric):
    Sb, Sr = ragged_sets(650, 277, 21, 107)
    G = oracle.exact_graph(Sb, 10, metric)
    oi, od, ost = oracle.jmerge(Sb, G, Sr, 10, metric, sample=7, seed=5)
    gi, gd, gst = hip.expand(dev(Sb), (dev(G[0]), dev(G[1])), dev(Sr), 10, metric, sample=7,
                             seed=5, precision="bf16")
    assert_same_graph(host(gi), host(gd), oi, od, f"bf16 jmerge {metric}")
    _same_stats(gst, ost)
    assert gst["screen_violations"] == 0


def test_bf16_l1_runs_the_fp32_path(hip):
    S1, S2 = ragged_sets(300, 200, 9, 112)
    G1 = oracle.exact_graph(S1, 8, "l1")
    G2 = oracle.exact_graph(S2, 8, "l1")
    oi, od, _ = oracle.smerge(S1, G1, S2, G2, 8, "l1", sample=5, seed=2)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2), (dev(G2[0]), dev(G2[1])),
                            8, "l1", sample=5, seed=2, precision="bf16")
    assert_same_graph(host(gi), host(gd), oi, od, "bf16 l1")
    assert gst["rescored"] == 0


# ---------------------------------------------------------------- merge tree

@pytest.mark.parametrize("sizes,metric", [((300, 257, 310, 280), "l1"), ((260, 240, 301), "l2")])
def test_merge_tree_identical_to_oracle(hip, sizes, metric):
    # blocks merged pairwise level by level (an odd block moves up unchanged)
    g = synth.rng(113)
    X = np.concatenate([(g.standard_normal((n, 10)) + 0.5 * b).astype(np.float32)
                        for b, n in enumerate(sizes)])
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    graphs = [oracle.exact_graph(X[starts[b]:starts[b + 1]], 8, metric) for b in range(len(sizes))]
    oi, od = oracle.merge_tree(X, starts, graphs, 8, metric, sample=6, seed=21)
    gi, gd, gst = hip.merge_tree(dev(X), starts, [(dev(a), dev(b)) for a, b in graphs], 8, metric,
                                 sample=6, seed=21)
    assert_same_graph(host(gi), host(gd), oi, od, f"merge tree {metric}")
    assert len(gst["level_rounds"]) == (2 if len(sizes) == 4 else 2)


# ---------------------------------------------------------------- H-Merge

@pytest.mark.parametrize("metric", ["l2", "l1", "cos"])
def test_hmerge_identical_to_oracle(hip, metric):
    # layers of 150, 300, 600, 1200, 2400 and 2,517 rows (a ragged last block)
    X = synth.rng(131).standard_normal((2517, 9)).astype(np.float32) + 0.25
    oi, od, ost = oracle.hmerge(X, 10, 150, metric, sample=6, seed=41)
    gi, gd, gst = hip.hmerge(dev(X), 10, 150, metric, sample=6, seed=41)
    assert_same_graph(host(gi), host(gd), oi, od, f"hmerge {metric}")
    assert gst["layer_rounds"] == [s["rounds"] for s in ost]
    assert gst["layer_evals"] == [s["evals"] for s in ost]
    assert gst["evals"] == sum(s["evals"] for s in ost)


def test_hmerge_exact_when_lists_hold_every_row(hip):
    # k = n - 1 with n = 4 n_top: every layer starts from lists holding every
    # other row, so the result is the exact graph
    X = synth.rng(132).standard_normal((64, 7)).astype(np.float32)
    gi, gd, _ = hip.hmerge(dev(X), 63, 16, "l2", sample=5, seed=3)
    ei, ed = oracle.exact_graph(X, 63)
    assert_same_graph(host(gi), host(gd), ei, ed, "hmerge exact")


def test_hmerge_single_layer_and_bf16(hip):
    # n_top >= n: one NN-Descent layer; the BF16 screen gives the same graph
    X = synth.rng(133).standard_normal((700, 24)).astype(np.float32)
    oi, od, _ = oracle.hmerge(X, 8, 5000, "l2", sample=6, seed=8)
    for prec in ("fp32", "bf16"):
        gi, gd, gst = hip.hmerge(dev(X), 8, 5000, "l2", sample=6, seed=8, precision=prec)
        assert_same_graph(host(gi), host(gd), oi, od, f"hmerge one layer {prec}")
        assert len(gst["layer_rounds"]) == 1


def test_hmerge_invalid_inputs(hip):
    X = synth.rng(134).standard_normal((100, 4)).astype(np.float32)
    with pytest.raises(hip.KnngError, match="EINVAL"):
        hip.hmerge(dev(X), 8, 1, "l2")                  # top layer of one row
    with pytest.raises(hip.KnngError, match="EINVAL"):
        hip.hmerge(dev(X), 8, 10, "l2", keep_ratio=0.9)  # keeps more than a k/2 layer holds
    with pytest.raises(hip.KnngError, match="EINVAL"):
        hip.hmerge(dev(X), 100, 10, "l2")               # k > n - 1


# ---------------------------------------------------------------- limits

@pytest.mark.parametrize("case", ["k64_s32", "d1", "one_row_set", "k_near_n"])
def test_smerge_limits_identical_to_oracle(hip, case):
    # the largest list and sample (3s + k = 160 members per neighbourhood),
    # one coordinate, a second set of one row, and k close to n - 1
    g = synth.rng(150)
    if case == "k64_s32":
        n1, n2, d, k, s, kin1, kin2 = 400, 333, 3, 64, 32, 64, 64
    elif case == "d1":
        n1, n2, d, k, s, kin1, kin2 = 300, 257, 1, 12, 8, 12, 12
    elif case == "one_row_set":
        n1, n2, d, k, s, kin1, kin2 = 60, 1, 5, 10, 6, 10, 0
    else:
        n1, n2, d, k, s, kin1, kin2 = 20, 18, 6, 33, 10, 19, 17
    S1 = g.standard_normal((n1, d)).astype(np.float32)
    S2 = (g.standard_normal((n2, d)) + 0.5).astype(np.float32)
    if case == "one_row_set":
        # a one-row set has no neighbours of its own: merged as the raw side
        # of J-Merge instead
        G = oracle.exact_graph(S1, kin1)
        (gi, gd, gst), (oi, od, ost) = _jmerge_both(hip, S1, G, S2, k, "l2", sample=s, seed=4)
        assert_same_graph(gi, gd, oi, od, case)
        return
    G1 = oracle.exact_graph(S1, kin1)
    G2 = oracle.exact_graph(S2, kin2)
    precs = ("fp32", "bf16") if case == "k64_s32" else ("fp32",)
    oi, od, ost = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s, seed=12)
    for prec in precs:
        gi, gd, gst = hip.merge(dev(S1), (dev(G1[0]), dev(G1[1])), dev(S2),
                                (dev(G2[0]), dev(G2[1])), k, "l2", sample=s, seed=12,
                                precision=prec)
        assert_same_graph(host(gi), host(gd), oi, od, f"{case} {prec}")
        _same_stats(gst, ost)


def test_union_above_id_range_rejected(hip):
    # each set is in range, their union is not: rejected before any row or
    # list is read (the sets point at a few device bytes)
    import ctypes
    import torch
    lib = hip.load()
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    half = (1 << 29) - 8
    s1 = hip.Set(half, 1, x.data_ptr())
    s2 = hip.Set(half, 1, x.data_ptr())
    g = hip.Graph(0, 0, None, None)
    o = hip.opts()
    rc = lib.knng_merge(ctypes.byref(s1), ctypes.byref(g), ctypes.byref(s2), ctypes.byref(g), 6,
                        0, ctypes.byref(o), ctypes.byref(g), None, 0, None, None)
    with pytest.raises(hip.KnngError, match="rows out of range"):
        hip._check(rc)
    rc = lib.knng_expand(ctypes.byref(s1), ctypes.byref(g), ctypes.byref(s2), 6, 0,
                         ctypes.byref(o), ctypes.byref(g), None, 0, None, None)
    with pytest.raises(hip.KnngError, match="rows out of range"):
        hip._check(rc)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reverse_hub_reservoirs(hip, precision):
    # every list holds its set's row 0, so the reverse reservoirs of the two
    # hubs get thousands of offers each: one wave mixes the first s offers
    # (slot claims) with later ones, which wait until every claimed slot is
    # written; identical to the oracle
    S1, S2 = ragged_sets(3000, 2500, 16, 121)
    G1 = oracle.exact_graph(S1, 8)[0].copy()
    G2 = oracle.exact_graph(S2, 8)[0].copy()
    for G in (G1, G2):
        rows = np.arange(1, G.shape[0])
        has = (G[1:] == 0).any(axis=1)
        G[rows[~has], -1] = 0
    assert all((G == 0).any(axis=1)[1:].all() for G in (G1, G2))
    oi, od, ost = oracle.smerge(S1, (G1, None), S2, (G2, None), 8, "l2", sample=5, seed=12)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1), None), dev(S2), (dev(G2), None), 8, "l2",
                            sample=5, seed=12, precision=precision)
    assert_same_graph(host(gi), host(gd), oi, od, f"hub reservoirs {precision}")
    _same_stats(gst, ost)
