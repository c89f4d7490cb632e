"""GPU parity of the exact-arithmetic shortcuts for rows certified exact
(integer coordinates in [0, 256], squared norm below 2^23): l2 distances summed
by several lanes over the bf16 rows, in input preparation (lists given without
distances) and in Append, and the fall-back to one lane per distance in
canonical order when a row involved is not certified or a list is too long.
Against the oracle's canonical FP32 distances: identical graphs, bit-identical
distances and identical per-round counters."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import _same_stats, assert_same_graph, dev, host

pytestmark = pytest.mark.gpu


def _byte_sets(n1, n2, d, seed):
    g = synth.rng(seed)
    S1 = g.integers(0, 256, size=(n1, d)).astype(np.float32)
    S2 = g.integers(0, 256, size=(n2, d)).astype(np.float32)
    return S1, S2


def _merge_without_distances(hip, S1, S2, k, kin, sample, seed, what):
    G1 = oracle.exact_graph(S1, kin)
    G2 = oracle.exact_graph(S2, kin)
    # the lists come without distances and out of order: the library computes
    # and sorts them
    p = synth.rng(seed).permutation(kin)
    G1n, G2n = (G1[0][:, p], None), (G2[0][:, p], None)
    oi, od, ost = oracle.smerge(S1, G1n, S2, G2n, k, "l2", sample=sample, seed=seed)
    gi, gd, gst = hip.merge(dev(S1), (dev(G1n[0]), None), dev(S2), (dev(G2n[0]), None), k, "l2",
                            sample=sample, seed=seed, precision="bf16")
    assert_same_graph(host(gi), host(gd), oi, od, what)
    _same_stats(gst, ost)


def test_certified_rows(hip):
    # every row certified: input distances two lanes each, Append four lanes
    S1, S2 = _byte_sets(700, 650, 40, 901)
    _merge_without_distances(hip, S1, S2, 12, 12, 8, 31, "certified")


def test_rows_without_certificate_fall_back(hip):
    # a half-integer coordinate or one above 256 takes a row's certificate
    # away; every list holding such a row, and the row's own, is evaluated one
    # lane per distance in canonical order
    S1, S2 = _byte_sets(700, 650, 40, 902)
    for r in (0, 5, 77, 300, 699):
        S1[r, r % 40] += 0.5
    for r in (10, 11, 400):
        S2[r, 3] = 300.0
    _merge_without_distances(hip, S1, S2, 12, 12, 8, 32, "mixed certificates")


def test_long_lists_fall_back(hip):
    # k = 40: more list entries than two lanes each can take (32) and more
    # drawn partners than four lanes each can take (16)
    S1, S2 = _byte_sets(520, 480, 24, 903)
    _merge_without_distances(hip, S1, S2, 40, 40, 20, 33, "long lists")
