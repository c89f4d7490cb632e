"""knng_merge_noalloc (the merge on the library's static scratch, for callers
that cannot allocate) gives exactly knng_merge's result: ids, distance bits
and per-round counters, on two calls in a row, the second smaller than the first (the
scratch keeps the first call's contents).  Its size limit and its refusal of
the profiling flag are checked before any device work."""
import numpy as np
import pytest

import synth
from test_gpu_parity import assert_same_graph, dev, host

pytestmark = pytest.mark.gpu


def _case(n1, n2, d, k, metric, seed):
    g = synth.rng(seed)
    S1 = g.standard_normal((n1, d)).astype(np.float32)
    S2 = (g.standard_normal((n2, d)) + 0.25).astype(np.float32)
    return S1, S2


def _both(hip, S1, S2, k, metric, **kw):
    dS1, dS2 = dev(S1), dev(S2)
    G1 = hip.exact_graph(dS1, k, metric)
    G2 = hip.exact_graph(dS2, k, metric)
    ref = hip.merge(dS1, G1, dS2, G2, k, metric, **kw)
    got = hip.merge_noalloc(dS1, G1, dS2, G2, k, metric, **kw)
    return ref, got


def _same(ref, got, what):
    ri, rd, rst = ref
    gi, gd, gst = got
    assert_same_graph(host(gi), host(gd), host(ri), host(rd), what)
    # the deterministic counters (rescores and insert attempts depend on the
    # order in which concurrent inserts lower the lists' bounds)
    for key in ("rounds", "c", "pairs", "evals"):
        assert gst[key] == rst[key], (what, key)


def test_noalloc_equals_merge_twice_second_smaller(hip):
    assert hip.noalloc_scratch_bytes() == 64 << 20
    print("\n[no-alloc] call 1: 9,000 + 7,000 x 48, k=16, l2, bf16", flush=True)
    S1, S2 = _case(9000, 7000, 48, 16, "l2", 501)
    need = hip.merge_workspace_size(9000, 7000, 48, 16, 16, 16, "l2", sample=12,
                                    precision="bf16")
    assert need <= hip.noalloc_scratch_bytes()
    ref, got = _both(hip, S1, S2, 16, "l2", sample=12, delta=0.001, seed=7, precision="bf16")
    _same(ref, got, "first call")
    print("[no-alloc] call 2: 2,500 + 2,100 x 19, k=10, cosine, fp32", flush=True)
    S1, S2 = _case(2500, 2100, 19, 10, "cos", 502)
    ref, got = _both(hip, S1, S2, 10, "cos", sample=8, seed=9)
    _same(ref, got, "second, smaller call")


def test_noalloc_refuses_what_it_cannot_hold(hip):
    from paper_1908_00814_amd.knng import KnngError
    S1, S2 = _case(300, 200, 8, 6, "l2", 503)
    dS1, dS2 = dev(S1), dev(S2)
    G1 = hip.exact_graph(dS1, 6)
    G2 = hip.exact_graph(dS2, 6)
    with pytest.raises(KnngError, match="EINVAL"):
        hip.merge_noalloc(dS1, G1, dS2, G2, 6, "l2", profile=True)
    # a merge whose workspace exceeds the scratch: rejected from its sizes,
    # before anything runs (the set only has to be large on paper: n and d
    # are read, the rows are not)
    big = hip.merge_workspace_size(400_000, 400_000, 128, 20, 20, 20, "l2", sample=20)
    assert big > hip.noalloc_scratch_bytes()
    import ctypes
    from paper_1908_00814_amd import knng
    lib = knng.load()
    s1 = knng.Set(400_000, 128, dS1.data_ptr())
    s2 = knng.Set(400_000, 128, dS2.data_ptr())
    g1 = knng.Graph(400_000, 20, G1[0].data_ptr(), G1[1].data_ptr())
    g2 = knng.Graph(400_000, 20, G2[0].data_ptr(), G2[1].data_ptr())
    out = knng.Graph(800_000, 20, G1[0].data_ptr(), G1[1].data_ptr())
    o = knng.opts(sample=20)
    rc = lib.knng_merge_noalloc(ctypes.byref(s1), ctypes.byref(g1), ctypes.byref(s2),
                                ctypes.byref(g2), 20, 0, ctypes.byref(o), ctypes.byref(out),
                                None, None)
    assert rc == 2 and b"scratch" in lib.knng_last_error()
    # the entry point still works after the refusals
    ref = hip.merge(dS1, G1, dS2, G2, 6, "l2", sample=5, seed=3)
    got = hip.merge_noalloc(dS1, G1, dS2, G2, 6, "l2", sample=5, seed=3)
    _same(ref, got, "after the refusals")
