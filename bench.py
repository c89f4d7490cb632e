#!/usr/bin/env python3
"""Benchmark: symmetric merge (S-Merge, Algorithm 1 of Zhao et al., "On the
Merge of k-NN Graph") of two byte-valued cluster sets of 500,000 x 128 with
approximate k=20 input graphs, merged to k=20 under squared l2, on one MI355X.

A step is one whole merge call (layout, Divide/Append, all rounds of the
repeat loop, Merge and Sort) with inputs already resident in HBM.  The value
is points merged per second.  After the timed steps the script
  - checks recall@10 of the merged graph on 1,000 sampled rows (exact FP64
    ground truth; the metric is quoted at recall@10 >= 0.95),
  - re-runs one merge with per-phase HIP-event timing to price the local-join
    kernel against the HBM roofline,
  - serving: a J-Merge server over a resident base of 2,000,000 rows of the
    same mixture (exact k=20 graph) takes 1,000 requests of 1-20,000 rows
    (log-uniform sizes) arriving as a Poisson stream at 0.7x the capacity
    measured on a warm-up burst, several requests on the device at once;
    p50/p99 of submit-to-result latency,
  - NN-Descent from random lists, J-Merge (S1 with its graph, S2 raw) and
    H-Merge on the same 1M rows: distance evaluations relative to NN-Descent
    (Eqs. 3-4, Table 1),
  - Table 2's scanning rates of NN-Descent, S-Merge and J-Merge on 100,000
    uniform rows, d from 2 to 100, l1 and l2, and Fig. 4's keep-ratio sweep,
  - merge tree: 8 blocks of 125,000 x d100 Gaussian-mixture rows with exact
    k=16 l1 block graphs merged pairwise in 3 levels to 1,000,000 rows,
  - times the CPU oracle on a bounded sample of the headline workload.
Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("points merged/s at recall@10≥0.95 (FP32 vs BF16-MFMA); "
          "p50/p99 insert latency")
HBM_PEAK = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recall_at10(ids, X, rows, device, metric="l2"):
    """Tie-tolerant recall@10 on sampled rows: a returned neighbour counts when
    its FP64 distance is at most the exact 10th-nearest distance (self
    excluded).  l2 on integer rows uses the GEMM form, which is exact there;
    l1 is summed directly.  ids: host (n, k) array of the graph."""
    import torch
    Xd = torch.from_numpy(X).to(device=device, dtype=torch.float64)
    sq = (Xd * Xd).sum(1) if metric == "l2" else None
    hits = 0
    for lo in range(0, len(rows), 100):
        r = torch.from_numpy(rows[lo:lo + 100]).to(device)
        if metric == "l2":
            D = sq[r, None] + sq[None, :] - 2.0 * (Xd[r] @ Xd.T)
        else:
            D = torch.empty((len(r), Xd.shape[0]), dtype=torch.float64, device=device)
            for a in range(len(r)):        # explicit sum of |x - y| per query row
                D[a] = (Xd - Xd[r[a]]).abs_().sum(1)
        D[torch.arange(len(r), device=device), r] = float("inf")
        kth = torch.topk(D, 10, dim=1, largest=False, sorted=True)[0][:, 9]
        got = torch.from_numpy(ids[rows[lo:lo + 100], :10].astype(np.int64)).to(device)
        dv = torch.gather(D, 1, got.clamp(min=0))
        hits += ((dv <= kth[:, None]) & (got >= 0)).sum().item()
        del D
    return hits / (len(rows) * 10)


def fp64_error(X, ids, dist, rows, metric, floor=1e-6):
    """Error of stored FP32 distances against an FP64 recomputation from the
    stored FP32 rows (plain definitions): relative above `floor`, absolute
    below it.  X: host rows; ids/dist: host (n, k) graph; rows: sampled rows."""
    rel, ab = [], []
    for i in rows:
        j = ids[i]
        ok = j >= 0
        a = X[i].astype(np.float64)
        B = X[j[ok]].astype(np.float64)
        if metric == "l2":
            e = ((B - a) ** 2).sum(1)
        elif metric == "l1":
            e = np.abs(B - a).sum(1)
        else:
            e = 1.0 - (B @ a) / (np.linalg.norm(B, axis=1) * np.linalg.norm(a))
        g = dist[i][ok].astype(np.float64)
        big = e >= floor
        rel.extend((np.abs(g[big] - e[big]) / e[big]).tolist())
        ab.extend(np.abs(g[~big] - e[~big]).tolist())
    return {"max_rel": float(max(rel)) if rel else 0.0,
            "p999_rel": float(np.percentile(rel, 99.9)) if rel else 0.0,
            "max_abs_below_floor": float(max(ab)) if ab else 0.0, "floor": floor,
            "entries": len(rel) + len(ab), "rows": len(rows)}


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


JOIN_SOURCES = ["paper_1908_00814_amd/csrc/knng_join.hip", "paper_1908_00814_amd/csrc/knng_common.h",
                "paper_1908_00814_amd/csrc/knng_internal.h"]


def measured_traffic(kernel):
    """HBM bytes per join launch from the committed PMC record (FETCH_SIZE and
    WRITE_SIZE scaled by a copy of known size), or None when there is no
    record for this kernel or its sources changed after the counters were
    taken."""
    import hashlib
    p = os.path.join(ROOT, "profiles", "k_join_traffic.json")
    if not os.path.exists(p):
        return None
    h = hashlib.sha256()
    for f in JOIN_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    data = json.load(open(p))
    for rec in data.get("records", [data]):
        if rec.get("kernel") == kernel and rec.get("sources_sha256") == h.hexdigest():
            return rec["traffic_bytes_per_launch"]
    return None


def join_roofline(st, n, d, k, s, prec="fp32"):
    """Algorithmic bytes of the local-join launches of one or more merges
    (summed counters and durations) and the achieved rate:
      gathers   every neighbourhood member's row once per round,
                members * (d * b_e + 4) (b_e = 4 for FP32 rows, 2 for bf16;
                + 4 for its list's worst bound);
      rescores  BF16 path: the two FP32 rows of every rescored pair,
                rescored * 2 * d * 4;
      lists     one read and one write of every list per round,
                rounds * 2 * n * k * 8.
    List reads and swaps of the inserts beyond that are implementation
    traffic, reported apart (insert_scan_bytes: attempts * (8k + 16))."""
    b_e = 4 if prec == "fp32" else 2
    rounds = st["rounds"]
    members = st["members"]
    gathers = members * (d * b_e + 4)
    rescores = st["rescored"] * 2 * d * 4 if prec != "fp32" else 0
    lists = rounds * 2 * n * k * 8
    alg = gathers + rescores + lists
    launches = max(st["join_launches"], 1)
    secs = st["join_ms"] / 1e3
    per_launch = alg / launches
    avg_s = secs / launches
    achieved = per_launch / avg_s if avg_s > 0 else 0.0
    kernel = "k_join<0, 32, 4>" if prec == "fp32" else "k_join_bf16<0, 32>"
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": measured_traffic(kernel),
            "kernel": kernel, "launches": launches,
            "algorithmic_bytes_per_launch": per_launch,
            "algorithmic_terms_per_launch": {"gathers": gathers / launches,
                                             "rescores": rescores / launches,
                                             "lists": lists / launches},
            "insert_scan_bytes_per_launch": st["insert_attempts"] * (8 * k + 16) / launches,
            "avg_launch_ms": st["join_ms"] / launches}


def serve_bench(args, dev, precision):
    """Serving workload: J-Merge server over a resident base, Poisson arrivals,
    once with independent requests and once with batching."""
    import torch
    import synth
    from paper_1908_00814_amd import knng
    k, nb = 20, args.serve_base
    W, R = args.serve_warmup, args.serve_requests
    t = time.perf_counter()
    base = synth.byte_cluster_points(nb, workload=2, stream=51)
    sizes = synth.request_sizes(W + R)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    req = synth.byte_cluster_points(int(offs[-1]), workload=2, stream=55)
    log(f"[serve] base {nb:,} rows, {W}+{R} requests ({int(offs[-1]):,} rows) generated in "
        f"{time.perf_counter() - t:.1f}s")
    dB = torch.from_numpy(base).to(dev)
    dR = torch.from_numpy(req).to(dev)
    t = time.perf_counter()
    gi, gd = knng.exact_graph(dB, k, "l2")
    torch.cuda.synchronize()
    log(f"[serve] exact k={k} base graph in {time.perf_counter() - t:.1f}s")
    budget = args.serve_budget_gib << 30
    service = service_times(args, dB, (gi, gd), dR, offs, sizes, k, nb, precision)
    jsweep = jmerge_sweep(args, dB, (gi, gd), base, req, k, precision, dev)
    modes = {}
    for mode, slots, batching in (("independent", args.serve_slots, False),
                                  ("batched", args.serve_batched_slots, True)):
        modes[mode] = serve_run(args, dB, (gi, gd), dR, base, req, offs, sizes, k, nb, budget,
                                slots, batching, precision, dev)
    del gi, gd
    out = dict(modes["independent"])
    out["batched"] = modes["batched"]
    out["service_time_unloaded"] = service
    out["jmerge_recall_sweep"] = jsweep
    return out


def jmerge_sweep(args, dB, G, base, req, k, precision, dev):
    """recall@10 of the inserted rows of one balanced-append J-Merge (a server
    request) of raw batches of 2,000 and 20,000 rows of the same mixture into
    the 2M-row base, against the sample size s: the base's 1,000 clusters are
    well separated (its exact graph has no edge between clusters), so a raw
    row meets its cluster only through random Initialize/Append samples."""
    import torch
    from paper_1908_00814_amd import knng
    Xb = torch.from_numpy(base).to(device=dev, dtype=torch.float64)
    sqb = (Xb * Xb).sum(1)
    out = []
    for nr in (2000, 20000):
        raw = req[:nr]
        dRaw = torch.from_numpy(raw).to(dev)
        Xr = torch.from_numpy(raw).to(device=dev, dtype=torch.float64)
        rows = np.arange(0, nr, max(1, nr // 200))
        q = Xr[torch.from_numpy(rows).to(dev)]
        D = torch.cat([(q * q).sum(1)[:, None] + sqb[None, :] - 2.0 * (q @ Xb.T),
                       (q * q).sum(1)[:, None] + (Xr * Xr).sum(1)[None, :] - 2.0 * (q @ Xr.T)], 1)
        D[torch.arange(len(rows), device=dev), torch.from_numpy(rows + len(base)).to(dev)] = \
            float("inf")
        kth = torch.topk(D, 10, dim=1, largest=False)[0][:, 9]
        for s_ in (10, 20, 32):
            kw = dict(sample=s_, delta=args.delta, seed=args.seed + 11, precision=precision,
                      balanced=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ids, _, st = knng.expand(dB, G, dRaw, k, "l2", **kw)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t
            got = ids[torch.from_numpy(rows + len(base)).to(dev), :10].long()
            dv = torch.gather(D, 1, got.clamp(min=0))
            rec = float(((dv <= kth[:, None]) & (got >= 0)).float().mean().item())
            out.append({"raw_rows": nr, "sample": s_, "recall@10_inserted": rec,
                        "ms": secs * 1e3, "rounds": st["rounds"]})
            log(f"[serve] J-Merge of {nr:,} raw rows into the base, s={s_}: recall@10 of "
                f"inserted rows {rec:.4f}, {secs * 1e3:.1f} ms, {st['rounds']} rounds")
        del D, Xr, q
    del Xb
    return out


def service_times(args, dB, G, dR, offs, sizes, k, nb, precision):
    """Service time of single requests with nothing else running (one slot,
    requests one after another), by request size, with the rounds run as the
    slot's captured launch graph and as host round trips."""
    import torch
    from paper_1908_00814_amd import knng
    want = [1, 10, 100, 1000, 10000]
    # requests of the stream closest in size to each target, 8 of each
    pick = {w: [int(i) for i in np.argsort(np.abs(sizes - w), kind="stable")[:8]] for w in want}
    out = {}
    for host_rounds in (False, True):
        mode = "host_rounds" if host_rounds else "graph_rounds"
        srv = knng.Server(dB, G, k, "l2", capacity=nb + int(offs[-1]), max_request=20_000,
                          slots=0, sample=args.sample, delta=args.delta, seed=args.seed + 5,
                          precision=precision, host_rounds=host_rounds)
        try:
            for i in pick[100][:3]:                       # warm-up (graph capture)
                t = srv.submit(dR[offs[i]:offs[i + 1]], 10_000 + i)
                srv.step()
                srv.wait(t, int(sizes[i]))
            res = {}
            for w in want:
                ms, rounds = [], []
                for i in pick[w]:
                    t = srv.submit(dR[offs[i]:offs[i + 1]], 20_000 + i)
                    srv.step()
                    info = srv.wait(t, int(sizes[i]))[2]
                    ms.append((info["done_us"] - info["start_us"]) / 1e3)
                    rounds.append(info["rounds"])
                res[str(w)] = {"rows": [int(sizes[i]) for i in pick[w]],
                               "median_ms": float(np.median(ms)), "mean_rounds":
                               float(np.mean(rounds))}
            out[mode] = res
        finally:
            srv.close()
        torch.cuda.synchronize()
        log(f"[serve] unloaded service time, {mode}: " + ", ".join(
            f"{w} rows {res[str(w)]['median_ms']:.2f} ms" for w in want))
    return out


def serve_run(args, dB, G, dR, base, req, offs, sizes, k, nb, budget, slots, batching,
              precision, dev):
    """One serving run: warm-up burst, then Poisson arrivals at 0.7x capacity."""
    import queue
    import threading
    import synth
    from paper_1908_00814_amd import knng
    W, R = args.serve_warmup, args.serve_requests
    mode = "batched" if batching else "independent"
    srv = knng.Server(dB, G, k, "l2", capacity=nb + int(offs[-1]), max_request=20_000,
                      hbm_budget=budget, slots=slots, batching=batching, sample=args.sample,
                      delta=args.delta, seed=args.seed + 5, precision=precision)
    try:
        # warm-up burst: every request queued at once, all slots busy
        tk = [srv.submit(dR[offs[i]:offs[i + 1]], i) for i in range(W)]
        inf = [srv.wait(tk[i], int(sizes[i]))[2] for i in range(W)]
        span = (max(x["done_us"] for x in inf) - min(x["submit_us"] for x in inf)) / 1e6
        cap = float(sizes[:W].sum()) / span
        lam = 0.7 * cap / float(sizes[W:].mean())
        log(f"[serve] {mode}, {srv.slots} slots; warm-up: {int(sizes[:W].sum()):,} rows in "
            f"{span * 1e3:.0f} ms -> capacity {cap:,.0f} rows/s; offered {lam:.1f} requests/s")
        gaps = synth.rng(5006).exponential(1.0 / lam, size=R)
        arrive = np.cumsum(gaps)
        q = queue.Queue()

        def submitter():
            t0 = time.perf_counter()
            for j in range(R):
                i = W + j
                delay = arrive[j] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                q.put((i, srv.submit(dR[offs[i]:offs[i + 1]], i)))

        th = threading.Thread(target=submitter)
        th.start()
        infos, results, by_req = [], {}, {}
        for j in range(R):
            i, ticket = q.get()
            ids, dist, info = srv.wait(ticket, int(sizes[i]))
            infos.append(info)
            results[i] = (ids.numpy(), dist.numpy())
            by_req[i] = info
            if (j + 1) % 250 == 0:
                log(f"[serve] {j + 1}/{R} requests done")
        th.join()
        lat = np.array([x["done_us"] - x["submit_us"] for x in infos]) / 1e3
        wall = (max(x["done_us"] for x in infos) - min(x["submit_us"] for x in infos)) / 1e6
        rows_meas = float(sizes[W:].sum())
    finally:
        srv.close()
    rec, err = serve_recall(base, req, offs, sizes, results, W, dev, by_req)
    how = ("queued requests merged together as one raw set when a slot frees up"
           if batching else "each request merged with the base on its own")
    out = {
        "workload": (f"J-Merge server: resident base {nb:,} x d128 (same byte-valued "
                     f"mixture, exact k=20 graph), {R} requests of 1-20,000 rows "
                     f"(log-uniform) in Poisson arrivals at 0.7x the capacity measured on a "
                     f"warm-up burst; {how} (balanced append), {srv.slots} slots, "
                     f"{precision}"),
        "mode": mode,
        "mean_merged_rows": float(np.mean([x["merged_rows"] for x in infos])),
        "mean_rounds": float(np.mean([x["rounds"] for x in infos])),
        "mean_service_ms": float(np.mean([x["done_us"] - x["start_us"] for x in infos]) / 1e3),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
        "inserted_points_per_s": rows_meas / wall, "capacity_rows_per_s": cap,
        "offered_requests_per_s": lam, "requests": R, "rows": int(rows_meas),
        "slots": slots, "hbm_budget_bytes": budget,
        "recall@10_inserted": rec, "fp64_error_inserted": err,
        "resident_rows_end": int(nb + offs[-1]),
    }
    log(f"[serve] {mode}: p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms, "
        f"{out['inserted_points_per_s']:,.0f} rows/s, mean merged rows "
        f"{out['mean_merged_rows']:,.0f}, recall@10 of inserted rows {rec:.4f}")
    return out


def serve_recall(base, req, offs, sizes, results, W, dev, infos):
    """recall@10 of inserted rows against their exact neighbours among the
    base and the rows their merge covered (their own request's, or with
    batching the whole batch's), and the error of their stored distances
    against FP64 (the GEMM form in FP64 is exact on these integer rows)."""
    import torch
    import synth
    g = synth.rng(5007)
    Xb = torch.from_numpy(base).to(device=dev, dtype=torch.float64)
    sqb = (Xb * Xb).sum(1)
    nb = base.shape[0]
    picked = g.choice(np.arange(W, len(sizes)), 100, replace=False)
    hits = total = 0
    rel, ab = [], []
    for i in picked:
        lo, hi = int(offs[i]), int(offs[i + 1])
        # the raw rows of the merge that ran request i (its own, or its batch)
        mlo = int(infos[i]["merged_first"]) - nb
        mhi = mlo + int(infos[i]["merged_rows"])
        Xr = torch.from_numpy(req[mlo:mhi]).to(device=dev, dtype=torch.float64)
        rows = g.choice(hi - lo, min(10, hi - lo), replace=False) + (lo - mlo)
        q = Xr[rows]
        Db = (q * q).sum(1)[:, None] + sqb[None, :] - 2.0 * (q @ Xb.T)
        Dr = (q * q).sum(1)[:, None] + (Xr * Xr).sum(1)[None, :] - 2.0 * (q @ Xr.T)
        Dr[torch.arange(len(rows), device=dev), torch.from_numpy(rows).to(dev)] = float("inf")
        D = torch.cat([Db, Dr], 1)                      # columns: base rows, then merged rows
        kth = torch.topk(D, 10, dim=1, largest=False)[0][:, 9]
        first = nb + mlo
        allids = results[i][0][rows - (lo - mlo)].astype(np.int64)
        ok = (allids >= 0) & ((allids < nb) |
                              ((allids >= first) & (allids < first + (mhi - mlo))))
        col = np.where(ok, np.where(allids < nb, allids, nb + (allids - first)), 0)
        got_all = torch.gather(D, 1, torch.from_numpy(col).to(dev)).cpu().numpy()
        stored = results[i][1][rows - (lo - mlo)].astype(np.float64)
        e, gv = got_all[ok], stored[ok]
        big = e >= 1e-6
        rel.extend((np.abs(gv[big] - e[big]) / e[big]).tolist())
        ab.extend(np.abs(gv[~big] - e[~big]).tolist())
        got = torch.from_numpy(got_all[:, :10]).to(dev)
        okt = torch.from_numpy(ok[:, :10]).to(dev)
        hits += int(((got <= kth[:, None]) & okt).sum().item())
        total += 10 * len(rows)
    err = {"max_rel": float(max(rel)) if rel else 0.0,
           "p999_rel": float(np.percentile(rel, 99.9)) if rel else 0.0,
           "max_abs_below_floor": float(max(ab)) if ab else 0.0, "floor": 1e-6,
           "entries": len(rel) + len(ab)}
    return hits / total, err


def tree_bench(args, dev):
    """Merge tree: 8 blocks, exact l1 block graphs, 3 levels of S-Merge."""
    import torch
    import synth
    from paper_1908_00814_amd import knng
    k = 16
    blocks = synth.gmm_blocks()
    starts = np.concatenate([[0], np.cumsum([len(b) for b in blocks])]).astype(np.int64)
    X = np.concatenate(blocks)
    dX = torch.from_numpy(X).to(dev)
    t = time.perf_counter()
    graphs = [knng.exact_graph(dX[starts[b]:starts[b + 1]], k, "l1") for b in range(len(blocks))]
    torch.cuda.synchronize()
    t_blocks = time.perf_counter() - t
    kw = dict(sample=args.sample, delta=args.delta, seed=args.seed + 4)
    knng.merge_tree(dX, starts, graphs, k, "l1", **kw)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    ids, dist, st = knng.merge_tree(dX, starts, graphs, k, "l1", **kw)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t
    rows = synth.rng(4007).choice(len(X), 1000, replace=False)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    rec = recall_at10(ids, X, rows, dev, metric="l1")
    sweep = []
    for s_ in (5, 10, 20, 32):
        for dl in (0.0, 0.001):
            kw_ = dict(sample=s_, delta=dl, seed=args.seed + 4)
            torch.cuda.synchronize()
            t = time.perf_counter()
            ids_s, _, st_s = knng.merge_tree(dX, starts, graphs, k, "l1", **kw_)
            torch.cuda.synchronize()
            secs_s = time.perf_counter() - t
            rec_s = recall_at10(ids_s.cpu().numpy(), X, rows, dev, metric="l1")
            sweep.append({"sample": s_, "delta": dl, "recall@10": rec_s, "ms": secs_s * 1e3,
                          "points_per_s": len(X) / secs_s})
            log(f"[tree] sweep s={s_} delta={dl}: recall@10 {rec_s:.4f}, {secs_s * 1e3:.0f} ms")
    out = {"workload": "merge tree: 8 x 125,000 x d100 Gaussian mixture (50 components), "
                       "exact k=16 l1 block graphs, pairwise S-Merge in 3 levels",
           "sweep": sweep,
           "points_per_s": len(X) / secs, "seconds": secs, "level_ms": st["level_ms"],
           "level_rounds": st["level_rounds"], "recall@10": rec,
           "block_graphs_s": t_blocks,
           "fp64_error": fp64_error(X, ids, dist, rows, "l1"),
           "scanning_rate": st["evals"] / (len(X) * (len(X) - 1) / 2.0)}
    log(f"[tree] 1,000,000 rows in {secs * 1e3:.0f} ms (levels {st['level_ms']} ms), "
        f"recall@10 {rec:.4f}; block graphs {t_blocks:.1f}s")
    return out


def cosine_bench(args, dev):
    """High-dimensional cosine workload: S-Merge of 2 x 250,000 x d960, both
    precisions, with the stored distances' error against FP64."""
    import torch
    import oracle
    import synth
    from synth.graphs import approximate_graph
    from paper_1908_00814_amd import knng
    k = 20
    t = time.perf_counter()
    S1, S2 = synth.cosine_sets()
    G1 = approximate_graph(S1, k, 0.9, device=dev, workload=3, stream=6)[0]
    G2 = approximate_graph(S2, k, 0.9, device=dev, workload=3, stream=7)[0]
    log(f"[cosine] 2 x 250,000 x d960 and approximate k=20 inputs in "
        f"{time.perf_counter() - t:.1f}s")
    d = lambda a: torch.from_numpy(a).to(dev)
    dS1, dS2, g1, g2 = d(S1), d(S2), (d(G1), None), (d(G2), None)
    X = np.concatenate([S1, S2])
    n = len(X)
    rows = synth.rng(3008).choice(n, 500, replace=False)
    out = {"workload": "symmetric merge, 2 x 250,000 x d960 nonnegative rows (|N(0,1)| plus "
                       "one of 200 offsets), L2-normalised, approximate k=20 inputs without "
                       "distances, merged to k=20 under cosine"}
    graphs = {}
    for prec in ("fp32", "bf16"):
        kw = dict(sample=args.sample, delta=args.delta, seed=args.seed + 3, precision=prec)
        knng.merge(dS1, g1, dS2, g2, k, "cos", **kw)            # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        ids, dist, st = knng.merge(dS1, g1, dS2, g2, k, "cos", **kw)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t
        graphs[prec] = (ids.cpu().numpy(), dist.cpu().numpy())
        out[prec] = {"points_per_s": n / secs, "ms": secs * 1e3, "rounds": st["rounds"],
                     "rescored": st["rescored"], "screen_violations": st["screen_violations"]}
        log(f"[cosine] {prec}: {secs * 1e3:.0f} ms, {n / secs / 1e6:.2f} M points/s, "
            f"{st['rounds']} rounds")
    ids, dist = graphs["fp32"]
    out["paths_identical"] = bool(np.array_equal(ids, graphs["bf16"][0]) and np.array_equal(
        dist.view(np.uint32), graphs["bf16"][1].view(np.uint32)))
    # FP64 error of every stored distance of the sampled rows
    out["fp64_error"] = fp64_error(X, ids, dist, rows, "cos")
    Xd = torch.from_numpy(X).to(device=dev, dtype=torch.float64)
    nrm = Xd.norm(dim=1)
    Drows = []
    for lo in range(0, len(rows), 100):
        r = torch.from_numpy(rows[lo:lo + 100]).to(dev)
        D = 1.0 - (Xd[r] @ Xd.T) / (nrm[r, None] * nrm[None, :])
        D[torch.arange(len(r), device=dev), r] = float("inf")
        Drows.append(D)
    del Xd
    kth = [torch.topk(D, 10, dim=1, largest=False)[0][:, 9] for D in Drows]

    def recall(ids_):
        hits = 0
        for b_, (D, kt) in enumerate(zip(Drows, kth)):
            got = torch.from_numpy(ids_[rows[b_ * 100:(b_ + 1) * 100], :10].astype(np.int64)).to(dev)
            hits += (torch.gather(D, 1, got) <= kt[:, None] * (1 + 1e-12)).sum().item()
        return hits / (len(rows) * 10)

    out["recall@10"] = recall(ids)
    # recall against the sample size s and the stopping threshold delta (BF16)
    out["sweep"] = []
    for s_ in (5, 10, 20, 32):
        for dl in (0.0, 0.001):
            kw = dict(sample=s_, delta=dl, seed=args.seed + 3, precision="bf16")
            torch.cuda.synchronize()
            t = time.perf_counter()
            ids_s, _, st = knng.merge(dS1, g1, dS2, g2, k, "cos", **kw)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t
            rec = recall(ids_s.cpu().numpy())
            out["sweep"].append({"sample": s_, "delta": dl, "recall@10": rec, "ms": secs * 1e3,
                                 "points_per_s": n / secs, "rounds": st["rounds"]})
            log(f"[cosine] sweep s={s_} delta={dl}: recall@10 {rec:.4f}, {secs * 1e3:.0f} ms, "
                f"{st['rounds']} rounds")
    del Drows
    log(f"[cosine] identical paths {out['paths_identical']}, recall@10 {out['recall@10']:.4f}, "
        f"FP64 max rel err {out['fp64_error']['max_rel']:.2e}")
    return out


def complexity_bench(args, dev, dS1, dG1, dS2, X, rows, smerge):
    """Comparisons of S-Merge and J-Merge against NN-Descent on the same 1M rows
    (Eqs. 3-4: about one third and two thirds of NN-Descent's comparisons, or
    fewer when the inputs are good).  NN-Descent is J-Merge with an empty base
    (random initial lists); J-Merge is Algorithm 2 as printed (every base list
    appended to), S1 with its input graph and S2 raw."""
    import torch
    from paper_1908_00814_amd import knng
    k, n = args.k, X.shape[0]
    kw = dict(sample=args.sample, delta=args.delta, seed=args.seed + 11)
    dX = torch.cat([dS1, dS2])
    out = {"s_merge": {"evals": smerge["evals"], "rounds": smerge["rounds"],
                       "recall@10": smerge["recall@10"],
                       "points_per_s": smerge["value"]}}
    for name, call in (("nn_descent", lambda: knng.expand(None, None, dX, k, "l2", **kw)),
                       ("j_merge", lambda: knng.expand(dS1, dG1, dS2, k, "l2", **kw))):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ids, _, st = call()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rec = recall_at10(ids.cpu().numpy(), X, rows, dev)
        out[name] = {"ms": dt * 1e3, "points_per_s": n / dt, "rounds": st["rounds"],
                     "evals": st["evals"], "recall@10": rec}
        log(f"[nnd] {name}: {dt * 1e3:.0f} ms, {n / dt / 1e6:.2f} M points/s, "
            f"{st['rounds']} rounds, {st['evals'] / 1e6:.0f}M distance evaluations, "
            f"recall@10 {rec:.4f}")
        del ids
    # H-Merge (Section 3.3): NN-Descent on n/64 random rows, then J-Merges
    # doubling the graph to all rows (k/2 lists above the bottom layer)
    n_top = n // 64
    torch.cuda.synchronize()
    t = time.perf_counter()
    ids, _, st = knng.hmerge(dX, k, n_top, "l2", **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    rec = recall_at10(ids.cpu().numpy(), X, rows, dev)
    out["h_merge"] = {"ms": dt * 1e3, "points_per_s": n / dt, "n_top": n_top,
                      "layers": len(st["layer_rounds"]), "rounds": st["rounds"],
                      "evals": st["evals"], "recall@10": rec,
                      "layer_ms": [round(v, 2) for v in st["layer_ms"]],
                      "layer_rounds": st["layer_rounds"]}
    log(f"[nnd] h_merge: {dt * 1e3:.0f} ms, {n / dt / 1e6:.2f} M points/s, "
        f"{len(st['layer_rounds'])} layers from {n_top:,} rows, {st['evals'] / 1e6:.0f}M "
        f"distance evaluations, recall@10 {rec:.4f}; layer ms {out['h_merge']['layer_ms']}")
    del ids
    e = out["nn_descent"]["evals"]
    out["s_merge_over_nn_descent"] = out["s_merge"]["evals"] / e
    out["j_merge_over_nn_descent"] = out["j_merge"]["evals"] / e
    out["h_merge_over_nn_descent"] = out["h_merge"]["evals"] / e
    out["workload"] = ("1M rows of the headline set: NN-Descent from random lists, J-Merge of "
                       "S1 (input graph) with S2 raw, H-Merge from n/64 random rows, S-Merge "
                       "as timed above; k=20, s=20, delta=0.001")
    log(f"[nnd] comparisons relative to NN-Descent: S-Merge "
        f"{out['s_merge_over_nn_descent']:.3f}, J-Merge {out['j_merge_over_nn_descent']:.3f}, "
        f"H-Merge {out['h_merge_over_nn_descent']:.3f}")
    del dX
    return out


TABLE2 = [(2, 10), (5, 10), (10, 20), (20, 20), (50, 30), (100, 40)]


def table2_bench(args, dev):
    """Scanning rates of Table 2 on its synthetic sets: 100,000 uniform rows in
    [0, 1)^d, d from 2 to 100 with the table's k, l1 and l2.  NN-Descent builds
    the whole graph from random lists; for the merges it builds the graphs of
    the two halves first (not counted), then S-Merge merges them and J-Merge
    joins the second half raw into the first half's graph.  c = distance
    evaluations / (n (n - 1) / 2); sampling rate 1 (s = min(k, 32)),
    delta = 0.001."""
    import torch
    import synth
    from paper_1908_00814_amd import knng
    n = 100_000
    h = n // 2
    out = []
    pairs = n * (n - 1) / 2.0
    rows = synth.rng(6100).choice(n, 1000, replace=False)
    for metric in ("l1", "l2"):
        for d, k in TABLE2:
            X = synth.rng(6000 + d).random((n, d), dtype=np.float32)
            dX = torch.from_numpy(X).to(dev)
            kw = dict(sample=min(k, 32), delta=0.001, seed=args.seed + d)
            rec = {"metric": metric, "d": d, "k": k}

            def timed(fn):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = fn()
                torch.cuda.synchronize()
                return r, (time.perf_counter() - t) * 1e3

            (ids, _, st), ms = timed(lambda: knng.expand(None, None, dX, k, metric, **kw))
            rec["nn_descent"] = {"c": st["evals"] / pairs, "ms": ms,
                                 "recall@10": recall_at10(ids.cpu().numpy(), X, rows, dev, metric)}
            g1 = knng.expand(None, None, dX[:h], k, metric, **kw)
            g2 = knng.expand(None, None, dX[h:], k, metric, **kw)
            (ids, _, st), ms = timed(lambda: knng.merge(dX[:h], g1[:2], dX[h:], g2[:2], k, metric,
                                                        **kw))
            rec["s_merge"] = {"c": st["evals"] / pairs, "ms": ms,
                              "recall@10": recall_at10(ids.cpu().numpy(), X, rows, dev, metric)}
            (ids, _, st), ms = timed(lambda: knng.expand(dX[:h], g1[:2], dX[h:], k, metric, **kw))
            rec["j_merge"] = {"c": st["evals"] / pairs, "ms": ms,
                              "recall@10": recall_at10(ids.cpu().numpy(), X, rows, dev, metric)}
            log(f"[table2] {metric} d={d:3d} k={k}: c NN-Descent {rec['nn_descent']['c']:.4f} "
                f"S-Merge {rec['s_merge']['c']:.4f} J-Merge {rec['j_merge']['c']:.4f}; "
                f"recall@10 {rec['nn_descent']['recall@10']:.3f} / "
                f"{rec['s_merge']['recall@10']:.3f} / {rec['j_merge']['recall@10']:.3f}; ms "
                f"{rec['nn_descent']['ms']:.1f} / {rec['s_merge']['ms']:.1f} / "
                f"{rec['j_merge']['ms']:.1f}")
            out.append(rec)
            del dX, ids, g1, g2
    return {"workload": "Table 2 synthetic sets: 100,000 rows uniform in [0,1)^d, halves of "
                        "50,000; sampling rate 1, delta 0.001", "rows": out}


FIG4_R = [0.0, 0.2, 1.0 / 3.0, 0.5, 0.8]
FIG4_SPLIT = [(2, 8), (3, 7), (5, 5), (7, 3), (8, 2)]


def fig4_bench(args, dev):
    """Fig. 4's ablation of the keep ratio r on the uniform d = 100 set of
    100,000 rows, k = 30, l2: recall@10 of S-Merge and J-Merge for r from 0 to
    4/5 with |S1|:|S2| from 2:8 to 8:2 (subgraphs by NN-Descent; one seed,
    the paper averages 20)."""
    import torch
    import synth
    from paper_1908_00814_amd import knng
    n, d, k = 100_000, 100, 30
    X = synth.rng(6000 + d).random((n, d), dtype=np.float32)
    dX = torch.from_numpy(X).to(dev)
    rows = synth.rng(6101).choice(n, 1000, replace=False)
    kw = dict(sample=min(k, 32), delta=0.001, seed=args.seed)
    out = []
    for a, b in FIG4_SPLIT:
        h = n * a // (a + b)
        g1 = knng.expand(None, None, dX[:h], k, "l2", **kw)
        g2 = knng.expand(None, None, dX[h:], k, "l2", **kw)
        rec = {"split": f"{a}:{b}", "r": FIG4_R, "s_merge": [], "j_merge": []}
        for r in FIG4_R:
            ids = knng.merge(dX[:h], g1[:2], dX[h:], g2[:2], k, "l2", keep_ratio=r, **kw)[0]
            rec["s_merge"].append(recall_at10(ids.cpu().numpy(), X, rows, dev))
            ids = knng.expand(dX[:h], g1[:2], dX[h:], k, "l2", keep_ratio=r, **kw)[0]
            rec["j_merge"].append(recall_at10(ids.cpu().numpy(), X, rows, dev))
        log(f"[fig4] |S1|:|S2| = {a}:{b}: recall@10 for r = 0, 1/5, 1/3, 1/2, 4/5: S-Merge "
            f"{' '.join(f'{v:.3f}' for v in rec['s_merge'])}; J-Merge "
            f"{' '.join(f'{v:.3f}' for v in rec['j_merge'])}")
        out.append(rec)
        del g1, g2, ids
    del dX
    return {"workload": "Fig. 4: 100,000 uniform rows in [0,1)^100, k = 30, l2, keep ratio r "
                        "swept at five size ratios", "rows": out}


def search_bench(args, dev, Xclust):
    """NN search over the H-Merge hierarchy (Section 4): H-Merge (k = 40, as in
    the paper's search experiments) keeps its layers, each layer is
    diversified (Algorithm 3, at most k/2 = 20 neighbours), and 10,000 held-out
    queries descend the hierarchy; recall@1 against the exact nearest
    neighbour (FP64, tie-tolerant) and queries/s for several ranked-list sizes
    ef, beside the same search on the bottom layer alone ("flat").  Two sets
    of 1,000,000 rows: uniform in [0,1)^32 (like the paper's random d=32 set)
    and the byte-valued clusters of the merge workload (1,000 well separated
    clusters: the bottom graph has no edges between clusters)."""
    import torch
    import synth
    from paper_1908_00814_amd import knng
    k, n_top, nq = 40, 15_625, 10_000
    g = synth.rng(7001)
    sets = {"uniform_d32": (g.random((1_000_000, 32), dtype=np.float32),
                            g.random((nq, 32), dtype=np.float32)),
            "clusters_d128": (Xclust, synth.byte_cluster_points(nq, workload=2, stream=71))}
    res = {"workload": "H-Merge hierarchy (k=40, top block 15,625) of 1,000,000 rows, layers "
                       "diversified to at most 20 neighbours, 10,000 held-out queries of the "
                       "same law, squared l2, top-1; uniform [0,1)^32 and the byte-valued "
                       "clusters (d=128)"}
    kw = dict(sample=args.sample, delta=args.delta, seed=args.seed + 9)
    for name, (X, Q) in sets.items():
        dX = torch.from_numpy(X).to(dev)
        dQ = torch.from_numpy(Q).to(dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        perm, xp, layers, hst = knng.hmerge_hierarchy(dX, k, n_top, "l2", **kw)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t
        del dX
        t = time.perf_counter()
        div = [knng.diversify(xp[:L[0].shape[0]].contiguous(), L, k // 2)[0] for L in layers]
        torch.cuda.synchronize()
        t_div = time.perf_counter() - t
        deg = [float((d_ >= 0).sum(1).float().mean().item()) for d_ in div]
        del layers
        # FP64 distance of the exact nearest row (positions of xp) of each query
        Xd = xp.to(torch.float64)
        sq = (Xd * Xd).sum(1)
        best = torch.empty(nq, dtype=torch.float64, device=dev)
        for lo in range(0, nq, 500):
            qd = dQ[lo:lo + 500].to(torch.float64)
            D = (qd * qd).sum(1)[:, None] + sq[None, :] - 2.0 * (qd @ Xd.T)
            best[lo:lo + 500] = D.min(1)[0]
            del D
        out = {"build_ms": t_build * 1e3, "diversify_ms": t_div * 1e3,
               "layers": [[int(L_.shape[0]), int(L_.shape[1])] for L_ in div],
               "mean_degree": deg, "hierarchy": [], "flat": []}
        for mode, use in (("hierarchy", div), ("flat", div[-1:])):
            for ef in (10, 20, 40, 80, 160):
                knng.search(xp, use, dQ[:256], 1, ef, seed=3)      # warm-up
                torch.cuda.synchronize()
                t = time.perf_counter()
                ids, _, ev = knng.search(xp, use, dQ, 1, ef, seed=3)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t
                got = Xd[ids[:, 0].long()]
                dg = ((got - dQ.to(torch.float64)) ** 2).sum(1)
                rec = float((dg <= best + 1e-9 * (1.0 + best.abs())).float().mean().item())
                out[mode].append({"ef": ef, "recall@1": rec, "queries_per_s": nq / secs,
                                  "evals_per_query": ev / nq})
                log(f"[search] {name} {mode} ef={ef}: recall@1 {rec:.4f}, {nq / secs:,.0f} "
                    f"queries/s, {ev / nq:.0f} distances/query")
        log(f"[search] {name}: hierarchy built in {t_build * 1e3:.0f} ms, diversified in "
            f"{t_div * 1e3:.0f} ms, layers {out['layers']}, mean degree "
            f"{[round(v, 1) for v in deg]}")
        res[name] = out
        del xp, perm, div, Xd, dQ
        torch.cuda.empty_cache()
    return res


def c1_bench(args, dev):
    """The small workload: S-Merge of two sets of 5,000 x d32 i.i.d. N(0,1)
    rows with exact k=10 input graphs, merged to k=10 with s=10, delta 0,
    seed 1004.  10,000 points are too few to fill the GPU, so this reports
    absolute times (no roofline), beside the oracle run in full on the same
    inputs, and the brute-force cross merge."""
    import torch
    import oracle
    import synth
    from paper_1908_00814_amd import knng
    k, s_, seed = 10, 10, 1004
    S1, S2 = synth.gaussian_sets(5000, 5000, 32)
    G1 = oracle.exact_graph(S1, k)
    G2 = oracle.exact_graph(S2, k)
    t = time.perf_counter()
    oi, od, ost = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s_, seed=seed)
    t_or = time.perf_counter() - t
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    args_ = (d(S1), (d(G1[0]), d(G1[1])), d(S2), (d(G2[0]), d(G2[1])), k, "l2")
    out = {"workload": "symmetric merge, 2 x 5,000 x d32 N(0,1), exact k=10 input graphs, "
                       "merged to k=10, s=10, delta 0, squared l2",
           "oracle_s": t_or, "oracle_rounds": ost["rounds"], "cpu": host_cpu()}
    X = np.concatenate([S1, S2])
    for prec in ("fp32", "bf16"):
        ms = []
        for rep in range(6):
            torch.cuda.synchronize()
            t = time.perf_counter()
            gi, gd, gst = knng.merge(*args_, sample=s_, seed=seed, precision=prec)
            torch.cuda.synchronize()
            if rep:
                ms.append((time.perf_counter() - t) * 1e3)
        gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
        out[prec] = {"ms_median": float(np.median(ms)), "ms_min": float(min(ms)),
                     "rounds": gst["rounds"],
                     "identical_to_oracle": bool(np.array_equal(gi, oi) and np.array_equal(
                         gd.view(np.uint32), od.view(np.uint32)))}
    out["recall@10"] = recall_at10(gi, X, np.arange(len(X)), dev)
    ms = []
    for rep in range(6):
        torch.cuda.synchronize()
        t = time.perf_counter()
        bi, bd = knng.merge_bruteforce(*args_)
        torch.cuda.synchronize()
        if rep:
            ms.append((time.perf_counter() - t) * 1e3)
    t = time.perf_counter()
    ei, ed = oracle.merge_bruteforce(S1, G1, S2, G2, k)
    out["bruteforce"] = {"ms_median": float(np.median(ms)),
                         "oracle_s": time.perf_counter() - t,
                         "identical_to_oracle": bool(np.array_equal(bi.cpu().numpy(), ei))}
    log(f"[c1] S-Merge 2 x 5,000 x d32: FP32 {out['fp32']['ms_median']:.2f} ms, BF16 "
        f"{out['bf16']['ms_median']:.2f} ms ({ost['rounds']} rounds), oracle {t_or:.2f} s; "
        f"identical {out['fp32']['identical_to_oracle']}/{out['bf16']['identical_to_oracle']}; "
        f"recall@10 {out['recall@10']:.4f}; brute-force merge {out['bruteforce']['ms_median']:.2f}"
        f" ms (oracle {out['bruteforce']['oracle_s']:.2f} s)")
    return out


ORACLE_CHILD = """
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
z = np.load(sys.argv[2])
k, s, delta, seed = (int(sys.argv[3]), int(sys.argv[4]), float(sys.argv[5]), int(sys.argv[6]))
t0 = time.time()
oracle.smerge(z["S1"], (z["g1i"], z["g1d"]), z["S2"], (z["g2i"], z["g2d"]), k, "l2",
              sample=s, delta=delta, seed=seed)
print(json.dumps({"start": t0, "end": time.time()}))
"""


def cpu_baseline(n_per, k, s, delta, seed, dev, precision):
    """The oracle (plain single-threaded C) timed on a bounded sample of the
    headline workload: once alone, and as one copy per usable CPU (at most 16)
    running at once on the same sample, which is the host's whole oracle
    throughput for merges of this size.  The GPU merges the same sample and
    the two graphs are compared."""
    import subprocess
    import tempfile
    import torch
    import oracle
    import synth
    from synth.graphs import approximate_graph
    from paper_1908_00814_amd import knng
    S1, S2 = synth.byte_cluster_sets(n_per, n_per, workload=2)
    G1 = approximate_graph(S1, k, 0.9, device="cpu", stream=6)
    G2 = approximate_graph(S2, k, 0.9, device="cpu", stream=7)
    oracle.lib()
    t0 = time.perf_counter()
    oi, od, _ = oracle.smerge(S1, G1, S2, G2, k, "l2", sample=s, delta=delta, seed=seed)
    dt = time.perf_counter() - t0
    cpu = host_cpu()
    P = max(1, min(16, cpu["usable"]))
    with tempfile.TemporaryDirectory() as tmp:
        f = os.path.join(tmp, "sample.npz")
        np.savez(f, S1=S1, S2=S2, g1i=G1[0], g1d=G1[1], g2i=G2[0], g2d=G2[1])
        procs = [subprocess.Popen([sys.executable, "-c", ORACLE_CHILD, ROOT, f, str(k), str(s),
                                   str(delta), str(seed)], stdout=subprocess.PIPE, text=True)
                 for _ in range(P)]
        spans = []
        for p_ in procs:
            o, _ = p_.communicate()
            if p_.returncode != 0:
                raise RuntimeError("oracle child failed")
            spans.append(json.loads(o.strip().splitlines()[-1]))
    wall = max(x["end"] for x in spans) - min(x["start"] for x in spans)
    d = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    gi, gd, _ = knng.merge(d(S1), (d(G1[0]), d(G1[1])), d(S2), (d(G2[0]), d(G2[1])), k, "l2",
                           sample=s, delta=delta, seed=seed, precision=precision)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    X = np.concatenate([S1, S2])
    rows = synth.rng(2009).choice(len(X), 300, replace=False)
    parity = {"identical": bool(np.array_equal(gi, oi) and
                                np.array_equal(gd.view(np.uint32), od.view(np.uint32))),
              "recall@10_oracle": oracle.recall_at(oi, X, rows, 10)[0],
              "recall@10_gpu": oracle.recall_at(gi, X, rows, 10)[0], "rows": 300}
    return {"value": P * 2 * n_per / wall, "unit": "points/s", "cores": P, "kind": "oracle",
            "parity_with_gpu": parity, "cpu": cpu,
            "single_thread": {"value": 2 * n_per / dt, "seconds": dt, "cores": 1},
            "all_cores": {"processes": P, "wall_s": wall,
                          "per_process_s": [x["end"] - x["start"] for x in spans]},
            "sample": (f"S-Merge of 2 x {n_per:,} points drawn from the same byte-valued "
                       f"cluster law (d=128, k=20, s={s}, delta={delta}), approximate "
                       f"input graphs built the same way; the single-threaded C oracle run "
                       f"as {P} processes at once on {P} of {cpu['nproc']} CPUs "
                       f"({cpu['model']}), {wall:.1f} s wall; alone: {dt:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-per", type=int, default=500_000)
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--sample", type=int, default=20)
    ap.add_argument("--delta", type=float, default=0.001)
    ap.add_argument("--precision", default="best", choices=["best", "fp32", "bf16"],
                    help="path quoted as the headline value (both are timed)")
    ap.add_argument("--seed", type=int, default=2004)
    ap.add_argument("--cpu-n", type=int, default=25_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the 2 x 5,000 x d32 workload")
    ap.add_argument("--no-search", action="store_true",
                    help="skip the hierarchy / diversification / search workload")
    ap.add_argument("--only", choices=["fp32", "bf16"], default=None,
                    help="time one path only (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (scales PMC byte counters)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--serve-base", type=int, default=2_000_000)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-batched-slots", type=int, default=2)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--no-tree", action="store_true", help="skip the merge-tree workload")
    ap.add_argument("--no-cosine", action="store_true", help="skip the d960 cosine workload")
    ap.add_argument("--no-nnd", action="store_true",
                    help="skip NN-Descent and J-Merge on the headline rows")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip Table 2's scanning rates and Fig. 4's keep-ratio sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"path is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from synth.graphs import approximate_graph
    from paper_1908_00814_amd import knng

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    knng.load()
    n1 = n2 = args.n_per
    n, d, k = n1 + n2, 128, args.k
    t = time.perf_counter()
    S1, S2 = synth.byte_cluster_sets(n1, n2, workload=2)
    log(f"[bench] points generated in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    G1 = approximate_graph(S1, k, 0.9, device=dev, stream=6)
    G2 = approximate_graph(S2, k, 0.9, device=dev, stream=7)
    log(f"[bench] input graphs (recall@20 ~0.9) built in {time.perf_counter() - t:.1f}s")
    dS1, dS2 = torch.from_numpy(S1).to(dev), torch.from_numpy(S2).to(dev)
    dG1 = (torch.from_numpy(G1[0]).to(dev), torch.from_numpy(G1[1]).to(dev))
    dG2 = (torch.from_numpy(G2[0]).to(dev), torch.from_numpy(G2[1]).to(dev))
    common = dict(sample=args.sample, delta=args.delta, seed=args.seed)
    ws_bytes = max(knng.merge_workspace_size(n1, n2, d, k, k, k, "l2", precision=p, **common)
                   for p in ("fp32", "bf16"))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = (torch.empty((n, k), dtype=torch.int32, device=dev),
           torch.empty((n, k), dtype=torch.float32, device=dev))
    stream = torch.cuda.current_stream()
    X = np.concatenate([S1, S2])
    rows = synth.rng(2000 + 8).choice(n, 1000, replace=False)

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 1 GiB device to device")
    paths = {}
    for prec in ((args.only,) if args.only else ("fp32", "bf16")):
        kw = dict(precision=prec, **common)

        def step():
            # phase timing with HIP events on the library's stream (the loop
            # already synchronises once per round to read its counter)
            return knng.merge(dS1, dG1, dS2, dG2, k, "l2", stream=stream, workspace=ws, out=out,
                              profile=True, **kw)[2]

        for i in range(args.warmup):
            st = step()
            log(f"[bench] {prec} warmup {i}: {st['rounds']} rounds")
        torch.cuda.synchronize()
        acc = {"rounds": 0, "members": 0, "rescored": 0, "insert_attempts": 0, "join_ms": 0.0,
               "join_launches": 0}
        phase = {}
        t0 = time.perf_counter()
        for i in range(args.steps):
            st = step()
            acc["rounds"] += st["rounds"]
            acc["members"] += sum(st["gathered"])
            for key in ("rescored", "insert_attempts", "join_launches"):
                acc[key] += st[key]
            acc["join_ms"] += st["ms"]["join"]
            for a_, b_ in st["ms"].items():
                phase[a_] = phase.get(a_, 0.0) + b_ / args.steps
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ms_step = elapsed * 1e3 / max(args.steps, 1)
        value = n * args.steps / elapsed
        ids = out[0].cpu().numpy()
        dist = out[1].cpu().numpy()
        rec = recall_at10(ids, X, rows, dev)
        log(f"[bench] {prec}: {args.steps} steps, {ms_step:.1f} ms/step, {value / 1e6:.2f} M "
            f"points/s, {st['rounds']} rounds, recall@10 {rec:.4f} (1,000 sampled rows)")
        roof = join_roofline(acc, n, d, k, args.sample, prec)
        log(f"[bench] {prec} join: {roof['launches']} launches in the timed steps, "
            f"{roof['avg_launch_ms']:.3f} ms avg, {roof['achieved']:.0f} GB/s algorithmic "
            f"({100 * roof['frac']:.1f}% of HBM peak); phase ms per step "
            f"{json.dumps({a_: round(b_, 2) for a_, b_ in phase.items()})}")
        paths[prec] = {"value": value, "ms_per_step": ms_step, "recall@10": rec,
                       "rounds": st["rounds"], "evals": st["evals"], "ids": ids, "dist": dist,
                       "roofline": roof, "phase_ms": phase,
                       "rescored": st["rescored"], "screen_violations": st["screen_violations"]}
    same = (bool(np.array_equal(paths["fp32"]["ids"], paths["bf16"]["ids"]))
            if len(paths) == 2 else None)
    best = max(paths, key=lambda p: paths[p]["value"]) if args.precision == "best" else \
        args.precision
    head = paths[best]
    line = {
        "metric": METRIC, "value": head["value"], "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if best == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": "symmetric merge, 2 x 500,000 x d128 byte-valued clusters "
                               "(1,000 centres, sigma 20), approximate k=20 input graphs "
                               "(recall@20 ~0.9), merged to k=20, squared l2",
                   "n1": n1, "n2": n2, "d": d, "k": k, "keep_ratio": 0.5,
                   "sample": args.sample, "delta": args.delta, "seed": args.seed,
                   "precision": best},
        "recall@10": head["recall@10"],
        "rounds": head["rounds"], "scanning_rate": head["evals"] / (n * (n - 1) / 2.0),
        "roofline": head["roofline"],
        "paths": {p: {"value": paths[p]["value"], "ms_per_step": paths[p]["ms_per_step"],
                      "recall@10": paths[p]["recall@10"],
                      "join_roofline_frac": paths[p]["roofline"]["frac"],
                      "rescored": paths[p]["rescored"],
                      "screen_violations": paths[p]["screen_violations"]} for p in paths},
        "bf16_over_fp32": (paths["bf16"]["value"] / paths["fp32"]["value"]
                           if len(paths) == 2 else None),
        "paths_identical": same,
        "fp64_error": fp64_error(X, head["ids"], head["dist"], rows, "l2"),
    }
    log(f"[bench] FP64 error of the stored distances of 1,000 sampled rows: "
        f"{json.dumps(line['fp64_error'])}")
    del ws, out
    torch.cuda.empty_cache()
    if not args.no_nnd:
        line["complexity"] = complexity_bench(args, dev, dS1, dG1, dS2, X, rows, paths[best])
    del dS1, dS2, dG1, dG2
    torch.cuda.empty_cache()
    if not args.no_search:
        line["search"] = search_bench(args, dev, X)
        torch.cuda.empty_cache()
    if not args.no_table2:
        line["table2"] = table2_bench(args, dev)
        line["fig4"] = fig4_bench(args, dev)
        torch.cuda.empty_cache()
    if not args.no_tree:
        line["tree"] = tree_bench(args, dev)
        torch.cuda.empty_cache()
    if not args.no_cosine:
        line["cosine"] = cosine_bench(args, dev)
        torch.cuda.empty_cache()
    if not args.no_serve:
        line["serving"] = serve_bench(args, dev, best)
        line["p50_insert_latency_ms"] = line["serving"]["p50_ms"]
        line["p99_insert_latency_ms"] = line["serving"]["p99_ms"]
        torch.cuda.empty_cache()
    if not args.no_c1:
        line["c1"] = c1_bench(args, dev)
    if not args.no_cpu_baseline:
        log(f"[bench] timing the CPU oracle on 2 x {args.cpu_n} points ...")
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, k, args.sample, args.delta, args.seed,
                                            dev, best)
        log(f"[bench] oracle: {line['cpu_baseline']['value']:.0f} points/s; GPU graph on the "
            f"same sample identical: {line['cpu_baseline']['parity_with_gpu']['identical']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
