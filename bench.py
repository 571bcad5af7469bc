#!/usr/bin/env python3
"""Benchmark of the streaming temporal-walk hot path on one MI355X.

Default workload ("stream"): a 1B-edge synthetic stream (50M nodes, source
and destination Zipf(1.3), bursty Poisson arrivals) ingested in 100 batches
of 10M edges under a sliding window of 2e9 time units (about 200M active
edges once full). One step is one batch: ingest (validate, sort, evict to
the window, update both views of the dual index), an explicit eviction, then
2M walks of at most 40 nodes (uniform start edge, linear hops). The first
batches fill the window untimed; then --warmup untimed batches and --steps
timed ones. Inputs are resident in HBM before anything is timed.

Other workloads: "single" (2M nodes, 100M edges in one batch, 4M
exponential walks of length 80), "mixed" (batched walks of uneven lengths
and six hop biases in one persistent launch), "serve" (the serving loop),
"tiny".

Prints one JSON line: the metric and its value, the timed steps, the
workload, the roofline of the dominant kernel, the whole step against the
HBM roofline, and the oracle's baseline on the host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "temporal-walk hops/sec + ingest edges/sec, batched/served vs plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
SECTOR = 64
INT64_MAX = (1 << 63) - 1


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="stream",
                    choices=["single", "tiny", "stream", "mixed", "serve"])
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="serve workload: seconds of real-time arrivals")
    ap.add_argument("--batches", type=int, default=0,
                    help="stream workload: number of 10M-edge batches (0 = the whole stream)")
    ap.add_argument("--dispatch", default="auto", choices=["auto", "full_walk", "coop", "queue"])
    ap.add_argument("--hop-bias", default=None,
                    choices=["uniform", "linear", "exponential", "node2vec", "weight"],
                    help="single-batch workload: hop bias in place of the workload's "
                         "(weight: the weight-based picker, its build timed with the walks)")
    ap.add_argument("--direction", default="forward", choices=["forward", "backward"],
                    help="single-batch workload: backward walks (in-edges before the current "
                         "time); the in-view's update is part of every timed ingest")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true",
                    help="stream workload: skip the single-batch figures that follow it")
    ap.add_argument("--no-probe", action="store_true")
    return ap.parse_args()


def describe(name, w, tau):
    s = w["stream"]
    return {
        "workload": name,
        "directed": s.directed,
        "nodes": s.num_nodes,
        "edges": s.num_edges,
        "src_zipf": s.src_s, "dst_zipf": s.dst_s,
        "timestamps": s.ts_kind,
        "walks": w["walks"], "max_len": w["max_len"],
        "start_bias": w["start_bias"], "hop_bias": w["hop_bias"],
        "tau": tau, "window": w["window"],
    }


def probe_rates(torch, dev):
    """Random 64 B-sector read rate over 8 GiB and streaming copy bandwidth."""
    import paper_2605_16182_amd as tw
    lib = ctypes.CDLL(os.path.join(os.path.dirname(tw.__file__), "libtw_probe.so"))
    lib.probe_gather.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    lib.probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                               ctypes.c_void_p]
    stream = torch.cuda.current_stream()
    nbytes = 8 << 30
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    buf.random_(0, 255)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    threads, iters = 256 * 2048 * 4, 64
    best = 0.0
    for rep in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        assert lib.probe_gather(buf.data_ptr(), nbytes, threads, iters, rep + 1, sink.data_ptr(),
                                stream.cuda_stream) == 0
        e1.record()
        torch.cuda.synchronize()
        if rep:
            best = max(best, threads * iters / (e0.elapsed_time(e1) * 1e-3))
    cb = 2 << 30
    a = buf[:cb]
    b = buf[cb:2 * cb]
    copy_best = 0.0
    for rep in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        assert lib.probe_copy(a.data_ptr(), b.data_ptr(), cb, stream.cuda_stream) == 0
        e1.record()
        torch.cuda.synchronize()
        if rep:
            copy_best = max(copy_best, 2 * cb / (e0.elapsed_time(e1) * 1e-3))
    del buf
    torch.cuda.empty_cache()
    return best, copy_best


WALK_SOURCES = ("paper_2605_16182_amd/csrc/walk.hip", "paper_2605_16182_amd/csrc/walk_device.h",
                "paper_2605_16182_amd/csrc/tw_internal.h")
TRAFFIC_FILES = {"single": os.path.join(ROOT, "profiles", "walk_traffic_single_100M.txt"),
                 "stream": os.path.join(ROOT, "profiles", "walk_traffic_stream_1B.txt")}


def walk_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes of one walk launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None when that summary does not describe the current walk sources."""
    path = TRAFFIC_FILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.loads(fh.read().split("\n---\n")[0])
    if rec.get("source_sha256") != walk_source_hash():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def walk_bytes(walks, hops, hop_bias):
    """Algorithmic bytes of one walk launch: every hop (the start edge
    included) reads 4 random 64 B sectors (node record, search leaf, group
    bounds, chosen edge; 3 for a uniform pick, which needs no group bounds)
    and writes 12 B of output (node and timestamp); every walk also writes
    its length and first node (8 B). Padding slots of the output rows are
    not counted."""
    per_hop = 3 if hop_bias == "uniform" else 4
    return hops * (per_hop * SECTOR + 12) + walks * 8


def ingest_bytes(b_in, kept, evicted, jobs):
    """Algorithmic bytes of one incremental ingest: read the batch (16 B per
    input record), one read+write pass to order the kept records by source
    (32 B), append them to the timestamp view with its group starts (16 + 4
    B) and to their nodes' runs in the node view with group records (12 + 16
    B), read the sources of the evicted records (4 B), and read and write the
    record of every node whose run changed (2 x 48 B)."""
    return 16 * b_in + 80 * kept + 4 * evicted + 96 * jobs


def rebuild_bytes(b, m_old, m_new, V):
    """Bytes of an ingest that rebuilds both views from scratch: read the
    batch, one sort pass, read the old and write the new window in both
    views (28 B per edge), the node table (4 B per node)."""
    return 16 * b + 32 * b + 28 * (m_old + m_new) + 4 * V


def cpu_baseline(w, tau, gpu_hops_per_step):
    """The oracle on a bounded sample: ingest of the stream's first 20% of
    edges (scaled linearly to the full batch) and 1% of the walk ids on that
    graph (hop rate applied to the GPU step's hop count)."""
    import oracle
    spec = w["stream"]
    frac = 0.2 if spec.num_edges >= 10_000_000 else 1.0
    n = int(spec.num_edges * frac)
    src, dst, ts = next(spec.batches(n))
    og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed, window=w["window"])
    t0 = time.perf_counter()
    og.ingest_batch(src, dst, ts)
    og.sizes()  # builds the views
    t_ing = (time.perf_counter() - t0) / frac
    nw = max(1000, w["walks"] // 100)
    idx = np.arange(0, w["walks"], max(1, w["walks"] // nw))[:nw]
    threads = oracle.threads()
    t0 = time.perf_counter()
    r = og.sample_walks(w["walks"], w["max_len"], hop_bias=w["hop_bias"], hop_tau=tau,
                        start_bias=w["start_bias"], start_tau=tau, seed=42, walk_idx=idx,
                        threads=threads)
    t_walk = time.perf_counter() - t0
    hops = int(np.maximum(r["len"] - 1, 0).sum())
    hop_rate = hops / t_walk
    t_step = t_ing + gpu_hops_per_step / hop_rate
    return {
        "value": gpu_hops_per_step / t_step, "unit": "hops/s", "cores": threads,
        "kind": "oracle",
        "ingest_edges_per_s": spec.num_edges / t_ing, "walk_hops_per_s": hop_rate,
        "sample": (f"oracle ingest of the first {n} edges ({frac:.0%}, single-threaded), "
                   f"scaled linearly to {spec.num_edges}; {len(idx)} walk ids (1%) on that "
                   f"graph with {threads} OpenMP threads, hop rate applied to the GPU step's "
                   f"hop count"),
    }


def stream_cpu_baseline(w, gpu_hops_per_batch, first_batches, steady):
    """The oracle on the stream: the first batches (the window filling) and
    the steady-state batches in `steady` ({1-based first batch: (window
    content before it, [that batch and the ones after it])}; the state before
    the first is set up untimed by one ingest of the window content: for a
    stream whose timestamps never decrease the index is a function of the
    window content). Each batch is timed for ingest + evict + the view
    rebuild (single-threaded, as the oracle runs) and for walks on 1% of the
    walk ids, on one thread and on every host core."""
    import oracle
    spec = w["stream"]
    B, W, L, window = w["batch_edges"], w["walks"], w["max_len"], w["window"]
    threads = oracle.threads()
    idx = np.arange(0, W, 100, dtype=np.int64)  # 1% of the walk ids
    kw = dict(hop_bias=w["hop_bias"], start_bias=w["start_bias"], walk_idx=idx)

    def one(og, b, s, d, t):
        t0 = time.perf_counter()
        info = og.ingest_batch(s, d, t)
        og.evict_before(info["t_max"] - window)
        og.sizes()  # builds the views
        t_ing = time.perf_counter() - t0
        t0 = time.perf_counter()
        og.sample_walks(W, L, seed=b, threads=1, **kw)
        t_w1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = og.sample_walks(W, L, seed=b, threads=threads, **kw)
        t_wn = time.perf_counter() - t0
        hops = int(np.maximum(r["len"] - 1, 0).sum())
        return t_ing, hops / t_w1, hops / t_wn

    rows = {}
    og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed, window=window)
    for b, (s, d, t) in enumerate(first_batches):
        rows[b + 1] = one(og, b, s, d, t)
    del og
    for sb, (content, nxt) in sorted(steady.items()):
        og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed, window=window)
        og.ingest_batch(*content)
        for k, batch in enumerate(nxt):
            rows[sb + k] = one(og, sb + k - 1, *batch)
            print(f"# oracle batch {sb + k}", file=sys.stderr, flush=True)
        del og
    first = len(first_batches)
    steady_ids = sorted(b for b in rows if b > first)
    ss = [rows[b] for b in steady_ids]
    t_ing = float(np.mean([r[0] for r in ss]))
    rate1 = float(np.mean([r[1] for r in ss]))
    rate_n = float(np.mean([r[2] for r in ss]))
    per_batch = t_ing + gpu_hops_per_batch / rate_n
    return {
        "value": gpu_hops_per_batch / per_batch, "unit": "hops/s", "cores": threads,
        "kind": "oracle",
        "ingest_edges_per_s": B / t_ing, "walk_hops_per_s": rate_n,
        "walk_hops_per_s_single_thread": rate1,
        "per_batch": {str(b): {"ingest_evict_views_s": r[0], "walk_hops_per_s_1_thread": r[1],
                               f"walk_hops_per_s_{threads}_threads": r[2]}
                      for b, r in sorted(rows.items())},
        "sample": (f"oracle on stream batches 1-{first} (window filling) and "
                   f"{steady_ids[0]}-{steady_ids[-1]} (window full; the state before the first set up "
                   f"untimed by one ingest of the window content): ingest + evict + view "
                   f"rebuild single-threaded; walks on 1% of the walk ids ({len(idx)}), timed "
                   f"on 1 thread and on {threads}; value = the GPU's hops per steady-state "
                   f"batch over (oracle ingest + those hops at the {threads}-thread rate)"),
    }


def h2d_ms(torch, dev, batch):
    """Host-to-device copy of one batch from pinned host memory (median of 3)."""
    host = [torch.from_numpy(a).pin_memory() for a in batch]
    devs = [torch.empty_like(h, device=dev) for h in host]
    times = []
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for h, d in zip(host, devs):
            d.copy_(h, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times[1:]))


COOP_SWEEP = [  # (regroup, wave_min, panel, sync) of the cooperative dispatch
    (0, 64, 4096, 1), (0, 64, 4096, 4), (0, 16, 4096, 4), (0, 16, 8192, 4), (0, 1, 2048, 4),
    (1, 64, 2048, 1), (1, 64, 2048, 4), (1, 64, 2048, 16)]


def dispatch_sweep(torch, g, W, L, walk_kw, hops_ref):
    """The walk launch under every queue shape and cooperative setting
    (tw_set_tuning, then the AUTO dispatch): median of 3 timed runs after
    one untimed; every setting must give the same walk lengths."""
    out = walk_kw["out"]
    saved = g.tuning()
    rows = []
    cands = [dict(dispatch="queue", queue_bpc=b) for b in (0, 4, 2)] + [
        dict(dispatch="coop", coop_regroup=r, coop_wave_min=wm, coop_panel=p, coop_sync=sy)
        for r, wm, p, sy in COOP_SWEEP]
    for c in cands:
        g.set_tuning(**c)
        times = []
        for rep in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.sample_walks(W, L, **dict(walk_kw, dispatch="auto"))
            e1.record()
            torch.cuda.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1))
        h = int((out[2].to(torch.int64) - 1).clamp_min(0).sum().item())
        assert h == hops_ref, f"{c} walks differ in length"
        rows.append(dict(c, walk_ms=float(np.median(times))))
    g.set_tuning(**{k: v for k, v in saved.items()})
    return rows


WALK_KERNEL = "k_walk_full"


def serve_stream(torch, tw, spec, w, batches, first_timed, total, hops_last):
    """The stream through a tw_server: per batch an ingest and one request of
    the batch's walks (same seeds as the plain loop), at most three requests
    outstanding. The server plans each batch on its ingest stream while the
    walks before it run. Batches before first_timed fill the window untimed;
    the rest are timed from the first submission to the last result."""
    W, L = w["walks"], w["max_len"]
    g2 = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    srv = tw.Server(g2, arena_bytes=3 * (W * L * 12 + W * 4) + (64 << 20),
                    max_walks_per_launch=W, max_inflight=2)
    pending = []
    last = {}

    def submit(b):
        pending.append((b, srv.ingest(*batches[b]), srv.submit(
            W, L, hop_bias=w["hop_bias"], start_bias=w["start_bias"], seed=b)))

    def drain(keep):
        while len(pending) > keep:
            b, iid, rid = pending.pop(0)
            assert srv.wait(iid)["status"] == 0 and srv.wait(rid)["status"] == 0
            if b == total - 1:
                last["len"] = srv.result(rid)[2]
            srv.release(iid)
            srv.release(rid)

    for b in range(first_timed):
        submit(b)
        drain(2)
    drain(0)
    st0 = srv.stats()
    t0 = time.perf_counter()
    for b in range(first_timed, total):
        submit(b)
        drain(2)
    drain(0)
    wall = time.perf_counter() - t0
    st1 = srv.stats()
    srv.close()
    g2.close()
    h = int((last["len"].to(torch.int64) - 1).clamp_min(0).sum().item())
    assert h == hops_last, "served walks differ from the plain loop's"
    K = total - first_timed
    hops = st1["hops_done"] - st0["hops_done"]
    return {"batches": K, "ms_per_step": wall * 1e3 / K, "hops_per_s": hops / wall,
            "ingest_edges_per_s": K * w["batch_edges"] / wall, "launches": int(
                st1["launches"] - st0["launches"]),
            "note": "one tw_server: ingest planned on its own stream while the walks before "
                    "it run; one request of the batch's walks after each batch"}


def run_stream(args, torch, tw, w, dev, gather_rate, copy_bw):
    """Streaming window, the default workload: a 1B-edge stream in 100
    batches of 10M edges under a 2e9 window. Per batch: ingest (which
    evicts to the window), an explicit evict_before(t_max - window), then the
    batch's walks. One step is one batch: the first batches fill the window
    untimed, then `warmup` untimed batches, then `steps` timed batches."""
    spec = w["stream"]
    B = w["batch_edges"]
    total = spec.num_edges // B if args.batches <= 0 else args.batches
    K, Wu = args.steps, args.warmup
    if K < 1 or K + Wu > total:
        raise SystemExit(f"stream: need 1 <= steps and steps + warmup <= {total} batches")
    fill = total - K - Wu
    t0 = time.perf_counter()
    batches, host_keep = [], {}
    # host copies for the oracle baseline: the first batches, and the window
    # content before each steady-state batch it times (with that batch)
    want_cpu = not args.no_cpu_baseline
    first_n = min(5, total)
    # steady state: batches 96-100 of the 100 (or the last ones of a shorter run)
    steady_first = max(min(96, total - 4), first_n + 1)
    first_host, window_host, steady_host = [], [], {}
    t_now = []  # the clock after each batch (its largest timestamp so far), host-side
    for b, (s, d, t) in enumerate(spec.batches(B)):
        if b >= total:
            break
        t_now.append(max(int(t.max()), t_now[-1] if t_now else int(t.max())))
        batches.append((torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev),
                        torch.from_numpy(t).to(dev)))
        if b == total - 1:
            host_keep["last"] = (s, d, t)
        if want_cpu:
            if b < first_n:
                first_host.append((s, d, t))
            if b + 1 == steady_first and window_host:
                content = tuple(np.concatenate([x[i] for x in window_host]) for i in range(3))
                lo = int(np.searchsorted(content[2], int(window_host[-1][2][-1]) - w["window"]))
                steady_host[b + 1] = (tuple(x[lo:] for x in content), [])
            if steady_host and b + 1 >= steady_first:
                steady_host[steady_first][1].append((s, d, t))
            window_host.append((s, d, t))
            cut = int(t[-1]) - w["window"]
            while window_host and int(window_host[0][2][-1]) < cut:
                window_host.pop(0)
        if b % 10 == 0:
            print(f"# generated batch {b}", file=sys.stderr, flush=True)
    del window_host
    gen_s = time.perf_counter() - t0
    print(f"# {total} batches resident in HBM ({gen_s:.1f}s)", file=sys.stderr, flush=True)
    W, L = w["walks"], w["max_len"]
    out = (torch.empty((W, L), dtype=torch.int32, device=dev),
           torch.empty((W, L), dtype=torch.int64, device=dev))
    # every batch's walk lengths are kept and its hops counted after the
    # timed region, so that no counting runs between the batches
    lens_all = torch.empty((total, W), dtype=torch.int32, device=dev)
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    per_batch = []  # (accepted, evicted, node-view jobs, compaction, active) of every ingest
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(total)]

    def batch(b):
        s, d, t = batches[b]
        e = evs[b]
        e[0].record()
        g.ingest_batch(s, d, t, info=False)  # the window's range stays on the device
        lu = g.last_update()  # host counters of the ingest just done
        st = g.index_stats()
        per_batch.append((lu["accepted"], lu["evicted"], st["jobs"], st["full_rewrite"],
                          lu["active_edges"]))
        e[1].record()
        g.evict_before(t_now[b] - w["window"])
        e[2].record()
        g.sample_walks(W, L, hop_bias=w["hop_bias"], start_bias=w["start_bias"], seed=b,
                       dispatch=args.dispatch, out=(out[0], out[1], lens_all[b]))
        e[3].record()

    for b in range(fill + Wu):
        batch(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(fill + Wu, total):
        batch(b)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = slice(fill + Wu, total)
    hops = (lens_all - 1).clamp_min(0).sum(1, dtype=torch.int64).cpu().numpy()
    ing = np.array([e[0].elapsed_time(e[1]) for e in evs])
    ev = np.array([e[1].elapsed_time(e[2]) for e in evs])
    wk = np.array([e[2].elapsed_time(e[3]) for e in evs])
    pb = np.array(per_batch, dtype=np.float64)
    hops_t = float(np.mean(hops[timed]))
    ing_t, ev_t, wk_t = (float(np.mean(x[timed])) for x in (ing, ev, wk))
    step_ms = ing_t + ev_t + wk_t
    m_t = float(np.mean(pb[timed, 4]))

    # walk phase alone under each dispatch on the final window (plain
    # full-walk against the work queue and the cooperative regrouping)
    compare = {}
    last = total - 1
    for disp in ("full_walk", "queue", "coop"):
        times = []
        for rep in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.sample_walks(W, L, hop_bias=w["hop_bias"], start_bias=w["start_bias"], seed=last,
                           dispatch=disp, out=(out[0], out[1], lens_all[last]))
            e1.record()
            torch.cuda.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1))
        h = int((lens_all[last] - 1).clamp_min(0).sum(dtype=torch.int64).item())
        assert h == int(hops[last]), f"{disp} walks differ in length"
        ms = float(np.median(times))
        compare[disp] = {"walk_ms": ms, "walk_hops_per_s": h / (ms * 1e-3)}
    g.close()
    torch.cuda.empty_cache()
    served = serve_stream(torch, tw, spec, w, batches, fill + Wu, total, int(hops[last]))
    del batches
    torch.cuda.empty_cache()
    h2d = h2d_ms(torch, dev, host_keep["last"])

    wb = walk_bytes(W, hops_t, w["hop_bias"])
    ib = ingest_bytes(B, float(np.mean(pb[timed, 0])), float(np.mean(pb[timed, 1])),
                      float(np.mean(pb[timed, 2])))
    rb = rebuild_bytes(B, m_t, m_t, spec.num_nodes)
    peak = HBM_PEAK_GBS * 1e9
    per_hop = 3 if w["hop_bias"] == "uniform" else 4
    res = {
        "metric": METRIC,
        "value": float(hops[timed].sum()) / wall,
        "unit": "hops/s",
        "n_gpus": 1, "steps": K, "warmup": Wu,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64+f64", "data": "synthetic",
        "config": describe("stream", w, 0.0) | {
            "batches": total, "batch_edges": B, "window_fill_batches": fill,
            "timed_batches": f"{fill + Wu + 1}..{total}"},
        "dispatch": args.dispatch,
        "hops_per_step": hops_t,
        "active_edges": m_t,
        "ingest_ms": ing_t, "evict_ms": ev_t, "walk_ms": wk_t,
        "ingest_edges_per_s": B / ((ing_t + ev_t) * 1e-3),
        "ingest_edges_per_s_with_h2d": B / ((ing_t + ev_t + h2d) * 1e-3),
        "h2d_ms": h2d,
        "walk_hops_per_s": hops_t / (wk_t * 1e-3),
        "node_view_jobs": float(np.mean(pb[timed, 2])),
        "compactions": int(pb[timed, 3].sum()),
        "plain_vs_tuned": compare,
        "served": served,
        "served_vs_plain": served["hops_per_s"] / (float(hops[timed].sum()) / wall),
        "roofline": {"bound": "hbm", "kernel": WALK_KERNEL,
                     "achieved": wb / (wk_t * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": wb / (wk_t * 1e-3) / peak, "traffic": measured_traffic("stream"),
                     "algorithmic_bytes": wb,
                     "bytes_model": f"hops x ({per_hop} x 64 + 12) + walks x 8"},
        # the whole batch against 8 TB/s: the ingest as a rebuild of both
        # views would move it, plus the walks
        "roofline_step": {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "ingest_bytes_rebuild_model": rb, "walk_bytes": wb,
                          "roof_ms": (rb + wb) / peak * 1e3, "measured_ms": step_ms,
                          "frac": (rb + wb) / peak * 1e3 / step_ms},
        "roofline_step_incremental": {"ingest_bytes": ib, "walk_bytes": wb,
                                      "roof_ms": (ib + wb) / peak * 1e3,
                                      "frac": (ib + wb) / peak * 1e3 / step_ms},
        "roofline_step_probed": {
            "copy_GBps_measured": copy_bw / 1e9, "random_sectors_per_s": gather_rate,
            "ingest_roof_ms": ib / copy_bw * 1e3 if copy_bw else None,
            "walk_roof_ms": hops_t * per_hop / gather_rate * 1e3 if gather_rate else None,
            "frac": ((ib / copy_bw + hops_t * per_hop / gather_rate) * 1e3 / step_ms)
            if copy_bw and gather_rate else None},
    }
    if not args.no_cpu_baseline:
        print("# oracle baseline ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = stream_cpu_baseline(w, hops_t, first_host, steady_host)
    return res


def run_mixed(args, torch, tw, w, dev, gather_rate):
    """Batched mixed walks: one persistent work-queue launch of walks with
    lengths uniform in [min_len, max_len] and six hop biases (walk id mod 6)
    on an undirected power-law graph, against the same batch with one thread
    per walk and no queue."""
    import synth
    spec = w["stream"]
    src, dst, ts = spec.all()
    tau = float(w["tau_frac"] * int(ts.max() - ts.min()))
    d_src, d_dst, d_ts = (torch.from_numpy(a).to(dev) for a in (src, dst, ts))
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.ingest_batch(d_src, d_dst, d_ts)
    e1.record()
    torch.cuda.synchronize()
    ingest_ms = e0.elapsed_time(e1)
    W, L = w["walks"], w["max_len"]
    lims = torch.from_numpy(synth.walk_lengths(4, W, w["min_len"], L)).to(dev)
    biases = synth.mixed_biases(tau)
    rows = g.row_offsets(lims)
    out = (torch.empty(rows[1], dtype=torch.int32, device=dev),
           torch.empty(rows[1], dtype=torch.int64, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev))
    kw = dict(max_lens=lims, seed=42, ragged=True, rows=rows, out=out)
    res_d = {}
    hops = None
    for disp in ("full_walk", "queue"):
        for _ in range(max(args.warmup, 1)):
            g.sample_walks_batch(W, L, biases, dispatch=disp, **kw)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            g.sample_walks_batch(W, L, biases, dispatch=disp, **kw)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        h = int((out[2].to(torch.int64) - 1).clamp_min(0).sum().item())
        assert hops is None or h == hops, "dispatches gave different walks"
        hops = h
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        res_d[disp] = {"walk_ms": ms, "walk_hops_per_s": hops / (ms * 1e-3),
                       "ms_per_step": wall * 1e3 / args.steps}
    g.sync()
    # plain exponential walks on this hub-heavy graph under each dispatch,
    # then under the autotuner's choice (the dispatch plane's tunables)
    Wp, Lp = 2_000_000, 40
    pout = (out[0][:Wp * Lp].view(Wp, Lp), out[1][:Wp * Lp].view(Wp, Lp), out[2][:Wp])
    pkw = dict(hop_bias="exponential", hop_tau=tau, start_bias="uniform", seed=42, out=pout)
    plain = {}
    phops = None
    for disp in ("full_walk", "queue", "coop", "tuned"):
        if disp == "tuned":
            plain["tuning"] = g.autotune(Wp, Lp, sample=Wp, **{k: v for k, v in pkw.items()
                                                                if k != "out"})
            plain["tuning"] = g.tuning()
        times = []
        for rep in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.sample_walks(Wp, Lp, dispatch="auto" if disp == "tuned" else disp, **pkw)
            e1.record()
            torch.cuda.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1))
        h = int((pout[2].to(torch.int64) - 1).clamp_min(0).sum().item())
        assert phops is None or h == phops, f"{disp} walks differ in length"
        phops = h
        ms = float(np.median(times))
        plain[disp] = {"walk_ms": ms, "walk_hops_per_s": h / (ms * 1e-3)}
    plain["walks"], plain["max_len"], plain["hops"] = Wp, Lp, phops
    plain["sweep"] = dispatch_sweep(torch, g, Wp, Lp, pkw, phops)
    q = res_d["queue"]
    roof = gather_rate / 4 if gather_rate else None
    res = {
        "metric": METRIC, "value": q["walk_hops_per_s"], "unit": "hops/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": q["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64+f64", "data": "synthetic",
        "config": describe("mixed", w, tau) | {
            "min_len": w["min_len"], "hop_biases": [b[0] if b[0] != "node2vec" else
                                                    f"node2vec({b[2]},{b[3]})" for b in biases],
            "layout": "ragged rows"},
        "dispatch": "queue",
        "hops_per_step": hops,
        "batched_vs_plain": res_d,
        "plain_walks_by_dispatch": plain,
        "ingest_ms": ingest_ms,
        "ingest_edges_per_s": spec.num_edges * (1 if spec.directed else 2) / (ingest_ms * 1e-3),
        "gather_roofline": {"random_sectors_per_s": gather_rate, "sectors_per_hop": 4,
                            "hops_per_s_roof": roof,
                            "frac": q["walk_hops_per_s"] / roof if roof else None},
    }
    g.close()
    print(json.dumps(res), flush=True)


def serve_phase(torch, tw, srv, batches, rate_req, seconds, tau, seed):
    """One real-time serving phase through `srv`: `batches` (resident, one
    per 100 ms) are ingested on schedule while walk requests arrive Poisson at
    rate_req per second (walk count log-uniform in [1e2, 1e5], length 10, 40
    or 80, a random hop bias). Returns the phase's counts and latencies."""
    import threading
    rng = np.random.default_rng(seed)
    n_req = rng.poisson(rate_req * seconds)
    arrivals = np.sort(rng.uniform(0.0, seconds, n_req))
    counts = np.exp(rng.uniform(np.log(1e2), np.log(1e5), n_req)).astype(np.int64)
    lens = rng.choice([10, 40, 80], n_req)
    kinds = rng.choice(["uniform", "linear", "exponential", "node2vec"], n_req)
    before = srv.stats()
    lat, ing_lat = [], []
    submitted = []
    cond = threading.Condition()
    finished = [False]

    def reaper():
        k = 0
        while True:
            with cond:
                while k >= len(submitted) and not finished[0]:
                    cond.wait()
                if k >= len(submitted):
                    return
                rid, is_req = submitted[k]
            r = srv.wait(rid)
            if is_req:
                lat.append(r["latency_ms"])
                srv.release(rid)
            else:
                ing_lat.append(r["latency_ms"])
            k += 1

    th = threading.Thread(target=reaper)
    th.start()
    events = sorted([(i * 0.1, 0, i) for i in range(len(batches))] +
                    [(float(a), 1, i) for i, a in enumerate(arrivals)])
    t_start = time.perf_counter()
    for when, kind, i in events:
        now = time.perf_counter() - t_start
        if when > now:
            time.sleep(when - now)
        if kind == 0:
            rid = srv.ingest(*batches[i])
        else:
            rid = srv.submit(int(counts[i]), int(lens[i]), hop_bias=str(kinds[i]), hop_tau=tau,
                             p=0.5, q=2.0, seed=int(seed * 1_000_003 + i), walk_id_base=0)
        with cond:
            submitted.append((rid, kind == 1))
            cond.notify()
    with cond:
        finished[0] = True
        cond.notify()
    th.join()
    wall = time.perf_counter() - t_start
    st = srv.stats()
    lat = np.array(lat)
    hops = st["hops_done"] - before["hops_done"]
    return {"requests_per_s": rate_req, "seconds": seconds, "requests": int(n_req),
            "offered_walks": int(counts.sum()), "walks": int(st["walks_done"] - before["walks_done"]),
            "hops": int(hops), "wall_s": wall, "hops_per_s": hops / wall,
            "launches": int(st["launches"] - before["launches"]),
            "ingests": len(ing_lat), "ingested_edges": int(sum(b[0].numel() for b in batches)),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "max_ms": float(lat.max()) if len(lat) else None,
            "ingest_p50_ms": float(np.percentile(ing_lat, 50)) if ing_lat else None,
            "ingest_p99_ms": float(np.percentile(ing_lat, 99)) if ing_lat else None}


def run_serve(args, torch, tw, w, dev, gather_rate):
    """Serving loop in real time on the 300M-edge stream (5M edges/s, 10M
    nodes, Zipf 1.2, 60 s window): the first 40 s of edges are ingested up
    front; then, for --serve-seconds of wall time (20: the rest of the 300M
    edges), 5M edges/s arrive in 100 ms batches and walk requests arrive
    Poisson at 2k/s, all through one tw_server, whose ingest thread plans each
    batch while the walks before it run. Reports sustained hops/s and request
    latency; then a saturation sweep (the stream continues, requests at 2x to
    16x the rate for 3 s each) and a burst of 2,000 requests served against
    the same requests as one tw_sample_walks call each."""
    spec = w["stream"]
    rate = w["edges_per_s"]
    warm_edges = int(40 * rate)
    live_s = args.serve_seconds
    step = int(rate * 0.1)
    sweep = [2, 4, 8, 16]
    sweep_s = 3.0
    nb = int(round(live_s / 0.1))
    nsweep = int(round(sweep_s / 0.1))
    # the sweep continues the stream past its 300M edges (every element is a
    # function of its index, so the first 300M are the workload's)
    import dataclasses
    gen = dataclasses.replace(spec, num_edges=spec.num_edges + len(sweep) * nsweep * step
                              ).batches(step)
    warm = [next(gen) for _ in range(warm_edges // step)]
    s0, d0, t0_ = (np.concatenate([b[k] for b in warm]) for k in range(3))
    del warm
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    info = g.ingest_batch(*(torch.from_numpy(a).to(dev) for a in (s0, d0, t0_)))
    del s0, d0, t0_

    def resident(k):
        out = []
        for _ in range(k):
            try:
                out.append(tuple(torch.from_numpy(a).to(dev) for a in next(gen)))
            except StopIteration:
                break
        return out

    tau = 0.1 * float(w["window"])
    live = resident(nb)
    torch.cuda.synchronize()
    print(f"# warm window {info['active_edges']} edges; {len(live)} live batches of {step}",
          file=sys.stderr, flush=True)
    srv = tw.Server(g, arena_bytes=w["arena_bytes"], max_walks_per_launch=1 << 20,
                    max_inflight=2)
    main = serve_phase(torch, tw, srv, live, w["requests_per_s"], live_s, tau, seed=7)
    del live
    print(f"# served {main['requests']} requests: p50 {main['p50_ms']:.2f} ms, "
          f"p99 {main['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    sat = []
    for k, mult in enumerate(sweep):
        more = resident(nsweep)
        torch.cuda.synchronize()
        r = serve_phase(torch, tw, srv, more, w["requests_per_s"] * mult, sweep_s, tau,
                        seed=100 + k)
        del more
        sat.append(r)
        print(f"# {r['requests_per_s']} requests/s: {r['hops_per_s'] / 1e9:.2f} G hops/s, "
              f"p50 {r['p50_ms']:.2f} ms, p99 {r['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    srv.close()

    # a burst of requests submitted at once through a server, against the
    # same requests as one tw_sample_walks call each
    rng = np.random.default_rng(11)
    nburst = 2000
    counts = np.exp(rng.uniform(np.log(1e2), np.log(1e5), nburst)).astype(np.int64)
    lens = rng.choice([10, 40, 80], nburst)
    kinds = rng.choice(["uniform", "linear", "exponential", "node2vec"], nburst)
    burst = [dict(num_walks=int(counts[i]), max_len=int(lens[i]), hop_bias=str(kinds[i]),
                  hop_tau=tau, p=0.5, q=2.0, seed=int(i), walk_id_base=0) for i in range(nburst)]
    srv = tw.Server(g, arena_bytes=w["arena_bytes"], max_walks_per_launch=1 << 20,
                    max_inflight=2)
    t0 = time.perf_counter()
    ids = [srv.submit(**r) for r in burst]
    for rid in ids:
        srv.wait(rid)
        srv.release(rid)
    t_served = time.perf_counter() - t0
    bst = srv.stats()
    srv.close()
    Lmax, Wmax = 80, int(counts.max())
    out = (torch.empty((Wmax, Lmax), dtype=torch.int32, device=dev),
           torch.empty((Wmax, Lmax), dtype=torch.int64, device=dev),
           torch.empty(Wmax, dtype=torch.int32, device=dev))
    g.sample_walks(1000, 10, out=(out[0].view(-1)[:10_000].view(1000, 10),
                                  out[1].view(-1)[:10_000].view(1000, 10), out[2][:1000]))
    # each request's lengths land in its own slice, counted after the timing
    lens_all = torch.empty(sum(r["num_walks"] for r in burst), dtype=torch.int32, device=dev)
    g.sync()
    t0 = time.perf_counter()
    off = 0
    for r in burst:
        n, L = r["num_walks"], r["max_len"]
        o = (out[0].view(-1)[:n * L].view(n, L), out[1].view(-1)[:n * L].view(n, L),
             lens_all[off:off + n])
        g.sample_walks(n, L, hop_bias=r["hop_bias"], hop_tau=tau, p=0.5, q=2.0, seed=r["seed"],
                       out=o)
        off += n
    g.sync()
    t_plain = time.perf_counter() - t0
    plain_hops = int((lens_all - 1).clamp_min(0).sum(dtype=torch.int64).item())
    active = g.stats()["active_edges"]
    g.close()
    assert plain_hops == bst["hops_done"], "served and plain walks differ"
    # saturation: the highest offered rate whose hops/s still follows the
    # offered load (within 10%) with p99 under 100 ms
    ok = [r for r in [main] + sat
          if r["p99_ms"] is not None and r["p99_ms"] < 100.0 and r["walks"] >= 0.9 * r["offered_walks"]]
    res = {
        "metric": METRIC, "value": main["hops_per_s"], "unit": "hops/s", "n_gpus": 1,
        "steps": int(main["launches"]), "warmup": 0,
        "ms_per_step": main["wall_s"] * 1e3 / max(main["launches"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": "serve", "nodes": spec.num_nodes, "src_zipf": spec.src_s,
                   "stream_edges": spec.num_edges, "window_ns": w["window"],
                   "edges_per_s": rate, "warm_edges": warm_edges,
                   "requests_per_s": w["requests_per_s"], "walks_per_request": "log-uniform 1e2..1e5",
                   "max_len": [10, 40, 80], "hop_biases": ["uniform", "linear", "exponential",
                                                           "node2vec(0.5,2)"],
                   "seconds": live_s},
        "serving": main | {"active_edges_at_start": info["active_edges"],
                           "active_edges_at_end": active},
        "saturation": {"phases": sat,
                       "highest_rate_served": max(r["requests_per_s"] for r in ok) if ok else None,
                       "rule": "hops/s within 10% of the offered walks and p99 < 100 ms"},
        "batched_vs_plain": {
            "requests": nburst, "walks": int(bst["walks_done"]), "hops": plain_hops,
            "served": {"seconds": t_served, "hops_per_s": plain_hops / t_served,
                       "launches": int(bst["launches"])},
            "plain_per_request": {"seconds": t_plain, "hops_per_s": plain_hops / t_plain,
                                  "launches": nburst}},
        "gather_roofline": {"random_sectors_per_s": gather_rate, "sectors_per_hop": 4,
                            "frac": main["hops_per_s"] / (gather_rate / 4) if gather_rate else None},
    }
    print(json.dumps(res), flush=True)


def run_single(args, torch, tw, w, dev, gather_rate, copy_bw):
    """One batch at scale (the "single" workload): each step empties the
    window, ingests the whole 100M-edge batch and samples the 4M walks."""
    if args.hop_bias:
        w = dict(w, hop_bias=args.hop_bias)
    name = args.workload if args.workload != "stream" else "single"
    spec = w["stream"]
    t0 = time.perf_counter()
    src, dst, ts = spec.all()
    gen_s = time.perf_counter() - t0
    span = int(ts.max() - ts.min())
    tau = float(w.get("tau_frac", 0.0) * span)
    d_src = torch.from_numpy(src).to(dev)
    d_dst = torch.from_numpy(dst).to(dev)
    d_ts = torch.from_numpy(ts).to(dev)
    W, L = w["walks"], w["max_len"]
    out = (torch.empty((W, L), dtype=torch.int32, device=dev),
           torch.empty((W, L), dtype=torch.int64, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev))
    print(f"# inputs generated in {gen_s:.1f}s; span {span}; tau {tau}", file=sys.stderr, flush=True)
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    walk_kw = dict(hop_bias=w["hop_bias"], hop_tau=tau, start_bias=w["start_bias"],
                   start_tau=tau, seed=42, dispatch=args.dispatch, out=out,
                   direction=args.direction,
                   **({"p": 0.5, "q": 2.0} if w["hop_bias"] == "node2vec" else {}))

    def step(events=None):
        g.evict_before(INT64_MAX)
        if events:
            events[0].record()
        g.ingest_batch(d_src, d_dst, d_ts)
        if events:
            events[1].record()
        g.sample_walks(W, L, **walk_kw)
        if events:
            events[2].record()

    def count_hops():
        return int((out[2].to(torch.int64) - 1).clamp_min(0).sum().item())

    hops = None
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.warmup:
        hops = count_hops()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ingest_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    walk_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_per_step = wall * 1e3 / args.steps
    hops_check = count_hops()
    assert hops is None or hops_check == hops, "walks changed between steps"
    hops = hops_check
    m_active = g.view_sizes()["m"]

    # walk phase alone under each dispatch (index built once): plain full-walk
    # against the work queue and the cooperative per-step regrouping
    compare = {}
    for disp in ("full_walk", "queue", "coop") if args.direction == "forward" else ("full_walk",):
        kw = dict(walk_kw, dispatch=disp)
        times = []
        for rep in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.sample_walks(W, L, **kw)
            e1.record()
            torch.cuda.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1))
        assert count_hops() == hops, f"{disp} walks differ in length"
        ms = float(np.median(times))
        compare[disp] = {"walk_ms": ms, "walk_hops_per_s": hops / (ms * 1e-3)}

    sweep = (dispatch_sweep(torch, g, W, L, walk_kw, hops)
             if args.direction == "forward" and w["hop_bias"] != "weight" else None)
    weight_build_ms = None
    if w["hop_bias"] == "weight":
        # the build alone: the first walk call after an ingest builds the
        # cumulative weights, the second reuses them
        g.evict_before(INT64_MAX)
        g.ingest_batch(d_src, d_dst, d_ts)
        pair = []
        for rep in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.sample_walks(W, L, **dict(walk_kw, dispatch="full_walk"))
            e1.record()
            torch.cuda.synchronize()
            pair.append(e0.elapsed_time(e1))
        weight_build_ms = pair[0] - pair[1]
    wb = walk_bytes(W, hops, w["hop_bias"])
    st = g.index_stats()
    ib = ingest_bytes(spec.num_edges, m_active, 0, st["jobs"])
    walk_gbs = wb / (walk_ms * 1e-3) / 1e9
    ingest_gbs = ib / (ingest_ms * 1e-3) / 1e9
    per_hop_sectors = 3 if w["hop_bias"] == "uniform" else 4
    gather_roof_hops = gather_rate / per_hop_sectors if gather_rate else None
    walk_hops_s = hops / (walk_ms * 1e-3)
    res = {
        "metric": METRIC,
        "value": hops / (ms_per_step * 1e-3),
        "unit": "hops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+f64",
        "data": "synthetic",
        "config": dict(describe(name, w, tau),
                       **({"direction": "backward"} if args.direction == "backward" else {})),
        "dispatch": args.dispatch,
        "hops_per_step": hops,
        "plain_vs_tuned": compare,
        "dispatch_sweep": sweep,
        "walk_ms": walk_ms,
        "ingest_ms": ingest_ms,
        "walk_hops_per_s": walk_hops_s,
        "ingest_edges_per_s": spec.num_edges / (ingest_ms * 1e-3),
        "roofline": {"bound": "hbm", "kernel": WALK_KERNEL,
                     "achieved": walk_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": walk_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(name),
                     "algorithmic_bytes": wb},
        "roofline_ingest": {"bound": "hbm", "achieved": ingest_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": ingest_gbs / HBM_PEAK_GBS,
                            "algorithmic_bytes": ib,
                            "copy_GBps_measured": copy_bw / 1e9},
        "gather_roofline": {"random_sectors_per_s": gather_rate,
                            "sectors_per_hop": per_hop_sectors,
                            "hops_per_s_roof": gather_roof_hops,
                            "frac": (walk_hops_s / gather_roof_hops) if gather_roof_hops else None},
    }
    if weight_build_ms is not None:
        res["weight_build_ms"] = weight_build_ms
        res["gather_roofline"]["note"] = ("weight-based hops: the binary search's reads come on "
                                          "top of the 4 sectors counted per hop")
    g.close()
    if not args.no_cpu_baseline and w["hop_bias"] != "weight" and args.direction == "forward":
        print("# oracle baseline ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(w, tau, hops)
    return res




def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    import paper_2605_16182_amd as tw

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = synth.workload(args.workload)
    gather_rate, copy_bw = (0.0, 0.0) if args.no_probe else probe_rates(torch, dev)
    print(f"# probe: {gather_rate / 1e9:.2f} G random sectors/s, copy {copy_bw / 1e9:.0f} GB/s",
          file=sys.stderr, flush=True)
    if args.workload == "serve":
        return run_serve(args, torch, tw, w, dev, gather_rate)
    if args.workload == "mixed":
        return run_mixed(args, torch, tw, w, dev, gather_rate)
    if args.workload == "stream":
        res = run_stream(args, torch, tw, w, dev, gather_rate, copy_bw)
        if not args.no_single:
            # the single-batch workload's figures beside the stream's (its
            # own timed steps, after the stream's)
            one = argparse.Namespace(**{**vars(args), "steps": 5, "warmup": 1,
                                        "no_cpu_baseline": True})
            r = run_single(one, torch, tw, synth.workload("single"), dev, gather_rate, copy_bw)
            res["single_batch"] = {k: r[k] for k in (
                "config", "ms_per_step", "value", "hops_per_step", "walk_ms", "ingest_ms",
                "walk_hops_per_s", "ingest_edges_per_s", "plain_vs_tuned", "dispatch_sweep",
                "roofline", "gather_roofline")}
        print(json.dumps(res), flush=True)
        return
    print(json.dumps(run_single(args, torch, tw, w, dev, gather_rate, copy_bw)), flush=True)


if __name__ == "__main__":
    main()
