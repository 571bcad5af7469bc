"""The serving loop (tw_server_*): continuous batching of walk requests
interleaved with ingestion. Every request must return exactly the walks the
plain tw_sample_walks gives on the same window (the ingest batches submitted
before it) with the same parameters, whatever else shares its launch; the
output arena must hold requests back until memory is released."""
import threading

import numpy as np
import pytest

import synth
from gpu_util import gpu_or_skip, to_dev

pytestmark = pytest.mark.gpu


def _stream(V, nb, n):
    w = synth.scaled("serve", V, nb * n)
    return [b for b in w["stream"].batches(n)][:nb]


def _requests(tau, V, torch, seed0):
    starts = to_dev(torch, synth.start_nodes(seed0, 2000, V))[0]
    return [dict(num_walks=3000, max_len=10, hop_bias="uniform", seed=seed0 + 1),
            dict(num_walks=20000, max_len=40, hop_bias="linear", seed=seed0 + 2, walk_id_base=100),
            dict(num_walks=500, max_len=80, hop_bias="exponential", hop_tau=tau,
                 start_bias="exponential", start_tau=tau, seed=seed0 + 3),
            dict(num_walks=4000, max_len=20, hop_bias="node2vec", hop_tau=tau, p=0.5, q=2.0,
                 seed=seed0 + 4),
            dict(num_walks=2000, max_len=15, hop_bias="linear", start_mode="node",
                 start_nodes=starts, seed=seed0 + 5)]


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_server_matches_plain_walks():
    torch, tw = gpu_or_skip()
    V, n = 5000, 40_000
    bs = _stream(V, 3, n)
    span = int(bs[0][2][-1] - bs[0][2][0])
    window = int(1.5 * span)
    tau = 0.1 * span
    dev = [to_dev(torch, *b) for b in bs]
    torch.cuda.synchronize()
    g1 = tw.Graph(V, window=window)
    srv = tw.Server(g1, arena_bytes=256 << 20, max_walks_per_launch=25_000, max_inflight=2)
    ing = [srv.ingest(*dev[0]), srv.ingest(*dev[1])]
    reqs1 = _requests(tau, V, torch, 10)
    ids1 = [srv.submit(**r) for r in reqs1]
    ing.append(srv.ingest(*dev[2]))  # an epoch boundary
    reqs2 = _requests(tau, V, torch, 20)[:3]
    ids2 = [srv.submit(**r) for r in reqs2]
    got1 = [srv.result(i) for i in ids1]
    got2 = [srv.result(i) for i in ids2]
    for i in ing:
        assert srv.wait(i)["status"] == tw.TW_OK
    st = srv.stats()
    assert st["requests_done"] == len(ids1) + len(ids2)
    assert st["ingests"] == 3 and st["launches"] >= 3  # the boundary and the walk cap split them
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["walks_done"] == sum(r["num_walks"] for r in reqs1 + reqs2)
    hops = sum(int((x[2].to(torch.int64) - 1).clamp_min(0).sum()) for x in got1 + got2)
    assert st["hops_done"] == hops
    for i in ids1 + ids2:
        srv.release(i)
    srv.close()
    g2 = tw.Graph(V, window=window)
    g2.ingest_batch(*dev[0])
    g2.ingest_batch(*dev[1])
    for r, got in zip(reqs1, got1):
        _same(got, g2.sample_walks(**r))
    g2.ingest_batch(*dev[2])
    for r, got in zip(reqs2, got2):
        _same(got, g2.sample_walks(**r))
    g2.sync()
    g1.close()
    g2.close()


def test_server_admission_by_memory_and_errors():
    torch, tw = gpu_or_skip()
    V = 3000
    (s, d, t), = _stream(V, 1, 30_000)
    dev = to_dev(torch, s, d, t)
    torch.cuda.synchronize()
    g = tw.Graph(V)
    W, L = 10_000, 20
    one = 4 * W * L + 8 * W * L + 4 * W + 3 * 256  # one request's outputs, aligned
    # a fixed arena: admission by the arena alone
    srv = tw.Server(g, arena_bytes=one + one // 2, max_walks_per_launch=1 << 20,
                    hbm_reserve_bytes=-1)
    srv.wait(srv.ingest(*dev))
    a = srv.submit(W, L, hop_bias="linear", seed=1)
    b = srv.submit(W, L, hop_bias="linear", seed=2)
    assert srv.wait(a) is not None
    # b needs a's memory: it stays queued until a is released
    assert srv.wait(b, timeout_s=0.3) is None
    with pytest.raises(tw.TwError) as ei:
        srv.release(b)  # not finished
    assert ei.value.code == tw.TW_EINVAL
    got_a = srv.result(a)
    srv.release(a)
    got_b = srv.result(b)
    with pytest.raises(tw.TwError) as ei:
        srv.submit(3 * W, L)  # can never fit
    assert ei.value.code == tw.TW_EINVAL
    with pytest.raises(tw.TwError) as ei:
        # the weight-based picker walks forward only
        srv.submit(10, L, hop_bias="weight", hop_tau=100.0, direction="backward")
    assert ei.value.code == tw.TW_EINVAL
    with pytest.raises(tw.TwError):
        srv.wait(a)  # released: unknown
    srv.release(b)
    srv.close()
    g2 = tw.Graph(V)
    g2.ingest_batch(*dev)
    _same(got_a, g2.sample_walks(W, L, hop_bias="linear", seed=1))
    _same(got_b, g2.sample_walks(W, L, hop_bias="linear", seed=2))
    g2.sync()
    g.close()
    g2.close()


def test_server_admission_by_free_device_memory():
    # the same two requests with a reserve the device can keep: the second
    # gets an arena chunk of its own instead of waiting; with a reserve no
    # device has, it waits for the first one's release
    torch, tw = gpu_or_skip()
    V = 3000
    (s, d, t), = _stream(V, 1, 30_000)
    dev = to_dev(torch, s, d, t)
    torch.cuda.synchronize()
    W, L = 10_000, 20
    one = 4 * W * L + 8 * W * L + 4 * W + 3 * 256
    for reserve, grows in ((1 << 30, True), (1 << 50, False)):
        g = tw.Graph(V)
        srv = tw.Server(g, arena_bytes=one + one // 2, max_walks_per_launch=1 << 20,
                        hbm_reserve_bytes=reserve)
        srv.wait(srv.ingest(*dev))
        a = srv.submit(W, L, hop_bias="linear", seed=1)
        b = srv.submit(W, L, hop_bias="linear", seed=2)
        c = srv.submit(3 * W, L, hop_bias="uniform", seed=3)  # larger than the first chunk
        assert srv.wait(a) is not None
        if grows:
            assert srv.wait(b, timeout_s=30.0) is not None
            assert srv.wait(c, timeout_s=30.0) is not None
            st = srv.stats()
            assert st["arena_chunks_added"] >= 2 and st["arena_bytes"] > one + one // 2
        else:
            assert srv.wait(b, timeout_s=0.3) is None
            srv.release(a)
            assert srv.wait(b, timeout_s=30.0) is not None
            assert srv.wait(c, timeout_s=0.3) is None  # fits no chunk, none added
            assert srv.stats()["arena_chunks_added"] == 0
        got = {k: srv.result(k) for k in (b,) + ((a, c) if grows else ())}
        srv.close()
        g.close()
        g2 = tw.Graph(V)
        g2.ingest_batch(*dev)
        _same(got[b], g2.sample_walks(W, L, hop_bias="linear", seed=2))
        if grows:
            _same(got[a], g2.sample_walks(W, L, hop_bias="linear", seed=1))
            _same(got[c], g2.sample_walks(3 * W, L, hop_bias="uniform", seed=3))
        g2.sync()
        g2.close()


def test_server_large_requests_alone():
    # a request of 2^16 walks or more launched alone runs the full-walk
    # kernel on its own rows (rows of a multiple of 4 slots): its walks, hop
    # count and error words must match the plain walks and the other path
    torch, tw = gpu_or_skip()
    V = 4000
    (s, d, t), = _stream(V, 1, 60_000)
    dev = to_dev(torch, s, d, t)
    tau = 0.1 * float(t[-1] - t[0])
    starts_np = synth.start_nodes(9, 70_000, V)
    starts_np[123] = V + 7  # out of range: the request fails with TW_ERANGE
    starts = to_dev(torch, starts_np)[0]
    torch.cuda.synchronize()
    g = tw.Graph(V)
    # one request per launch: the next one would pass the walk cap
    srv = tw.Server(g, arena_bytes=1 << 30, max_walks_per_launch=80_000, max_inflight=1)
    srv.wait(srv.ingest(*dev))
    reqs = [dict(num_walks=70_000, max_len=16, hop_bias="linear", seed=1),
            dict(num_walks=70_000, max_len=18, hop_bias="exponential", hop_tau=tau, seed=2),
            dict(num_walks=80_000, max_len=12, hop_bias="node2vec", hop_tau=tau, p=0.5, q=2.0,
                 seed=3)]
    ids = [srv.submit(**r) for r in reqs]
    bad = srv.submit(70_000, 8, start_mode="node", start_nodes=starts, seed=4)
    got = [srv.result(i) for i in ids]
    assert srv.wait(bad)["status"] == tw.TW_ERANGE
    for i in ids:
        r = srv.wait(i)
        assert r["status"] == tw.TW_OK and r["trial_cap_hits"] == 0
    st = srv.stats()
    hops = sum(int((x[2].to(torch.int64) - 1).clamp_min(0).sum()) for x in got)
    srv.close()
    g.close()
    g2 = tw.Graph(V)
    g2.ingest_batch(*dev)
    plain_hops = 0
    for r, x in zip(reqs, got):
        ref = g2.sample_walks(**r)
        _same(x, ref)
        plain_hops += int((ref[2].to(torch.int64) - 1).clamp_min(0).sum())
    assert hops == plain_hops
    g2.sample_walks(70_000, 8, start_mode="node", start_nodes=starts, seed=4)
    with pytest.raises(tw.TwError):
        g2.sync()
    assert st["hops_done"] >= hops  # the failed request's walks count too
    g2.close()


def test_server_concurrent_submitters():
    # requests from two host threads at once, small and mixed: every result
    # equals the plain walks of its own parameters
    torch, tw = gpu_or_skip()
    V = 4000
    (s, d, t), = _stream(V, 1, 60_000)
    dev = to_dev(torch, s, d, t)
    torch.cuda.synchronize()
    tau = 0.1 * float(t[-1] - t[0])
    g = tw.Graph(V)
    srv = tw.Server(g, arena_bytes=512 << 20, max_walks_per_launch=40_000, max_inflight=3)
    srv.wait(srv.ingest(*dev))
    kinds = ["uniform", "linear", "exponential", "node2vec"]
    params = {}
    lock = threading.Lock()

    def client(k0):
        for j in range(40):
            r = dict(num_walks=100 + 37 * j, max_len=5 + j % 30, hop_bias=kinds[(k0 + j) % 4],
                     hop_tau=tau, p=2.0, q=0.5, seed=1000 * k0 + j, walk_id_base=j)
            rid = srv.submit(**r)
            with lock:
                params[rid] = r

    th = [threading.Thread(target=client, args=(k,)) for k in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    got = {rid: srv.result(rid) for rid in params}
    st = srv.stats()
    assert st["requests_done"] == len(params)
    srv.close()
    g2 = tw.Graph(V)
    g2.ingest_batch(*dev)
    for rid, r in params.items():
        _same(got[rid], g2.sample_walks(**r))
    g2.sync()
    g.close()
    g2.close()


def _served_case(V, tau, torch, seed0, starts):
    """Requests of every hop kind, EDGE and NODE starts, sizes that share and
    split launches."""
    kinds = [("uniform", 0.0, 1.0, 1.0), ("linear", 0.0, 1.0, 1.0),
             ("exponential", tau, 1.0, 1.0), ("node2vec", tau, 0.5, 2.0),
             ("node2vec", tau, 2.0, 0.5), ("node2vec", tau, 1.0, 1.0)]
    reqs = []
    for j in range(7):
        kind, ht, p, q = kinds[(seed0 + j) % len(kinds)]
        r = dict(num_walks=[700, 3000, 150, 12_000, 1200, 450, 5000][j],
                 max_len=[10, 40, 80, 12, 25, 6, 30][j], hop_bias=kind, hop_tau=ht, p=p, q=q,
                 seed=seed0 * 100 + j, walk_id_base=37 * j)
        if j % 3 == 1:
            r.update(start_mode="node", start_nodes=starts)
        if j % 2 == 0:
            r.update(start_bias="exponential", start_tau=tau)
        reqs.append(r)
    return reqs


def test_served_mix_matches_oracle():
    # ingest batches interleaved with 21 requests through one server; each
    # request's walks are compared with the oracle's on that request's epoch
    # window (the batches submitted before it), on sampled walk ids, under
    # the boundary tolerance
    import oracle
    from gpu_util import compare_walks
    torch, tw = gpu_or_skip()
    V, n = 6000, 50_000
    bs = _stream(V, 4, n)
    span = int(bs[0][2][-1] - bs[0][2][0])
    window = int(1.5 * span)
    tau = 0.1 * window
    dev = [to_dev(torch, *b) for b in bs]
    starts_np = synth.start_nodes(31, 12_000, V)
    starts = to_dev(torch, starts_np)[0]
    torch.cuda.synchronize()
    g = tw.Graph(V, window=window)
    srv = tw.Server(g, arena_bytes=512 << 20, max_walks_per_launch=8_000, max_inflight=3)
    plan = []  # (epoch, request params, id)
    ingests = [srv.ingest(*dev[0]), srv.ingest(*dev[1])]
    for ep in (2, 3, 4):
        for r in _served_case(V, tau, torch, ep, starts):
            plan.append((ep, r, srv.submit(**r)))
        if ep < 4:
            ingests.append(srv.ingest(*dev[ep]))
    results = {rid: srv.result(rid) for _, _, rid in plan}
    for i in ingests:
        assert srv.wait(i)["status"] == tw.TW_OK
    for _, _, rid in plan:
        assert srv.wait(rid)["status"] == tw.TW_OK
    st = srv.stats()
    assert st["requests_done"] == len(plan) >= 20
    assert st["launches"] < len(plan)  # requests shared launches
    srv.close()
    g.close()
    og = oracle.OracleGraph(V, window=window)
    og.ingest_batch(*bs[0])
    epoch = 1
    rng = np.random.default_rng(5)
    totals = {}
    for ep, r, rid in plan:
        while epoch < ep:
            og.ingest_batch(*bs[epoch])
            epoch += 1
        W, L = r["num_walks"], r["max_len"]
        idx = np.unique(np.concatenate([[0, W - 1], rng.integers(0, W, 600)])).astype(np.int64)
        kw = {k: v for k, v in r.items() if k not in ("num_walks", "max_len", "start_nodes")}
        if r.get("start_mode") == "node":
            kw["start_nodes"] = starts_np
        ref = og.sample_walks(W, L, walk_idx=idx, with_margin=True, **kw)
        nodes, ts, lens = (x.cpu().numpy() for x in results[rid])
        exact = r["hop_bias"] in ("uniform", "linear") and r.get("start_bias") is None
        same, boundary = compare_walks((nodes[idx], ts[idx], lens[idx]), ref, exact,
                                       label=f"served epoch {ep} {r['hop_bias']} "
                                             f"{r.get('start_mode', 'edge')}",
                                       kind=r["hop_bias"])
        totals[r["hop_bias"]] = totals.get(r["hop_bias"], 0) + boundary
        assert boundary <= 2, (ep, r["hop_bias"], same, boundary)


def test_served_out_of_range_start_fails_only_its_request():
    torch, tw = gpu_or_skip()
    V = 2000
    (s, d, t), = _stream(V, 1, 20_000)
    dev = to_dev(torch, s, d, t)
    bad = to_dev(torch, np.array([3, V + 5, 7], np.int32))[0]
    torch.cuda.synchronize()
    g = tw.Graph(V)
    srv = tw.Server(g, arena_bytes=64 << 20)
    srv.wait(srv.ingest(*dev))
    ok1 = srv.submit(500, 8, hop_bias="linear", seed=1)
    bad_id = srv.submit(3, 8, start_mode="node", start_nodes=bad, seed=2)
    ok2 = srv.submit(500, 8, hop_bias="uniform", seed=3)
    assert srv.wait(ok1)["status"] == tw.TW_OK
    assert srv.wait(bad_id)["status"] == tw.TW_ERANGE
    assert srv.wait(ok2)["status"] == tw.TW_OK
    for i in (ok1, bad_id, ok2):
        srv.release(i)
    # the graph's own flags are untouched: later calls succeed
    assert srv.wait(srv.ingest(*dev))["status"] == tw.TW_OK
    srv.close()
    g.ingest_batch(*dev)
    g.sync()
    g.close()


def test_backward_walks_after_a_server_session():
    # the in-view of a directed graph receives the batches the server ingests
    import oracle
    from gpu_util import compare_walks
    torch, tw = gpu_or_skip()
    V, n = 3000, 30_000
    bs = _stream(V, 3, n)
    dev = [to_dev(torch, *b) for b in bs]
    torch.cuda.synchronize()
    g = tw.Graph(V)
    og = oracle.OracleGraph(V, backward=True)
    g.ingest_batch(*dev[0])
    og.ingest_batch(*bs[0])
    g.sample_walks(100, 5, direction="backward")  # creates the in-view
    g.sync()
    srv = tw.Server(g, arena_bytes=64 << 20)
    for b in dev[1:]:
        assert srv.wait(srv.ingest(*b))["status"] == tw.TW_OK
    srv.close()
    for b in bs[1:]:
        og.ingest_batch(*b)
    W, L = 5000, 12
    nodes, ts, lens = g.sample_walks(W, L, hop_bias="linear", direction="backward", seed=4)
    g.sync()
    ref = og.sample_walks(W, L, hop_bias="linear", direction="backward", seed=4,
                          with_margin=True)
    same, boundary = compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()),
                                   ref, exact=True)
    assert same == W
    g.close()


def test_served_backward_and_weight_requests_match_oracle():
    # backward requests (the first one makes the in-view from the window; the
    # server's later batches reach it) and weight-based requests (two time
    # scales: they take separate launches) mixed with forward ones, each
    # compared with the oracle on its epoch window
    import oracle
    from gpu_util import compare_walks
    torch, tw = gpu_or_skip()
    V, n = 4000, 40_000
    bs = _stream(V, 3, n)
    span = int(bs[0][2][-1] - bs[0][2][0])
    window = int(1.5 * span)
    tau = 0.1 * window
    dev = [to_dev(torch, *b) for b in bs]
    torch.cuda.synchronize()
    g = tw.Graph(V, window=window)
    srv = tw.Server(g, arena_bytes=256 << 20, max_walks_per_launch=6_000, max_inflight=3)
    cases = [dict(hop_bias="linear", direction="backward"),
             dict(hop_bias="weight", hop_tau=tau),
             dict(hop_bias="exponential", hop_tau=tau, direction="backward",
                  start_bias="exponential", start_tau=tau),
             dict(hop_bias="uniform"),
             dict(hop_bias="weight", hop_tau=2 * tau),
             dict(hop_bias="node2vec", hop_tau=tau, p=0.5, q=2.0, direction="backward"),
             dict(hop_bias="weight", hop_tau=tau),
             dict(hop_bias="uniform", direction="backward")]
    plan = []
    ingests = [srv.ingest(*dev[0]), srv.ingest(*dev[1])]
    for ep in (2, 3):
        for j, c in enumerate(cases):
            r = dict(num_walks=[900, 2500, 400, 3000][j % 4], max_len=[12, 20, 30, 8][j % 4],
                     seed=ep * 50 + j, walk_id_base=11 * j, **c)
            plan.append((ep, r, srv.submit(**r)))
        if ep == 2:
            ingests.append(srv.ingest(*dev[2]))
    results = {rid: srv.result(rid) for _, _, rid in plan}
    for i in ingests:
        assert srv.wait(i)["status"] == tw.TW_OK
    for _, _, rid in plan:
        assert srv.wait(rid)["status"] == tw.TW_OK
    # a backward weight-based request is refused at submission
    with pytest.raises(tw.TwError) as ei:
        srv.submit(10, 5, hop_bias="weight", hop_tau=tau, direction="backward")
    assert ei.value.code == tw.TW_EINVAL
    srv.close()
    g.close()
    og = oracle.OracleGraph(V, window=window, backward=True)
    og.ingest_batch(*bs[0])
    og.ingest_batch(*bs[1])
    epoch = 2
    rng = np.random.default_rng(9)
    for ep, r, rid in plan:
        while epoch < ep:
            og.ingest_batch(*bs[epoch])
            epoch += 1
        W, L = r["num_walks"], r["max_len"]
        idx = np.unique(np.concatenate([[0, W - 1], rng.integers(0, W, 500)])).astype(np.int64)
        kw = {k: v for k, v in r.items() if k not in ("num_walks", "max_len")}
        ref = og.sample_walks(W, L, walk_idx=idx, with_margin=True, **kw)
        nodes, ts, lens = (x.cpu().numpy() for x in results[rid])
        exact = r["hop_bias"] in ("uniform", "linear") and r.get("start_bias") is None
        same, boundary = compare_walks((nodes[idx], ts[idx], lens[idx]), ref, exact,
                                       label=f"served {r.get('direction', 'forward')} "
                                             f"{r['hop_bias']} epoch {ep}",
                                       kind=r["hop_bias"])
        assert boundary <= 2, (ep, r, same, boundary)
        assert float(ref["len"].mean()) > 1.5, (ep, r)
