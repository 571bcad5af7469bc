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
    srv = tw.Server(g, arena_bytes=one + one // 2, max_walks_per_launch=1 << 20)
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
        srv.submit(10, L, hop_bias="weight", hop_tau=100.0)  # not served
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
