"""Batched walks (uneven lengths, mixed hop biases) through the persistent
work-queue kernel, the queue dispatch of plain walks, the autotuner and
hipGraph replay of a walk launch, all against the oracle or the full-walk
kernel.

A batched walk must be the walk the oracle draws for the same id, start and
hop bias, cut to the walk's length limit (the RNG is keyed by walk, hop and
trial), under the same boundary tolerance as the plain walks.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_walks, gpu_or_skip, to_dev

pytestmark = pytest.mark.gpu


def _mixed_graph(torch, tw, V=3000, m=40_000):
    w = synth.scaled("mixed", V, m)
    spec = w["stream"]
    s, d, t = spec.all()
    g = tw.Graph(V, directed=spec.directed)
    g.ingest_batch(*to_dev(torch, s, d, t))
    og = oracle.OracleGraph(V, directed=spec.directed)
    og.ingest_batch(s, d, t)
    tau = 0.1 * float(t.max() - t.min())
    return g, og, tau


def _oracle_batch(og, W, L, biases, lims, bidx, seed, base, start_mode="edge", starts=None,
                  direction="forward"):
    """Oracle walks of a batch: every bias group at length L, then each walk
    cut to its limit."""
    nodes = np.full((W, L), -1, np.int32)
    ts = np.full((W, L), np.iinfo(np.int64).min, np.int64)
    lens = np.zeros(W, np.int32)
    margin = np.ones((W, L))
    for b, (kind, tau, p, q) in enumerate(biases):
        idx = np.flatnonzero(bidx == b)
        if len(idx) == 0:
            continue
        r = og.sample_walks(W, L, hop_bias=kind, hop_tau=tau, p=p, q=q, start_mode=start_mode,
                            start_nodes=starts, seed=seed, walk_id_base=base, walk_idx=idx,
                            with_margin=True, direction=direction)
        nodes[idx], ts[idx], lens[idx], margin[idx] = r["nodes"], r["ts"], r["len"], r["margin"]
    for i in range(W):
        k = lims[i]
        nodes[i, k:] = -1
        ts[i, k:] = np.iinfo(np.int64).min
        lens[i] = min(lens[i], k)
    return dict(nodes=nodes, ts=ts, len=lens, margin=margin)


@pytest.mark.parametrize("dispatch", ["queue", "full_walk"])
@pytest.mark.parametrize("ragged", [False, True])
@pytest.mark.parametrize("start_mode", ["edge", "node"])
def test_batch_mixed_parity(ragged, start_mode, dispatch):
    torch, tw = gpu_or_skip()
    g, og, tau = _mixed_graph(torch, tw)
    biases = synth.mixed_biases(tau)
    W, L, seed, base = 12_000, 30, 7, 1000
    lims = synth.walk_lengths(3, W, 1, L)
    bidx = ((base + np.arange(W)) % len(biases)).astype(np.uint8)
    starts = synth.start_nodes(4, W, 3000)
    st = to_dev(torch, starts)[0] if start_mode == "node" else None
    nodes, ts, lens, row = g.sample_walks_batch(
        W, L, biases, max_lens=to_dev(torch, lims)[0], start_mode=start_mode, start_nodes=st,
        seed=seed, walk_id_base=base, ragged=ragged, dispatch=dispatch)
    g.sync()
    ref = _oracle_batch(og, W, L, biases, lims, bidx, seed, base, start_mode, starts)
    if ragged:
        r = row.cpu().numpy()
        assert r[0] == 0 and np.array_equal(np.diff(r), lims) and r[-1] == lims.sum()
        fn, ft = nodes.cpu().numpy(), ts.cpu().numpy()
        gn = np.full((W, L), -1, np.int32)
        gt = np.full((W, L), np.iinfo(np.int64).min, np.int64)
        for i in range(W):
            gn[i, :lims[i]] = fn[r[i]:r[i + 1]]
            gt[i, :lims[i]] = ft[r[i]:r[i + 1]]
    else:
        gn, gt = nodes.cpu().numpy(), ts.cpu().numpy()
    same, boundary = compare_walks((gn, gt, lens.cpu().numpy()), ref, exact=False,
                                   label=f"batch {dispatch} ragged={ragged} {start_mode}",
                                   kind="mixed")
    print(f"batch {dispatch} ragged={ragged} {start_mode}: {same}/{W} identical, "
          f"{boundary} at a boundary")
    assert boundary <= max(2, W // 2000)
    g.close()


@pytest.mark.parametrize("dispatch", ["queue", "full_walk"])
@pytest.mark.parametrize("directed", [True, False])
def test_batch_backward_parity(directed, dispatch):
    # backward walks of uneven lengths and mixed biases on the in-view (a
    # directed graph builds it on this first backward call)
    torch, tw = gpu_or_skip()
    V, m = 3000, 40_000
    w = synth.scaled("mixed", V, m)
    spec = w["stream"]
    spec.directed = directed
    s, d, t = spec.all()
    g = tw.Graph(V, directed=directed)
    g.ingest_batch(*to_dev(torch, s, d, t))
    og = oracle.OracleGraph(V, directed=directed, backward=True)
    og.ingest_batch(s, d, t)
    tau = 0.1 * float(t.max() - t.min())
    biases = synth.mixed_biases(tau)
    W, L, seed, base = 12_000, 24, 17, 300
    lims = synth.walk_lengths(5, W, 1, L)
    bidx = ((base + np.arange(W)) % len(biases)).astype(np.uint8)
    nodes, ts, lens, _ = g.sample_walks_batch(W, L, biases, max_lens=to_dev(torch, lims)[0],
                                              seed=seed, walk_id_base=base, dispatch=dispatch,
                                              direction="backward")
    g.sync()
    ref = _oracle_batch(og, W, L, biases, lims, bidx, seed, base, direction="backward")
    same, boundary = compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()),
                                   ref, exact=False,
                                   label=f"backward batch {dispatch} directed={directed}",
                                   kind="mixed")
    print(f"backward batch {dispatch} directed={directed}: {same}/{W} identical, "
          f"{boundary} at a boundary; mean length {float(ref['len'].mean()):.2f}")
    assert boundary <= max(2, W // 2000)
    assert float(ref["len"].mean()) > 2.5
    # the weight-based picker walks forward only
    with pytest.raises(tw.TwError) as ei:
        g.sample_walks_batch(10, 5, [("weight", 5.0, 1.0, 1.0)], direction="backward")
    assert ei.value.code == tw.TW_EINVAL
    g.close()


def test_batch_explicit_bias_indices_and_errors():
    torch, tw = gpu_or_skip()
    g, og, tau = _mixed_graph(torch, tw, V=2000, m=20_000)
    biases = synth.mixed_biases(tau)[:3]
    W, L = 3000, 12
    lims = np.full(W, L, np.int32)
    bidx = synth.uniform_i64(8, 1, 0, W, 0, 3).astype(np.uint8)
    nodes, ts, lens, _ = g.sample_walks_batch(W, L, biases, max_lens=to_dev(torch, lims)[0],
                                              bias_idx=to_dev(torch, bidx)[0], seed=5)
    g.sync()
    ref = _oracle_batch(og, W, L, biases, lims, bidx, 5, 0)
    compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()), ref,
                  exact=False)
    # a limit above max_len and a bias index past the table: length 0, EINVAL
    bad_l = lims.copy()
    bad_l[5] = L + 1
    _, _, lens, _ = g.sample_walks_batch(W, L, biases, max_lens=to_dev(torch, bad_l)[0], seed=5)
    with pytest.raises(tw.TwError) as ei:
        g.sync()
    assert ei.value.code == tw.TW_EINVAL and int(lens[5].item()) == 0
    bad_b = bidx.copy()
    bad_b[7] = 3
    g.sample_walks_batch(W, L, biases, bias_idx=to_dev(torch, bad_b)[0], seed=5)
    with pytest.raises(tw.TwError) as ei:
        g.sync()
    assert ei.value.code == tw.TW_EINVAL
    g.sync()  # cleared once reported
    with pytest.raises(tw.TwError):
        g.sample_walks_batch(W, L, [])
    g.close()


@pytest.mark.parametrize("dispatch", ["queue", "full_walk"])
def test_batch_with_weight_bias(dispatch):
    # the weight-based picker among the other biases of one launch; two
    # weight-based biases of one launch must share their time scale
    torch, tw = gpu_or_skip()
    g, og, tau = _mixed_graph(torch, tw)
    biases = synth.mixed_biases(tau)[:4] + [("weight", tau, 1.0, 1.0), ("weight", tau, 1.0, 1.0)]
    W, L, seed, base = 9_000, 24, 11, 50
    lims = synth.walk_lengths(6, W, 1, L)
    bidx = ((base + np.arange(W)) % len(biases)).astype(np.uint8)
    nodes, ts, lens, _ = g.sample_walks_batch(W, L, biases, max_lens=to_dev(torch, lims)[0],
                                              seed=seed, walk_id_base=base, dispatch=dispatch)
    g.sync()
    ref = _oracle_batch(og, W, L, biases, lims, bidx, seed, base)
    same, boundary = compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()),
                                   ref, exact=False)
    assert boundary <= max(2, W // 2000), (same, boundary)
    with pytest.raises(tw.TwError) as ei:
        g.sample_walks_batch(W, L, [("weight", tau, 1.0, 1.0), ("weight", 2 * tau, 1.0, 1.0)])
    assert ei.value.code == tw.TW_EINVAL
    g.close()


@pytest.mark.parametrize("ci", range(4))
def test_queue_dispatch_equals_full_walk(ci):
    torch, tw = gpu_or_skip()
    case = [("exponential", "exponential", "edge", 80), ("linear", "uniform", "node", 40),
            ("node2vec", "uniform", "edge", 20), ("uniform", "linear", "edge", 1)][ci]
    hop, start, mode, L = case
    w = synth.scaled("single", 20_000, 1_000_000)
    s, d, t = w["stream"].all()
    g = tw.Graph(20_000)
    g.ingest_batch(*to_dev(torch, s, d, t))
    tau = 0.1 * float(t.max() - t.min())
    starts = to_dev(torch, synth.start_nodes(2, 100_000, 20_000))[0]
    outs = []
    for disp in ("full_walk", "queue"):
        r = g.sample_walks(100_000, L, hop_bias=hop, hop_tau=tau, p=0.5, q=2.0,
                           start_bias=start, start_tau=tau, start_mode=mode, start_nodes=starts,
                           seed=3, walk_id_base=11, dispatch=disp)
        g.sync()
        outs.append([x.cpu().numpy() for x in r])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    g.close()


def test_autotune_then_auto_equals_full_walk():
    torch, tw = gpu_or_skip()
    w = synth.scaled("single", 20_000, 1_000_000)
    s, d, t = w["stream"].all()
    g = tw.Graph(20_000)
    g.ingest_batch(*to_dev(torch, s, d, t))
    tau = 0.1 * float(t.max() - t.min())
    kw = dict(hop_bias="exponential", hop_tau=tau, start_bias="exponential", start_tau=tau)
    best = g.autotune(200_000, 40, sample=100_000, **kw)
    assert best["dispatch"] in ("full_walk", "coop", "queue")
    ref = [x.cpu().numpy() for x in g.sample_walks(50_000, 40, dispatch="full_walk", **kw)]
    got = [x.cpu().numpy() for x in g.sample_walks(50_000, 40, dispatch="auto", **kw)]
    g.sync()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    g.close()


@pytest.mark.parametrize("dispatch", ["full_walk", "queue"])
def test_walk_launch_graph_replay(dispatch):
    # one walk launch captured in a HIP graph (after a warm-up call that
    # allocates what it needs), replayed with eager work in between; every
    # replay must equal the eager result
    torch, tw = gpu_or_skip()
    w = synth.scaled("single", 20_000, 1_000_000)
    s, d, t = w["stream"].all()
    cap = torch.cuda.Stream()
    g = tw.Graph(20_000, stream=cap)
    batch = to_dev(torch, s, d, t)
    torch.cuda.synchronize()
    g.ingest_batch(*batch)
    tau = 0.1 * float(t.max() - t.min())
    W, L = 50_000, 40
    out = (torch.empty((W, L), dtype=torch.int32, device="cuda"),
           torch.empty((W, L), dtype=torch.int64, device="cuda"),
           torch.empty(W, dtype=torch.int32, device="cuda"))
    kw = dict(hop_bias="exponential", hop_tau=tau, seed=21, dispatch=dispatch, out=out)
    g.sample_walks(W, L, **kw)
    g.sync()
    eager = [x.cpu().numpy().copy() for x in out]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        g.sample_walks(W, L, **kw)
    for rep in range(3):
        for x in out:
            x.fill_(7)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, out):
            assert np.array_equal(a, b.cpu().numpy()), f"replay {rep} differs"
    del graph
    g.close()


@pytest.mark.parametrize("mode", ["full_walk", "queue", "noalloc", "batch"])
def test_walk_graph_replays_over_a_stream(mode):
    # a walk launch recorded once in a HIP graph reads the window from
    # device-side state that every update keeps current: replayed after each
    # later batch (ingest and eviction run eagerly in between) it must equal
    # an eager call with the same parameters; when the buffers moved
    # (walk_layout changed) the launch is recorded again
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(31)
    V, window = 3001, 40_000
    cap = torch.cuda.Stream()
    g = tw.Graph(V, window=window, stream=cap)
    W, L, tau = 20_000, 16, 8_000.0
    biases = [("uniform", 0.0, 1.0, 1.0), ("linear", 0.0, 1.0, 1.0),
              ("exponential", tau, 1.0, 1.0), ("node2vec", tau, 0.5, 2.0)]
    lims = to_dev(torch, synth.walk_lengths(6, W, 2, L))[0]

    def alloc():
        return (torch.empty((W, L), dtype=torch.int32, device="cuda"),
                torch.empty((W, L), dtype=torch.int64, device="cuda"),
                torch.empty(W, dtype=torch.int32, device="cuda"))

    def walk(out, seed):
        kw = dict(hop_bias="exponential", hop_tau=tau, start_bias="exponential",
                  start_tau=tau, seed=seed)
        if mode == "batch":
            g.sample_walks_batch(W, L, biases, max_lens=lims, seed=seed, out=out)
        elif mode == "noalloc":
            g.sample_walks_noalloc(W, L, out, **kw)
        else:
            g.sample_walks(W, L, dispatch=mode, out=out, **kw)

    eager_out, graph_out = alloc(), alloc()
    graph, token, records, replays = None, None, 0, 0
    t0 = 0
    for b in range(14):
        n = int(rng.integers(20_000, 40_000))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = np.sort(t0 + rng.integers(0, 5_000, n)).astype(np.int64)
        t0 += 5_000
        torch.cuda.synchronize()
        g.ingest_batch(*to_dev(torch, s, d, t))
        if b % 4 == 3:
            g.evict_before(t0 - window // 2)
        if b < 2:
            continue
        walk(eager_out, 77)
        g.sync()
        eager = [x.cpu().numpy().copy() for x in eager_out]
        if graph is None or g.walk_layout() != token:
            del graph
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=cap):
                walk(graph_out, 77)
            token = g.walk_layout()
            records += 1
            continue
        for x in graph_out:
            x.fill_(7)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, x in zip(eager, graph_out):
            assert np.array_equal(a, x.cpu().numpy()), f"batch {b}: replay differs"
        replays += 1
    print(f"walk graph {mode}: {records} recordings, {replays} replays checked")
    assert replays >= 3
    del graph
    g.close()
