"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Indices, eviction, uniform and linear walks must be bit-exact. Exponential
and node2vec walks must be identical except where a pick's draw lies within
1e-6 of a CDF boundary of the exact law; the rate is reported.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_walks, gpu_or_skip, to_dev

pytestmark = pytest.mark.gpu


def _views_equal(g, og):
    v = {k: t.cpu().numpy() for k, t in g.export_views().items()}
    o = og.views()
    for k in o:
        assert np.array_equal(v[k], o[k]), f"view {k} differs"


def _stream_batches(rng, V, nb, n_lo, n_hi, step, spread):
    t_base = 0
    for _ in range(nb):
        n = int(rng.integers(n_lo, n_hi))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V, n).astype(np.int32)
        ts = (t_base + rng.integers(-spread, spread, n)).astype(np.int64)
        t_base += step
        yield src, dst, ts


@pytest.mark.parametrize("directed", [True, False])
@pytest.mark.parametrize("window", [0, 700])
def test_stream_index_parity_small(directed, window):
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(7 + window + directed)
    V = 53
    g = tw.Graph(V, directed=directed, window=window)
    og = oracle.OracleGraph(V, directed=directed, window=window)
    for b, (s, d, t) in enumerate(_stream_batches(rng, V, 10, 0, 300, 150, 400)):
        s_, d_, t_ = to_dev(torch, s, d, t)
        info = g.ingest_batch(s_, d_, t_)
        oinfo = og.ingest_batch(s, d, t)
        assert info == oinfo, (b, info, oinfo)
        _views_equal(g, og)
        if b == 5:
            cut = 600
            assert g.evict_before(cut) == og.evict_before(cut)
            assert g.evict_before(cut) == 0
            _views_equal(g, og)
    g.close()


@pytest.mark.parametrize("directed", [True, False])
def test_wide_and_narrow_timestamp_spans(directed):
    # a batch whose timestamps span 2^32 or more is sorted by source with
    # 12-byte records, a narrower one as packed 8-byte words; mixed batches
    # (late ones merged into the runs) must give the same index and walks
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(23 + directed)
    V = 97
    g = tw.Graph(V, directed=directed)
    og = oracle.OracleGraph(V, directed=directed)
    t_base = 1 << 40
    for b in range(8):
        n = int(rng.integers(200, 3000))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V, n).astype(np.int32)
        wide = b % 3 != 1
        span = (1 << 34) if wide else 5000
        ts = (t_base + rng.integers(-span, span, n)).astype(np.int64)
        t_base += span // 2
        s_, d_, t_ = to_dev(torch, src, dst, ts)
        assert g.ingest_batch(s_, d_, t_) == og.ingest_batch(src, dst, ts), b
        _views_equal(g, og)
    W, L = 4000, 12
    for kind in ("uniform", "linear"):
        nodes, tts, lens = g.sample_walks(W, L, hop_bias=kind, start_bias=kind, seed=5)
        g.sync()
        r = og.sample_walks(W, L, hop_bias=kind, start_bias=kind, seed=5)
        assert np.array_equal(lens.cpu().numpy(), r["len"])
        assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
        assert np.array_equal(tts.cpu().numpy(), r["ts"])
    # every node's run here spans more than 2^30 time units, so its fence
    # keys are shifted and the exponential rate reads the first candidate's
    # timestamp from its group record (the other tests' graphs, with narrower
    # spans, read it from the level-0 fence key)
    for kind, tau in (("exponential", 3.0e8), ("exponential", 2.0e3), ("node2vec", 3.0e8)):
        kw = dict(hop_bias=kind, hop_tau=tau, start_bias="exponential", start_tau=tau, seed=6,
                  **({"p": 0.5, "q": 2.0} if kind == "node2vec" else {}))
        for disp in ("full_walk", "queue"):
            nodes, tts, lens = g.sample_walks(W, L, dispatch=disp, **kw)
            g.sync()
            r = og.sample_walks(W, L, with_margin=True, **kw)
            compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()), r,
                          exact=False, label=f"spans/{directed}/{kind}/{tau:g}/{disp}",
                          kind=kind)
    g.close()


def test_index_parity_multi_tile_ragged():
    # several radix / scan tiles (4096) with a ragged tail, duplicate timestamps
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(11)
    V = 5003
    g = tw.Graph(V, window=3_000)
    og = oracle.OracleGraph(V, window=3_000)
    for s, d, t in _stream_batches(rng, V, 6, 40_000, 90_001, 1000, 2500):
        s_, d_, t_ = to_dev(torch, s, d, t)
        assert g.ingest_batch(s_, d_, t_) == og.ingest_batch(s, d, t)
    _views_equal(g, og)
    g.close()


@pytest.mark.parametrize("V,spread", [(300, 200), (100_003, 60_000), (5003, 50_000_000)])
def test_index_parity_nine_bit_digits(V, spread):
    # sorts whose key bits take one radix pass fewer with 9-bit digits: node
    # ids of 9 and 17 bits, timestamp keys of 17 and 27 bits (unsorted batches)
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(V + spread)
    g = tw.Graph(V)
    og = oracle.OracleGraph(V)
    for s, d, t in _stream_batches(rng, V, 4, 40_000, 90_001, 1000, spread):
        s_, d_, t_ = to_dev(torch, s, d, t)
        assert g.ingest_batch(s_, d_, t_) == og.ingest_batch(s, d, t)
    _views_equal(g, og)
    g.close()


def test_ingest_rejects_out_of_range_ids():
    torch, tw = gpu_or_skip()
    g = tw.Graph(10)
    s, d, t = to_dev(torch, np.array([1, 2], np.int32), np.array([3, 4], np.int32),
                     np.array([5, 6], np.int64))
    g.ingest_batch(s, d, t)
    bad = to_dev(torch, np.array([1, 10], np.int32), np.array([3, 4], np.int32),
                 np.array([7, 8], np.int64))
    with pytest.raises(tw.TwError) as ei:
        g.ingest_batch(*bad)
    assert ei.value.code == tw.TW_ERANGE
    assert g.view_sizes()["m"] == 2
    g.close()


def _tiny_workload(V=4000, m=60000, **over):
    w = synth.scaled("tiny", V, m, **over)
    return w, w["stream"].all()


WALK_CASES = [
    # hop, hop tau, p, q, start, start tau, mode
    ("uniform", 0.0, 1, 1, "uniform", 0.0, "edge"),
    ("linear", 0.0, 1, 1, "linear", 0.0, "edge"),
    ("linear", 0.0, 1, 1, "uniform", 0.0, "node"),
    ("exponential", 0.0, 1, 1, "exponential", 0.0, "edge"),
    ("exponential", 5e4, 1, 1, "exponential", 1e5, "edge"),
    ("exponential", 2e4, 1, 1, "linear", 0.0, "node"),
    ("node2vec", 5e4, 0.5, 2.0, "uniform", 0.0, "edge"),
    ("node2vec", 5e4, 2.0, 0.5, "exponential", 5e4, "node"),
    ("node2vec", 5e4, 1.0, 1.0, "uniform", 0.0, "edge"),
    ("weight", 5e4, 1, 1, "uniform", 0.0, "edge"),
    ("weight", 2e4, 1, 1, "exponential", 5e4, "node"),
    ("weight", 0.0, 1, 1, "linear", 0.0, "edge"),
]


@pytest.mark.parametrize("dispatch", ["full_walk", "coop", "queue"])
@pytest.mark.parametrize("ci", range(len(WALK_CASES)),
                         ids=["-".join(map(str, c[:1] + c[4:])) for c in WALK_CASES])
@pytest.mark.parametrize("directed", [True, False])
def test_walk_parity(ci, directed, dispatch):
    torch, tw = gpu_or_skip()
    hk, ht, p, q, sk, st, mode = WALK_CASES[ci]
    V, m = 4000, 60000
    w = synth.scaled("tiny", V, m)
    w["stream"].directed = directed
    src, dst, ts = w["stream"].all()
    g = tw.Graph(V, directed=directed)
    og = oracle.OracleGraph(V, directed=directed)
    g.ingest_batch(*to_dev(torch, src, dst, ts))
    og.ingest_batch(src, dst, ts)
    W, L, seed, base = 20000, 16, 42, 777
    starts = synth.start_nodes(9, W, V)
    st_dev = to_dev(torch, starts)[0]
    nodes, tts, lens = g.sample_walks(W, L, hop_bias=hk, hop_tau=ht, p=p, q=q, start_bias=sk,
                                      start_tau=st, start_mode=mode, start_nodes=st_dev,
                                      seed=seed, walk_id_base=base, dispatch=dispatch)
    g.sync()
    r = og.sample_walks(W, L, hop_bias=hk, hop_tau=ht, p=p, q=q, start_bias=sk, start_tau=st,
                        start_mode=mode, start_nodes=starts, seed=seed, walk_id_base=base,
                        with_margin=True)
    exact = hk in ("uniform", "linear") and sk in ("uniform", "linear")
    same, boundary = compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()),
                                   r, exact, label=f"walk_parity {dispatch} directed={directed} "
                                                   f"{hk}/{sk}/{mode}", kind=hk)
    hops = int(np.maximum(r["len"] - 1, 0).sum())
    print(f"{dispatch} {hk}/{sk}/{mode}: {same}/{W} identical, boundary mismatches {boundary} "
          f"({boundary / max(hops, 1):.2e} per hop)")
    assert boundary <= max(2, W // 2000)
    g.close()


def test_empty_graph_and_degenerate_walks():
    torch, tw = gpu_or_skip()
    g = tw.Graph(6)
    nodes, ts, lens = g.sample_walks(4, 5)
    g.sync()
    assert (lens.cpu().numpy() == 0).all() and (nodes.cpu().numpy() == -1).all()
    st = to_dev(torch, np.array([0, 5, 3, 1], np.int32))[0]
    nodes, ts, lens = g.sample_walks(4, 5, start_mode="node", start_nodes=st)
    g.sync()
    assert (lens.cpu().numpy() == 1).all()
    s, d, t = (np.array([0, 1, 2, 0], np.int32), np.array([1, 2, 0, 2], np.int32),
               np.array([1, 2, 3, 1], np.int64))
    g.ingest_batch(*to_dev(torch, s, d, t))
    og = oracle.OracleGraph(6)
    og.ingest_batch(s, d, t)
    for L in (1, 2, 7):
        for mode in ("edge", "node"):
            stn = np.array([0, 1, 4, 2, 5], np.int32)
            nodes, ts, lens = g.sample_walks(5, L, start_mode=mode, start_nodes=to_dev(torch, stn)[0],
                                             seed=3)
            g.sync()
            r = og.sample_walks(5, L, start_mode=mode, start_nodes=stn, seed=3)
            assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
            assert np.array_equal(ts.cpu().numpy(), r["ts"])
            assert np.array_equal(lens.cpu().numpy(), r["len"])
    bad = to_dev(torch, np.array([0, 6], np.int32))[0]
    g.sample_walks(2, 4, start_mode="node", start_nodes=bad)
    with pytest.raises(tw.TwError) as ei:
        g.sync()
    assert ei.value.code == tw.TW_ERANGE
    g.sync()  # the flag is cleared once reported
    for kw in (dict(max_len=0), dict(hop_bias="node2vec", p=0.0), dict(start_mode="node")):
        args = dict(num_walks=2, max_len=4)
        args.update(kw)
        with pytest.raises(tw.TwError) as ei:
            g.sample_walks(**args)
        assert ei.value.code == tw.TW_EINVAL
    g.close()


def test_windowed_stream_walks_parity():
    # streaming window: walks after every batch, linear hops, uniform start
    torch, tw = gpu_or_skip()
    w = synth.scaled("stream", 20000, 400_000)
    spec = w["stream"]
    window = 150_000 * 10
    g = tw.Graph(spec.num_nodes, window=window)
    og = oracle.OracleGraph(spec.num_nodes, window=window)
    for b, (s, d, t) in enumerate(spec.batches(50_000)):
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t)
        nodes, ts, lens = g.sample_walks(4000, 40, hop_bias="linear", seed=b)
        g.sync()
        r = og.sample_walks(4000, 40, hop_bias="linear", seed=b)
        assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
        assert np.array_equal(ts.cpu().numpy(), r["ts"])
        assert np.array_equal(lens.cpu().numpy(), r["len"])
    g.close()


@pytest.mark.parametrize("directed", [True, False])
def test_node2vec_pairs_follow_the_window(directed):
    # node2vec's pair table is built by the first node2vec walk and then kept
    # current by every ingest and eviction (unsorted batches, late drops,
    # explicit evictions); a small window on a few nodes makes pairs leave
    # and come back, and fills the table past three quarters so it is also
    # rebuilt; every batch's node2vec walks against the oracle's
    from gpu_util import compare_walks
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(61)
    V, window = 40, 3_000
    g = tw.Graph(V, directed=directed, window=window)
    og = oracle.OracleGraph(V, directed=directed, window=window)
    t0 = 0
    for b in range(16):
        n = int(rng.integers(100, 400))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (t0 + rng.integers(-300, 1000, n)).astype(np.int64)
        t0 += 1000
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        if b % 5 == 3:
            cut = t0 - 1500
            assert g.evict_before(cut) == og.evict_before(cut)
        for p_, q_ in ((0.5, 2.0), (2.0, 0.25)):
            kw = dict(hop_bias="node2vec", hop_tau=200.0, p=p_, q=q_, seed=b)
            nodes, ts, lens = g.sample_walks(3000, 12, **kw)
            g.sync()
            r = og.sample_walks(3000, 12, with_margin=True, **kw)
            same, boundary = compare_walks(
                (nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()), r, False,
                label=f"node2vec pairs batch {b} directed={directed}", kind="node2vec")
            assert boundary <= 2, (b, same, boundary)
    g.close()


@pytest.mark.parametrize("groups", [1, 15, 16, 17, 255, 256, 257, 4097, 70_001])
def test_fence_search_depths(groups):
    # one hub whose out-edges all loop back to itself, so every hop searches
    # the hub's groups again with a later time; two edges share each
    # timestamp, and a second node keeps the hub off position 0 of the view
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(groups)
    V = 3
    ts_groups = np.sort(rng.choice(np.arange(10 * groups + 10), groups, replace=False))
    t = np.repeat(ts_groups, 2).astype(np.int64)
    src = np.full(len(t), 1, np.int32)
    dst = np.where(np.arange(len(t)) % 2 == 0, 1, 2).astype(np.int32)
    src = np.concatenate([src, np.array([0, 2], np.int32)])
    dst = np.concatenate([dst, np.array([1, 1], np.int32)])
    t = np.concatenate([t, np.array([0, 5], np.int64)])
    g = tw.Graph(V)
    og = oracle.OracleGraph(V)
    g.ingest_batch(*to_dev(torch, src, dst, t))
    og.ingest_batch(src, dst, t)
    _views_equal(g, og)
    W, L = 3000, 24
    starts = np.full(W, 1, np.int32)
    for kind, dispatch in (("uniform", "full_walk"), ("linear", "full_walk"),
                           ("uniform", "coop"), ("linear", "coop")):
        nodes, tts, lens = g.sample_walks(W, L, hop_bias=kind, start_bias=kind,
                                          start_mode="node",
                                          start_nodes=to_dev(torch, starts)[0], seed=5,
                                          dispatch=dispatch)
        g.sync()
        r = og.sample_walks(W, L, hop_bias=kind, start_bias=kind, start_mode="node",
                            start_nodes=starts, seed=5)
        assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
        assert np.array_equal(tts.cpu().numpy(), r["ts"])
        assert np.array_equal(lens.cpu().numpy(), r["len"])
    # the exponential rate takes the first candidate's timestamp from its
    # level-0 fence key (the keys are unshifted here) at every fence depth
    tau = 0.1 * float(ts_groups[-1] - ts_groups[0] + 1)
    for kind, dispatch in (("exponential", "full_walk"), ("exponential", "queue"),
                           ("exponential", "coop"), ("node2vec", "full_walk")):
        kw = dict(hop_bias=kind, hop_tau=tau, start_bias="exponential", start_tau=tau,
                  start_mode="node", seed=7, **({"p": 0.5, "q": 2.0} if kind == "node2vec" else {}))
        nodes, tts, lens = g.sample_walks(W, L, start_nodes=to_dev(torch, starts)[0],
                                          dispatch=dispatch, **kw)
        g.sync()
        r = og.sample_walks(W, L, start_nodes=starts, with_margin=True, **kw)
        compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()), r,
                      exact=False, label=f"fence/{groups}/{kind}/{dispatch}", kind=kind)
    g.close()


@pytest.mark.parametrize("L", [1, 2, 3, 40])
def test_dispatches_agree_on_lengths_and_edge_cases(L):
    # the cooperative and queue paths against the full-walk path on a hub-heavy graph:
    # identical bytes for every walk, including walks that end at the start
    torch, tw = gpu_or_skip()
    w = synth.scaled("single", 5000, 300_000)
    s, d, t = w["stream"].all()
    g = tw.Graph(5000)
    g.ingest_batch(*to_dev(torch, s, d, t))
    span = float(t.max() - t.min())
    outs = []
    for dispatch in ("full_walk", "coop", "queue"):
        r = g.sample_walks(30_000, L, hop_bias="exponential", hop_tau=0.1 * span,
                           start_bias="exponential", start_tau=0.1 * span, seed=9,
                           dispatch=dispatch)
        g.sync()
        outs.append([x.cpu().numpy() for x in r])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)
    g.close()


COOP_TUNINGS = [
    # regroup, wave_min, panel, sync
    (0, 64, 4096, 1), (0, 1, 64, 1), (0, 16, 8192, 4), (0, 40, 2048, 7),
    (1, 64, 2048, 1), (1, 8, 512, 4), (1, 1, 8192, 64),
]


@pytest.mark.parametrize("ci", range(len(COOP_TUNINGS)),
                         ids=["-".join(map(str, c)) for c in COOP_TUNINGS])
@pytest.mark.parametrize("hop", ["linear", "node2vec"])
def test_coop_tunings_equal_full_walk(ci, hop):
    # every setting of the cooperative dispatch's tunables gives the walks
    # of the full-walk kernel byte for byte (the RNG is keyed by walk and
    # hop), on a hub-heavy graph whose hubs engage the wavefront and
    # workgroup tiers; uniform walks also against the oracle
    torch, tw = gpu_or_skip()
    regroup, wave_min, panel, sync = COOP_TUNINGS[ci]
    w = synth.scaled("mixed", 4000, 200_000)
    spec = w["stream"]
    s, d, t = spec.all()
    g = tw.Graph(4000, directed=spec.directed)
    g.ingest_batch(*to_dev(torch, s, d, t))
    tau = 0.1 * float(t.max() - t.min())
    kw = dict(hop_bias=hop, hop_tau=tau, p=0.5, q=2.0, start_bias="linear", seed=21,
              walk_id_base=3)
    ref = [x.cpu().numpy() for x in g.sample_walks(20_000, 30, dispatch="full_walk", **kw)]
    g.set_tuning("coop", coop_regroup=regroup, coop_wave_min=wave_min, coop_panel=panel,
                 coop_sync=sync)
    assert g.tuning()["coop_sync"] == sync
    got = [x.cpu().numpy() for x in g.sample_walks(20_000, 30, dispatch="auto", **kw)]
    g.sync()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    if hop == "linear":
        og = oracle.OracleGraph(4000, directed=spec.directed)
        og.ingest_batch(s, d, t)
        idx = np.arange(0, 20_000, 7)
        r = og.sample_walks(20_000, 30, walk_idx=idx, with_margin=True,
                            **{k: v for k, v in kw.items() if k not in ("p", "q", "hop_tau")})
        assert compare_walks(tuple(x[idx] for x in got), r, exact=True) == (len(idx), 0)
    with pytest.raises(tw.TwError):
        g.set_tuning("coop", coop_panel=100)  # not a multiple of 64
    g.close()


@pytest.mark.parametrize("sorted_arrivals", [True, False])
def test_long_stream_compactions(sorted_arrivals):
    # many batches under a short window: the window's start moves through
    # the edge-store buffers and forces repeated compaction / regrowth;
    # explicit evictions in between
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(21 + sorted_arrivals)
    V, window = 997, 4_000
    g = tw.Graph(V, window=window)
    og = oracle.OracleGraph(V, window=window)
    t0 = 0
    for b in range(60):
        n = int(rng.integers(500, 3000))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        if sorted_arrivals:
            t = (t0 + np.sort(rng.integers(0, 1000, n))).astype(np.int64)
        else:
            t = (t0 + rng.integers(-1500, 1000, n)).astype(np.int64)
        t0 += 1000
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        if b % 7 == 3:
            cut = t0 - 2500
            assert g.evict_before(cut) == og.evict_before(cut)
        if b % 10 == 9:
            _views_equal(g, og)
            nodes, ts, lens = g.sample_walks(500, 12, hop_bias="linear",
                                             start_bias="exponential", start_tau=300.0, seed=b)
            g.sync()
            r = og.sample_walks(500, 12, hop_bias="linear", start_bias="exponential",
                                start_tau=300.0, seed=b, with_margin=True)
            compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()), r, False)
    g.close()


def test_sorted_batches_staged_in_place():
    # sorted batches of mixed sizes, so that they are staged in the free tail
    # of the window buffers, in the alternate buffers or in the staging
    # buffers; each kind of update in turn: appended after the window, merged
    # into its end, a late prefix under the window cut followed by records
    # after the window, and a jump that evicts the whole window
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(31)
    V, window = 101, 5_000
    g = tw.Graph(V, window=window)
    og = oracle.OracleGraph(V, window=window)
    t0 = 0
    for b in range(48):
        n = int(rng.choice([50, 400, 1500, 5000, 20000]))
        kind = b % 4
        if kind == 0:
            t = rng.integers(t0 + 1, t0 + 1001, n)
        elif kind == 1:
            t = rng.integers(t0 - 800, t0 + 500, n)
        elif kind == 2:
            late = n // 3
            t = np.concatenate([rng.integers(t0 - 6500, t0 - 4100, late),
                                rng.integers(t0 + 1, t0 + 999, n - late - 1), [t0 + 999]])
        else:
            t = rng.integers(t0 + 3 * window, t0 + 3 * window + 1000, n)
        t = np.sort(t).astype(np.int64)
        t0 = max(t0, int(t[-1]))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        _views_equal(g, og)
        if b % 8 == 7:
            nodes, ts, lens = g.sample_walks(300, 10, hop_bias="uniform", seed=b)
            g.sync()
            r = og.sample_walks(300, 10, hop_bias="uniform", seed=b)
            assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
            assert np.array_equal(ts.cpu().numpy(), r["ts"])
            assert np.array_equal(lens.cpu().numpy(), r["len"])
    g.close()


@pytest.mark.parametrize("directed", [True, False])
def test_sorted_batches_continuing_the_last_timestamp(directed):
    # sorted batches whose first timestamp equals the window's last one: the
    # batch's first record continues the window's last timestamp group, so
    # the group starts counted while the batch is staged must compare it with
    # the window's last record; batch sizes span several 4096-record tiles,
    # end raggedly, and some batches hold that one timestamp only
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(53 + directed)
    V = 211
    g = tw.Graph(V, directed=directed)
    og = oracle.OracleGraph(V, directed=directed)
    t_last = 100
    for b in range(14):
        n = int(rng.choice([1, 63, 4096, 4097, 9000, 13001]))
        if b % 5 == 4:
            t = np.full(n, t_last, np.int64)
        else:
            t = np.sort(rng.integers(t_last, t_last + 300, n)).astype(np.int64)
            t[0] = t_last
        t_last = int(t[-1])
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        _views_equal(g, og)
    for kind in ("uniform", "exponential"):
        nodes, ts, lens = g.sample_walks(500, 12, hop_bias=kind, hop_tau=50.0, start_bias=kind,
                                         start_tau=50.0, seed=9)
        g.sync()
        r = og.sample_walks(500, 12, hop_bias=kind, hop_tau=50.0, start_bias=kind,
                            start_tau=50.0, seed=9, with_margin=True)
        same, boundary = compare_walks((nodes.cpu().numpy(), ts.cpu().numpy(),
                                        lens.cpu().numpy()), r, kind == "uniform")
        assert boundary <= 2 and same >= 490, (kind, same, boundary)
    g.close()


@pytest.mark.parametrize("groups", [9, 100, 5_000, 100_000])
def test_weight_search_on_uneven_timestamps(groups):
    # a hub whose group timestamps grow as the cube of their rank (gaps far
    # from even), some groups of two edges: the weight picker's search starts
    # at the group an even spacing predicts and must gallop from there to
    # the group a bisection of all candidates finds
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(groups + 5)
    V = 3
    t_groups = (np.arange(1, groups + 1, dtype=np.int64) ** 3) * 7
    reps = np.where(rng.random(groups) < 0.2, 2, 1)
    t = np.repeat(t_groups, reps)
    src = np.full(len(t), 1, np.int32)
    dst = np.where(rng.random(len(t)) < 0.8, 1, 2).astype(np.int32)
    src = np.concatenate([src, np.array([0, 2], np.int32)])
    dst = np.concatenate([dst, np.array([1, 1], np.int32)])
    t = np.concatenate([t, np.array([0, 3], np.int64)])
    g = tw.Graph(V)
    og = oracle.OracleGraph(V)
    g.ingest_batch(*to_dev(torch, src, dst, t))
    og.ingest_batch(src, dst, t)
    W, L = 3000, 24
    starts = np.full(W, 1, np.int32)
    span = float(t_groups[-1] - t_groups[0])
    for tau in (1e-3 * span, 0.1 * span, 10.0 * span):
        for dispatch in ("full_walk", "queue"):
            kw = dict(hop_bias="weight", hop_tau=tau, start_bias="uniform", start_mode="node",
                      seed=21)
            nodes, tts, lens = g.sample_walks(W, L, start_nodes=to_dev(torch, starts)[0],
                                              dispatch=dispatch, **kw)
            g.sync()
            r = og.sample_walks(W, L, start_nodes=starts, with_margin=True, **kw)
            compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()), r,
                          exact=False, label=f"weight_uneven/{groups}/{tau:g}/{dispatch}",
                          kind="weight")
    g.close()


@pytest.mark.parametrize("at_ingest", [False, True])
def test_weight_walks_follow_the_window(at_ingest):
    # the weight-based picker's cumulative weights are rebuilt after every
    # change of the window (ingest, eviction) and of the time scale, either
    # by the first weight-based walk or by the ingest itself
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(41)
    V, window = 301, 6_000
    g = tw.Graph(V, window=window)
    if at_ingest:
        g.set_ingest_weights(300.0)
    og = oracle.OracleGraph(V, window=window)
    t0 = 0
    for b in range(12):
        n = int(rng.integers(2000, 8000))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (t0 + rng.integers(-500, 1000, n)).astype(np.int64)
        t0 += 1000
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        if b % 4 == 2:
            cut = t0 - 4000
            assert g.evict_before(cut) == og.evict_before(cut)
        for tau in ((300.0, 3000.0) if b % 3 == 0 else (300.0,)):
            nodes, ts, lens = g.sample_walks(4000, 12, hop_bias="weight", hop_tau=tau, seed=b)
            g.sync()
            r = og.sample_walks(4000, 12, hop_bias="weight", hop_tau=tau, seed=b,
                                with_margin=True)
            same, boundary = compare_walks(
                (nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()), r, False,
                label=f"weight window batch {b} tau {tau} at ingest {at_ingest}", kind="weight")
            assert boundary <= 2, (b, tau, same, boundary)
    g.set_ingest_weights(None)
    g.close()


BACK_CASES = [
    # hop, hop tau, p, q, start, start tau, mode
    ("uniform", 0.0, 1, 1, "uniform", 0.0, "edge"),
    ("linear", 0.0, 1, 1, "linear", 0.0, "node"),
    ("exponential", 5e4, 1, 1, "exponential", 1e5, "edge"),
    ("exponential", 0.0, 1, 1, "uniform", 0.0, "node"),
    ("node2vec", 5e4, 0.5, 2.0, "uniform", 0.0, "edge"),
]


@pytest.mark.parametrize("ci", range(len(BACK_CASES)),
                         ids=["-".join(map(str, c[:1] + c[4:])) for c in BACK_CASES])
@pytest.mark.parametrize("directed", [True, False])
def test_backward_walk_parity(ci, directed):
    torch, tw = gpu_or_skip()
    hk, ht, p, q, sk, st, mode = BACK_CASES[ci]
    V, m = 4000, 60000
    w = synth.scaled("tiny", V, m)
    w["stream"].directed = directed
    src, dst, ts = w["stream"].all()
    g = tw.Graph(V, directed=directed)
    og = oracle.OracleGraph(V, directed=directed, backward=True)
    g.ingest_batch(*to_dev(torch, src, dst, ts))
    og.ingest_batch(src, dst, ts)
    W, L, seed, base = 20000, 16, 43, 9
    starts = synth.start_nodes(10, W, V)
    kw = dict(hop_bias=hk, hop_tau=ht, p=p, q=q, start_bias=sk, start_tau=st, start_mode=mode,
              seed=seed, walk_id_base=base)
    nodes, tts, lens = g.sample_walks(W, L, start_nodes=to_dev(torch, starts)[0],
                                      direction="backward", **kw)
    # the work queue runs the same walks
    qn, qt, ql = g.sample_walks(W, L, start_nodes=to_dev(torch, starts)[0],
                                direction="backward", dispatch="queue", **kw)
    g.sync()
    assert torch.equal(qn, nodes) and torch.equal(qt, tts) and torch.equal(ql, lens)
    r = og.sample_walks(W, L, start_nodes=starts, with_margin=True, direction="backward", **kw)
    exact = hk in ("uniform", "linear") and sk in ("uniform", "linear")
    same, boundary = compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()),
                                   r, exact, label=f"backward directed={directed} {hk}/{sk}/{mode}",
                                   kind=hk)
    print(f"backward {hk}/{sk}/{mode} directed={directed}: {same}/{W} identical, "
          f"{boundary} at a boundary; mean length {float(r['len'].mean()):.2f}")
    assert boundary <= max(2, W // 2000)
    assert float(r["len"].mean()) > 2.5
    g.close()


def test_backward_walks_follow_the_stream():
    # the in-view is created mid-stream from the window, then fed every batch
    # and eviction; forward walks are unchanged by it
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(71)
    V, window = 401, 5_000
    g = tw.Graph(V, window=window)
    og = oracle.OracleGraph(V, window=window, backward=True)
    t0 = 0
    for b in range(14):
        n = int(rng.integers(2000, 9000))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (t0 + rng.integers(-700, 1000, n)).astype(np.int64)
        t0 += 1000
        assert g.ingest_batch(*to_dev(torch, s, d, t)) == og.ingest_batch(s, d, t), b
        if b % 5 == 3:
            cut = t0 - 3500
            assert g.evict_before(cut) == og.evict_before(cut)
        if b < 4:
            continue  # the in-view appears at batch 4
        for direction in ("backward", "forward"):
            nodes, ts, lens = g.sample_walks(3000, 10, hop_bias="linear", seed=b,
                                             direction=direction)
            g.sync()
            r = og.sample_walks(3000, 10, hop_bias="linear", seed=b, direction=direction)
            assert np.array_equal(nodes.cpu().numpy(), r["nodes"]), (b, direction)
            assert np.array_equal(ts.cpu().numpy(), r["ts"]), (b, direction)
            assert np.array_equal(lens.cpu().numpy(), r["len"]), (b, direction)
    with pytest.raises(tw.TwError) as ei:
        g.sample_walks(10, 5, hop_bias="weight", hop_tau=5.0, direction="backward")
    assert ei.value.code == tw.TW_EINVAL
    with pytest.raises(tw.TwError) as ei:
        g.sample_walks(10, 5, dispatch="coop", direction="backward")
    assert ei.value.code == tw.TW_EINVAL
    g.close()


def test_fresh_graph_reports_no_error():
    # device error flags start cleared: a fresh graph's first synchronising
    # calls succeed, before and after edge-start walks
    torch, tw = gpu_or_skip()
    for _ in range(3):
        g = tw.Graph(50)
        g.sync()
        s, d, t = to_dev(torch, np.arange(10, dtype=np.int32), np.arange(10, dtype=np.int32)[::-1].copy(),
                         np.arange(10, dtype=np.int64))
        g.ingest_batch(s, d, t)
        g.sample_walks(100, 5)
        g.sync()
        g.ingest_batch(s, d, t + 100)
        g.close()


@pytest.mark.parametrize("directed", [True, False])
def test_ingest_without_info(directed):
    # ingests that leave the window's range and group count on the device
    # (no info requested): explicit evictions, biased start picks (which read
    # them on the device) and the counts must match the oracle's, and the
    # range is read back on request
    from gpu_util import compare_walks
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(17)
    V, window = 400, 5_000
    g = tw.Graph(V, directed=directed, window=window)
    og = oracle.OracleGraph(V, directed=directed, window=window)
    t0 = 0
    for b in range(10):
        n = int(rng.integers(1000, 3000))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (t0 + rng.integers(-400, 1000, n)).astype(np.int64)
        t0 += 1000
        assert g.ingest_batch(*to_dev(torch, s, d, t), info=False) is None
        oi = og.ingest_batch(s, d, t)
        lu = g.last_update()
        assert (lu["accepted"], lu["dropped_late"], lu["evicted"], lu["active_edges"]) == (
            oi["accepted"], oi["dropped_late"], oi["evicted"], oi["active_edges"]), b
        cut = t0 - window + (300 if b % 3 == 0 else -2000)  # sometimes nothing to evict
        assert g.evict_before(cut) == og.evict_before(cut), b
        for kind in ("linear", "exponential"):
            nodes, ts, lens = g.sample_walks(2000, 8, hop_bias="uniform", start_bias=kind,
                                             start_tau=300.0, seed=b)
            g.sync()
            r = og.sample_walks(2000, 8, hop_bias="uniform", start_bias=kind, start_tau=300.0,
                                seed=b, with_margin=True)
            same, boundary = compare_walks(
                (nodes.cpu().numpy(), ts.cpu().numpy(), lens.cpu().numpy()), r, kind == "linear")
            assert boundary <= 2, (b, kind, same, boundary)
    st = g.stats()
    ots = og.views()["ts"]
    assert (st["t_min"], st["t_max"], st["active_edges"]) == (int(ots[0]), int(ots[-1]), len(ots))
    _views_equal(g, og)
    g.close()


def test_walk_errors_reported_by_the_next_ingest():
    # a walk's out-of-range start node is reported by the next ingest, which
    # then ingests nothing; an eviction with nothing to evict neither
    # synchronises nor reports it
    torch, tw = gpu_or_skip()
    w = synth.scaled("tiny", 500, 6000)
    s, d, t = w["stream"].all()
    half = len(s) // 2
    g = tw.Graph(500, window=int(t.max()) // 2)
    og = oracle.OracleGraph(500, window=int(t.max()) // 2)
    order = np.argsort(t, kind="stable")
    s, d, t = s[order], d[order], t[order]
    g.ingest_batch(*to_dev(torch, s[:half], d[:half], t[:half]))
    og.ingest_batch(s[:half], d[:half], t[:half])
    bad = to_dev(torch, np.array([3, 900], np.int32))[0]
    g.sample_walks(2, 4, start_mode="node", start_nodes=bad)
    assert g.evict_before(int(t[0]) - 1) == 0  # nothing to evict: no report
    batch = to_dev(torch, s[half:], d[half:], t[half:])
    with pytest.raises(tw.TwError) as ei:
        g.ingest_batch(*batch)
    assert ei.value.code == tw.TW_ERANGE
    _views_equal(g, og)  # nothing ingested
    assert g.ingest_batch(*batch) == og.ingest_batch(s[half:], d[half:], t[half:])
    _views_equal(g, og)
    g.sync()
    g.close()


def test_deep_fence_hub():
    # a hub with millions of timestamp groups: many fence levels for any fan
    torch, tw = gpu_or_skip()
    rng = np.random.default_rng(77)
    G = 3_000_000
    t = np.sort(rng.choice(np.arange(4 * G), G, replace=False)).astype(np.int64)
    src = np.zeros(G, np.int32)
    dst = np.where(rng.random(G) < 0.9, 0, 1).astype(np.int32)
    src = np.concatenate([src, np.array([1], np.int32)])
    dst = np.concatenate([dst, np.array([0], np.int32)])
    t = np.concatenate([t, np.array([1], np.int64)])
    g = tw.Graph(2)
    og = oracle.OracleGraph(2)
    g.ingest_batch(*to_dev(torch, src, dst, t))
    og.ingest_batch(src, dst, t)
    W, L = 20_000, 30
    for kind in ("uniform", "linear"):
        nodes, tts, lens = g.sample_walks(W, L, hop_bias=kind, start_bias=kind, seed=13)
        g.sync()
        r = og.sample_walks(W, L, hop_bias=kind, start_bias=kind, seed=13)
        assert np.array_equal(nodes.cpu().numpy(), r["nodes"])
        assert np.array_equal(tts.cpu().numpy(), r["ts"])
    tau = 0.1 * float(t[:G].max() - t[:G].min())
    kw = dict(hop_bias="exponential", hop_tau=tau, start_bias="exponential", start_tau=tau,
              seed=14)
    nodes, tts, lens = g.sample_walks(W, L, **kw)
    g.sync()
    r = og.sample_walks(W, L, with_margin=True, **kw)
    compare_walks((nodes.cpu().numpy(), tts.cpu().numpy(), lens.cpu().numpy()), r,
                  exact=False, label="deep_fence_hub/exponential", kind="exponential")
    g.close()
