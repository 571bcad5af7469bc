"""GPU parity at the full sizes the benchmark runs, in its launch
configuration (dispatch AUTO, the same walk parameters and seeds).

* single batch: 2M nodes, 100M edges, 4M exponential walks of length 80.
  Every view array is compared with the oracle's element by element; walks
  are compared on a sample of walk ids that the oracle computes one by one,
  and every walk is checked for the properties that hold at any size.
* stream: 50M nodes, 10M-edge batches under a 2e9 window, 30 batches, so
  the window has filled (about 200M active edges) and eviction runs on every
  later batch. The oracle ingests the final window content in one batch: for
  a stream whose timestamps never decrease, the canonical order of the window
  is its arrival order, so the index is a function of the window content
  alone. Views are compared in full and the last batch's walks (uniform start,
  linear hops: exact pickers) bit for bit on sampled ids.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_walks, gpu_or_skip, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

INT64_MIN = np.iinfo(np.int64).min


def _views_equal(g, og):
    o = og.views()
    v = g.export_views()
    for k in list(o):
        got = v.pop(k).cpu().numpy()
        assert got.shape == o[k].shape, f"view {k}: shape {got.shape} vs {o[k].shape}"
        assert np.array_equal(got, o[k]), f"view {k} differs"
        del o[k], got


def _walk_properties(torch, nodes, ts, lens, V, L):
    """Checks on every walk that hold at any size: length in [0, L], node ids
    in range inside the walk and -1 after it, ts[0] = INT64_MIN, strictly
    increasing timestamps inside the walk, INT64_MIN after it."""
    assert int(lens.min()) >= 0 and int(lens.max()) <= L
    pos = torch.arange(L, device=nodes.device).unsqueeze(0)
    inside = pos < lens.unsqueeze(1).to(torch.int64)
    assert bool(((nodes >= 0) & (nodes < V))[inside].all())
    assert bool((nodes[~inside] == -1).all())
    assert bool((ts[~inside] == INT64_MIN).all())
    assert bool((ts[:, 0] == INT64_MIN).all())
    inc = ts[:, 1:] > ts[:, :-1]
    need = inside[:, 1:] & (pos[:, 1:] >= 2)
    assert bool(inc[need].all())


def _sample_ids(W, n, seed):
    rng = np.random.default_rng(seed)
    ids = np.concatenate([[0, 1, W - 2, W - 1], np.linspace(0, W - 1, n // 2).astype(np.int64),
                          rng.integers(0, W, n // 2)])
    return np.unique(ids).astype(np.int64)


@pytest.mark.timeout(900)
def test_single_batch_full_scale():
    torch, tw = gpu_or_skip()
    w = synth.workload("single")
    spec = w["stream"]
    src, dst, ts = spec.all()
    tau = float(w["tau_frac"] * int(ts.max() - ts.min()))
    W, L = w["walks"], w["max_len"]
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=w["window"])
    info = g.ingest_batch(*to_dev(torch, src, dst, ts))
    assert info["accepted"] == spec.num_edges and info["active_edges"] == spec.num_edges
    kw = dict(hop_bias=w["hop_bias"], hop_tau=tau, start_bias=w["start_bias"], start_tau=tau,
              seed=42)
    nodes, wts, lens = g.sample_walks(W, L, **kw)
    g.sync()
    _walk_properties(torch, nodes, wts, lens, spec.num_nodes, L)
    # the cooperative dispatch gives the same walks at full size
    c_nodes, c_ts, c_lens = g.sample_walks(W, L, dispatch="coop", **kw)
    g.sync()
    assert torch.equal(c_lens, lens) and torch.equal(c_nodes, nodes) and torch.equal(c_ts, wts)
    del c_nodes, c_ts, c_lens

    og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed, window=w["window"])
    og.ingest_batch(src, dst, ts)
    del src, dst, ts
    _views_equal(g, og)
    idx = _sample_ids(W, 4096, 5)
    r = og.sample_walks(W, L, walk_idx=idx, with_margin=True, threads=oracle.threads(), **kw)
    sel = torch.from_numpy(idx).to(nodes.device)
    gpu = (nodes.index_select(0, sel).cpu().numpy(), wts.index_select(0, sel).cpu().numpy(),
           lens.index_select(0, sel).cpu().numpy())
    same, boundary = compare_walks(gpu, r, exact=False)
    print(f"single full scale: {same}/{len(idx)} sampled walks identical, {boundary} at a "
          f"CDF boundary")
    assert boundary <= max(2, len(idx) // 2000)
    g.close()


@pytest.mark.timeout(900)
def test_stream_window_full_scale():
    torch, tw = gpu_or_skip()
    w = synth.workload("stream")
    spec = w["stream"]
    B, W, L, window = w["batch_edges"], w["walks"], w["max_len"], w["window"]
    nb = 30
    g = tw.Graph(spec.num_nodes, directed=spec.directed, window=window)
    kept = []          # host copies of what may still be in the window
    t_prev = INT64_MIN
    for b, (s, d, t) in enumerate(spec.batches(B)):
        if b >= nb:
            break
        assert t[0] >= t_prev and bool((np.diff(t) >= 0).all())
        t_prev = int(t[-1])
        info = g.ingest_batch(*to_dev(torch, s, d, t))
        cut = info["t_max"] - window
        g.evict_before(cut)
        kept.append((s, d, t))
        while kept and kept[0][2][-1] < cut:
            kept.pop(0)
        nodes, wts, lens = g.sample_walks(W, L, hop_bias=w["hop_bias"],
                                          start_bias=w["start_bias"], seed=b)
    g.sync()
    assert kept
    _walk_properties(torch, nodes, wts, lens, spec.num_nodes, L)
    # the window content: the kept suffix of the arrivals
    s = np.concatenate([k[0] for k in kept])
    d = np.concatenate([k[1] for k in kept])
    t = np.concatenate([k[2] for k in kept])
    first = int(np.searchsorted(t, cut, side="left"))
    s, d, t = s[first:], d[first:], t[first:]
    del kept
    st = g.stats()
    assert st["active_edges"] == len(t) and st["t_min"] == int(t[0])
    assert len(t) > 150_000_000, "the window should have filled"
    og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed, window=window)
    og.ingest_batch(s, d, t)
    del s, d, t
    _views_equal(g, og)
    idx = _sample_ids(W, 4096, 6)
    r = og.sample_walks(W, L, hop_bias=w["hop_bias"], start_bias=w["start_bias"], seed=nb - 1,
                        walk_idx=idx, threads=oracle.threads())
    sel = torch.from_numpy(idx).to(nodes.device)
    assert np.array_equal(nodes.index_select(0, sel).cpu().numpy(), r["nodes"])
    assert np.array_equal(wts.index_select(0, sel).cpu().numpy(), r["ts"])
    assert np.array_equal(lens.index_select(0, sel).cpu().numpy(), r["len"])
    g.close()
