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
    same, boundary = compare_walks(gpu, r, exact=False, label="single full scale (sampled ids)",
                                   kind="exponential")
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


def _ragged_properties(torch, nodes, ts, lens, row, lims, V):
    """The per-walk properties of _walk_properties on packed rows: walk i owns
    slots [row[i], row[i] + lims[i])."""
    W = lens.numel()
    lim = lims.to(torch.int64)
    assert int((lens < 0).sum()) == 0 and bool((lens.to(torch.int64) <= lim).all())
    owner = torch.repeat_interleave(torch.arange(W, device=nodes.device), lim)
    pos = torch.arange(owner.numel(), device=nodes.device) - row[:-1].index_select(0, owner)
    inside = pos < lens.to(torch.int64).index_select(0, owner)
    assert bool(((nodes >= 0) & (nodes < V))[inside].all())
    assert bool((nodes[~inside] == -1).all())
    assert bool((ts[~inside] == INT64_MIN).all())
    assert bool((ts.index_select(0, row[:-1]) == INT64_MIN).all())
    nxt = torch.zeros_like(inside)
    nxt[:-1] = inside[1:] & (pos[1:] >= 2)
    assert bool((ts[1:] > ts[:-1])[nxt[:-1]].all())
    del owner, pos, inside, nxt


@pytest.mark.timeout(900)
def test_mixed_batch_full_scale():
    # 1M nodes, 20M undirected edges (40M records), Zipf-Mandelbrot 1.5 with
    # rank offset 200 (hubs of about 1e5 edges); 8M walks with lengths
    # uniform in [5, 120] and six hop biases (walk id mod 6) in one work-queue
    # launch on packed rows, as the mixed-batch benchmark runs it
    torch, tw = gpu_or_skip()
    w = synth.workload("mixed")
    spec = w["stream"]
    src, dst, ts = spec.all()
    deg = np.bincount(np.concatenate([src, dst]), minlength=spec.num_nodes)
    assert 5e4 < deg.max() < 5e5, deg.max()
    tau = float(w["tau_frac"] * int(ts.max() - ts.min()))
    g = tw.Graph(spec.num_nodes, directed=spec.directed)
    info = g.ingest_batch(*to_dev(torch, src, dst, ts))
    assert info["active_edges"] == 2 * spec.num_edges
    W, L = w["walks"], w["max_len"]
    lims_np = synth.walk_lengths(4, W, w["min_len"], L)
    lims = to_dev(torch, lims_np)[0]
    biases = synth.mixed_biases(tau)
    rows = g.row_offsets(lims)
    nodes, wts, lens, row = g.sample_walks_batch(W, L, biases, max_lens=lims, seed=42,
                                                 ragged=True, rows=rows, dispatch="queue")
    g.sync()
    _ragged_properties(torch, nodes, wts, lens, row, lims, spec.num_nodes)
    og = oracle.OracleGraph(spec.num_nodes, directed=spec.directed)
    og.ingest_batch(src, dst, ts)
    del src, dst, ts
    rng = np.random.default_rng(9)
    row_np = row.cpu().numpy()
    for b, (kind, ht, p, q) in enumerate(biases):
        ids = np.arange(b, W, len(biases), dtype=np.int64)
        idx = np.unique(np.concatenate([ids[:4], ids[-4:], rng.choice(ids, 4096, False)]))
        r = og.sample_walks(W, L, hop_bias=kind, hop_tau=ht, p=p, q=q, seed=42, walk_idx=idx,
                            with_margin=True, threads=oracle.threads())
        assert r["cap_hits"] == 0
        lim = lims_np[idx]
        gn = np.full((len(idx), L), -1, np.int32)
        gt = np.full((len(idx), L), INT64_MIN, np.int64)
        sel = torch.from_numpy(np.concatenate([np.arange(row_np[i], row_np[i] + lim[k])
                                               for k, i in enumerate(idx)])).to(nodes.device)
        fn, ft = nodes.index_select(0, sel).cpu().numpy(), wts.index_select(0, sel).cpu().numpy()
        o = 0
        for k in range(len(idx)):
            gn[k, :lim[k]] = fn[o:o + lim[k]]
            gt[k, :lim[k]] = ft[o:o + lim[k]]
            o += lim[k]
        for k in range(len(idx)):  # the oracle's walk cut to the limit
            r["nodes"][k, lim[k]:] = -1
            r["ts"][k, lim[k]:] = INT64_MIN
            r["len"][k] = min(r["len"][k], lim[k])
        gl = lens.index_select(0, torch.from_numpy(idx).to(nodes.device)).cpu().numpy()
        same, boundary = compare_walks((gn, gt, gl), r, exact=kind in ("uniform", "linear"),
                                       label=f"mixed full scale {kind}({p},{q})", kind=kind)
        print(f"mixed full scale {kind}({p},{q}): {same}/{len(idx)} identical, {boundary} at a "
              f"CDF boundary; mean length {float(r['len'].mean()):.1f}")
        assert boundary <= max(2, len(idx) // 2000)
    g.close()
