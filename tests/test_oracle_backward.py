"""Pins of the oracle's backward walks (the backward case of Gamma, which the
paper defines by analogy, Sec. "Design Constraints").

A backward walk moves from node v at time t to an in-edge (u, v, t') with
t' < t. The oracle's reading: the candidates are listed in reverse canonical
order and every pick is the forward pick over that listing. Pinned by
(a) the brute-force reference, which filters the edge list and reverses the
listing literally; (b) time reflection: without equal timestamps a backward
walk on G is exactly a forward walk on G' = {(v, u, -t)}, computed by the
oracle's forward path; (c) chi-square of the per-hop law; (d) invariants.
"""
from collections import defaultdict

import numpy as np
import pytest
from scipy import stats

import brute
import oracle

TS_NONE = -(1 << 63)


def _graphs(seed, V=7, n=45, directed=True, window=0, tspan=40, batches=3):
    rng = np.random.default_rng(seed)
    og = oracle.OracleGraph(V, directed=directed, window=window, backward=True)
    bg = brute.BruteGraph(V, directed=directed, window=window)
    rev = brute.BruteGraph(V, directed=directed, window=window) if directed else bg
    for b in range(batches):
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (rng.integers(0, tspan, n) + b * tspan // 2).astype(np.int64)
        og.ingest_batch(s, d, t)
        bg.ingest(s, d, t)
        if directed:
            rev.ingest(d, s, t)
    return og, bg, rev


CASES = [
    # hop kind, hop tau, p, q, start kind, start tau, start mode, directed, window
    ("uniform", 0.0, 1, 1, "uniform", 0.0, "edge", True, 0),
    ("linear", 0.0, 1, 1, "linear", 0.0, "node", True, 0),
    ("exponential", 5.0, 1, 1, "exponential", 9.0, "edge", True, 0),
    ("exponential", 0.0, 1, 1, "uniform", 0.0, "node", False, 0),
    ("linear", 0.0, 1, 1, "exponential", 3.0, "edge", False, 30),
    ("uniform", 0.0, 1, 1, "linear", 0.0, "node", True, 25),
    ("node2vec", 6.0, 0.5, 2.0, "uniform", 0.0, "edge", True, 0),
    ("node2vec", 0.0, 2.0, 0.5, "exponential", 2.0, "node", False, 0),
]


@pytest.mark.parametrize("ci", range(len(CASES)),
                         ids=[f"{c[0]}-{c[4]}-{c[6]}-{c[7]}-{c[8]}" for c in CASES])
def test_backward_walks_match_brute_force(ci):
    hk, ht, p, q, sk, st, mode, directed, window = CASES[ci]
    og, bg, rev = _graphs(2000 + ci, directed=directed, window=window)
    W, L, seed, base = 120, 7, 31, 500
    starts = np.random.default_rng(4).integers(0, 7, W).astype(np.int32)
    r = og.sample_walks(W, L, hop_bias=hk, hop_tau=ht, p=p, q=q, start_bias=sk, start_tau=st,
                        start_mode=mode, start_nodes=starts, seed=seed, walk_id_base=base,
                        with_margin=True, direction="backward")
    walked = 0
    for w in range(W):
        nodes, ts, margins = brute.walk(rev, base + w, L, seed, hk, ht, p, q, sk, st, mode,
                                        int(starts[w]), backward=True)
        got_n = list(r["nodes"][w, :r["len"][w]])
        got_t = list(r["ts"][w, :r["len"][w]])
        walked += len(nodes) > 2
        if got_n == nodes and got_t == ts:
            continue
        k = next(j for j in range(min(len(nodes), len(got_n)) + 1)
                 if j == min(len(nodes), len(got_n)) or got_n[j] != nodes[j] or got_t[j] != ts[j])
        assert min(margins[k], r["margin"][w, k]) < 1e-9, (w, k, got_n, nodes)
    assert walked > 10


@pytest.mark.parametrize("kind,tau,p,q", [("uniform", 0.0, 1, 1), ("linear", 0.0, 1, 1),
                                          ("exponential", 7.0, 1, 1), ("exponential", 0.0, 1, 1),
                                          ("node2vec", 7.0, 0.5, 2.0)])
@pytest.mark.parametrize("mode", ["edge", "node"])
def test_backward_is_forward_on_the_time_reversed_graph(kind, tau, p, q, mode):
    # distinct timestamps: reversing every edge and negating its timestamp
    # turns backward walks into forward walks, draw for draw
    rng = np.random.default_rng(9)
    V, n = 40, 900
    s = rng.integers(0, V, n).astype(np.int32)
    d = rng.integers(0, V, n).astype(np.int32)
    t = rng.permutation(10 * n)[:n].astype(np.int64)
    og = oracle.OracleGraph(V, backward=True)
    og.ingest_batch(s, d, t)
    ogr = oracle.OracleGraph(V)
    ogr.ingest_batch(d, s, -t)
    W, L = 3000, 12
    starts = rng.integers(0, V, W).astype(np.int32)
    # biased starts of the window pick its latest (forward) or earliest
    # (backward) edges, where walks end at once: uniform starts here
    kw = dict(hop_bias=kind, hop_tau=tau, p=p, q=q, start_bias="uniform", start_mode=mode,
              start_nodes=starts, seed=77, walk_id_base=3)
    b = og.sample_walks(W, L, direction="backward", **kw)
    f = ogr.sample_walks(W, L, **kw)
    assert np.array_equal(b["len"], f["len"])
    assert np.array_equal(b["nodes"], f["nodes"])
    inside = np.arange(L)[None, :] < b["len"][:, None]
    inside[:, 0] = False
    assert np.array_equal(b["ts"][inside], -f["ts"][inside])
    assert (b["len"] > 3).sum() > 10


def _chi2(og, rev, kind, tau, p, q, W=60000, L=6, seed=5):
    r = og.sample_walks(W, L, hop_bias=kind, hop_tau=tau, p=p, q=q, seed=seed,
                        direction="backward")
    counts = defaultdict(lambda: defaultdict(int))
    for w in range(W):
        n, t, ln = r["nodes"][w], r["ts"][w], r["len"][w]
        for j in range(2, ln):
            counts[(int(n[j - 1]), int(t[j - 1]), int(n[j - 2]))][(int(n[j]), int(t[j]))] += 1
    chi2, dof, states = 0.0, 0, 0
    for (cur, tc, prev), obs in counts.items():
        tot = sum(obs.values())
        if tot < 40:
            continue
        law = brute.transition_law(rev, cur, tc, prev, kind, tau, p, q, backward=True)
        assert set(obs) <= set(law), "walk took an edge outside the backward Gamma"
        big = [k for k, pr in law.items() if pr * tot >= 5]
        small = [k for k in law if k not in big]
        cells = [(obs.get(k, 0), law[k] * tot) for k in big]
        if small:
            cells.append((sum(obs.get(k, 0) for k in small), sum(law[k] for k in small) * tot))
        if len(cells) < 2:
            continue
        chi2 += sum((o - e) ** 2 / e for o, e in cells)
        dof += len(cells) - 1
        states += 1
    return chi2, dof, states


@pytest.mark.parametrize("kind,tau,p,q", [("uniform", 0, 1, 1), ("linear", 0, 1, 1),
                                          ("exponential", 6.0, 1, 1),
                                          ("node2vec", 6.0, 0.5, 2.0)])
def test_backward_per_hop_law_chi_square(kind, tau, p, q):
    og, bg, rev = _graphs(88, V=5, n=30, tspan=30)
    chi2, dof, states = _chi2(og, rev, kind, tau, p, q)
    assert states >= 10 and dof >= 20
    assert stats.chi2.sf(chi2, dof) > 0.01, (chi2, dof)


def test_backward_invariants():
    og, bg, rev = _graphs(17, V=30, n=400, tspan=300, batches=4)
    edges = set(bg.ts_view())  # (src, dst, ts)
    r = og.sample_walks(5000, 10, hop_bias="exponential", hop_tau=20.0, seed=3,
                        direction="backward")
    for w in range(5000):
        ln = int(r["len"][w])
        n, t = r["nodes"][w], r["ts"][w]
        assert t[0] == TS_NONE and np.all(n[ln:] == -1)
        for j in range(1, ln):
            # hop j took the edge (n[j] -> n[j-1]) at time t[j], earlier than t[j-1]
            assert (int(n[j]), int(n[j - 1]), int(t[j])) in edges
            if j >= 2:
                assert t[j] < t[j - 1]
    with pytest.raises(oracle.OracleError):
        og.sample_walks(10, 5, hop_bias="weight", hop_tau=5.0, direction="backward")
