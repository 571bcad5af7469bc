"""Pins for the oracle's walks.

- Bit-exact agreement with the independent brute force (tests/brute.py) on
  tiny graphs for every bias kind and start mode; exponential-law picks may
  differ only where the draw sits within 1e-12 of a CDF boundary.
- A pooled chi-square test (p > 0.01) of every visited state's transition
  counts against the exact per-hop law enumerated by the brute force.
- Walk invariants on a scaled copy of the tiny workload: strictly
  increasing timestamps, every hop an active edge, and maximality (a walk
  shorter than max_len ends where Gamma is empty).
- node2vec with p = q = 1 reduces to the exponential picker exactly.
- Error handling and degenerate cases.
"""
import math
from collections import defaultdict

import numpy as np
import pytest
from scipy import stats

import brute
import oracle
import synth

TS_NONE = -(1 << 63)


def _tiny_graph(seed, V=7, n=45, directed=True, window=0, tspan=40, batches=3):
    rng = np.random.default_rng(seed)
    og = oracle.OracleGraph(V, directed=directed, window=window)
    bg = brute.BruteGraph(V, directed=directed, window=window)
    for b in range(batches):
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (rng.integers(0, tspan, n) + b * tspan // 2).astype(np.int64)
        og.ingest_batch(s, d, t)
        bg.ingest(s, d, t)
    return og, bg


CASES = [
    # hop kind, hop tau, p, q, start kind, start tau, start mode, directed, window
    ("uniform", 0.0, 1, 1, "uniform", 0.0, "edge", True, 0),
    ("linear", 0.0, 1, 1, "linear", 0.0, "edge", True, 0),
    ("exponential", 0.0, 1, 1, "exponential", 0.0, "edge", True, 0),
    ("exponential", 5.0, 1, 1, "uniform", 0.0, "edge", False, 0),
    ("exponential", 40.0, 1, 1, "exponential", 9.0, "node", True, 0),
    ("linear", 0.0, 1, 1, "exponential", 3.0, "node", False, 30),
    ("uniform", 0.0, 1, 1, "linear", 0.0, "node", True, 25),
    ("node2vec", 6.0, 0.5, 2.0, "uniform", 0.0, "edge", True, 0),
    ("node2vec", 0.0, 2.0, 0.5, "exponential", 2.0, "edge", False, 0),
    ("node2vec", 3.0, 1.0, 1.0, "linear", 0.0, "node", True, 0),
    ("weight", 6.0, 1, 1, "uniform", 0.0, "edge", True, 0),
    ("weight", 0.0, 1, 1, "exponential", 4.0, "node", False, 30),
    ("weight", 40.0, 1, 1, "linear", 0.0, "edge", True, 25),
]


@pytest.mark.parametrize("ci", range(len(CASES)),
                         ids=[f"{c[0]}-{c[4]}-{c[6]}-{c[7]}-{c[8]}" for c in CASES])
def test_walks_match_brute_force(ci):
    hk, ht, p, q, sk, st, mode, directed, window = CASES[ci]
    og, bg = _tiny_graph(1000 + ci, directed=directed, window=window)
    W, L, seed, base = 120, 7, 99, 1000
    starts = np.random.default_rng(3).integers(0, 7, W).astype(np.int32)
    r = og.sample_walks(W, L, hop_bias=hk, hop_tau=ht, p=p, q=q, start_bias=sk, start_tau=st,
                        start_mode=mode, start_nodes=starts, seed=seed, walk_id_base=base,
                        with_margin=True)
    boundary = 0
    for w in range(W):
        nodes, ts, margins = brute.walk(bg, base + w, L, seed, hk, ht, p, q, sk, st, mode,
                                        int(starts[w]))
        got_n = list(r["nodes"][w, :r["len"][w]])
        got_t = list(r["ts"][w, :r["len"][w]])
        if got_n == nodes and got_t == ts:
            assert np.all(r["nodes"][w, r["len"][w]:] == -1)
            continue
        # first divergence must sit on an exponential CDF boundary
        k = next(j for j in range(min(len(nodes), len(got_n)) + 1)
                 if j >= len(nodes) or j >= len(got_n) or nodes[j] != got_n[j] or ts[j] != got_t[j])
        assert k < len(margins) and margins[k] < 1e-12, (w, k, nodes, got_n)
        boundary += 1
    assert boundary <= 2


def _law_chi2(og, bg, kind, tau, p, q, W=60000, L=6, seed=5):
    r = og.sample_walks(W, L, hop_bias=kind, hop_tau=tau, p=p, q=q, seed=seed)
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
        law = brute.transition_law(bg, cur, tc, prev, kind, tau, p, q)
        assert set(obs) <= set(law), "walk took an edge outside Gamma"
        assert abs(sum(law.values()) - 1.0) < 1e-9
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
                                          ("exponential", 0.0, 1, 1), ("exponential", 8.0, 1, 1),
                                          ("node2vec", 8.0, 0.5, 2.0), ("node2vec", 0.0, 2.0, 0.5),
                                          ("weight", 4.0, 1, 1), ("weight", 0.0, 1, 1)])
def test_per_hop_law_chi_square(kind, tau, p, q):
    og, bg = _tiny_graph(77, V=5, n=30, tspan=30)
    chi2, dof, states = _law_chi2(og, bg, kind, tau, p, q)
    assert states >= 10 and dof >= 20
    pval = stats.chi2.sf(chi2, dof)
    assert pval > 0.01, (chi2, dof, pval)


def test_chi_square_detects_a_wrong_law():
    # the same statistic rejects linear walks judged against the uniform law
    og, bg = _tiny_graph(77, V=5, n=30, tspan=30)
    r = og.sample_walks(60000, 6, hop_bias="linear", seed=5)
    counts = defaultdict(lambda: defaultdict(int))
    for w in range(60000):
        n, t, ln = r["nodes"][w], r["ts"][w], r["len"][w]
        for j in range(2, ln):
            counts[(int(n[j - 1]), int(t[j - 1]))][(int(n[j]), int(t[j]))] += 1
    chi2, dof = 0.0, 0
    for (cur, tc), obs in counts.items():
        tot = sum(obs.values())
        if tot < 200:
            continue
        law = brute.transition_law(bg, cur, tc, None, "uniform", 0)
        cells = [(obs.get(k, 0), pr * tot) for k, pr in law.items() if pr * tot >= 5]
        if len(cells) >= 2:
            chi2 += sum((o - e) ** 2 / e for o, e in cells)
            dof += len(cells) - 1
    assert dof > 0 and stats.chi2.sf(chi2, dof) < 1e-6


def test_invariants_on_scaled_tiny_workload():
    w = synth.scaled("tiny", 2000, 20000)
    s, d, t = w["stream"].all()
    og = oracle.OracleGraph(2000)
    og.ingest_batch(s, d, t)
    edges = set(zip(s.tolist(), d.tolist(), t.tolist()))
    by_src = defaultdict(list)
    for u, v, tt in edges:
        by_src[u].append(tt)
    maxts = {u: max(v) for u, v in by_src.items()}
    for kind in ("uniform", "linear", "exponential"):
        r = og.sample_walks(3000, 20, hop_bias=kind, hop_tau=5e4, seed=11)
        assert r["len"].min() >= 2
        for i in range(3000):
            n, tt, ln = r["nodes"][i], r["ts"][i], r["len"][i]
            assert tt[0] == TS_NONE
            for j in range(1, ln):
                assert (int(n[j - 1]), int(n[j]), int(tt[j])) in edges
                if j >= 2:
                    assert tt[j] > tt[j - 1]
            if ln < 20:  # maximal: nothing later leaves the last node
                assert maxts.get(int(n[ln - 1]), TS_NONE) <= tt[ln - 1]
            assert np.all(n[ln:] == -1) and np.all(tt[ln:] == TS_NONE)


def test_node2vec_unit_pq_equals_exponential():
    og, _ = _tiny_graph(4, V=9, n=80)
    a = og.sample_walks(2000, 8, hop_bias="exponential", hop_tau=7.0, seed=3)
    b = og.sample_walks(2000, 8, hop_bias="node2vec", hop_tau=7.0, p=1.0, q=1.0, seed=3)
    assert np.array_equal(a["nodes"], b["nodes"]) and np.array_equal(a["ts"], b["ts"])
    assert b["trials"] == int(np.maximum(b["len"] - 2, 0).sum())


def test_walk_subset_and_id_base():
    og, _ = _tiny_graph(8)
    full = og.sample_walks(300, 6, hop_bias="linear", seed=2, walk_id_base=50)
    idx = np.array([0, 7, 299, 123, 7])
    sub = og.sample_walks(300, 6, hop_bias="linear", seed=2, walk_id_base=50, walk_idx=idx)
    assert np.array_equal(sub["nodes"], full["nodes"][idx])
    shifted = og.sample_walks(250, 6, hop_bias="linear", seed=2, walk_id_base=100)
    assert np.array_equal(shifted["nodes"], full["nodes"][50:])


def test_degenerate_cases():
    og, _ = _tiny_graph(1, V=7)
    one = og.sample_walks(10, 1, seed=1)
    assert np.all(one["len"] == 1) and np.all(one["nodes"][:, 0] >= 0)
    iso = oracle.OracleGraph(4)
    iso.ingest_batch(np.array([0], np.int32), np.array([1], np.int32), np.array([3], np.int64))
    r = iso.sample_walks(2, 5, start_mode="node", start_nodes=np.array([2, 0], np.int32))
    assert list(r["len"]) == [1, 2] and list(r["nodes"][1, :2]) == [0, 1]
    bad = iso.sample_walks(2, 5, start_mode="node", start_nodes=np.array([4, 0], np.int32),
                           check=False)
    assert bad["status"] == oracle.ST_ERANGE and bad["len"][0] == 0 and bad["len"][1] == 2
    for kw in (dict(max_len=0), dict(hop_bias="node2vec", p=0.0),
               dict(hop_bias="node2vec", q=-1.0), dict(start_mode="node")):
        args = dict(num_walks=2, max_len=4)
        args.update(kw)
        with pytest.raises(oracle.OracleError) as ei:
            iso.sample_walks(**args)
        assert ei.value.code == oracle.ST_EINVAL


def test_equal_timestamps_never_chained():
    # a ring where every edge has the same timestamp: walks stop after one hop
    og = oracle.OracleGraph(5)
    og.ingest_batch(np.arange(5, dtype=np.int32), (np.arange(5, dtype=np.int32) + 1) % 5,
                    np.full(5, 42, np.int64))
    r = og.sample_walks(50, 6, seed=3)
    assert np.all(r["len"] == 2)
