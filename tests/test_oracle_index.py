"""Pins for the oracle's ingest, window eviction and dual index.

The expected views come from numpy's stable lexsort and np.unique over a
list of edges tagged with their arrival sequence, and from a filter over
the edge multiset for the window; none of it goes through the oracle's
std::merge / std::stable_sort path.
"""
import numpy as np
import pytest

import brute
import oracle


def _np_views(edges):
    """edges: array rows (ts, seq, src, dst) of the active multiset."""
    if len(edges) == 0:
        e = np.zeros((0, 4), np.int64)
    else:
        e = np.asarray(edges, np.int64)
    order = np.lexsort((e[:, 1], e[:, 0]))          # by ts, then arrival
    tv = e[order]
    norder = np.lexsort((tv[:, 1], tv[:, 0], tv[:, 2]))  # by src, ts, arrival
    nv = tv[norder]
    g_ts, g_first = np.unique(tv[:, 0], return_index=True)
    key = nv[:, 2] * (1 << 40) + (nv[:, 0] - (nv[:, 0].min() if len(nv) else 0))
    _, n_first = np.unique(key, return_index=True)
    return tv, nv, g_ts, g_first, n_first


def _check(og: oracle.OracleGraph, active, V):
    tv, nv, g_ts, g_first, n_first = _np_views(active)
    v = og.views()
    m = len(tv)
    assert np.array_equal(v["src"], tv[:, 2]) and np.array_equal(v["dst"], tv[:, 3])
    assert np.array_equal(v["ts"], tv[:, 0])
    assert np.array_equal(v["g_ts"], g_ts)
    assert np.array_equal(v["g_off"], np.append(g_first, m))
    assert np.array_equal(v["n_dst"], nv[:, 3]) and np.array_equal(v["n_ts"], nv[:, 0])
    assert np.array_equal(v["n_gts"], nv[n_first, 0] if m else np.zeros(0, np.int64))
    assert np.array_equal(v["n_goff"], np.append(n_first, m))
    # node table: first edge / first group of each node (CSR-style, V+1)
    ebeg = np.searchsorted(nv[:, 2], np.arange(V + 1), side="left")
    gsrc = nv[n_first, 2] if m else np.zeros(0, np.int64)
    gbeg = np.searchsorted(gsrc, np.arange(V + 1), side="left")
    assert np.array_equal(v["n_ebeg"], ebeg)
    assert np.array_equal(v["n_gbeg"], gbeg)


@pytest.mark.parametrize("directed", [True, False])
@pytest.mark.parametrize("window", [0, 300, 5000])
def test_stream_views_match_numpy(directed, window):
    rng = np.random.default_rng(100 + window + directed)
    V = 37
    og = oracle.OracleGraph(V, directed=directed, window=window)
    active = []  # rows (ts, seq, src, dst)
    seq = 0
    t_now = None
    t_base = 0
    for b in range(12):
        n = int(rng.integers(0, 60))
        src = rng.integers(0, V, n).astype(np.int32)
        dst = rng.integers(0, V, n).astype(np.int32)
        # mostly advancing time with heavy duplicates and some late edges
        ts = (t_base + rng.integers(-400, 250, n) // 7 * 7).astype(np.int64)
        t_base += 200
        info = og.ingest_batch(src, dst, ts)
        batch = []
        for u, w, t in zip(src, dst, ts):
            batch.append((int(t), seq, int(u), int(w))); seq += 1
            if not directed:
                batch.append((int(t), seq, int(w), int(u))); seq += 1
        if batch:
            bm = max(r[0] for r in batch)
            t_now = bm if t_now is None else max(t_now, bm)
        dropped = evicted = 0
        if window > 0 and t_now is not None:
            cut = t_now - window
            dropped = sum(r[0] < cut for r in batch)
            batch = [r for r in batch if r[0] >= cut]
            evicted = sum(r[0] < cut for r in active)
            active = [r for r in active if r[0] >= cut]
        active = active + batch
        assert info["accepted"] == len(batch)
        assert info["dropped_late"] == dropped
        assert info["evicted"] == evicted
        assert info["active_edges"] == len(active)
        _check(og, active, V)
        if b == 6:
            cut = t_base - 350
            assert og.evict_before(cut) == sum(r[0] < cut for r in active)
            active = [r for r in active if r[0] >= cut]
            assert og.evict_before(cut) == 0  # idempotent
            _check(og, active, V)


def test_incremental_equals_single_batch():
    rng = np.random.default_rng(5)
    V, n = 50, 3000
    src = rng.integers(0, V, n).astype(np.int32)
    dst = rng.integers(0, V, n).astype(np.int32)
    ts = rng.integers(0, 400, n).astype(np.int64)
    a = oracle.OracleGraph(V)
    a.ingest_batch(src, dst, ts)
    b = oracle.OracleGraph(V)
    for s in range(0, n, 271):
        b.ingest_batch(src[s:s + 271], dst[s:s + 271], ts[s:s + 271])
    va, vb = a.views(), b.views()
    for k in va:
        assert np.array_equal(va[k], vb[k]), k


def test_out_of_range_batch_rejected_whole():
    og = oracle.OracleGraph(10)
    og.ingest_batch(np.array([1], np.int32), np.array([2], np.int32), np.array([5], np.int64))
    with pytest.raises(oracle.OracleError) as ei:
        og.ingest_batch(np.array([1, 10], np.int32), np.array([2, 3], np.int32),
                        np.array([6, 7], np.int64))
    assert ei.value.code == oracle.ST_ERANGE
    assert og.sizes()["m"] == 1
    with pytest.raises(oracle.OracleError):
        og.ingest_batch(np.array([-1], np.int32), np.array([2], np.int32), np.array([5], np.int64))


def test_empty_graph_and_batches():
    og = oracle.OracleGraph(4, window=10)
    info = og.ingest_batch(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert info["active_edges"] == 0
    v = og.views()
    assert len(v["src"]) == 0 and np.array_equal(v["n_ebeg"], np.zeros(5))
    w = og.sample_walks(5, 4)
    assert np.all(w["len"] == 0) and np.all(w["nodes"] == -1)


def test_brute_graph_agrees_with_oracle_views():
    # the brute-force graph used by the walk tests sees the same window
    rng = np.random.default_rng(9)
    V = 12
    og = oracle.OracleGraph(V, directed=False, window=60)
    bg = brute.BruteGraph(V, directed=False, window=60)
    for _ in range(6):
        n = int(rng.integers(1, 25))
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = rng.integers(0, 120, n).astype(np.int64) + _ * 30
        i1, i2 = og.ingest_batch(s, d, t), bg.ingest(s, d, t)
        for k in ("accepted", "dropped_late", "evicted", "active_edges"):
            assert i1[k] == i2[k]
        v = og.views()
        assert list(zip(v["src"], v["dst"], v["ts"])) == bg.ts_view()
