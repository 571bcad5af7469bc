"""The law of the GPU's walks, tested directly: on tiny graphs every visited
state's transition counts are compared with the exact per-hop law that the
brute force (tests/brute.py) enumerates, pooled into one chi-square
statistic that must pass at p > 0.01. This covers the pickers whose GPU
results may differ from the oracle's at a CDF boundary (exponential,
node2vec, weight-based) as well as the exact ones."""
from collections import defaultdict

import numpy as np
import pytest
from scipy import stats

import brute
from gpu_util import gpu_or_skip, to_dev

pytestmark = pytest.mark.gpu


def _tiny_batches(seed, V=5, n=30, tspan=30, batches=3):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(batches):
        s = rng.integers(0, V, n).astype(np.int32)
        d = rng.integers(0, V, n).astype(np.int32)
        t = (rng.integers(0, tspan, n) + b * tspan // 2).astype(np.int64)
        out.append((s, d, t))
    return out


def _pooled_chi2(bg, nodes, ts, lens, kind, tau, p, q, min_visits=40):
    """Pooled chi-square over the states (current node, arrival time, previous
    node) visited at least min_visits times; cells with expectation < 5 are
    merged."""
    L = nodes.shape[1]
    pos = np.arange(2, L)
    keep = pos[None, :] < lens[:, None]
    rows = np.stack([nodes[:, 1:L - 1][keep], ts[:, 1:L - 1][keep], nodes[:, 0:L - 2][keep],
                     nodes[:, 2:L][keep], ts[:, 2:L][keep]], axis=1)
    uniq, cnt = np.unique(rows, axis=0, return_counts=True)
    counts = defaultdict(dict)
    for (cur, tc, prev, nx, tn), c in zip(uniq.tolist(), cnt.tolist()):
        counts[(cur, tc, prev)][(nx, tn)] = c
    chi2, dof, states = 0.0, 0, 0
    for (cur, tc, prev), obs in counts.items():
        tot = sum(obs.values())
        if tot < min_visits:
            continue
        law = brute.transition_law(bg, cur, tc, prev, kind, tau, p, q)
        assert set(obs) <= set(law), "a GPU walk took an edge outside Gamma"
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


@pytest.mark.parametrize("kind,tau,p,q", [("uniform", 0.0, 1, 1), ("linear", 0.0, 1, 1),
                                          ("exponential", 0.0, 1, 1), ("exponential", 8.0, 1, 1),
                                          ("node2vec", 8.0, 0.5, 2.0),
                                          ("node2vec", 0.0, 2.0, 0.5),
                                          ("weight", 4.0, 1, 1), ("weight", 0.0, 1, 1)])
@pytest.mark.parametrize("dispatch", ["full_walk", "queue"])
def test_gpu_per_hop_law_chi_square(kind, tau, p, q, dispatch):
    torch, tw = gpu_or_skip()
    V = 5
    bg = brute.BruteGraph(V)
    g = tw.Graph(V)
    for s, d, t in _tiny_batches(77, V=V):
        bg.ingest(s, d, t)
        g.ingest_batch(*to_dev(torch, s, d, t))
    W, L = 120_000, 6
    nodes, ts, lens = g.sample_walks(W, L, hop_bias=kind, hop_tau=tau, p=p, q=q, seed=23,
                                     dispatch=dispatch if kind != "weight" else "full_walk")
    g.sync()
    chi2, dof, states = _pooled_chi2(bg, nodes.cpu().numpy(), ts.cpu().numpy(),
                                     lens.cpu().numpy(), kind, tau, p, q)
    pval = stats.chi2.sf(chi2, dof)
    print(f"{kind} tau={tau} p={p} q={q} {dispatch}: chi2 {chi2:.1f}, dof {dof}, "
          f"{states} states, p = {pval:.3f}")
    assert states >= 10 and dof >= 20
    assert pval > 0.01, (chi2, dof, pval)
    g.close()
