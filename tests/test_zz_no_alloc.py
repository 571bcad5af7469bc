"""tw_sample_walks_noalloc: the queue dispatch's walks with the call's lists
in the library's own device array instead of allocated buffers. Its walks
must equal tw_sample_walks with TW_DISPATCH_QUEUE (same kernels, so bit for
bit, for every hop bias), on two calls in a row with the second smaller, and
the graph's device memory must not grow. Uniform and linear walks are also
checked against the oracle, exactly."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import compare_walks, gpu_or_skip, to_dev

pytestmark = pytest.mark.gpu


def _graph(torch, tw, V=4000, m=60_000):
    w = synth.scaled("tiny", V, m)
    s, d, t = w["stream"].all()
    g = tw.Graph(V, directed=True)
    g.ingest_batch(*to_dev(torch, s, d, t))
    og = oracle.OracleGraph(V)
    og.ingest_batch(s, d, t)
    return g, og, 0.1 * float(t.max() - t.min()), (s, d, t)


def _out(torch, W, L):
    dev = torch.device("cuda", 0)
    return (torch.empty((W, L), dtype=torch.int32, device=dev),
            torch.empty((W, L), dtype=torch.int64, device=dev),
            torch.empty(W, dtype=torch.int32, device=dev))


def _np(x):
    return tuple(a.cpu().numpy() for a in x)


@pytest.mark.parametrize("kind", ["uniform", "linear", "exponential", "node2vec"])
def test_noalloc_equals_queue_dispatch(kind):
    torch, tw = gpu_or_skip()
    g, og, tau, _ = _graph(torch, tw)
    kw = dict(hop_bias=kind, hop_tau=tau, p=0.5, q=2.0, start_bias="linear")
    if kind == "node2vec":
        g.sample_walks(16, 4, **kw)  # builds the adjacency (allocates)
    torch.cuda.synchronize()
    # first call at the maximum walk count, then a smaller one with another
    # seed, id base and length: the array keeps the first call's contents
    for W, L, seed, base in ((tw.MAX_NOALLOC_WALKS, 24, 7, 0), (3001, 9, 8, 12345)):
        ref = g.sample_walks(W, L, seed=seed, walk_id_base=base, dispatch="queue", **kw)
        out = _out(torch, W, L)
        torch.cuda.synchronize()
        before = g.device_bytes()
        g.sample_walks_noalloc(W, L, out, seed=seed, walk_id_base=base, **kw)
        torch.cuda.synchronize()
        assert g.device_bytes() == before
        got, want = _np(out), _np(ref)
        for a, b in zip(got, want):
            assert np.array_equal(a, b), kind
        assert int(got[2].sum()) > W  # walks do move
        if kind in ("uniform", "linear") and W < 5000:
            r = og.sample_walks(W, L, hop_bias=kind, start_bias="linear", seed=seed,
                                walk_id_base=base, with_margin=True)
            same, boundary = compare_walks(got, r, exact=True)
            assert same == W and boundary == 0
    g.sync()
    g.close()


def test_noalloc_node_starts_and_errors():
    torch, tw = gpu_or_skip()
    g, og, tau, (s, d, t) = _graph(torch, tw)
    V = 4000
    starts = to_dev(torch, synth.start_nodes(3, 5000, V))[0]
    out = _out(torch, 5000, 12)
    g.sample_walks_noalloc(5000, 12, out, hop_bias="linear", start_mode="node",
                           start_nodes=starts, seed=3)
    ref = g.sample_walks(5000, 12, hop_bias="linear", start_mode="node", start_nodes=starts,
                         seed=3, dispatch="queue")
    for a, b in zip(_np(out), _np(ref)):
        assert np.array_equal(a, b)
    r = og.sample_walks(5000, 12, hop_bias="linear", start_mode="node",
                        start_nodes=starts.cpu().numpy(), seed=3, with_margin=True)
    assert compare_walks(_np(out), r, exact=True) == (5000, 0)

    def rejects(fn, match):
        with pytest.raises(tw.TwError) as ei:
            fn()
        assert ei.value.code == tw.TW_EINVAL and match in str(ei.value)

    big = tw.MAX_NOALLOC_WALKS + 1
    rejects(lambda: g.sample_walks_noalloc(big, 2, _out(torch, big, 2)), "exceeds")
    rejects(lambda: g.sample_walks_noalloc(10, 4, out, hop_bias="weight", hop_tau=tau), "TW_WEIGHT")
    # a new ingest drops the node2vec adjacency; the call refuses to build it
    g.ingest_batch(*to_dev(torch, s[:100], d[:100], t[:100] + int(t.max()) + 1))
    rejects(lambda: g.sample_walks_noalloc(10, 4, out, hop_bias="node2vec", hop_tau=tau, p=2.0,
                                           q=0.5), "adjacency")
    fresh = tw.Graph(V)
    rejects(lambda: fresh.sample_walks_noalloc(10, 4, out), "no index")
    fresh.close()
    g.sync()
    g.close()
