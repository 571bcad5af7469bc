"""Brute-force reference for tiny graphs, written independently of the oracle.

It keeps the active window as a plain Python list of edges tagged with their
arrival sequence number, finds the causal neighbourhood Gamma_t(v) by
filtering that list, draws Philox4x64-10 from numpy's own implementation,
and evaluates each picker's law exactly: `fractions` for the linear law and
50-digit `decimal` for the exponential law, both from sums of the
probability mass function rather than from any closed-form inverse.
"""
from __future__ import annotations

import decimal
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional, Tuple

import numpy as np

TS_NONE = -(1 << 63)
M64 = (1 << 64) - 1
decimal.getcontext().prec = 60


# ------------------------------------------------------------------ RNG

def philox_numpy(seed: int, walk_id: int, hop: int, trial: int) -> List[int]:
    """Philox4x64-10 block for counter (walk_id, hop, trial, 0), key (seed, 0),
    taken from numpy's bit generator, which emits the block of counter+1."""
    c = walk_id + (hop << 64) + (trial << 128)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & M64 for i in range(4)]
    g = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                         key=np.array([seed, 0], dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


def u_open(x: int) -> Fraction:
    return Fraction(2 * (x >> 12) + 1, 1 << 53)


def u_closed(x: int) -> Fraction:
    return Fraction(x >> 11, 1 << 53)


def scaled(x: int, n: int) -> int:
    return (x * n) >> 64


# --------------------------------------------------------------- laws

def linear_cdf(n: int, k: int) -> Fraction:
    """P(i < k) under P(i) proportional to i+1, by summing the mass."""
    tot = sum(range(1, n + 1))
    return Fraction(sum(range(1, k + 1)), tot)


def linear_pick(n: int, x: int) -> int:
    u = Fraction(x >> 11, 1 << 53)
    tot = n * (n + 1) // 2
    acc = 0
    for i in range(n):
        acc += i + 1
        if u < Fraction(acc, tot):
            return i
    return n - 1


def exp_masses(n: int, lam: float) -> List[decimal.Decimal]:
    L = decimal.Decimal(lam)
    return [(L * i).exp() for i in range(n)]


def exp_pick(n: int, lam: float, x: int) -> Tuple[int, float]:
    """Index under P(i) proportional to exp(lam*i) and the distance of the
    uniform draw from the nearest CDF boundary."""
    w = exp_masses(n, lam)
    tot = sum(w)
    u = decimal.Decimal(u_open(x).numerator) / decimal.Decimal(u_open(x).denominator)
    acc = decimal.Decimal(0)
    prev = decimal.Decimal(0)
    for i in range(n):
        acc += w[i]
        hi = acc / tot
        if u < hi or i == n - 1:
            return i, float(min(u - prev, hi - u))
        prev = hi
    raise AssertionError


def weight_masses(ts: List[int], tau: float) -> List[decimal.Decimal]:
    """The weight-based sampler's weights exactly as printed: exp(t_i - t_min),
    with tau the time scale (tau <= 0: 1)."""
    sc = decimal.Decimal(tau if tau > 0 else 1.0)
    return [(decimal.Decimal(t - ts[0]) / sc).exp() for t in ts]


def weight_pick(ts: List[int], tau: float, x: int) -> Tuple[int, float]:
    """Smallest k with W[k] >= u W[n-1] over the cumulative weights W, and the
    distance of u from the nearest interior boundary W[k] / W[n-1]."""
    w = weight_masses(ts, tau)
    tot = sum(w)
    u = decimal.Decimal(u_open(x).numerator) / decimal.Decimal(u_open(x).denominator)
    r = u * tot
    acc = decimal.Decimal(0)
    for k, wk in enumerate(w):
        lo = acc
        acc += wk
        if acc >= r:
            m = decimal.Decimal("Infinity")
            if k > 0:
                m = u - lo / tot
            if k < len(w) - 1:
                m = min(m, acc / tot - u)
            return k, float(m)
    raise AssertionError


def exp_lambda(t_first: int, t_last: int, n: int, tau: float) -> float:
    if tau <= 0 or n <= 1:
        return 1.0
    return float(t_last - t_first) / (float(n - 1) * tau)


# --------------------------------------------------------------- graph

@dataclass
class BruteGraph:
    num_nodes: int
    directed: bool = True
    window: int = 0
    t_now: Optional[int] = None
    seq: int = 0
    edges: List[Tuple[int, int, int, int]] = field(default_factory=list)  # (ts, seq, src, dst)

    def ingest(self, src, dst, ts):
        batch = []
        for u, v, t in zip(src, dst, ts):
            batch.append((int(t), self.seq, int(u), int(v)))
            self.seq += 1
            if not self.directed:
                batch.append((int(t), self.seq, int(v), int(u)))
                self.seq += 1
        for e in batch:
            self.t_now = e[0] if self.t_now is None else max(self.t_now, e[0])
        dropped = 0
        evicted = 0
        if self.window > 0 and self.t_now is not None:
            cut = self.t_now - self.window
            keep = [e for e in batch if e[0] >= cut]
            dropped = len(batch) - len(keep)
            batch = keep
            evicted = self.evict_before(cut)
        self.edges = sorted(self.edges + batch)  # by (ts, seq)
        return dict(accepted=len(batch), dropped_late=dropped, evicted=evicted,
                    active_edges=len(self.edges))

    def evict_before(self, cut: int) -> int:
        before = len(self.edges)
        self.edges = [e for e in self.edges if e[0] >= cut]
        return before - len(self.edges)

    # views, built from the definitions
    def ts_view(self):
        return [(s, d, t) for (t, q, s, d) in self.edges]

    def node_view(self):
        return sorted(self.edges, key=lambda e: (e[2], e[0], e[1]))

    def gamma(self, v: int, t: int) -> List[Tuple[int, int, int, int]]:
        """Out-edges of v strictly after t, in node-view order."""
        return [e for e in self.node_view() if e[2] == v and e[0] > t]

    def gamma_before(self, v: int, t: int) -> List[Tuple[int, int, int, int]]:
        """Candidates of a backward hop: v's edges in this graph (the in-view
        of a backward walk) with timestamp strictly before t, canonical order."""
        return [e for e in self.node_view() if e[2] == v and e[0] < t]

    def has_edge(self, u: int, w: int) -> bool:
        return any(e[2] == u and e[3] == w for e in self.edges)


def _groups(cands):
    """Split a timestamp-ordered candidate list into equal-timestamp groups."""
    out = []
    for e in cands:
        if out and out[-1][0][0] == e[0]:
            out[-1].append(e)
        else:
            out.append([e])
    return out


def pick(cands, kind: str, tau: float, d: List[int], backward: bool = False):
    """Returns (edge, margin). cands are in view order (timestamp ascending);
    a backward walk lists them in reverse and picks over that listing."""
    if backward:
        cands = list(reversed(cands))
    if kind == "uniform":
        return cands[scaled(d[0], len(cands))], float("inf")
    if kind == "weight":
        k, margin = weight_pick([e[0] for e in cands], tau, d[0])
        return cands[k], margin
    groups = _groups(cands)
    n = len(groups)
    margin = float("inf")
    if kind == "linear":
        i = linear_pick(n, d[0])
    else:
        # the rate from the candidates' time span (either listing order)
        span_lo = min(grp[0][0] for grp in groups)
        span_hi = max(grp[0][0] for grp in groups)
        lam = exp_lambda(span_lo, span_hi, n, tau)
        if n == 1:
            i = 0
        else:
            i, margin = exp_pick(n, lam, d[0])
    g = groups[i]
    return g[scaled(d[1], len(g))], margin


def walk(g: BruteGraph, walk_id: int, max_len: int, seed: int, hop_kind="uniform",
         hop_tau=0.0, p=1.0, q=1.0, start_kind="uniform", start_tau=0.0, start_mode="edge",
         start_node: int = 0, backward: bool = False):
    """One walk: (nodes, ts, min margin per position). backward: g is the
    in-view and each hop goes to an edge strictly before the current time."""
    nodes, ts, margins = [], [], []
    d0 = philox_numpy(seed, walk_id, 0, 0)
    bw = backward
    if start_mode == "edge":
        if not g.edges:
            return nodes, ts, margins
        e, mg = pick(g.edges, start_kind, start_tau, d0, bw)
        nodes.append(e[2]); ts.append(TS_NONE); margins.append(mg)
        if max_len == 1:
            return nodes, ts, margins
        nodes.append(e[3]); ts.append(e[0]); margins.append(mg)
        prev, cur, t = e[2], e[3], e[0]
    else:
        nodes.append(start_node); ts.append(TS_NONE); margins.append(float("inf"))
        if max_len == 1:
            return nodes, ts, margins
        run = [e for e in g.node_view() if e[2] == start_node]
        if not run:
            return nodes, ts, margins
        e, mg = pick(run, start_kind, start_tau, d0, bw)
        nodes.append(e[3]); ts.append(e[0]); margins.append(mg)
        prev, cur, t = start_node, e[3], e[0]
    hop = 1
    while len(nodes) < max_len:
        cands = g.gamma_before(cur, t) if bw else g.gamma(cur, t)
        if not cands:
            break
        if hop_kind == "node2vec":
            bmax = max(1.0 / p, 1.0, 1.0 / q)
            chosen, worst = None, float("inf")
            for trial in range(4096):
                d = philox_numpy(seed, walk_id, hop, trial)
                e, mg = pick(cands, "exponential", hop_tau, d, bw)
                worst = min(worst, mg)
                w = e[3]
                beta = 1.0 / p if w == prev else (1.0 if g.has_edge(prev, w) else 1.0 / q)
                if float(u_closed(d[2])) * bmax < beta:
                    chosen = e
                    break
            if chosen is None:
                break
            e, mg = chosen, worst
        else:
            e, mg = pick(cands, hop_kind, hop_tau, philox_numpy(seed, walk_id, hop, 0), bw)
        nodes.append(e[3]); ts.append(e[0]); margins.append(mg)
        prev, cur, t = cur, e[3], e[0]
        hop += 1
    return nodes, ts, margins


# --------------------------------------------------------------- laws for chi-square

def transition_law(g: BruteGraph, cur: int, t: int, prev: Optional[int], kind: str,
                   tau: float, p: float = 1.0, q: float = 1.0, backward: bool = False):
    """Exact probability of each next (dst, ts) pair from state (cur, t, prev);
    backward: over g's edges before t, listed latest first."""
    cands = list(reversed(g.gamma_before(cur, t))) if backward else g.gamma(cur, t)
    if not cands:
        return {}
    groups = _groups(cands)
    n = len(groups)
    probs = {}

    def add(key, pr):
        probs[key] = probs.get(key, 0.0) + pr

    if kind == "uniform":
        for e in cands:
            add((e[3], e[0]), 1.0 / len(cands))
        return probs
    if kind == "weight":
        w = weight_masses([e[0] for e in cands], tau)
        s = sum(w)
        for e, x in zip(cands, w):
            add((e[3], e[0]), float(x / s))
        return probs
    if kind == "linear":
        tot = n * (n + 1) / 2
        gp = [(i + 1) / tot for i in range(n)]
    else:
        lam = exp_lambda(min(grp[0][0] for grp in groups), max(grp[0][0] for grp in groups), n,
                         tau)
        w = [float(x) for x in exp_masses(n, lam)]
        s = sum(w)
        gp = [x / s for x in w]
    per_edge = []
    for i, grp in enumerate(groups):
        for e in grp:
            per_edge.append((e, gp[i] / len(grp)))
    if kind == "node2vec":
        wts = []
        for e, pr in per_edge:
            beta = 1.0 / p if e[3] == prev else (1.0 if g.has_edge(prev, e[3]) else 1.0 / q)
            wts.append(pr * beta)
        s = sum(wts)
        per_edge = [(e, x / s) for (e, _), x in zip(per_edge, wts)]
    for e, pr in per_edge:
        add((e[3], e[0]), pr)
    return probs
