"""Seeded synthetic temporal edge streams shared by the tests, the benchmark
and the oracle's callers.

Nothing here implements the walk method: this module only draws node ids
(uniform, or bounded Zipf / Zipf-Mandelbrot through a fixed id bijection)
and timestamps (uniform, sorted Poisson arrivals, or Markov-modulated
"bursty" Poisson arrivals). The C kernel in ``synth.c`` does the per-element
work; every value is a pure function of (seed, stream, element index), so a
stream can be produced batch by batch, in any thread count, and always gives
the same bytes.

The workload recipes (`workload`) follow the five configurations the
benchmark and the parity tests use; `scaled` shrinks one while keeping its
distribution shapes, for tests the CPU oracle finishes in seconds.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Iterator, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libsynth.so")
_lib = None

# stream ids inside one seed
_S_SRC, _S_DST, _S_TS, _S_SEG, _S_START, _S_LEN = 1, 2, 3, 4, 5, 6


def build(verbose: bool = False) -> str:
    """Compile synth.c into _build/libsynth.so (gcc, OpenMP)."""
    import subprocess

    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           os.path.join(_HERE, "synth.c"), "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, u64, i32, dbl, p = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                             ctypes.c_double, ctypes.c_void_p)
    lib.synth_nodes.argtypes = [u64, u64, i64, i64, i64, dbl, dbl, u64, p]
    lib.synth_nodes.restype = None
    lib.synth_zipf_pmf.argtypes = [i64, dbl, dbl, p]
    lib.synth_zipf_pmf.restype = None
    lib.synth_perm_apply.argtypes = [i64, u64, i64]
    lib.synth_perm_apply.restype = i64
    lib.synth_uniform_i64.argtypes = [u64, u64, i64, i64, i64, i64, p]
    lib.synth_uniform_i64.restype = None
    lib.synth_poisson_ts.argtypes = [u64, u64, i64, i64, i32, p, p, i64, p, p]
    lib.synth_poisson_ts.restype = None
    lib.synth_raw.argtypes = [u64, u64, i64, i64, p]
    lib.synth_raw.restype = None
    lib.synth_threads.argtypes = []
    lib.synth_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# --------------------------------------------------------------------------
# primitive draws

def nodes(seed: int, stream: int, start: int, n: int, num_nodes: int, s: float,
          k0: float = 0.0, perm_seed: Optional[int] = None) -> np.ndarray:
    """Node ids for draws [start, start+n). s <= 0 means uniform."""
    out = np.empty(n, dtype=np.int32)
    _load().synth_nodes(seed, stream, start, n, num_nodes, float(s), float(k0),
                        seed if perm_seed is None else perm_seed, _ptr(out))
    return out


def zipf_pmf(num_nodes: int, s: float, k0: float = 0.0) -> np.ndarray:
    out = np.empty(num_nodes, dtype=np.float64)
    _load().synth_zipf_pmf(num_nodes, float(s), float(k0), _ptr(out))
    return out


def rank_to_id(num_nodes: int, perm_seed: int, rank: int) -> int:
    return int(_load().synth_perm_apply(num_nodes, perm_seed, rank))


def uniform_i64(seed: int, stream: int, start: int, n: int, lo: int, hi: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _load().synth_uniform_i64(seed, stream, start, n, lo, hi, _ptr(out))
    return out


def raw(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_raw(seed, stream, start, n, _ptr(out))
    return out


def threads() -> int:
    return int(_load().synth_threads())


# --------------------------------------------------------------------------
# edge streams

@dataclasses.dataclass
class StreamSpec:
    """A synthetic temporal edge stream.

    ts_kind: "uniform" (i.i.d. in [ts_lo, ts_hi), unsorted arrival),
             "poisson" (sorted arrivals, Exp(mean_gap) gaps),
             "bursty"  (sorted arrivals, two-state Markov-modulated Poisson:
                        the burst state's rate is burst_factor times the base
                        rate; dwell lengths in edges are exponential with
                        means dwell_base / dwell_burst; the base gap is solved
                        so that the overall mean gap is mean_gap).
    src_s / dst_s: Zipf exponent, <= 0 for uniform ids. zipf_k0 shifts ranks
    (Zipf-Mandelbrot).
    """
    num_nodes: int
    num_edges: int
    directed: bool = True
    src_s: float = 0.0
    dst_s: float = 0.0
    zipf_k0: float = 0.0
    ts_kind: str = "uniform"
    ts_lo: int = 0
    ts_hi: int = 1_000_000
    mean_gap: float = 10.0
    burst_factor: float = 10.0
    dwell_base: float = 1e6
    dwell_burst: float = 1e5
    seed: int = 1

    def _segments(self, upto: int):
        """State segments covering edge indices [0, upto)."""
        if self.ts_kind != "bursty":
            return np.zeros(1, np.int64), np.array([self.mean_gap], np.float64)
        frac_base = self.dwell_base / (self.dwell_base + self.dwell_burst)
        base_gap = self.mean_gap / (frac_base + (1 - frac_base) / self.burst_factor)
        # dwell lengths come from the generator's own uniform stream
        starts, means = [0], [base_gap]
        pos, g = 0, 0
        while pos < upto:
            u = (int(raw(self.seed, _S_SEG, g, 1)[0]) >> 11) * 2.0 ** -53
            dwell = self.dwell_base if g % 2 == 0 else self.dwell_burst
            pos += max(1, int(-dwell * math.log1p(-u)))
            g += 1
            starts.append(pos)
            means.append(base_gap if g % 2 == 0 else base_gap / self.burst_factor)
        return np.array(starts, np.int64), np.array(means, np.float64)

    def batches(self, batch_edges: int, ts0: int = 0) -> Iterator[tuple]:
        """Yield (src, dst, ts) numpy batches in stream order."""
        acc = ctypes.c_int64(0)
        seg_s, seg_m = self._segments(self.num_edges)
        for start in range(0, self.num_edges, batch_edges):
            n = min(batch_edges, self.num_edges - start)
            yield self._batch(start, n, seg_s, seg_m, acc, ts0)

    def all(self, ts0: int = 0) -> tuple:
        return next(self.batches(max(1, self.num_edges), ts0)) if self.num_edges else (
            np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.int64))

    def _batch(self, start, n, seg_s, seg_m, acc, ts0):
        perm = self.seed * 7919 + 1
        src = nodes(self.seed, _S_SRC, start, n, self.num_nodes, self.src_s, self.zipf_k0, perm)
        dst = nodes(self.seed, _S_DST, start, n, self.num_nodes, self.dst_s, self.zipf_k0, perm)
        if self.ts_kind == "uniform":
            ts = uniform_i64(self.seed, _S_TS, start, n, self.ts_lo, self.ts_hi)
        elif self.ts_kind in ("poisson", "bursty"):
            ts = np.empty(n, np.int64)
            _load().synth_poisson_ts(self.seed, _S_TS, start, n, len(seg_s), _ptr(seg_s),
                                     _ptr(seg_m), ts0, ctypes.byref(acc), _ptr(ts))
        else:
            raise ValueError(f"unknown ts_kind {self.ts_kind!r}")
        return src, dst, ts


def start_nodes(seed: int, n: int, num_nodes: int) -> np.ndarray:
    """Uniformly drawn start nodes for NODE-mode walks."""
    return nodes(seed, _S_START, 0, n, num_nodes, 0.0)


def walk_lengths(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    """Per-walk length limits, uniform in [lo, hi] (int32)."""
    return uniform_i64(seed, _S_LEN, 0, n, lo, hi + 1).astype(np.int32)


def mixed_biases(tau: float) -> list:
    """The six hop biases of the batched mixed workload, walk i taking
    entry (walk id mod 6): uniform, linear, exponential and temporal node2vec
    with (p, q) = (0.5, 2), (1, 1), (2, 0.5); (kind, tau, p, q) tuples."""
    return [("uniform", 0.0, 1.0, 1.0), ("linear", 0.0, 1.0, 1.0),
            ("exponential", tau, 1.0, 1.0), ("node2vec", tau, 0.5, 2.0),
            ("node2vec", tau, 1.0, 1.0), ("node2vec", tau, 2.0, 0.5)]


# --------------------------------------------------------------------------
# the five workloads

WORKLOADS = {
    # plain method, tiny
    "tiny": dict(stream=dict(num_nodes=10_000, num_edges=100_000, src_s=1.1, dst_s=0.0,
                             ts_kind="uniform", ts_lo=0, ts_hi=1_000_000, seed=1),
                 window=0, walks=10_000, max_len=20, start_bias="uniform", hop_bias="uniform",
                 batch_edges=100_000),
    # single batch at scale
    "single": dict(stream=dict(num_nodes=2_000_000, num_edges=100_000_000, src_s=1.2, dst_s=1.2,
                               ts_kind="poisson", mean_gap=10.0, seed=2),
                   window=0, walks=4_000_000, max_len=80, start_bias="exponential",
                   hop_bias="exponential", tau_frac=0.1, batch_edges=100_000_000),
    # streaming window
    "stream": dict(stream=dict(num_nodes=50_000_000, num_edges=1_000_000_000, src_s=1.3,
                               dst_s=1.3, ts_kind="bursty", mean_gap=10.0, seed=3),
                   window=2_000_000_000, walks=2_000_000, max_len=40, start_bias="uniform",
                   hop_bias="linear", batch_edges=10_000_000),
    # batched mixed walks (undirected)
    "mixed": dict(stream=dict(num_nodes=1_000_000, num_edges=20_000_000, directed=False,
                              src_s=1.5, dst_s=1.5, zipf_k0=200.0, ts_kind="poisson",
                              mean_gap=10.0, seed=4),
                  window=0, walks=8_000_000, max_len=120, min_len=5, start_bias="uniform",
                  hop_bias="mixed", tau_frac=0.1, batch_edges=20_000_000),
    # serving loop: ns timestamps at 5M edges/s
    "serve": dict(stream=dict(num_nodes=10_000_000, num_edges=300_000_000, src_s=1.2, dst_s=1.2,
                              ts_kind="poisson", mean_gap=200.0, seed=5),
                  window=60_000_000_000, walks=None, max_len=80, start_bias="uniform",
                  hop_bias="mixed", tau_frac=0.1, batch_edges=5_000_000,
                  edges_per_s=5_000_000, requests_per_s=2000, arena_bytes=8 << 30),
}


def workload(name: str) -> dict:
    w = dict(WORKLOADS[name])
    w["stream"] = StreamSpec(**w["stream"])
    return w


def scaled(name: str, num_nodes: int, num_edges: int, **over) -> dict:
    """The named workload's distributions at a smaller size."""
    w = workload(name)
    w["stream"] = dataclasses.replace(w["stream"], num_nodes=num_nodes, num_edges=num_edges)
    w.update(over)
    return w
