"""ctypes wrapper around the CPU oracle (``tw_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers. The product path never
imports this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libtw_oracle.so")
_lib = None

KINDS = {"uniform": 0, "linear": 1, "exponential": 2, "node2vec": 3, "weight": 4}
START_MODES = {"edge": 0, "node": 1}
ST_OK, ST_EINVAL, ST_ERANGE = 0, 1, 4


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           os.path.join(_HERE, "tw_oracle.cpp"), "-o", tmp]
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
    p, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_double)
    lib.oracle_philox.argtypes = [p, p, p]
    lib.oracle_philox.restype = None
    lib.oracle_pick_uniform.argtypes = [i64, u64]
    lib.oracle_pick_uniform.restype = i64
    lib.oracle_pick_linear.argtypes = [i64, u64]
    lib.oracle_pick_linear.restype = i64
    lib.oracle_pick_exponential.argtypes = [i64, dbl, u64, p]
    lib.oracle_pick_exponential.restype = i64
    lib.oracle_exp_lambda.argtypes = [i64, i64, i64, dbl]
    lib.oracle_exp_lambda.restype = dbl
    lib.oracle_pick_weight.argtypes = [p, i64, dbl, u64, p]
    lib.oracle_pick_weight.restype = i64
    lib.oracle_unit_open.argtypes = [u64]
    lib.oracle_unit_open.restype = dbl
    lib.oracle_create.argtypes = [i32, i32, i64]
    lib.oracle_create.restype = p
    lib.oracle_destroy.argtypes = [p]
    lib.oracle_destroy.restype = None
    lib.oracle_ingest.argtypes = [p, p, p, p, i64, p]
    lib.oracle_ingest.restype = ctypes.c_int
    lib.oracle_evict_before.argtypes = [p, i64]
    lib.oracle_evict_before.restype = i64
    lib.oracle_sizes.argtypes = [p, p]
    lib.oracle_sizes.restype = None
    lib.oracle_views.argtypes = [p] * 12
    lib.oracle_views.restype = None
    lib.oracle_sample_walks.argtypes = [p, i32, i32, dbl, dbl, dbl, i32, dbl, i32, p, u64, u64,
                                        p, i64, p, p, p, p, p, i32, i32]
    lib.oracle_sample_walks.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be contiguous"
    return a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, np.uint64)
    _load().oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def pick_uniform(n: int, x: int) -> int:
    return int(_load().oracle_pick_uniform(n, x))


def pick_linear(n: int, x: int) -> int:
    return int(_load().oracle_pick_linear(n, x))


def pick_exponential(n: int, lam: float, x: int):
    m = ctypes.c_double(0.0)
    i = _load().oracle_pick_exponential(n, lam, x, ctypes.byref(m))
    return int(i), float(m.value)


def pick_weight(ts, tau: float, x: int):
    """Weight-based pick over candidate edges with timestamps ts (ascending):
    (index, distance of the draw from the nearest boundary)."""
    a = np.ascontiguousarray(ts, np.int64)
    m = ctypes.c_double(0.0)
    i = _load().oracle_pick_weight(_ptr(a), len(a), float(tau), x, ctypes.byref(m))
    return int(i), float(m.value)


def exp_lambda(t_first: int, t_last: int, n: int, tau: float) -> float:
    return float(_load().oracle_exp_lambda(t_first, t_last, n, tau))


def unit_open(x: int) -> float:
    return float(_load().oracle_unit_open(x))


def threads() -> int:
    return int(_load().oracle_threads())


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class OracleGraph:
    """The oracle's graph: ingest / evict / views / walks, all on the CPU.

    backward: also keep the in-view for backward walks. A directed graph
    keeps it as a second graph fed every batch with source and destination
    swapped (and the same evictions); an undirected graph is its own."""

    def __init__(self, num_nodes: int, directed: bool = True, window: int = 0,
                 backward: bool = False):
        self._lib = _load()
        self._h = self._lib.oracle_create(num_nodes, 1 if directed else 0, int(window))
        if not self._h:
            raise OracleError(ST_EINVAL, "create")
        self._rev = None
        if backward and directed:
            self._rev = self._lib.oracle_create(num_nodes, 1, int(window))
        self._backward = backward
        self.num_nodes = num_nodes

    def __del__(self):
        for name in ("_h", "_rev"):
            h = getattr(self, name, None)
            if h:
                self._lib.oracle_destroy(h)
                setattr(self, name, None)

    def ingest_batch(self, src, dst, ts) -> dict:
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        ts = np.ascontiguousarray(ts, np.int64)
        assert len(src) == len(dst) == len(ts)
        info = np.zeros(6, np.int64)
        rc = self._lib.oracle_ingest(self._h, _ptr(src), _ptr(dst), _ptr(ts), len(src), _ptr(info))
        if rc != ST_OK:
            raise OracleError(rc, "ingest_batch")
        if self._rev:
            rinfo = np.zeros(6, np.int64)
            rc = self._lib.oracle_ingest(self._rev, _ptr(dst), _ptr(src), _ptr(ts), len(src),
                                         _ptr(rinfo))
            if rc != ST_OK:
                raise OracleError(rc, "ingest_batch (in-view)")
        keys = ("accepted", "dropped_late", "evicted", "active_edges", "t_min", "t_max")
        return dict(zip(keys, (int(v) for v in info)))

    def evict_before(self, cutoff: int) -> int:
        if self._rev:
            self._lib.oracle_evict_before(self._rev, int(cutoff))
        return int(self._lib.oracle_evict_before(self._h, int(cutoff)))

    def sizes(self) -> dict:
        s = np.zeros(4, np.int64)
        self._lib.oracle_sizes(self._h, _ptr(s))
        return dict(m=int(s[0]), gg=int(s[1]), gn=int(s[2]), V=int(s[3]))

    def views(self) -> dict:
        s = self.sizes()
        m, gg, gn, V = s["m"], s["gg"], s["gn"], s["V"]
        out = dict(src=np.empty(m, np.int32), dst=np.empty(m, np.int32), ts=np.empty(m, np.int64),
                   g_ts=np.empty(gg, np.int64), g_off=np.empty(gg + 1, np.int64),
                   n_dst=np.empty(m, np.int32), n_ts=np.empty(m, np.int64),
                   n_gts=np.empty(gn, np.int64), n_goff=np.empty(gn + 1, np.int64),
                   n_ebeg=np.empty(V + 1, np.int64), n_gbeg=np.empty(V + 1, np.int64))
        self._lib.oracle_views(self._h, *(_ptr(out[k]) for k in (
            "src", "dst", "ts", "g_ts", "g_off", "n_dst", "n_ts", "n_gts", "n_goff",
            "n_ebeg", "n_gbeg")))
        return out

    def sample_walks(self, num_walks: int, max_len: int, hop_bias: str = "uniform",
                     hop_tau: float = 0.0, p: float = 1.0, q: float = 1.0,
                     start_bias: str = "uniform", start_tau: float = 0.0,
                     start_mode: str = "edge", start_nodes=None, seed: int = 42,
                     walk_id_base: int = 0, walk_idx=None, with_margin: bool = False,
                     threads: int = 0, check: bool = True, direction: str = "forward") -> dict:
        """Walks for ids walk_idx (default: all num_walks); direction
        "backward" needs a graph created with backward=True."""
        backward = direction == "backward"
        if backward and not self._backward:
            raise OracleError(ST_EINVAL, "sample_walks: created without backward")
        h = self._rev if (backward and self._rev) else self._h
        idx = None if walk_idx is None else np.ascontiguousarray(walk_idx, np.int64)
        n_out = num_walks if idx is None else len(idx)
        sn = None if start_nodes is None else np.ascontiguousarray(start_nodes, np.int32)
        nodes = np.empty((n_out, max(max_len, 1)), np.int32)
        ts = np.empty((n_out, max(max_len, 1)), np.int64)
        lens = np.empty(n_out, np.int32)
        margin = np.empty((n_out, max(max_len, 1)), np.float64) if with_margin else None
        stats = np.zeros(2, np.int64)
        rc = self._lib.oracle_sample_walks(
            h, int(max_len), KINDS[hop_bias], float(hop_tau), float(p), float(q),
            KINDS[start_bias], float(start_tau), START_MODES[start_mode], _ptr(sn),
            int(seed), int(walk_id_base), _ptr(idx), int(n_out), _ptr(nodes), _ptr(ts),
            _ptr(lens), _ptr(margin), _ptr(stats), int(threads), 1 if backward else 0)
        if check and rc != ST_OK:
            raise OracleError(rc, "sample_walks")
        return dict(nodes=nodes, ts=ts, len=lens, margin=margin, status=rc,
                    cap_hits=int(stats[0]), trials=int(stats[1]))
