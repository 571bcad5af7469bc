"""Python binding of the MI355X streaming temporal random-walk library.

Argument marshalling only: every step of ingest, eviction and walk sampling
runs in the HIP kernels of ``libtw.so`` (C ABI in ``include/tw.h``). PyTorch
supplies device memory (tensors) and the HIP stream. The library must be
built (``__graft_entry__.build()``); importing works without it, but every
call raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtw.so")

UNIFORM, LINEAR, EXPONENTIAL, NODE2VEC, WEIGHT = 0, 1, 2, 3, 4
KINDS = {"uniform": UNIFORM, "linear": LINEAR, "exponential": EXPONENTIAL, "node2vec": NODE2VEC,
         "weight": WEIGHT}
DIRECTIONS = {"forward": 0, "backward": 1}
START_EDGE, START_NODE = 0, 1
START_MODES = {"edge": START_EDGE, "node": START_NODE}
DISPATCH = {"auto": 0, "full_walk": 1, "coop": 2, "queue": 3}
DISPATCH_NAMES = {v: k for k, v in DISPATCH.items()}
MAX_BIASES = 8
MAX_NOALLOC_WALKS = 262144  # TW_NOALLOC_MAX_WALKS
TW_OK, TW_EINVAL, TW_ENOMEM, TW_EDEVICE, TW_ERANGE, TW_ETIMEOUT = 0, 1, 2, 3, 4, 5
TS_NONE = -(1 << 63)

_c = ctypes


class _Bias(_c.Structure):
    _fields_ = [("kind", _c.c_int32), ("tau", _c.c_double), ("p", _c.c_double),
                ("q", _c.c_double)]


class _Config(_c.Structure):
    _fields_ = [("num_nodes", _c.c_int32), ("directed", _c.c_int32), ("window", _c.c_int64),
                ("hip_stream", _c.c_void_p)]


class _WalkParams(_c.Structure):
    _fields_ = [("num_walks", _c.c_int64), ("max_len", _c.c_int32), ("hop_bias", _Bias),
                ("start_bias", _Bias), ("start_mode", _c.c_int32),
                ("d_start_nodes", _c.c_void_p), ("seed", _c.c_uint64),
                ("walk_id_base", _c.c_uint64), ("dispatch", _c.c_int32),
                ("direction", _c.c_int32)]


class _BatchParams(_c.Structure):
    _fields_ = [("num_walks", _c.c_int64), ("max_len", _c.c_int32),
                ("d_max_len", _c.c_void_p), ("num_biases", _c.c_int32),
                ("hop_biases", _Bias * MAX_BIASES), ("d_bias", _c.c_void_p),
                ("start_bias", _Bias), ("start_mode", _c.c_int32),
                ("d_start_nodes", _c.c_void_p), ("seed", _c.c_uint64),
                ("walk_id_base", _c.c_uint64), ("d_row", _c.c_void_p),
                ("out_slots", _c.c_int64), ("dispatch", _c.c_int32),
                ("direction", _c.c_int32)]


class _Info(_c.Structure):
    _fields_ = [(k, _c.c_int64) for k in ("accepted", "dropped_late", "evicted",
                                          "active_edges", "t_min", "t_max")]


class _Tuning(_c.Structure):
    _fields_ = [(k, _c.c_int32) for k in ("dispatch", "queue_bpc", "coop_regroup",
                                          "coop_wave_min", "coop_panel", "coop_sync")]


class _ServerConfig(_c.Structure):
    _fields_ = [("arena_bytes", _c.c_int64), ("max_walks_per_launch", _c.c_int64),
                ("max_inflight", _c.c_int32), ("hbm_reserve_bytes", _c.c_int64)]


class _RequestResult(_c.Structure):
    _fields_ = [("status", _c.c_int), ("d_nodes", _c.c_void_p), ("d_ts", _c.c_void_p),
                ("d_len", _c.c_void_p), ("num_walks", _c.c_int64), ("max_len", _c.c_int32),
                ("queue_ms", _c.c_double), ("latency_ms", _c.c_double), ("ingest", _Info),
                ("trial_cap_hits", _c.c_int64)]


class _ServerCounters(_c.Structure):
    _fields_ = [(k, _c.c_int64) for k in ("requests_done", "walks_done", "hops_done",
                                          "launches", "ingests")] + \
               [(k, _c.c_double) for k in ("p50_ms", "p99_ms", "max_ms", "mean_ms", "wall_s")] + \
               [(k, _c.c_int64) for k in ("arena_bytes", "arena_chunks_added")]


_lib = None


def lib():
    """The loaded libtw.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = _c.CDLL(LIB_PATH)
    P, I64 = _c.c_void_p, _c.c_int64
    sig = {
        "tw_create": ([_c.POINTER(_Config), _c.POINTER(P)], _c.c_int),
        "tw_destroy": ([P], _c.c_int),
        "tw_set_stream": ([P, P], _c.c_int),
        "tw_ingest_batch": ([P, P, P, P, I64, _c.POINTER(_Info)], _c.c_int),
        "tw_evict_before": ([P, I64, _c.POINTER(I64)], _c.c_int),
        "tw_sample_walks": ([P, _c.POINTER(_WalkParams), P, P, P], _c.c_int),
        "tw_sample_walks_noalloc": ([P, _c.POINTER(_WalkParams), P, P, P], _c.c_int),
        "tw_set_ingest_weights": ([P, _c.c_double], _c.c_int),
        "tw_last_update": ([P, _c.POINTER(I64)], _c.c_int),
        "tw_walk_layout": ([P, _c.POINTER(_c.c_uint64)], _c.c_int),
        "tw_get_tuning": ([P, _c.POINTER(_Tuning)], _c.c_int),
        "tw_set_tuning": ([P, _c.POINTER(_Tuning)], _c.c_int),
        "tw_sync": ([P], _c.c_int),
        "tw_stats": ([P, _c.POINTER(_Info)], _c.c_int),
        "tw_view_sizes": ([P, _c.POINTER(I64)], _c.c_int),
        "tw_export_views": ([P] * 12, _c.c_int),
        "tw_device_bytes": ([P], I64),
        "tw_index_stats": ([P, _c.POINTER(I64)], _c.c_int),
        "tw_server_create": ([P, _c.POINTER(_ServerConfig), _c.POINTER(P)], _c.c_int),
        "tw_server_submit": ([P, _c.POINTER(_WalkParams), _c.POINTER(_c.c_uint64)], _c.c_int),
        "tw_server_ingest": ([P, P, P, P, I64, _c.POINTER(_c.c_uint64)], _c.c_int),
        "tw_server_wait": ([P, _c.c_uint64, I64, _c.POINTER(_RequestResult)], _c.c_int),
        "tw_server_release": ([P, _c.c_uint64], _c.c_int),
        "tw_server_copy_out": ([P, _c.c_uint64, P, P, P], _c.c_int),
        "tw_server_stats": ([P, _c.POINTER(_ServerCounters)], _c.c_int),
        "tw_server_destroy": ([P], _c.c_int),
        "tw_sample_walks_batch": ([P, _c.POINTER(_BatchParams), P, P, P], _c.c_int),
        "tw_row_offsets": ([P, P, I64, P, _c.POINTER(I64)], _c.c_int),
        "tw_autotune": ([P, _c.POINTER(_WalkParams), I64, P, P, P, _c.POINTER(_c.c_int32)],
                        _c.c_int),
        "tw_last_error": ([], _c.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class TwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[tw status {code}] {msg}")
        self.code = code


def _check(rc: int):
    if rc != TW_OK:
        raise TwError(rc, lib().tw_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tw arrays must be device tensors")
    if not t.is_contiguous():
        raise ValueError("tw arrays must be contiguous")
    return _c.c_void_p(t.data_ptr())


def _info(i: _Info) -> dict:
    return {k: int(getattr(i, k)) for k, _ in _Info._fields_}


class Graph:
    """A sliding-window temporal graph resident on one GPU."""

    def __init__(self, num_nodes: int, directed: bool = True, window: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.num_nodes = int(num_nodes)
        self._lib = lib()
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream()
            self.stream = s
            cfg = _Config(self.num_nodes, 1 if directed else 0, int(window),
                          _c.c_void_p(s.cuda_stream))
            h = _c.c_void_p()
            _check(self._lib.tw_create(_c.byref(cfg), _c.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.tw_destroy(h)
            self._h = None

    __del__ = close

    def set_stream(self, stream: torch.cuda.Stream):
        _check(self._lib.tw_set_stream(self._h, _c.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def ingest_batch(self, src: torch.Tensor, dst: torch.Tensor, ts: torch.Tensor,
                     info: bool = True) -> Optional[dict]:
        """The batch's counts and the window's range (info=False: None, and
        the window summary stays on the device; one read-back fewer)."""
        assert src.dtype == torch.int32 and dst.dtype == torch.int32 and ts.dtype == torch.int64
        n = src.numel()
        assert dst.numel() == n and ts.numel() == n
        out = _Info() if info else None
        _check(self._lib.tw_ingest_batch(self._h, _ptr(src), _ptr(dst), _ptr(ts), n,
                                         _c.byref(out) if info else None))
        return _info(out) if info else None

    def last_update(self) -> dict:
        """Counts of the last ingest or eviction, host-side (tw_last_update)."""
        out = (_c.c_int64 * 4)()
        _check(self._lib.tw_last_update(self._h, out))
        return dict(zip(("accepted", "dropped_late", "evicted", "active_edges"), map(int, out)))

    def set_ingest_weights(self, tau: Optional[float]):
        """Build the weight-based picker's weights at every ingest and
        eviction for this tau (None: on the first weight-based walk)."""
        _check(self._lib.tw_set_ingest_weights(self._h, float("nan") if tau is None
                                               else float(tau)))

    def evict_before(self, cutoff: int) -> int:
        n = _c.c_int64(0)
        _check(self._lib.tw_evict_before(self._h, int(cutoff), _c.byref(n)))
        return int(n.value)

    def sample_walks(self, num_walks: int, max_len: int, hop_bias: str = "uniform",
                     hop_tau: float = 0.0, p: float = 1.0, q: float = 1.0,
                     start_bias: str = "uniform", start_tau: float = 0.0,
                     start_mode: str = "edge", start_nodes: Optional[torch.Tensor] = None,
                     seed: int = 42, walk_id_base: int = 0, dispatch: str = "auto",
                     out=None, direction: str = "forward"):
        """Returns (nodes int32[W, L], ts int64[W, L], len int32[W]) on the device.
        direction "backward": each hop takes an in-edge strictly before the
        current time (tw_direction)."""
        W, L = int(num_walks), int(max_len)
        if out is None:
            nodes = torch.empty((W, max(L, 1)), dtype=torch.int32, device=self.device)
            ts = torch.empty((W, max(L, 1)), dtype=torch.int64, device=self.device)
            lens = torch.empty(W, dtype=torch.int32, device=self.device)
        else:
            nodes, ts, lens = out
        if start_nodes is not None:
            assert start_nodes.dtype == torch.int32 and start_nodes.numel() >= W
        prm = _WalkParams(W, L, _Bias(KINDS[hop_bias], float(hop_tau), float(p), float(q)),
                          _Bias(KINDS[start_bias], float(start_tau), 1.0, 1.0),
                          START_MODES[start_mode], _ptr(start_nodes), int(seed),
                          int(walk_id_base), DISPATCH[dispatch], DIRECTIONS[direction])
        _check(self._lib.tw_sample_walks(self._h, _c.byref(prm), _ptr(nodes), _ptr(ts),
                                         _ptr(lens)))
        return nodes, ts, lens

    def sample_walks_noalloc(self, num_walks: int, max_len: int, out, hop_bias: str = "uniform",
                             hop_tau: float = 0.0, p: float = 1.0, q: float = 1.0,
                             start_bias: str = "uniform", start_tau: float = 0.0,
                             start_mode: str = "edge", start_nodes: Optional[torch.Tensor] = None,
                             seed: int = 42, walk_id_base: int = 0):
        """tw_sample_walks_noalloc into the caller's out = (nodes int32[W, L],
        ts int64[W, L], len int32[W]): the queue dispatch's walks with no
        device allocation (at most MAX_NOALLOC_WALKS walks)."""
        W, L = int(num_walks), int(max_len)
        nodes, ts, lens = out
        if start_nodes is not None:
            assert start_nodes.dtype == torch.int32 and start_nodes.numel() >= W
        prm = _WalkParams(W, L, _Bias(KINDS[hop_bias], float(hop_tau), float(p), float(q)),
                          _Bias(KINDS[start_bias], float(start_tau), 1.0, 1.0),
                          START_MODES[start_mode], _ptr(start_nodes), int(seed),
                          int(walk_id_base), DISPATCH["queue"], DIRECTIONS["forward"])
        _check(self._lib.tw_sample_walks_noalloc(self._h, _c.byref(prm), _ptr(nodes), _ptr(ts),
                                                 _ptr(lens)))
        return nodes, ts, lens

    def sample_walks_batch(self, num_walks: int, max_len: int, hop_biases,
                           max_lens: Optional[torch.Tensor] = None,
                           bias_idx: Optional[torch.Tensor] = None,
                           start_bias: str = "uniform", start_tau: float = 0.0,
                           start_mode: str = "edge", start_nodes: Optional[torch.Tensor] = None,
                           seed: int = 42, walk_id_base: int = 0, ragged: bool = False,
                           dispatch: str = "queue", rows=None, out=None,
                           direction: str = "forward"):
        """Walks of uneven lengths and mixed hop biases in one persistent
        launch. hop_biases: list of (kind, tau, p, q); max_lens: int32[W] or
        None; bias_idx: uint8[W] or None (walk id mod len(hop_biases)).
        Returns (nodes, ts, len, row): rows of width max_len (row None), or,
        with ragged=True, packed rows starting at row[i] (int64[W + 1]; pass
        rows=(row, total) from row_offsets to skip computing them).
        dispatch "queue" (persistent work queue) or "full_walk" (one thread
        per walk, no queue); direction "forward" or "backward"."""
        W, L = int(num_walks), int(max_len)
        nb = len(hop_biases)  # the library rejects 0 or more than MAX_BIASES
        biases = (_Bias * MAX_BIASES)()
        for i, (k, tau, p, q) in enumerate(hop_biases[:MAX_BIASES]):
            biases[i] = _Bias(KINDS[k], float(tau), float(p), float(q))
        if max_lens is not None:
            assert max_lens.dtype == torch.int32 and max_lens.numel() >= W
        if bias_idx is not None:
            assert bias_idx.dtype == torch.uint8 and bias_idx.numel() >= W
        if start_nodes is not None:
            assert start_nodes.dtype == torch.int32 and start_nodes.numel() >= W
        row = None
        slots = W * L
        if ragged:
            assert max_lens is not None
            row, total = rows if rows is not None else self.row_offsets(max_lens, W)
            slots = max(int(total), 1)
        if out is None:
            nodes = torch.empty(max(slots, 1), dtype=torch.int32, device=self.device)
            ts = torch.empty(max(slots, 1), dtype=torch.int64, device=self.device)
            lens = torch.empty(max(W, 1), dtype=torch.int32, device=self.device)
        else:
            nodes, ts, lens = out
            assert nodes.numel() >= slots and ts.numel() >= slots
        prm = _BatchParams(W, L, _ptr(max_lens), nb, biases, _ptr(bias_idx),
                           _Bias(KINDS[start_bias], float(start_tau), 1.0, 1.0),
                           START_MODES[start_mode], _ptr(start_nodes), int(seed),
                           int(walk_id_base), _ptr(row), slots if ragged else 0,
                           DISPATCH[dispatch], DIRECTIONS[direction])
        _check(self._lib.tw_sample_walks_batch(self._h, _c.byref(prm), _ptr(nodes), _ptr(ts),
                                               _ptr(lens)))
        if not ragged:
            nodes, ts = nodes[:W * L].view(W, L), ts[:W * L].view(W, L)
        return nodes, ts, lens[:W], row

    def row_offsets(self, max_lens: torch.Tensor, n: Optional[int] = None):
        """Packed row starts for per-walk limits: (row int64[n + 1], total)."""
        n = max_lens.numel() if n is None else int(n)
        assert max_lens.dtype == torch.int32
        row = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        total = _c.c_int64(0)
        _check(self._lib.tw_row_offsets(self._h, _ptr(max_lens), n, _ptr(row), _c.byref(total)))
        return row, int(total.value)

    def autotune(self, num_walks: int, max_len: int, sample: int = 1 << 20,
                 hop_bias: str = "uniform", hop_tau: float = 0.0, p: float = 1.0,
                 q: float = 1.0, start_bias: str = "uniform", start_tau: float = 0.0,
                 start_mode: str = "edge", start_nodes: Optional[torch.Tensor] = None,
                 seed: int = 42) -> dict:
        """Time the dispatches on the current window and keep the fastest for
        dispatch="auto"; returns {"dispatch": name, "blocks_per_cu": n}."""
        W = min(int(num_walks), int(sample))
        L = int(max_len)
        nodes = torch.empty((max(W, 1), L), dtype=torch.int32, device=self.device)
        ts = torch.empty((max(W, 1), L), dtype=torch.int64, device=self.device)
        lens = torch.empty(max(W, 1), dtype=torch.int32, device=self.device)
        prm = _WalkParams(int(num_walks), L, _Bias(KINDS[hop_bias], float(hop_tau), float(p),
                                                   float(q)),
                          _Bias(KINDS[start_bias], float(start_tau), 1.0, 1.0),
                          START_MODES[start_mode], _ptr(start_nodes), int(seed), 0, 0)
        best = (_c.c_int32 * 2)()
        _check(self._lib.tw_autotune(self._h, _c.byref(prm), int(sample), _ptr(nodes), _ptr(ts),
                                     _ptr(lens), best))
        return {"dispatch": DISPATCH_NAMES[int(best[0])], "blocks_per_cu": int(best[1])}

    def tuning(self) -> dict:
        """The dispatch tuning (tw_tuning); dispatch as a name."""
        t = _Tuning()
        _check(self._lib.tw_get_tuning(self._h, _c.byref(t)))
        d = {k: getattr(t, k) for k, _ in _Tuning._fields_}
        d["dispatch"] = DISPATCH_NAMES[d["dispatch"]]
        return d

    def set_tuning(self, dispatch: str = "full_walk", queue_bpc: int = 0, coop_regroup: int = 0,
                   coop_wave_min: int = 64, coop_panel: int = 4096, coop_sync: int = 1):
        t = _Tuning(DISPATCH[dispatch], int(queue_bpc), int(coop_regroup), int(coop_wave_min),
                    int(coop_panel), int(coop_sync))
        _check(self._lib.tw_set_tuning(self._h, _c.byref(t)))

    def sync(self):
        _check(self._lib.tw_sync(self._h))

    def stats(self) -> dict:
        info = _Info()
        _check(self._lib.tw_stats(self._h, _c.byref(info)))
        return _info(info)

    def view_sizes(self) -> dict:
        out = (_c.c_int64 * 4)()
        _check(self._lib.tw_view_sizes(self._h, out))
        return dict(m=out[0], gg=out[1], gn=out[2], V=out[3])

    def export_views(self) -> dict:
        s = self.view_sizes()
        m, gg, gn, V = s["m"], s["gg"], s["gn"], s["V"]
        d = self.device
        t = dict(src=torch.empty(m, dtype=torch.int32, device=d),
                 dst=torch.empty(m, dtype=torch.int32, device=d),
                 ts=torch.empty(m, dtype=torch.int64, device=d),
                 g_ts=torch.empty(gg, dtype=torch.int64, device=d),
                 g_off=torch.empty(gg + 1, dtype=torch.int64, device=d),
                 n_dst=torch.empty(m, dtype=torch.int32, device=d),
                 n_ts=torch.empty(m, dtype=torch.int64, device=d),
                 n_gts=torch.empty(gn, dtype=torch.int64, device=d),
                 n_goff=torch.empty(gn + 1, dtype=torch.int64, device=d),
                 n_ebeg=torch.empty(V + 1, dtype=torch.int64, device=d),
                 n_gbeg=torch.empty(V + 1, dtype=torch.int64, device=d))
        order = ("src", "dst", "ts", "g_ts", "g_off", "n_dst", "n_ts", "n_gts", "n_goff",
                 "n_ebeg", "n_gbeg")
        _check(self._lib.tw_export_views(self._h, *(_ptr(t[k]) if t[k].numel() else None
                                                    for k in order)))
        return t

    def walk_layout(self) -> int:
        """Where the device buffers lie (see tw_walk_layout): a recorded walk
        launch replays correctly while this value is unchanged."""
        out = _c.c_uint64(0)
        _check(self._lib.tw_walk_layout(self._h, _c.byref(out)))
        return int(out.value)

    def index_stats(self) -> dict:
        """Counters of the last index update (see tw_index_stats)."""
        out = (_c.c_int64 * 8)()
        _check(self._lib.tw_index_stats(self._h, out))
        keys = ("jobs", "written", "new_slots", "full_rewrite", "edge_slots", "group_slots",
                "fence_slots", "edge_capacity")
        return {k: int(out[i]) for i, k in enumerate(keys)}

    def device_bytes(self) -> int:
        return int(self._lib.tw_device_bytes(self._h))


class Server:
    """Continuous batching of walk requests over a Graph (see tw_server_* in
    include/tw.h). The graph must not be used directly while the server
    exists."""

    def __init__(self, graph: Graph, arena_bytes: int = 1 << 30,
                 max_walks_per_launch: int = 1 << 21, max_inflight: int = 2,
                 hbm_reserve_bytes: int = 8 << 30):
        """hbm_reserve_bytes < 0: a fixed arena; else more arena chunks are
        added while the device keeps that much memory free."""
        self._lib = lib()
        self.graph = graph
        self.device = graph.device
        cfg = _ServerConfig(int(arena_bytes), int(max_walks_per_launch), int(max_inflight),
                            int(hbm_reserve_bytes))
        h = _c.c_void_p()
        _check(self._lib.tw_server_create(graph._h, _c.byref(cfg), _c.byref(h)))
        self._h = h
        self._keep = {}  # input tensors of queued work, by id

    def submit(self, num_walks: int, max_len: int, hop_bias: str = "uniform",
               hop_tau: float = 0.0, p: float = 1.0, q: float = 1.0,
               start_bias: str = "uniform", start_tau: float = 0.0, start_mode: str = "edge",
               start_nodes: Optional[torch.Tensor] = None, seed: int = 42,
               walk_id_base: int = 0, direction: str = "forward") -> int:
        prm = _WalkParams(int(num_walks), int(max_len),
                          _Bias(KINDS[hop_bias], float(hop_tau), float(p), float(q)),
                          _Bias(KINDS[start_bias], float(start_tau), 1.0, 1.0),
                          START_MODES[start_mode], _ptr(start_nodes), int(seed),
                          int(walk_id_base), 0, DIRECTIONS[direction])
        rid = _c.c_uint64(0)
        _check(self._lib.tw_server_submit(self._h, _c.byref(prm), _c.byref(rid)))
        if start_nodes is not None:
            self._keep[rid.value] = start_nodes
        return int(rid.value)

    def ingest(self, src: torch.Tensor, dst: torch.Tensor, ts: torch.Tensor) -> int:
        assert src.dtype == torch.int32 and dst.dtype == torch.int32 and ts.dtype == torch.int64
        rid = _c.c_uint64(0)
        _check(self._lib.tw_server_ingest(self._h, _ptr(src), _ptr(dst), _ptr(ts), src.numel(),
                                          _c.byref(rid)))
        self._keep[rid.value] = (src, dst, ts)
        return int(rid.value)

    def wait(self, rid: int, timeout_s: Optional[float] = None) -> Optional[dict]:
        """The finished request's result record, or None on timeout."""
        out = _RequestResult()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        rc = self._lib.tw_server_wait(self._h, _c.c_uint64(rid), us, _c.byref(out))
        if rc == TW_ETIMEOUT:
            return None
        _check(rc)
        self._keep.pop(rid, None)
        return {"status": int(out.status), "num_walks": int(out.num_walks),
                "max_len": int(out.max_len), "queue_ms": out.queue_ms,
                "latency_ms": out.latency_ms, "ingest": _info(out.ingest),
                "trial_cap_hits": int(out.trial_cap_hits)}

    def result(self, rid: int):
        """(nodes, ts, len) of a finished request, copied into new tensors."""
        r = self.wait(rid)
        W, L = r["num_walks"], r["max_len"]
        nodes = torch.empty((max(W, 1), max(L, 1)), dtype=torch.int32, device=self.device)
        ts = torch.empty((max(W, 1), max(L, 1)), dtype=torch.int64, device=self.device)
        lens = torch.empty(max(W, 1), dtype=torch.int32, device=self.device)
        _check(self._lib.tw_server_copy_out(self._h, _c.c_uint64(rid), _ptr(nodes), _ptr(ts),
                                            _ptr(lens)))
        return nodes[:W], ts[:W], lens[:W]

    def release(self, rid: int):
        _check(self._lib.tw_server_release(self._h, _c.c_uint64(rid)))

    def stats(self) -> dict:
        c = _ServerCounters()
        _check(self._lib.tw_server_stats(self._h, _c.byref(c)))
        return {k: getattr(c, k) for k, _ in _ServerCounters._fields_}

    def close(self):
        if self._h:
            _check(self._lib.tw_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
