// Walk sampling (Tempest, Sec. "Temporal Bias Sampling" and "The Full-Walk
// Baseline"). A walk is keyed by (seed, walk id); hop h, trial r draws
// Philox4x64-10 at counter (id, h, r, 0), so every dispatch produces the
// same walks.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "walk_device.h"

namespace tw {
namespace {

// A hop bias with node2vec's constants precomputed.
struct HopBias {
    int32_t kind;
    double tau, inv_p, inv_q, beta_max;
};

HopBias make_hop_bias(const tw_bias& b) {
    HopBias h;
    h.kind = b.kind;
    h.tau = b.tau;
    h.inv_p = b.kind == TW_NODE2VEC ? 1.0 / b.p : 1.0;
    h.inv_q = b.kind == TW_NODE2VEC ? 1.0 / b.q : 1.0;
    h.beta_max = std::max(std::max(h.inv_p, 1.0), h.inv_q);
    return h;
}

struct WalkArgs {
    // timestamp view and its groups
    const int32_t* e_src;
    const int32_t* e_dst;
    const int64_t* e_ts;
    const uint32_t* gg_off;  // first record of each timestamp group (from gg_base), then the end
    // read from the graph's scalar slots, where the last update wrote them: the
    // window's first and last timestamps, its global group count, and
    // win = (e_base, m, gg_base): the window is e_*[e_base, e_base + m), its
    // groups start at gg_off[gg_base]
    const int64_t* wsum;
    const int64_t* wgg;
    const int64_t* win;
    // node view
    const int32_t* n_dst;
    const int64_t* n_ts;
    const GroupRec* ng;
    const NodeRec* rec;
    const uint32_t* fence;
    const AdjSlot* adj_tab;  // node2vec pair table (adj_mask + 1 slots)
    uint64_t adj_mask;
    const double* cw;  // cumulative group weights (weight-based picker)
    int32_t V;
    // parameters
    int64_t num_walks;
    int32_t L;
    HopBias hop;
    int32_t start_kind, start_mode;
    double start_tau;
    const int32_t* start_nodes;
    uint64_t seed, base;
    // outputs
    int32_t* nodes;
    int64_t* ts;
    int32_t* len;
    uint32_t* err;  // [0] start node out of range, [2] node2vec trial cap hits
};

// The start of a walk: RNG seed, start bias and mode, start nodes.
struct StartParams {
    uint64_t seed;
    int32_t kind, mode;
    double tau;
    const int32_t* nodes;
};

__device__ __forceinline__ StartParams start_of(const WalkArgs& a) {
    return StartParams{a.seed, a.start_kind, a.start_mode, a.start_tau, a.start_nodes};
}

constexpr int WALK_THREADS = 256;

// Kernels are instantiated per hop kind HK and start kind SK (-1: read at
// run time). A fixed kind leaves only that picker's arithmetic in the
// kernel: the full-walk kernel takes 52-56 VGPRs for uniform and linear hops
// (8 wavefronts per SIMD) and about 100 for exponential hops, against 129
// for the kernel that carries every picker (3 wavefronts per SIMD).
template <int HK>
__device__ __forceinline__ HopBias fixed_hop(HopBias h) {
    if (HK >= 0) h.kind = HK;
    return h;
}
template <int SK>
__device__ __forceinline__ StartParams fixed_start(StartParams sp) {
    if (SK >= 0) sp.kind = SK;
    return sp;
}
constexpr uint32_t N2V_MAX_TRIALS = 4096;

// Walk state after the first pick (RNG hop 0).
struct StartState {
    int32_t len;   // nodes written so far
    int32_t cur, prev;
    int64_t t;
    int32_t first; // the node at position 0 (when len >= 1)
};

// First pick of walk w: EDGE mode draws from the whole window, NODE mode from
// the start node's run; writes output positions 0 and 1 (out_n null: writes
// nothing, the caller takes them from the state). rev: a backward walk
// (candidates listed in reverse). A start node out of range sets
// *range_flag (the graph's flag word when null).
__device__ __forceinline__ StartState walk_start(const WalkArgs& a, const StartParams& sp, int64_t w,
                                                 uint64_t id, int32_t L, int32_t* out_n,
                                                 int64_t* out_t, bool rev = false,
                                                 uint32_t* range_flag = nullptr) {
    StartState st{0, 0, 0, 0, -1};
    const Draw d0 = philox(id, 0, 0, sp.seed);
    if (sp.mode == TW_START_EDGE) {
        const uint32_t m = (uint32_t)a.win[1];
        if (m == 0) return st;
        uint32_t e;
        if (sp.kind == TW_UNIFORM) {
            const uint32_t i = (uint32_t)scale_u64(d0.x0, m);
            e = (uint32_t)a.win[0] + (rev ? m - 1 - i : i);
        } else {
            e = pick_global(a.gg_off + a.win[2], (uint32_t)*a.wgg, a.wsum[0], a.wsum[1], sp.kind,
                            sp.tau, d0, rev);
        }
        const int32_t s = a.e_src[e], t_dst = a.e_dst[e];
        const int64_t t = a.e_ts[e];
        if (out_n) out_n[0] = s;
        st.first = s;
        st.len = 1;
        if (L == 1) return st;
        if (out_n) {
            out_n[1] = t_dst;
            out_t[1] = t;
        }
        st.len = 2;
        st.prev = s;
        st.cur = t_dst;
        st.t = t;
        return st;
    }
    const int32_t v0 = sp.nodes[w];
    if (v0 < 0 || v0 >= a.V) {
        atomicOr(range_flag ? range_flag : &a.err[0], 1u);
        return st;
    }
    if (out_n) out_n[0] = v0;
    st.first = v0;
    st.len = 1;
    if (L == 1) return st;
    const NodeRec r = a.rec[v0];
    if (r.gb == r.ge) return st;
    const int64_t t_first = reads_first_ts(sp.kind) ? a.ng[r.gb].ts : 0;
    Pick p = pick_node(a.ng, a.n_dst, a.n_ts, r.gb, r.ge, r.ee, sp.kind, sp.tau, t_first,
                       r.t_last, d0, rev);
    const int32_t nx = p.dst;
    if (out_n) {
        out_n[1] = nx;
        out_t[1] = p.t;
    }
    st.len = 2;
    st.prev = v0;
    st.cur = nx;
    st.t = p.t;
    return st;
}

// The pick of hop `hop` among groups [gc, r.ge) of node cur (previous node
// prev): the hop bias, or node2vec's rejection loop. Returns false when
// node2vec exhausts its trials (the walk ends; counted in *cap_count, the
// graph's counter word when null).
__device__ __forceinline__ bool hop_pick(const WalkArgs& a, const HopBias& hb, uint64_t seed,
                                         const NodeRec& r, uint32_t gc, uint64_t id, uint64_t hop,
                                         int32_t prev, Pick& p, int32_t& nx,
                                         uint32_t* cap_count = nullptr) {
    if (hb.kind == TW_WEIGHT) {
        const Draw d = philox(id, hop, 0, seed);
        p = pick_weight(a.ng, a.n_dst, a.cw, r.gb, gc, r.ge, r.ee, hb.tau > 0.0 ? hb.tau : 1.0,
                        group_ts(a.ng, a.fence, r, gc), r.t_last, d);
        nx = p.dst;
        return true;
    }
    if (hb.kind != TW_NODE2VEC) {
        const Draw d = philox(id, hop, 0, seed);
        const int64_t t_first = reads_first_ts(hb.kind) ? group_ts(a.ng, a.fence, r, gc) : 0;
        p = pick_node(a.ng, a.n_dst, a.n_ts, gc, r.ge, r.ee, hb.kind, hb.tau, t_first, r.t_last,
                      d);
        nx = p.dst;
        return true;
    }
    const int64_t t_first = group_ts(a.ng, a.fence, r, gc);
    for (uint32_t trial = 0; trial < N2V_MAX_TRIALS; ++trial) {
        const Draw d = philox(id, hop, trial, seed);
        p = pick_node(a.ng, a.n_dst, a.n_ts, gc, r.ge, r.ee, TW_EXPONENTIAL, hb.tau, t_first,
                      r.t_last, d);
        nx = p.dst;
        double beta;
        if (nx == prev) beta = hb.inv_p;
        else if (adj_has(a.adj_tab, a.adj_mask, prev, nx)) beta = 1.0;
        else beta = hb.inv_q;
        if (unit_closed_open(d.x2) * hb.beta_max < beta) return true;
    }
    atomicAdd(cap_count ? cap_count : &a.err[2], 1u);
    return false;
}

// the output rows were pre-filled with -1 / INT64_MIN, so ending a walk
// only records its length
__device__ __forceinline__ void finish_walk(const WalkArgs& a, int64_t w, int32_t len) {
    a.len[w] = len;
}

// Padding values (-1 nodes, INT64_MIN timestamps) for the output slots
// [b, e), written by threads tid, tid + stride, ... with 16-byte stores where
// the arrays are 16-byte aligned. The bulk stores are non-temporal: the
// padding is not read back, and cached it displaces index records the walk
// reads next (fill + walk measured 0.3% faster; the fill alone is slower).
typedef int v4i __attribute__((ext_vector_type(4)));
typedef long long v2l __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void fill_span(int32_t* __restrict__ nodes, int64_t* __restrict__ ts,
                                          int64_t b, int64_t e, int64_t tid, int64_t stride) {
    if (b >= e) return;
    // nodes: scalar head up to a 16-byte boundary, int4 body, scalar tail
    const int64_t nb = std::min<int64_t>(
        e, b + (int64_t)(((16 - ((uintptr_t)(nodes + b) & 15)) & 15) / 4));
    for (int64_t i = b + tid; i < nb; i += stride) nodes[i] = -1;
    const int64_t nv = (e - nb) / 4;
    int4* nv4 = reinterpret_cast<int4*>(nodes + nb);
    for (int64_t i = tid; i < nv; i += stride)
        __builtin_nontemporal_store((v4i){-1, -1, -1, -1}, reinterpret_cast<v4i*>(nv4) + i);
    for (int64_t i = nb + 4 * nv + tid; i < e; i += stride) nodes[i] = -1;
    const int64_t tb = std::min<int64_t>(
        e, b + (int64_t)(((16 - ((uintptr_t)(ts + b) & 15)) & 15) / 8));
    for (int64_t i = b + tid; i < tb; i += stride) ts[i] = TS_NONE;
    const int64_t tv = (e - tb) / 2;
    longlong2* tv2 = reinterpret_cast<longlong2*>(ts + tb);
    for (int64_t i = tid; i < tv; i += stride)
        __builtin_nontemporal_store((v2l){TS_NONE, TS_NONE}, reinterpret_cast<v2l*>(tv2) + i);
    for (int64_t i = tb + 2 * tv + tid; i < e; i += stride) ts[i] = TS_NONE;
}

// Fill every output slot with the padding values, fully coalesced; the walk
// kernels then write only the slots their walks reach. (Padding inside the
// walk kernel, block by block, measured slower: the stores compete with the
// walks' dependent gathers.)
__global__ void k_fill_outputs(int32_t* __restrict__ nodes, int64_t* __restrict__ ts,
                               int64_t n) {
    fill_span(nodes, ts, 0, n, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
              (int64_t)gridDim.x * blockDim.x);
}

// The last four output slots of a walk in registers (a shift register, so
// no slot is ever indexed at run time): when a walk has filled slots
// 4k..4k+3 they leave as one 16-byte store of nodes and two of timestamps.
struct RowChunk {
    int32_t n0 = -1, n1 = -1, n2 = -1, n3 = -1;
    int64_t t0 = TS_NONE, t1 = TS_NONE, t2 = TS_NONE, t3 = TS_NONE;
    __device__ __forceinline__ void push(int32_t v, int64_t t) {
        n0 = n1;
        n1 = n2;
        n2 = n3;
        n3 = v;
        t0 = t1;
        t1 = t2;
        t2 = t3;
        t3 = t;
    }
    // slots [at, at + 4) of a row; both pointers 16-byte aligned there
    __device__ __forceinline__ void store(int32_t* __restrict__ on, int64_t* __restrict__ ot,
                                          int32_t at) const {
        *reinterpret_cast<int4*>(on + at) = make_int4(n0, n1, n2, n3);
        *reinterpret_cast<longlong2*>(ot + at) = make_longlong2(t0, t1);
        *reinterpret_cast<longlong2*>(ot + at + 2) = make_longlong2(t2, t3);
    }
};

// Ends a row whose first len slots were pushed through c (and stored up to
// the last multiple of 4): the partial chunk is completed with padding, then
// every slot up to L (a multiple of 4) is padded with 16-byte stores.
__device__ __forceinline__ void finish_row(RowChunk& c, int32_t* __restrict__ on,
                                           int64_t* __restrict__ ot, int32_t len, int32_t L) {
    int32_t at = len & ~3;
    if (len & 3) {
        for (int32_t k = len & 3; k < 4; ++k) c.push(-1, TS_NONE);
        c.store(on, ot, at);
        at += 4;
    }
    const RowChunk pad;
    for (; at < L; at += 4) pad.store(on, ot, at);
}

// A lane's current four output slots in LDS, slot p in row p & 3 of the
// lane's column (registers the FP64 pickers need instead): when slots
// 4k..4k+3 are complete they leave as one 16-byte store of nodes and two of
// timestamps. Each lane touches its own column only.
struct RowRing {
    int32_t (*n)[WALK_THREADS];
    int64_t (*t)[WALK_THREADS];
    int tid;
    __device__ __forceinline__ void put(int32_t p, int32_t v, int64_t x) const {
        n[p & 3][tid] = v;
        t[p & 3][tid] = x;
    }
    // slots [at, at + 4) of a row; both pointers 16-byte aligned there
    __device__ __forceinline__ void flush(int32_t* __restrict__ on, int64_t* __restrict__ ot,
                                          int32_t at) const {
        *reinterpret_cast<int4*>(on + at) = make_int4(n[0][tid], n[1][tid], n[2][tid], n[3][tid]);
        *reinterpret_cast<longlong2*>(ot + at) = make_longlong2(t[0][tid], t[1][tid]);
        *reinterpret_cast<longlong2*>(ot + at + 2) = make_longlong2(t[2][tid], t[3][tid]);
    }
    // ends a row of len slots (stored up to the last multiple of 4): the
    // partial chunk is completed with padding, then every slot up to L (a
    // multiple of 4) is padded with 16-byte stores
    __device__ __forceinline__ void finish(int32_t* __restrict__ on, int64_t* __restrict__ ot,
                                           int32_t len, int32_t L) const {
        int32_t at = len & ~3;
        if (len & 3) {
            for (int32_t k = len & 3; k < 4; ++k) put(k, -1, TS_NONE);
            flush(on, ot, at);
            at += 4;
        }
        const RowChunk pad;
        for (; at < L; at += 4) pad.store(on, ot, at);
    }
};

// One full walk per thread: the full-walk baseline (Sec. "The Full-Walk
// Baseline"). The walk is bound by dependent random loads, so waves in flight
// count: the uniform and linear pickers are held to 5 waves per SIMD (they
// fit 8), the exponential and weight pickers' FP64 code and the mixed-kind
// instantiation to 4 (no spills; 5 waves spill 14-16 registers there);
// node2vec (more live state) keeps its own allocation. ROWS: the walk writes
// its whole output row itself, four slots per store, padding included (rows
// of a multiple of 4 slots, 16-byte aligned outputs); otherwise the rows were
// pre-filled with padding and the walk writes the slots it reaches.
template <int HK, int SK, bool ROWS>
__global__ void __launch_bounds__(WALK_THREADS)
__attribute__((amdgpu_waves_per_eu(HK == TW_NODE2VEC ? 1
                                     : HK < 0 || HK == TW_EXPONENTIAL || HK == TW_WEIGHT
                                         ? 4
                                         : 5)))
k_walk_full(const WalkArgs a) {
    const int64_t w = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (w >= a.num_walks) return;
    const uint64_t id = a.base + (uint64_t)w;
    int32_t* out_n = a.nodes + w * a.L;
    int64_t* out_t = a.ts + w * a.L;
    StartState st = walk_start(a, fixed_start<SK>(start_of(a)), w, id, a.L,
                               ROWS ? nullptr : out_n, out_t);
    // ROWS: the row's current four slots in LDS, slot p at [p & 3] (each
    // thread its own column): registers the FP64 pickers need instead
    // (exponential walks 4.57 -> 4.39 ms, node2vec 5.49 -> 4.69 ms on the
    // 100M-edge graph)
    __shared__ int32_t ring_n[4][WALK_THREADS];
    __shared__ int64_t ring_t[4][WALK_THREADS];
    const RowRing ring{ring_n, ring_t, (int)threadIdx.x};
    if (ROWS) {
        ring.put(0, st.len >= 1 ? st.first : -1, TS_NONE);
        ring.put(1, st.len >= 2 ? st.cur : -1, st.len >= 2 ? st.t : TS_NONE);
    }
    const HopBias hb = fixed_hop<HK>(a.hop);
    int32_t len = st.len, cur = st.cur, prev = st.prev;
    int64_t tcur = st.t;
    if (len >= 2) {
        for (uint64_t hop = 1; len < a.L; ++hop) {
            const NodeRec r = a.rec[cur];
            if (tcur >= r.t_last) break;  // Gamma_t(cur) is empty
            const uint32_t gc = fence_search(a.ng, a.fence, r, tcur, nullptr, 0, 0);
            Pick p;
            int32_t nx;
            if (!hop_pick(a, hb, a.seed, r, gc, id, hop, prev, p, nx)) break;
            if (ROWS) {
                ring.put(len, nx, p.t);
                if ((len & 3) == 3) ring.flush(out_n, out_t, len - 3);
            } else {
                out_n[len] = nx;
                out_t[len] = p.t;
            }
            ++len;
            prev = cur;
            cur = nx;
            tcur = p.t;
        }
    }
    if (ROWS) ring.finish(out_n, out_t, len, a.L);
    finish_walk(a, w, len);
}

// Backward walks (Gamma-_t(v): in-edges of v with t' < t, the backward case
// of Sec. "Design Constraints") on the in-view: the candidates of a hop at
// node v and time t are the groups [gb, hi) of v before the first group at
// or after t, listed from the latest, so every pick index is mirrored.
__device__ __forceinline__ bool back_pick(const WalkArgs& a, const HopBias& hb, uint64_t seed,
                                          const NodeRec& r, uint32_t hi, uint64_t id,
                                          uint64_t hop, int32_t prev, Pick& p, int32_t& nx,
                                          uint32_t* cap_count = nullptr) {
    const uint32_t end = hi < r.ge ? a.ng[hi].first : r.ee;  // the candidates' edges end
    const bool rate = reads_first_ts(hb.kind);
    const int64_t t_lo = rate ? group_ts(a.ng, a.fence, r, r.gb) : 0;
    const int64_t t_hi = rate ? group_ts(a.ng, a.fence, r, hi - 1) : 0;
    if (hb.kind != TW_NODE2VEC) {
        const Draw d = philox(id, hop, 0, seed);
        p = pick_node(a.ng, a.n_dst, a.n_ts, r.gb, hi, end, hb.kind, hb.tau, t_lo, t_hi, d,
                      true);
        nx = p.dst;
        return true;
    }
    // the edge candidate -> prev of the graph is prev -> candidate here
    for (uint32_t trial = 0; trial < N2V_MAX_TRIALS; ++trial) {
        const Draw d = philox(id, hop, trial, seed);
        p = pick_node(a.ng, a.n_dst, a.n_ts, r.gb, hi, end, TW_EXPONENTIAL, hb.tau, t_lo, t_hi,
                      d, true);
        nx = p.dst;
        double beta;
        if (nx == prev) beta = hb.inv_p;
        else if (adj_has(a.adj_tab, a.adj_mask, prev, nx)) beta = 1.0;
        else beta = hb.inv_q;
        if (unit_closed_open(d.x2) * hb.beta_max < beta) return true;
    }
    atomicAdd(cap_count ? cap_count : &a.err[2], 1u);
    return false;
}

// One backward walk per thread (full-walk form).
template <int HK, int SK>
__global__ void __launch_bounds__(WALK_THREADS) k_walk_back(const WalkArgs a) {
    const int64_t w = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (w >= a.num_walks) return;
    const uint64_t id = a.base + (uint64_t)w;
    int32_t* out_n = a.nodes + w * a.L;
    int64_t* out_t = a.ts + w * a.L;
    StartState st = walk_start(a, fixed_start<SK>(start_of(a)), w, id, a.L, out_n, out_t, true);
    const HopBias hb = fixed_hop<HK>(a.hop);
    int32_t len = st.len, cur = st.cur, prev = st.prev;
    int64_t tcur = st.t;
    if (len >= 2) {
        for (uint64_t hop = 1; len < a.L; ++hop) {
            const NodeRec r = a.rec[cur];
            if (r.gb == r.ge) break;  // no in-edge at all
            // the first group at or after tcur (first with a timestamp > tcur - 1)
            const uint32_t hi = tcur - 1 >= r.t_last
                                    ? r.ge
                                    : fence_search(a.ng, a.fence, r, tcur - 1, nullptr, 0, 0);
            if (hi == r.gb) break;  // Gamma- is empty
            Pick p;
            int32_t nx;
            if (!back_pick(a, hb, a.seed, r, hi, id, hop, prev, p, nx)) break;
            out_n[len] = nx;
            out_t[len] = p.t;
            ++len;
            prev = cur;
            cur = nx;
            tcur = p.t;
        }
    }
    finish_walk(a, w, len);
}

// ----------------------------------------------------------------- queue
//
// Persistent dispatch with a device work queue. Every lane of a wavefront
// carries one walk at a time; when walks end, the wavefront takes as many
// new walk ids as it has idle lanes with one atomic add on a counter. The
// ids are split in QUEUE_SLICES contiguous slices, each with its own counter,
// and a wavefront starts on slice blockIdx % QUEUE_SLICES (consecutive
// workgroups go to different XCDs), moving to the next slice when one runs
// out, so the counters see little contention. Per walk: its length limit,
// its hop bias (one of up to TW_MAX_BIASES) and its output row.

constexpr int QUEUE_SLICES = 8;
constexpr int QUEUE_REFILL_MIN = 32;  // idle lanes that trigger a refill (hop-only queue)

struct QueueArgs {
    unsigned long long* counters;  // QUEUE_SLICES counters, zero at launch
    const int32_t* max_len;        // per-walk limit, or null (a.L)
    const uint8_t* bias_idx;       // per-walk hop bias, or null (id mod n_bias)
    const int64_t* row;            // per-walk row start, or null (w * a.L)
    int64_t out_slots;             // slots of the outputs: a row must end inside
    int32_t n_bias;
    HopBias bias[TW_MAX_BIASES];
};

__global__ void k_queue_reset(unsigned long long* counters) {
    if (threadIdx.x < QUEUE_SLICES) counters[threadIdx.x] = 0;
}

// REFILL = false is the same per-walk work without the queue: thread i runs
// walk i only (the full-walk form of a batch). REV: backward walks on the
// in-view (each hop as in k_walk_back).
template <bool REFILL, int HK, int SK, bool REV = false>
// The instantiation for mixed hop kinds (HK < 0) carries every picker's
// registers (about 160 VGPRs, 3 waves per SIMD); it is held to 4 waves, which
// spills a few registers and measured 11 % faster on mixed batches.
__global__ void __launch_bounds__(WALK_THREADS)
__attribute__((amdgpu_waves_per_eu(HK < 0 ? 4 : 1)))
k_walk_queue(const WalkArgs a, const QueueArgs q) {
    const int lane = threadIdx.x & 63;
    const int64_t W = a.num_walks;
    const int64_t slice_len = REFILL ? (W + QUEUE_SLICES - 1) / QUEUE_SLICES : W;
    int slice = REFILL ? (int)(blockIdx.x % QUEUE_SLICES) : 0;
    int exhausted = 0;  // slices this wavefront found empty (wave-uniform)
    int64_t w = -1;
    uint64_t id = 0, hop = 0;
    int32_t len = 0, lim = 0, cur = 0, prev = 0;
    int64_t tcur = 0;
    int32_t* out_n = nullptr;
    int64_t* out_t = nullptr;
    HopBias hb{};
    while (true) {
        const uint64_t idle = __ballot(w < 0);
        if (idle && exhausted < QUEUE_SLICES) {
            const int n = __popcll(idle);
            const int leader = __ffsll((unsigned long long)idle) - 1;
            unsigned long long got = 0;
            if (REFILL) {
                if (lane == leader) got = atomicAdd(&q.counters[slice], (unsigned long long)n);
                got = __shfl(got, leader, 64);
            } else {
                // each lane its own walk, once: the wave's first walk id
                got = (unsigned long long)blockIdx.x * WALK_THREADS + (threadIdx.x & ~63);
            }
            const int64_t lo = (int64_t)slice * slice_len;
            const int64_t hi = lo + slice_len < W ? lo + slice_len : W;
            if (w < 0) {
                const int rank = __popcll(idle & ((1ull << lane) - 1));
                const int64_t cand = lo + (int64_t)got + rank;
                if (cand < hi) {
                    w = cand;
                    id = a.base + (uint64_t)w;
                    lim = q.max_len ? q.max_len[w] : a.L;
                    const uint32_t b = q.bias_idx ? q.bias_idx[w] : (uint32_t)(id % (uint64_t)q.n_bias);
                    const int64_t row = q.row ? q.row[w] : w * (int64_t)a.L;
                    if (lim < 1 || lim > a.L || b >= (uint32_t)q.n_bias || row < 0 ||
                        row + lim > q.out_slots) {
                        atomicOr(&a.err[3], 1u);
                        a.len[w] = 0;
                        w = -1;
                    } else {
                        hb = fixed_hop<HK>(q.bias[b]);
                        out_n = a.nodes + row;
                        out_t = a.ts + row;
                        const StartState st = walk_start(a, fixed_start<SK>(start_of(a)), w, id,
                                                         lim, out_n, out_t, REV);
                        len = st.len;
                        cur = st.cur;
                        prev = st.prev;
                        tcur = st.t;
                        hop = 1;
                        if (len < 2 || len >= lim) {
                            a.len[w] = len;
                            w = -1;
                        }
                    }
                }
            }
            if (!REFILL) {
                exhausted = QUEUE_SLICES;  // no more walks for this wavefront
            } else if (lo + (int64_t)got + n >= hi) {
                slice = (slice + 1) % QUEUE_SLICES;
                ++exhausted;
            }
        }
        if (__ballot(w >= 0) == 0) {
            if (exhausted >= QUEUE_SLICES) break;
            continue;
        }
        if (w >= 0) {
            bool done = true;
            const NodeRec r = a.rec[cur];
            // forward: Gamma_t(cur) is empty when t >= the last timestamp;
            // backward: when cur has no in-edge or none before t
            bool live = REV ? r.gb != r.ge : tcur < r.t_last;
            uint32_t g = 0;
            if (live) {
                if (REV) {
                    g = tcur - 1 >= r.t_last
                            ? r.ge
                            : fence_search(a.ng, a.fence, r, tcur - 1, nullptr, 0, 0);
                    live = g != r.gb;
                } else {
                    g = fence_search(a.ng, a.fence, r, tcur, nullptr, 0, 0);
                }
            }
            if (live) {
                Pick p;
                int32_t nx;
                if (REV ? back_pick(a, hb, a.seed, r, g, id, hop, prev, p, nx)
                        : hop_pick(a, hb, a.seed, r, g, id, hop, prev, p, nx)) {
                    out_n[len] = nx;
                    out_t[len] = p.t;
                    ++len;
                    ++hop;
                    prev = cur;
                    cur = nx;
                    tcur = p.t;
                    done = len >= lim;
                }
            }
            if (done) {
                a.len[w] = len;
                w = -1;
            }
        }
    }
}

// Live walks between steps: current node, walk index, current timestamp.
struct Live {
    uint32_t* node;
    uint32_t* walk;
    uint64_t* t;
};

// Hops of the live walks after their start (k_coop_start and
// k_compact_live leave them in `live`, n_live of them): the work queue
// without the start pick, so a lane that takes a walk only loads its state
// and the kernel keeps the registers of the full-walk kernel. ROWS: each
// lane writes its walk's whole output row, four slots per store, padding
// included; otherwise the rows were pre-filled. node2vec and mixed kinds
// keep a walk's current four slots in an LDS ring (as k_walk_full) and are
// held to 4 waves per SIMD: 4.47 ms against 5.00 with the slots in
// registers at 3 waves (2M walks of length 40, 100M-edge graph). The other
// kinds keep the slots in registers at the occupancy their registers give:
// there the ring and more waves measured slower (exponential 5.33 against
// 4.98 ms at 5 waves, linear 2.45 against 2.30 at 8).
template <int HK, bool ROWS>
__global__ void __launch_bounds__(WALK_THREADS)
__attribute__((amdgpu_waves_per_eu(HK == TW_NODE2VEC || HK < 0 ? 4 : 1)))
k_walk_hops(const WalkArgs a, Live live, const int32_t* __restrict__ prev_of,
            const uint32_t* __restrict__ n_live_p, unsigned long long* counters) {
    constexpr bool RING = HK == TW_NODE2VEC || HK < 0;
    const int lane = threadIdx.x & 63;
    const int64_t W = *n_live_p;
    const int64_t slice_len = (W + QUEUE_SLICES - 1) / QUEUE_SLICES;
    int slice = (int)(blockIdx.x % QUEUE_SLICES);
    int exhausted = 0;
    int64_t w = -1;
    uint64_t id = 0, hop = 0;
    int32_t len = 0, cur = 0, prev = 0;
    int64_t tcur = 0;
    __shared__ int32_t ring_n[RING ? 4 : 1][WALK_THREADS];
    __shared__ int64_t ring_t[RING ? 4 : 1][WALK_THREADS];
    const RowRing ring{ring_n, ring_t, (int)threadIdx.x};
    RowChunk c;
    // the walk's output row: kept as pointers (fewer instructions), or
    // recomputed from w where registers are short (RING)
    int32_t* out_n = nullptr;
    int64_t* out_t = nullptr;
    auto row_n = [&]() { return RING ? a.nodes + w * (int64_t)a.L : out_n; };
    auto row_t = [&]() { return RING ? a.ts + w * (int64_t)a.L : out_t; };
    const HopBias hb = fixed_hop<HK>(a.hop);
    while (true) {
        const uint64_t idle = __ballot(w < 0);
        // refill once half the lanes are idle: a refill is an atomic round
        // trip and three dependent loads on the wavefront's critical path,
        // and plain walks end after a few hops
        if (exhausted < QUEUE_SLICES &&
            (idle == ~0ull || (idle && __popcll(idle) >= QUEUE_REFILL_MIN))) {
            const int n = __popcll(idle);
            const int leader = __ffsll((unsigned long long)idle) - 1;
            unsigned long long got = 0;
            if (lane == leader) got = atomicAdd(&counters[slice], (unsigned long long)n);
            got = __shfl(got, leader, 64);
            const int64_t lo = (int64_t)slice * slice_len;
            const int64_t hi = lo + slice_len < W ? lo + slice_len : W;
            if (w < 0) {
                const int rank = __popcll(idle & ((1ull << lane) - 1));
                const int64_t j = lo + (int64_t)got + rank;
                if (j < hi) {
                    w = live.walk[j];
                    cur = (int32_t)live.node[j];
                    tcur = (int64_t)live.t[j];
                    prev = prev_of[w];
                    id = a.base + (uint64_t)w;
                    if (!RING) {
                        out_n = a.nodes + w * (int64_t)a.L;
                        out_t = a.ts + w * (int64_t)a.L;
                    }
                    len = 2;
                    hop = 1;
                    // positions 0 and 1: the start edge's source and target
                    if (ROWS && RING) {
                        ring.put(0, prev, TS_NONE);
                        ring.put(1, cur, tcur);
                    } else if (ROWS) {
                        c = RowChunk();
                        c.push(prev, TS_NONE);
                        c.push(cur, tcur);
                    }
                }
            }
            if (lo + (int64_t)got + n >= hi) {
                slice = (slice + 1) % QUEUE_SLICES;
                ++exhausted;
            }
        }
        if (__ballot(w >= 0) == 0) {
            if (exhausted >= QUEUE_SLICES) break;
            continue;
        }
        if (w >= 0) {
            bool done = true;
            const NodeRec r = a.rec[cur];
            if (tcur < r.t_last) {
                const uint32_t gc = fence_search(a.ng, a.fence, r, tcur, nullptr, 0, 0);
                Pick p;
                int32_t nx;
                if (hop_pick(a, hb, a.seed, r, gc, id, hop, prev, p, nx)) {
                    if (ROWS && RING) {
                        ring.put(len, nx, p.t);
                        if ((len & 3) == 3) ring.flush(row_n(), row_t(), len - 3);
                    } else if (ROWS) {
                        c.push(nx, p.t);
                        if ((len & 3) == 3) c.store(row_n(), row_t(), len - 3);
                    } else {
                        row_n()[len] = nx;
                        row_t()[len] = p.t;
                    }
                    ++len;
                    ++hop;
                    prev = cur;
                    cur = nx;
                    tcur = p.t;
                    done = len >= a.L;
                }
            }
            if (done) {
                if (ROWS && RING) ring.finish(row_n(), row_t(), len, a.L);
                else if (ROWS) finish_row(c, row_n(), row_t(), len, a.L);
                a.len[w] = len;
                w = -1;
            }
        }
    }
}

// ----------------------------------------------------------------- serve
//
// A serving launch: the walks of several requests, each with its own seed,
// id base, length limit, hop and start bias, start nodes and output rows,
// through the same work queue. Walk w of the launch belongs to the request r
// with walk0[r] <= w < walk0[r] + count[r] and is that request's walk
// w - walk0[r], so a request's result does not depend on what else shares
// the launch.

constexpr int SERVE_MAX_REQ = 1024;

struct ServeReqDev {
    int64_t walk0, count;
    uint64_t seed, base;
    int32_t L, start_kind, start_mode, pad;
    double start_tau;
    HopBias hop;
    const int32_t* start_nodes;
    int32_t* nodes;
    int64_t* ts;
    int32_t* len;
    uint32_t* err;  // the request's own words: [0] start node out of range, [1] trial-cap hits
};

// every picker's registers (about 180 VGPRs): held to 3 waves per SIMD
// (a burst of 2,000 mixed requests: 3.53 G hops/s, against 3.37 at the 2
// waves 180 VGPRs allow and 3.34 at 4, which spills 47 registers)
// REV: backward requests on the in-view (each hop as in k_walk_back).
template <bool REV>
__global__ void __launch_bounds__(WALK_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_walk_serve(const WalkArgs a, const ServeReqDev* __restrict__ reqs, int nreq,
             unsigned long long* counters, unsigned long long* hops_out) {
    __shared__ int64_t w0[SERVE_MAX_REQ];
    for (int r = threadIdx.x; r < nreq; r += WALK_THREADS) w0[r] = reqs[r].walk0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t W = a.num_walks;  // walks of the launch
    const int64_t slice_len = (W + QUEUE_SLICES - 1) / QUEUE_SLICES;
    int slice = (int)(blockIdx.x % QUEUE_SLICES);
    int exhausted = 0;
    int64_t w = -1, i = 0;
    uint64_t id = 0, hop = 0, hops = 0;
    int32_t len = 0, lim = 0, cur = 0, prev = 0;
    int64_t tcur = 0;
    int32_t* out_n = nullptr;
    int64_t* out_t = nullptr;
    int32_t* out_len = nullptr;
    uint32_t* rerr = nullptr;
    StartParams sp{};
    uint64_t seed = 0;
    HopBias hb{};
    while (true) {
        const uint64_t idle = __ballot(w < 0);
        if (idle && exhausted < QUEUE_SLICES) {
            const int n = __popcll(idle);
            const int leader = __ffsll((unsigned long long)idle) - 1;
            unsigned long long got = 0;
            if (lane == leader) got = atomicAdd(&counters[slice], (unsigned long long)n);
            got = __shfl(got, leader, 64);
            const int64_t lo = (int64_t)slice * slice_len;
            const int64_t hi = lo + slice_len < W ? lo + slice_len : W;
            if (w < 0) {
                const int rank = __popcll(idle & ((1ull << lane) - 1));
                const int64_t cand = lo + (int64_t)got + rank;
                if (cand < hi) {
                    w = cand;
                    int rl = 0, rh = nreq;  // last request with walk0 <= w
                    while (rh - rl > 1) {
                        const int mid = (rl + rh) >> 1;
                        if (w0[mid] <= w) rl = mid; else rh = mid;
                    }
                    const ServeReqDev& R = reqs[rl];
                    i = w - R.walk0;
                    seed = R.seed;
                    sp = StartParams{R.seed, R.start_kind, R.start_mode, R.start_tau,
                                     R.start_nodes};
                    hb = R.hop;
                    lim = R.L;
                    id = R.base + (uint64_t)i;
                    out_n = R.nodes + i * (int64_t)R.L;
                    out_t = R.ts + i * (int64_t)R.L;
                    out_len = R.len + i;
                    rerr = R.err;
                    const StartState st = walk_start(a, sp, i, id, lim, out_n, out_t, REV, rerr);
                    len = st.len;
                    cur = st.cur;
                    prev = st.prev;
                    tcur = st.t;
                    hop = 1;
                    if (len < 2 || len >= lim) {
                        *out_len = len;
                        hops += len > 1 ? (uint64_t)(len - 1) : 0;
                        w = -1;
                    }
                }
            }
            if (lo + (int64_t)got + n >= hi) {
                slice = (slice + 1) % QUEUE_SLICES;
                ++exhausted;
            }
        }
        if (__ballot(w >= 0) == 0) {
            if (exhausted >= QUEUE_SLICES) break;
            continue;
        }
        if (w >= 0) {
            bool done = true;
            const NodeRec r = a.rec[cur];
            // forward: Gamma_t(cur) is empty when t >= the last timestamp;
            // backward: when cur has no in-edge or none before t
            bool live = REV ? r.gb != r.ge : tcur < r.t_last;
            uint32_t g = 0;
            if (live) {
                if (REV) {
                    g = tcur - 1 >= r.t_last
                            ? r.ge
                            : fence_search(a.ng, a.fence, r, tcur - 1, nullptr, 0, 0);
                    live = g != r.gb;
                } else {
                    g = fence_search(a.ng, a.fence, r, tcur, nullptr, 0, 0);
                }
            }
            if (live) {
                Pick p;
                int32_t nx;
                if (REV ? back_pick(a, hb, seed, r, g, id, hop, prev, p, nx, rerr + 1)
                        : hop_pick(a, hb, seed, r, g, id, hop, prev, p, nx, rerr + 1)) {
                    out_n[len] = nx;
                    out_t[len] = p.t;
                    ++len;
                    ++hop;
                    prev = cur;
                    cur = nx;
                    tcur = p.t;
                    done = len >= lim;
                }
            }
            if (done) {
                *out_len = len;
                hops += (uint64_t)(len - 1);
                w = -1;
            }
        }
    }
    // hops of the launch: one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1) hops += __shfl_down(hops, off, 64);
    if (lane == 0 && hops) atomicAdd(hops_out, (unsigned long long)hops);
}

// ------------------------------------------------------------------ coop
//
// Cooperative dispatch (Sec. "Hierarchical Cooperative Scheduling"): each
// step sorts the live walks by current node, and k_hop_coop advances them
// in that order. A wavefront whose 64 walks share one node, or a workgroup
// whose 256 walks do, reads the node record once and stages the top levels
// of the node's fence in LDS (the panel); mixed chunks run one walk per
// thread. Walks at a node with W walks thus get the workgroup tier for each
// full 256-walk chunk, the wavefront tier for each remaining full 64-walk
// chunk, and the thread tier otherwise; a node's walks beyond one
// workgroup are split over several workgroups.

// Live walks of one step, structure of arrays in one order: current node,
// walk index, time of arrival.
// ROWS: the rows are not pre-filled; a walk that ends at its start writes
// its whole padded row here, and the hop kernel writes the rows of the others.
template <int SK, bool ROWS = false>
__global__ void __launch_bounds__(WALK_THREADS) k_coop_start(const WalkArgs a, Live nx,
                                                              int32_t* __restrict__ prev,
                                                              uint32_t* __restrict__ alive) {
    const int64_t w = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (w >= a.num_walks) return;
    const uint64_t id = a.base + (uint64_t)w;
    int32_t* out_n = a.nodes + w * a.L;
    int64_t* out_t = a.ts + w * a.L;
    StartState st = walk_start(a, fixed_start<SK>(start_of(a)), w, id, a.L,
                               ROWS ? nullptr : out_n, out_t);
    bool live = st.len >= 2 && st.len < a.L;
    if (live) {
        nx.node[w] = (uint32_t)st.cur;
        nx.walk[w] = (uint32_t)w;
        nx.t[w] = (uint64_t)st.t;
        prev[w] = st.prev;
    } else {
        if (ROWS) {
            RowChunk c;
            if (st.len >= 1) c.push(st.first, TS_NONE);
            if (st.len >= 2) c.push(st.cur, st.t);
            finish_row(c, out_n, out_t, st.len, a.L);
        }
        finish_walk(a, w, st.len);
    }
    alive[w] = live ? 1u : 0u;
}

// in-order compaction of the walks flagged alive
__global__ void k_compact_live(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                               int64_t n, Live in, Live out) {
    int64_t i = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (i < n && flags[i]) {
        uint32_t o = pos[i];
        out.node[o] = in.node[i];
        out.walk[o] = in.walk[i];
        out.t[o] = in.t[i];
    }
}

// One hop for the live walks of `cur` (*n_live of the n_ub entries; the
// rest are idle), in node order when the step sorted them. Results go to
// `nx` at the same positions, with alive[i] set for walks that continue (0
// for idle entries). A wavefront engages the wavefront tier for the node of
// its first lane when at least wave_min of its lanes are at that node: the
// record is read once and the top levels of the node's fence are staged in
// LDS for those lanes; a workgroup whose four wavefronts engage it for one
// node stages a panel four times larger.
template <int HK>
__global__ void __launch_bounds__(WALK_THREADS)
k_hop_coop(const WalkArgs a, Live cur, Live nxt, int32_t* __restrict__ prev_of,
           const uint32_t* __restrict__ n_live, int64_t n_ub, uint64_t hop, uint32_t panel_cap,
           int wave_min, uint32_t* __restrict__ alive) {
    extern __shared__ __align__(16) uint32_t panel[];
    __shared__ int32_t wave_node[WALK_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    const bool valid = i < (int64_t)*n_live;
    const int32_t v = valid ? (int32_t)cur.node[i] : -1;
    const int32_t v0 = __shfl(v, 0, 64);
    const int at_v0 = __popcll(__ballot(valid && v == v0));
    const bool wave_tier = v0 >= 0 && at_v0 >= wave_min;
    if (lane == 0) wave_node[wave] = wave_tier ? v0 : -1;
    __syncthreads();
    bool wg_tier = wave_node[0] >= 0;
#pragma unroll
    for (int k = 1; k < WALK_THREADS / 64; ++k) wg_tier &= wave_node[k] == wave_node[0];

    // stage the top levels of the node's fence: the whole panel for a
    // workgroup of one node, a quarter of it per wavefront otherwise.
    // Levels are stored bottom-up, so levels K down to some m are one
    // contiguous range.
    const uint32_t* my_panel = nullptr;
    uint64_t my_base = 0;
    uint32_t my_cap = 0;
    int32_t panel_node = -1;
    if (wg_tier || wave_tier) {
        panel_node = wg_tier ? wave_node[0] : v0;
        const NodeRec r = a.rec[panel_node];
        const uint32_t slice = wg_tier ? panel_cap : panel_cap / (WALK_THREADS / 64);
        uint32_t* dst = wg_tier ? panel : panel + wave * slice;
        const int K = (int)rec_levels(r.lv);
        if (K > 0) {
            const uint64_t cap = seg_groups(rec_code(r.lv));
            const uint64_t top = (uint64_t)r.fence_off + fence_level_off(cap, K) +
                                 fence_level_len(cap, K);  // end of level K
            uint64_t from = top;
            for (int k = K; k >= 0; --k) {
                const uint32_t len = fence_level_len(cap, k);
                if (top - (from - len) > slice) break;
                from -= len;
            }
            my_base = from;
            my_cap = (uint32_t)(top - from);
        }
        const int first = wg_tier ? threadIdx.x : lane;
        const int stride = wg_tier ? WALK_THREADS : 64;
        for (uint32_t j = first; j < my_cap; j += stride) dst[j] = a.fence[my_base + j];
        my_panel = dst;
    }
    __syncthreads();
    if (!valid) {
        if (i < n_ub) alive[i] = 0u;
        return;
    }
    if (v != panel_node) {
        my_panel = nullptr;
        my_base = 0;
        my_cap = 0;
    }

    const uint32_t w = cur.walk[i];
    const uint64_t id = a.base + (uint64_t)w;
    const NodeRec r = a.rec[v];
    const int64_t tcur = (int64_t)cur.t[i];
    const int32_t len = (int32_t)hop + 1;  // nodes written before this hop
    bool live = false;
    if (tcur < r.t_last) {
        const uint32_t gc = fence_search(a.ng, a.fence, r, tcur, my_panel, my_base, my_cap);
        Pick p;
        int32_t nx;
        const int32_t prev = a.hop.kind == TW_NODE2VEC ? prev_of[w] : 0;
        if (hop_pick(a, fixed_hop<HK>(a.hop), a.seed, r, gc, id, hop, prev, p, nx)) {
            a.nodes[(int64_t)w * a.L + len] = nx;
            a.ts[(int64_t)w * a.L + len] = p.t;
            if (len + 1 < a.L) {
                nxt.node[i] = (uint32_t)nx;
                nxt.walk[i] = w;
                nxt.t[i] = (uint64_t)p.t;
                if (a.hop.kind == TW_NODE2VEC) prev_of[w] = v;
                live = true;
            } else {
                a.len[w] = len + 1;
            }
        } else {
            finish_walk(a, w, len);
        }
    } else {
        finish_walk(a, w, len);
    }
    alive[i] = live ? 1u : 0u;
}

// entries [*n_live, n_ub) of a live list get a node id above every real
// one, so a sort by node leaves them last
__global__ void k_live_tail(Live live, const uint32_t* __restrict__ n_live, int64_t n_ub,
                            uint32_t sentinel) {
    const int64_t i = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (i < n_ub && i >= (int64_t)*n_live) live.node[i] = sentinel;
}

bool valid_tau(double t) { return std::isfinite(t); }

template <int V>
using Kind = std::integral_constant<int, V>;

// f(Kind<HK>, Kind<SK>) for the run-time hop kind hk (-1: left dynamic, for
// batches that mix hop biases) and start kind sk
template <typename F>
void with_kinds(int hk, int sk, F&& f) {
    auto by_start = [&](auto h) {
        switch (sk) {
            case TW_LINEAR: f(h, Kind<TW_LINEAR>{}); break;
            case TW_EXPONENTIAL: f(h, Kind<TW_EXPONENTIAL>{}); break;
            default: f(h, Kind<TW_UNIFORM>{}); break;
        }
    };
    switch (hk) {
        case TW_UNIFORM: by_start(Kind<TW_UNIFORM>{}); break;
        case TW_LINEAR: by_start(Kind<TW_LINEAR>{}); break;
        case TW_EXPONENTIAL: by_start(Kind<TW_EXPONENTIAL>{}); break;
        case TW_NODE2VEC: by_start(Kind<TW_NODE2VEC>{}); break;
        case TW_WEIGHT: by_start(Kind<TW_WEIGHT>{}); break;
        default: by_start(Kind<-1>{}); break;
    }
}

// Host loop of the cooperative dispatch: per step, regroup the live walks
// by node (a stable sort, or none), one hop, in-order compaction. The live
// count is read back every coop_sync steps; in between, launches cover the
// last count read (an upper bound) and their threads past the device count
// idle.
tw_status coop_walks(tw_graph* g, const WalkArgs& a, Error& err) {
    hipStream_t s = g->stream;
    const int64_t W = a.num_walks;
    DevBuf* bufs32[] = {&g->c_node0, &g->c_walk0, &g->c_node1, &g->c_walk1, &g->c_node2,
                        &g->c_walk2, &g->c_flags, &g->c_pos, &g->c_prev};
    for (DevBuf* b : bufs32) TW_HIP(ensure(*b, sizeof(uint32_t) * W, g->stream));
    TW_HIP(ensure(g->c_t0, sizeof(uint64_t) * W, g->stream));
    TW_HIP(ensure(g->c_t1, sizeof(uint64_t) * W, g->stream));
    TW_HIP(ensure(g->c_t2, sizeof(uint64_t) * W, g->stream));
    // live (compacted) -> sorted (by node) -> next (after the hop) -> live
    Live live{g->c_node0.as<uint32_t>(), g->c_walk0.as<uint32_t>(), g->c_t0.as<uint64_t>()};
    Live sorted{g->c_node1.as<uint32_t>(), g->c_walk1.as<uint32_t>(), g->c_t1.as<uint64_t>()};
    Live next{g->c_node2.as<uint32_t>(), g->c_walk2.as<uint32_t>(), g->c_t2.as<uint64_t>()};
    int32_t* prev = g->c_prev.as<int32_t>();
    uint32_t* flags = g->c_flags.as<uint32_t>();
    uint32_t* pos = g->c_pos.as<uint32_t>();
    uint32_t* n_live_d = g->scal.as<uint32_t>() + SLOT_U32_N_LIVE;
    // node ids and the sentinel V sort in bits_for(V) bits
    const int vbits = bits_for((uint64_t)g->V);
    const uint32_t panel_cap = g->coop_panel;
    const int sync_every = std::max(g->coop_sync, 1);
    const dim3 wgrid((unsigned)ceil_div(W, WALK_THREADS));

    with_kinds(-1, a.start_kind, [&](auto, auto sk) {
        hipLaunchKernelGGL((k_coop_start<decltype(sk)::value>), wgrid, dim3(WALK_THREADS), 0, s, a,
                           next, prev, flags);
    });
    TW_HIP(scan_exclusive_u32(flags, pos, W, n_live_d, g->ws, s));
    hipLaunchKernelGGL(k_compact_live, wgrid, dim3(WALK_THREADS), 0, s, flags, pos, W, next, live);
    TW_HIP(hipGetLastError());
    int64_t n_ub = W;
    for (uint64_t hop = 1; hop + 1 < (uint64_t)a.L; ++hop) {
        if ((hop - 1) % (uint64_t)sync_every == 0) {
            if (pull_scalars(g, false, err) != TW_OK) return err.code;
            n_ub = host_u32(g, SLOT_U32_N_LIVE);
            if (n_ub == 0) break;
        }
        const dim3 grid((unsigned)ceil_div(n_ub, WALK_THREADS));
        Live in = live;
        if (g->coop_regroup == 0) {
            if (sync_every > 1)
                hipLaunchKernelGGL(k_live_tail, grid, dim3(WALK_THREADS), 0, s, live, n_live_d,
                                   n_ub, (uint32_t)g->V);
            TW_HIP(radix_sort_u32_kv(live.node, live.walk, live.t, sorted.node, sorted.walk,
                                     sorted.t, n_ub, 0, vbits, g->ws, s));
            in = sorted;
        }
        with_kinds(a.hop.kind, TW_UNIFORM, [&](auto hk, auto) {
            hipLaunchKernelGGL((k_hop_coop<decltype(hk)::value>), grid, dim3(WALK_THREADS),
                               sizeof(uint32_t) * panel_cap, s, a, in, next, prev, n_live_d,
                               n_ub, hop, panel_cap, g->coop_wave_min, flags);
        });
        TW_HIP(scan_exclusive_u32(flags, pos, n_ub, n_live_d, g->ws, s));
        hipLaunchKernelGGL(k_compact_live, grid, dim3(WALK_THREADS), 0, s, flags, pos, n_ub, next,
                           live);
        TW_HIP(hipGetLastError());
    }
    return TW_OK;
}

}  // namespace

namespace {

tw_status check_bias(const tw_bias& b, bool hop, Error& err) {
    if (b.kind < TW_UNIFORM || b.kind > (hop ? TW_WEIGHT : TW_EXPONENTIAL) || !valid_tau(b.tau)) {
        err = Error{TW_EINVAL, "sample_walks: bad bias kind or tau (start bias cannot be node2vec)"};
        return err.code;
    }
    if (b.kind == TW_NODE2VEC &&
        !(b.p > 0.0 && b.q > 0.0 && std::isfinite(b.p) && std::isfinite(b.q))) {
        err = Error{TW_EINVAL, "sample_walks: node2vec needs p > 0 and q > 0"};
        return err.code;
    }
    return TW_OK;
}

tw_status check_start(int mode, const int32_t* starts, int64_t num_walks, Error& err) {
    if (mode != TW_START_EDGE && mode != TW_START_NODE) {
        err = Error{TW_EINVAL, "sample_walks: bad start mode"};
        return err.code;
    }
    if (mode == TW_START_NODE && !starts && num_walks > 0) {
        err = Error{TW_EINVAL, "sample_walks: start mode NODE needs d_start_nodes"};
        return err.code;
    }
    return TW_OK;
}

// The index part of the walk arguments and the common parameters.
// Walk arguments over the graph's current views. node2vec: the adjacency
// is needed; weight_tau (NaN: none) the cumulative weights at that scale.
tw_status fill_args(tw_graph* g, int64_t num_walks, int32_t L, const tw_bias& sb, int start_mode,
                    const int32_t* starts, uint64_t seed, uint64_t base, bool node2vec,
                    double weight_tau, int32_t* nodes, int64_t* ts, int32_t* len, WalkArgs& a,
                    Error& err) {
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    if (node2vec && g->m > 0 && build_adjacency(g, err) != TW_OK) return err.code;
    if (!std::isnan(weight_tau) && build_weights(g, weight_tau, err) != TW_OK) return err.code;
    a = WalkArgs{};
    a.e_src = g->e_src.as<int32_t>();
    a.e_dst = g->e_dst.as<int32_t>();
    a.e_ts = g->e_ts.as<int64_t>();
    a.wsum = g->scal.as<int64_t>() + SLOT_I64_SUMMARY;
    a.wgg = g->scal.as<int64_t>() + SLOT_I64_GG;
    a.gg_off = g->gg_off.as<uint32_t>();
    a.win = g->scal.as<int64_t>() + SLOT_I64_WIN;
    a.n_dst = g->n_dst.as<int32_t>();
    a.n_ts = g->n_ts.as<int64_t>();
    a.ng = g->ng.as<GroupRec>();

    a.rec = g->rec.as<NodeRec>();
    a.fence = g->fence.as<uint32_t>();
    a.adj_tab = g->adj_tab.as<AdjSlot>();
    a.adj_mask = g->adj_mask;
    a.cw = g->cw.as<double>();
    a.V = g->V;
    a.num_walks = num_walks;
    a.L = L;
    a.start_kind = sb.kind;
    a.start_mode = start_mode;
    a.start_tau = sb.tau;
    a.start_nodes = starts;
    a.seed = seed;
    a.base = base;
    a.nodes = nodes;
    a.ts = ts;
    a.len = len;
    a.err = g->err.as<uint32_t>();
    return TW_OK;
}

void launch_fill(tw_graph* g, int32_t* nodes, int64_t* ts, int64_t slots) {
    hipLaunchKernelGGL(k_fill_outputs,
                       dim3((unsigned)std::max<int64_t>(
                           std::min<int64_t>(ceil_div(slots, 4 * WALK_THREADS), 8192), 1)),
                       dim3(WALK_THREADS), 0, g->stream, nodes, ts, slots);
}

// compute units and the workgroups of k_walk_queue one of them holds at
// once, queried once per graph (host-side queries only, so a walk launch can
// be captured in a graph afterwards)
tw_status queue_shape(tw_graph* g, Error& err) {
    if (g->cu_count) return TW_OK;
    int n = 0, nb = 0;
    TW_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, g->device));
    TW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_queue<true, -1, -1>,
                                                         WALK_THREADS, 0));
    g->cu_count = std::max(n, 1);
    g->queue_bpc_max = std::max(nb, 1);
    return TW_OK;
}

// resident workgroups per compute unit of one queue kernel instantiation
template <typename K>
int resident_bpc(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, WALK_THREADS, 0) != hipSuccess)
        nb = 1;
    return std::max(nb, 1);
}

// Calls f with the direction as a compile-time constant. Backward walks
// never take the weight-based picker (refused before any launch), so its
// backward instantiations are not built.
template <typename F>
void with_direction(bool rev, int hk, F&& f) {
    if (!rev) f(std::false_type{});
    else if (hk != TW_WEIGHT) f(std::true_type{});
}

// rev: backward walks (a is the in-view's)
tw_status queue_walks(tw_graph* g, const WalkArgs& a, const QueueArgs& q0, int bpc, Error& err,
                      bool rev = false) {
    if (queue_shape(g, err) != TW_OK) return err.code;
    TW_HIP(ensure(g->wq, sizeof(unsigned long long) * QUEUE_SLICES, g->stream));
    QueueArgs q = q0;
    q.counters = g->wq.as<unsigned long long>();
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, g->stream, q.counters);
    const int hk = q.n_bias == 1 ? q.bias[0].kind : -1;
    with_kinds(hk, a.start_kind, [&](auto h, auto st) {
        with_direction(rev, decltype(h)::value, [&](auto r) {
            auto kernel =
                k_walk_queue<true, decltype(h)::value, decltype(st)::value, decltype(r)::value>;
            static const int maxb = resident_bpc(kernel);  // per instantiation
            const int b = (bpc <= 0 || bpc > maxb) ? maxb : bpc;
            const int64_t blocks =
                std::min<int64_t>(ceil_div(a.num_walks, WALK_THREADS), (int64_t)g->cu_count * b);
            hipLaunchKernelGGL(kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)),
                               dim3(WALK_THREADS), 0, g->stream, a, q);
        });
    });
    TW_HIP(hipGetLastError());
    return TW_OK;
}

// the batch with one thread per walk and no queue
tw_status batch_full_walk(tw_graph* g, const WalkArgs& a, const QueueArgs& q, Error& err,
                          bool rev = false) {
    const int hk = q.n_bias == 1 ? q.bias[0].kind : -1;
    with_kinds(hk, a.start_kind, [&](auto h, auto st) {
        with_direction(rev, decltype(h)::value, [&](auto r) {
            hipLaunchKernelGGL((k_walk_queue<false, decltype(h)::value, decltype(st)::value,
                                             decltype(r)::value>),
                               dim3((unsigned)ceil_div(a.num_walks, WALK_THREADS)),
                               dim3(WALK_THREADS), 0, g->stream, a, q);
        });
    });
    TW_HIP(hipGetLastError());
    return TW_OK;
}

// Whether the full-walk and queue kernels write whole output rows themselves (four slots
// per 16-byte store, padding included): rows of a multiple of 4 slots and
// 16-byte aligned outputs.
bool own_rows(const WalkArgs& a) {
    return a.L % 4 == 0 && (reinterpret_cast<uintptr_t>(a.nodes) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(a.ts) & 15) == 0;
}

// Per-call lists of the queue dispatch of plain walks: the walks alive after
// their start (current node, walk, time) before and after compaction, each
// walk's previous node, the alive flags and their scan, the live count, the
// scan's partial sums (scan_parts_u32(walks) words) and the queue counters.
struct HopLists {
    Live live, next;
    int32_t* prev;
    uint32_t* flags;
    uint32_t* pos;
    uint32_t* n_live;
    uint32_t* scan_part;
    unsigned long long* counters;
};

// The queue dispatch of plain walks: every start in one pass (as the
// cooperative dispatch starts), the live walks compacted, then one
// persistent launch of k_walk_hops over them. Allocates nothing.
tw_status queue_hops_in(tw_graph* g, const WalkArgs& a, int bpc, const HopLists& h,
                        Error& err) {
    hipStream_t s = g->stream;
    const int64_t W = a.num_walks;
    if (queue_shape(g, err) != TW_OK) return err.code;
    const dim3 wgrid((unsigned)ceil_div(W, WALK_THREADS));
    const bool rows = own_rows(a);
    with_kinds(-1, a.start_kind, [&](auto, auto sk) {
        if (rows)
            hipLaunchKernelGGL((k_coop_start<decltype(sk)::value, true>), wgrid,
                               dim3(WALK_THREADS), 0, s, a, h.next, h.prev, h.flags);
        else
            hipLaunchKernelGGL((k_coop_start<decltype(sk)::value, false>), wgrid,
                               dim3(WALK_THREADS), 0, s, a, h.next, h.prev, h.flags);
    });
    TW_HIP(scan_exclusive_u32_into(h.flags, h.pos, W, h.n_live, h.scan_part, s));
    hipLaunchKernelGGL(k_compact_live, wgrid, dim3(WALK_THREADS), 0, s, h.flags, h.pos, W, h.next,
                       h.live);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, h.counters);
    with_kinds(a.hop.kind, TW_UNIFORM, [&](auto hk, auto) {
        auto launch = [&](auto kernel) {
            static const int maxb = resident_bpc(kernel);  // per instantiation
            const int b = (bpc <= 0 || bpc > maxb) ? maxb : bpc;
            const int64_t blocks =
                std::min<int64_t>(ceil_div(W, WALK_THREADS), (int64_t)g->cu_count * b);
            hipLaunchKernelGGL(kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)),
                               dim3(WALK_THREADS), 0, s, a, h.live, h.prev, h.n_live, h.counters);
        };
        if (rows)
            launch(k_walk_hops<decltype(hk)::value, true>);
        else
            launch(k_walk_hops<decltype(hk)::value, false>);
    });
    TW_HIP(hipGetLastError());
    return TW_OK;
}

// The same with the lists in the graph's buffers (grown as needed).
tw_status queue_hops(tw_graph* g, const WalkArgs& a, int bpc, Error& err) {
    const int64_t W = a.num_walks;
    DevBuf* bufs32[] = {&g->c_node0, &g->c_walk0, &g->c_node2, &g->c_walk2, &g->c_flags,
                        &g->c_pos, &g->c_prev};
    for (DevBuf* b : bufs32) TW_HIP(ensure(*b, sizeof(uint32_t) * W, g->stream));
    TW_HIP(ensure(g->c_t0, sizeof(uint64_t) * W, g->stream));
    TW_HIP(ensure(g->c_t2, sizeof(uint64_t) * W, g->stream));
    TW_HIP(ensure(g->wq, sizeof(unsigned long long) * QUEUE_SLICES, g->stream));
    TW_HIP(ensure(g->ws.scan_part, sizeof(uint32_t) * scan_parts_u32(W), g->stream));
    HopLists h;
    h.live = Live{g->c_node0.as<uint32_t>(), g->c_walk0.as<uint32_t>(), g->c_t0.as<uint64_t>()};
    h.next = Live{g->c_node2.as<uint32_t>(), g->c_walk2.as<uint32_t>(), g->c_t2.as<uint64_t>()};
    h.prev = g->c_prev.as<int32_t>();
    h.flags = g->c_flags.as<uint32_t>();
    h.pos = g->c_pos.as<uint32_t>();
    h.n_live = g->scal.as<uint32_t>() + SLOT_U32_N_LIVE;
    h.scan_part = g->ws.scan_part.as<uint32_t>();
    h.counters = g->wq.as<unsigned long long>();
    return queue_hops_in(g, a, bpc, h, err);
}


// run the walks of `a` under a dispatch; the output rows are padded first
// unless the walk kernel writes them whole
tw_status run_dispatch(tw_graph* g, const WalkArgs& a, int dispatch, int bpc, Error& err) {
    if ((dispatch != TW_DISPATCH_FULL_WALK && dispatch != TW_DISPATCH_QUEUE) || !own_rows(a))
        launch_fill(g, a.nodes, a.ts, a.num_walks * (int64_t)a.L);
    if (dispatch == TW_DISPATCH_COOP) return coop_walks(g, a, err);
    if (dispatch == TW_DISPATCH_QUEUE) return queue_hops(g, a, bpc, err);
    const bool rows = own_rows(a);
    with_kinds(a.hop.kind, a.start_kind, [&](auto h, auto st) {
        const dim3 grid((unsigned)ceil_div(a.num_walks, WALK_THREADS));
        if (rows)
            hipLaunchKernelGGL((k_walk_full<decltype(h)::value, decltype(st)::value, true>), grid,
                               dim3(WALK_THREADS), 0, g->stream, a);
        else
            hipLaunchKernelGGL((k_walk_full<decltype(h)::value, decltype(st)::value, false>),
                               grid, dim3(WALK_THREADS), 0, g->stream, a);
    });
    TW_HIP(hipGetLastError());
    return TW_OK;
}

tw_status prepare_plain(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                        int32_t* len, WalkArgs& a, Error& err) {
    if (!p || p->num_walks < 0 || p->max_len < 1) {
        err = Error{TW_EINVAL, "sample_walks: need num_walks >= 0 and max_len >= 1"};
        return err.code;
    }
    if (check_bias(p->hop_bias, true, err) != TW_OK) return err.code;
    if (check_bias(p->start_bias, false, err) != TW_OK) return err.code;
    if (check_start(p->start_mode, p->d_start_nodes, p->num_walks, err) != TW_OK) return err.code;
    if (p->dispatch < TW_DISPATCH_AUTO || p->dispatch > TW_DISPATCH_QUEUE) {
        err = Error{TW_EINVAL, "sample_walks: bad dispatch"};
        return err.code;
    }
    if (p->num_walks > 0 && (!nodes || !ts || !len)) {
        err = Error{TW_EINVAL, "sample_walks: null output"};
        return err.code;
    }
    if (fill_args(g, p->num_walks, p->max_len, p->start_bias, p->start_mode, p->d_start_nodes,
                  p->seed, p->walk_id_base, p->hop_bias.kind == TW_NODE2VEC,
                  p->hop_bias.kind == TW_WEIGHT ? p->hop_bias.tau : NAN, nodes, ts, len, a,
                  err) != TW_OK)
        return err.code;
    a.hop = make_hop_bias(p->hop_bias);
    return TW_OK;
}

}  // namespace

// Backward walks on the in-view: the full-walk kernel k_walk_back (AUTO,
// FULL_WALK) or the work queue (QUEUE).
tw_status sample_backward(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                          int32_t* len, Error& err) {
    if (p->hop_bias.kind == TW_WEIGHT) {
        err = Error{TW_EINVAL, "sample_walks: the weight-based picker walks forward only"};
        return err.code;
    }
    if (p->dispatch == TW_DISPATCH_COOP) {
        err = Error{TW_EINVAL,
                    "sample_walks: backward walks run on the full-walk or the queue dispatch"};
        return err.code;
    }
    tw_graph* b = nullptr;
    if (backward_view(g, &b, err) != TW_OK) return err.code;
    WalkArgs a;
    if (prepare_plain(b, p, nodes, ts, len, a, err) != TW_OK) return err.code;
    if (p->num_walks == 0) return TW_OK;
    launch_fill(b, nodes, ts, p->num_walks * (int64_t)p->max_len);
    if (p->dispatch == TW_DISPATCH_QUEUE) {
        // the work queue with the one hop bias
        QueueArgs q{};
        q.n_bias = 1;
        q.bias[0] = a.hop;
        q.out_slots = p->num_walks * (int64_t)p->max_len;
        return queue_walks(b, a, q, g->auto_bpc, err, true);
    }
    const dim3 grid((unsigned)ceil_div(p->num_walks, WALK_THREADS));
    with_kinds(a.hop.kind, a.start_kind, [&](auto h, auto sk) {
        hipLaunchKernelGGL((k_walk_back<decltype(h)::value, decltype(sk)::value>), grid,
                           dim3(WALK_THREADS), 0, b->stream, a);
    });
    TW_HIP(hipGetLastError());
    return TW_OK;
}

tw_status sample_walks(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                       int32_t* len, Error& err) {
    if (p && p->direction == TW_BACKWARD) return sample_backward(g, p, nodes, ts, len, err);
    if (p && p->direction != TW_FORWARD) {
        err = Error{TW_EINVAL, "sample_walks: bad direction"};
        return err.code;
    }
    WalkArgs a;
    if (prepare_plain(g, p, nodes, ts, len, a, err) != TW_OK) return err.code;
    if (p->num_walks == 0) return TW_OK;
    int dispatch = p->dispatch;
    // AUTO: the autotuned choice, else the full-walk kernel
    if (dispatch == TW_DISPATCH_AUTO)
        dispatch = g->auto_dispatch ? g->auto_dispatch : TW_DISPATCH_FULL_WALK;
    return run_dispatch(g, a, dispatch, g->auto_bpc, err);
}

tw_status sample_walks_batch(tw_graph* g, const tw_batch_params* p, int32_t* nodes, int64_t* ts,
                             int32_t* len, Error& err) {
    if (!p || p->num_walks < 0 || p->max_len < 1 || p->num_biases < 1 ||
        p->num_biases > TW_MAX_BIASES) {
        err = Error{TW_EINVAL,
                    "sample_walks_batch: need num_walks >= 0, max_len >= 1, 1..8 hop biases"};
        return err.code;
    }
    bool n2v = false;
    double wtau = NAN;  // the weight-based biases' time scale: one per launch
    for (int b = 0; b < p->num_biases; ++b) {
        const tw_bias& hb = p->hop_biases[b];
        if (check_bias(hb, true, err) != TW_OK) return err.code;
        n2v |= hb.kind == TW_NODE2VEC;
        if (hb.kind == TW_WEIGHT) {
            const double sc = hb.tau > 0.0 ? hb.tau : 1.0;
            if (!std::isnan(wtau) && wtau != sc) {
                err = Error{TW_EINVAL,
                            "sample_walks_batch: weight-based biases of one launch need one tau"};
                return err.code;
            }
            wtau = sc;
        }
    }
    if (check_bias(p->start_bias, false, err) != TW_OK) return err.code;
    if (check_start(p->start_mode, p->d_start_nodes, p->num_walks, err) != TW_OK) return err.code;
    if (p->dispatch != TW_DISPATCH_AUTO && p->dispatch != TW_DISPATCH_QUEUE &&
        p->dispatch != TW_DISPATCH_FULL_WALK) {
        err = Error{TW_EINVAL, "sample_walks_batch: dispatch must be AUTO, QUEUE or FULL_WALK"};
        return err.code;
    }
    if (p->direction != TW_FORWARD && p->direction != TW_BACKWARD) {
        err = Error{TW_EINVAL, "sample_walks_batch: bad direction"};
        return err.code;
    }
    const bool rev = p->direction == TW_BACKWARD;
    if (rev && !std::isnan(wtau)) {
        err = Error{TW_EINVAL, "sample_walks_batch: the weight-based picker walks forward only"};
        return err.code;
    }
    if (p->num_walks == 0) return TW_OK;
    if (!nodes || !ts || !len) {
        err = Error{TW_EINVAL, "sample_walks_batch: null output"};
        return err.code;
    }
    // backward walks run on the in-view, on the same stream
    tw_graph* vg = g;
    if (rev && backward_view(g, &vg, err) != TW_OK) return err.code;
    WalkArgs a;
    if (fill_args(vg, p->num_walks, p->max_len, p->start_bias, p->start_mode, p->d_start_nodes,
                  p->seed, p->walk_id_base, n2v, wtau, nodes, ts, len, a, err) != TW_OK)
        return err.code;
    a.hop = make_hop_bias(p->hop_biases[0]);
    QueueArgs q{};
    q.max_len = p->d_max_len;
    q.bias_idx = p->d_bias;
    q.row = p->d_row;
    q.n_bias = p->num_biases;
    for (int b = 0; b < p->num_biases; ++b) q.bias[b] = make_hop_bias(p->hop_biases[b]);
    if (p->d_row && p->out_slots < 1) {
        err = Error{TW_EINVAL, "sample_walks_batch: ragged rows need out_slots"};
        return err.code;
    }
    const int64_t slots = p->out_slots > 0 ? p->out_slots : p->num_walks * (int64_t)p->max_len;
    q.out_slots = slots;
    launch_fill(vg, nodes, ts, slots);
    if (p->dispatch == TW_DISPATCH_FULL_WALK) return batch_full_walk(vg, a, q, err, rev);
    return queue_walks(vg, a, q, g->auto_bpc, err, rev);
}

// ---------------------------------------------------------------------------
// Allocation-free walks: the queue dispatch of plain walks (queue_hops_in)
// with its per-call lists in one file-scope device array, for callers that
// cannot allocate device memory.

namespace {

constexpr int64_t NA_MAX = TW_NOALLOC_MAX_WALKS;
constexpr int64_t na_round(int64_t b) { return (b + 255) / 256 * 256; }
// byte offsets of the lists of NA_MAX walks inside the array
constexpr int64_t NA_NODE0 = 0;
constexpr int64_t NA_WALK0 = NA_NODE0 + na_round(4 * NA_MAX);
constexpr int64_t NA_T0 = NA_WALK0 + na_round(4 * NA_MAX);
constexpr int64_t NA_NODE2 = NA_T0 + na_round(8 * NA_MAX);
constexpr int64_t NA_WALK2 = NA_NODE2 + na_round(4 * NA_MAX);
constexpr int64_t NA_T2 = NA_WALK2 + na_round(4 * NA_MAX);
constexpr int64_t NA_PREV = NA_T2 + na_round(8 * NA_MAX);
constexpr int64_t NA_FLAGS = NA_PREV + na_round(4 * NA_MAX);
constexpr int64_t NA_POS = NA_FLAGS + na_round(4 * NA_MAX);
constexpr int64_t NA_NLIVE = NA_POS + na_round(4 * NA_MAX);
constexpr int64_t NA_COUNTERS = NA_NLIVE + 256;
constexpr int64_t NA_PART = NA_COUNTERS + na_round(8 * QUEUE_SLICES);
// the scan's partial sums: one word per 256 walks bounds scan_parts_u32
// (tiles of at least 256 elements, plus one); checked at set-up
constexpr int64_t NA_PART_WORDS = NA_MAX / 256 + 2;
constexpr int64_t NA_BYTES = NA_PART + na_round(4 * NA_PART_WORDS);

// The lists of every allocation-free call on a device. Host code never
// passes this name to a kernel: it stands for the device array only in
// device code and in hipGetSymbolAddress, whose result (per device) is
// what the kernels receive.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_DEVICES = 64;
std::mutex na_mu;
void* na_ptr[NA_DEVICES] = {};

template <typename T>
T* na_at(void* base, int64_t off) {
    return reinterpret_cast<T*>(static_cast<unsigned char*>(base) + off);
}

}  // namespace

// Once per device, with that device current: the device address of the
// array (each device holds its own copy).
tw_status noalloc_setup(int device, Error& err) {
    if (device < 0 || device >= NA_DEVICES) {
        err = Error{TW_EDEVICE, "allocation-free walks: device ordinal out of range"};
        return err.code;
    }
    if (scan_parts_u32(NA_MAX) > NA_PART_WORDS) {
        err = Error{TW_EDEVICE, "allocation-free walks: scan partials exceed their space"};
        return err.code;
    }
    std::lock_guard<std::mutex> lk(na_mu);
    if (na_ptr[device]) return TW_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        err = Error{TW_EDEVICE, std::string("allocation-free walks: hipGetSymbolAddress failed: ") +
                                    hipGetErrorString(e)};
        return err.code;
    }
    na_ptr[device] = p;
    return TW_OK;
}

int64_t noalloc_scratch_bytes() { return NA_BYTES; }

tw_status sample_walks_noalloc(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                               int32_t* len, Error& err) {
    if (!p) {
        err = Error{TW_EINVAL, "sample_walks_noalloc: null params"};
        return err.code;
    }
    if (p->num_walks > NA_MAX) {
        err = Error{TW_EINVAL, "sample_walks_noalloc: num_walks exceeds TW_NOALLOC_MAX_WALKS (" +
                                   std::to_string(NA_MAX) + ")"};
        return err.code;
    }
    if (p->direction != TW_FORWARD) {
        err = Error{TW_EINVAL, "sample_walks_noalloc: forward walks only"};
        return err.code;
    }
    if (p->hop_bias.kind == TW_WEIGHT) {
        err = Error{TW_EINVAL, "sample_walks_noalloc: TW_WEIGHT needs its weights built (allocates)"};
        return err.code;
    }
    // nothing may be built lazily: an index must exist, and node2vec needs
    // the adjacency of the current window
    if (!g->rec.p) {
        err = Error{TW_EINVAL, "sample_walks_noalloc: the graph holds no index yet (ingest first)"};
        return err.code;
    }
    if (p->hop_bias.kind == TW_NODE2VEC && g->m > 0 && !g->adj_ready) {
        err = Error{TW_EINVAL,
                    "sample_walks_noalloc: the node2vec adjacency of the current window is not "
                    "built (one tw_sample_walks call with a node2vec bias builds it)"};
        return err.code;
    }
    void* base = nullptr;
    if (g->device >= 0 && g->device < NA_DEVICES) {
        std::lock_guard<std::mutex> lk(na_mu);
        base = na_ptr[g->device];
    }
    if (!base) {
        err = Error{TW_EDEVICE, "sample_walks_noalloc: no device array for the graph's device"};
        return err.code;
    }
    WalkArgs a;
    if (prepare_plain(g, p, nodes, ts, len, a, err) != TW_OK) return err.code;
    if (p->num_walks == 0) return TW_OK;
    HopLists h;
    h.live = Live{na_at<uint32_t>(base, NA_NODE0), na_at<uint32_t>(base, NA_WALK0),
                  na_at<uint64_t>(base, NA_T0)};
    h.next = Live{na_at<uint32_t>(base, NA_NODE2), na_at<uint32_t>(base, NA_WALK2),
                  na_at<uint64_t>(base, NA_T2)};
    h.prev = na_at<int32_t>(base, NA_PREV);
    h.flags = na_at<uint32_t>(base, NA_FLAGS);
    h.pos = na_at<uint32_t>(base, NA_POS);
    h.n_live = na_at<uint32_t>(base, NA_NLIVE);
    h.scan_part = na_at<uint32_t>(base, NA_PART);
    h.counters = na_at<unsigned long long>(base, NA_COUNTERS);
    // the rows are padded first unless the kernels write them whole, as in
    // tw_sample_walks
    if (!own_rows(a)) launch_fill(g, a.nodes, a.ts, a.num_walks * (int64_t)a.L);
    return queue_hops_in(g, a, g->auto_bpc, h, err);
}

tw_status check_walk_params(const tw_walk_params* p, Error& err) {
    if (!p || p->num_walks < 0 || p->max_len < 1) {
        err = Error{TW_EINVAL, "walk request: need num_walks >= 0 and max_len >= 1"};
        return err.code;
    }
    if (check_bias(p->hop_bias, true, err) != TW_OK) return err.code;
    if (check_bias(p->start_bias, false, err) != TW_OK) return err.code;
    return check_start(p->start_mode, p->d_start_nodes, p->num_walks, err);
}

size_t serve_table_bytes(int n) { return sizeof(ServeReqDev) * (size_t)std::max(n, 1); }

// hops of n walks from their lengths, added to *out
__global__ void k_sum_hops(const int32_t* __restrict__ len, int64_t n,
                           unsigned long long* out) {
    uint64_t h = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        h += len[i] > 1 ? (uint64_t)(len[i] - 1) : 0;
    for (int off = 32; off > 0; off >>= 1) h += __shfl_down(h, off, 64);
    if ((threadIdx.x & 63) == 0 && h) atomicAdd(out, (unsigned long long)h);
}

// error words of a one-request launch run by the full-walk kernel: it
// counts trial-cap hits in word 2, the request's layout has them in word 1
__global__ void k_err_words(uint32_t* e, int finish) {
    if (threadIdx.x == 0) {
        if (finish) {
            e[1] = e[2];
            e[2] = 0u;
        } else {
            e[2] = 0u;
        }
    }
}

// Requests of at least this many walks launched alone run the full-walk
// kernel on their own rows (the fastest dispatch for one rectangular batch).
constexpr int64_t SERVE_FULL_MIN = 1 << 16;

tw_status serve_launch(tw_graph* g, const ServeReq* reqs, int n, void* d_table, void* h_table,
                       unsigned long long* d_hops, uint32_t* d_err, bool rev, Error& err) {
    if (n < 1 || n > SERVE_MAX_REQ) {
        err = Error{TW_EINVAL, "serve: 1..1024 requests per launch"};
        return err.code;
    }
    if (!rev && n == 1 && reqs[0].count >= SERVE_FULL_MIN && reqs[0].hop.kind != TW_WEIGHT) {
        const ServeReq& q = reqs[0];
        WalkArgs a;
        if (fill_args(g, q.count, q.max_len, q.start, q.start_mode, q.start_nodes, q.seed, q.base,
                      q.hop.kind == TW_NODE2VEC, NAN, q.nodes, q.ts, q.len, a, err) != TW_OK)
            return err.code;
        if (own_rows(a)) {
            a.hop = make_hop_bias(q.hop);
            a.err = d_err;  // [0] start node out of range, [2] trial-cap hits
            hipLaunchKernelGGL(k_err_words, dim3(1), dim3(64), 0, g->stream, d_err, 0);
            const dim3 grid((unsigned)ceil_div(q.count, WALK_THREADS));
            with_kinds(a.hop.kind, a.start_kind, [&](auto h, auto st) {
                hipLaunchKernelGGL((k_walk_full<decltype(h)::value, decltype(st)::value, true>),
                                   grid, dim3(WALK_THREADS), 0, g->stream, a);
            });
            hipLaunchKernelGGL(k_err_words, dim3(1), dim3(64), 0, g->stream, d_err, 1);
            hipLaunchKernelGGL(k_sum_hops, dim3(1024), dim3(256), 0, g->stream, q.len, q.count,
                               d_hops);
            TW_HIP(hipGetLastError());
            return TW_OK;
        }
    }
    bool n2v = false;
    double wtau = NAN;  // the weight-based requests' time scale: one per launch
    int64_t total = 0;
    ServeReqDev* tab = static_cast<ServeReqDev*>(h_table);
    for (int r = 0; r < n; ++r) {
        const ServeReq& q = reqs[r];
        if (q.hop.kind == TW_WEIGHT) {
            const double sc = q.hop.tau > 0.0 ? q.hop.tau : 1.0;
            if (rev || (!std::isnan(wtau) && wtau != sc)) {
                err = Error{TW_EINVAL, "serve: weight-based requests of one launch need one "
                                       "tau and walk forward"};
                return err.code;
            }
            wtau = sc;
        }
        n2v |= q.hop.kind == TW_NODE2VEC;
        ServeReqDev d{};
        d.walk0 = total;
        d.count = q.count;
        d.seed = q.seed;
        d.base = q.base;
        d.L = q.max_len;
        d.start_kind = q.start.kind;
        d.start_mode = q.start_mode;
        d.start_tau = q.start.tau;
        d.hop = make_hop_bias(q.hop);
        d.start_nodes = q.start_nodes;
        d.nodes = q.nodes;
        d.ts = q.ts;
        d.len = q.len;
        d.err = d_err + 2 * r;
        tab[r] = d;
        total += q.count;
    }
    WalkArgs a;
    tw_bias none{TW_UNIFORM, 0.0, 1.0, 1.0};
    if (fill_args(g, total, 1, none, TW_START_EDGE, nullptr, 0, 0, n2v, wtau, nullptr, nullptr,
                  nullptr, a, err) != TW_OK)
        return err.code;
    if (queue_shape(g, err) != TW_OK) return err.code;
    TW_HIP(ensure(g->wq, sizeof(unsigned long long) * QUEUE_SLICES, g->stream));
    TW_HIP(hipMemcpyAsync(d_table, h_table, sizeof(ServeReqDev) * n, hipMemcpyHostToDevice,
                          g->stream));
    for (int r = 0; r < n; ++r)
        if (reqs[r].count > 0)
            launch_fill(g, reqs[r].nodes, reqs[r].ts, reqs[r].count * (int64_t)reqs[r].max_len);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, g->stream,
                       g->wq.as<unsigned long long>());
    if (total > 0) {
        const int64_t blocks = std::min<int64_t>(ceil_div(total, WALK_THREADS),
                                                 (int64_t)g->cu_count * g->queue_bpc_max);
        const ServeReqDev* tab_d = static_cast<const ServeReqDev*>(d_table);
        if (rev)
            hipLaunchKernelGGL(k_walk_serve<true>, dim3((unsigned)blocks), dim3(WALK_THREADS), 0,
                               g->stream, a, tab_d, n, g->wq.as<unsigned long long>(), d_hops);
        else
            hipLaunchKernelGGL(k_walk_serve<false>, dim3((unsigned)blocks), dim3(WALK_THREADS), 0,
                               g->stream, a, tab_d, n, g->wq.as<unsigned long long>(), d_hops);
    }
    TW_HIP(hipGetLastError());
    return TW_OK;
}

tw_status row_offsets(tw_graph* g, const int32_t* max_len, int64_t n, int64_t* row,
                      int64_t* total, Error& err) {
    if (!row || n < 0 || (n > 0 && !max_len)) {
        err = Error{TW_EINVAL, "row_offsets: null argument or negative count"};
        return err.code;
    }
    uint64_t* out = reinterpret_cast<uint64_t*>(row);
    TW_HIP(scan_exclusive_i32_to_u64(max_len, out, n, out + n, g->ws, g->stream));
    int64_t t = 0;
    TW_HIP(hipMemcpyAsync(&t, row + n, sizeof(t), hipMemcpyDeviceToHost, g->stream));
    TW_HIP(hipStreamSynchronize(g->stream));
    if (total) *total = t;
    return TW_OK;
}

tw_status autotune(tw_graph* g, const tw_walk_params* p, int64_t sample, int32_t* nodes,
                   int64_t* ts, int32_t* len, int32_t best[2], Error& err) {
    if (!p || sample < 1 || p->direction != TW_FORWARD) {
        err = Error{TW_EINVAL, "autotune: need forward parameters and sample_walks >= 1"};
        return err.code;
    }
    tw_walk_params q = *p;
    q.num_walks = std::min<int64_t>(p->num_walks, sample);
    WalkArgs a;
    if (prepare_plain(g, &q, nodes, ts, len, a, err) != TW_OK) return err.code;
    if (q.num_walks == 0) return TW_OK;
    if (queue_shape(g, err) != TW_OK) return err.code;
    // full-walk; the queue at three launch shapes (as many workgroups as
    // fit, 4 or 2 per CU); the cooperative dispatch over its regroup, the
    // lanes that engage the wavefront tier, the LDS panel and the read-back
    // cadence of the live count
    std::vector<tw_tuning> cands;
    const tw_tuning base{TW_DISPATCH_FULL_WALK, 0, 0, 64, 4096, 1};
    cands.push_back(base);
    for (int bpc : {0, 4, 2}) {
        tw_tuning c = base;
        c.dispatch = TW_DISPATCH_QUEUE;
        c.queue_bpc = bpc;
        cands.push_back(c);
    }
    for (int regroup : {0, 1})
        for (int wave_min : {64, 16})
            for (int panel : {2048, 8192})
                for (int sync : {1, 4}) {
                    if (regroup == 1 && (wave_min != 64 || panel != 2048)) continue;
                    cands.push_back(tw_tuning{TW_DISPATCH_COOP, 0, regroup, wave_min, panel, sync});
                }
    const tw_tuning saved = get_tuning(g);
    hipEvent_t e0, e1;
    TW_HIP(hipEventCreate(&e0));
    TW_HIP(hipEventCreate(&e1));
    float best_ms = 0.0f;
    tw_tuning pick = base;
    bool first = true;
    for (const tw_tuning& c : cands) {
        set_tuning_fields(g, c);
        float ms_min = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {  // the first run warms up
            hipEventRecord(e0, g->stream);
            if (run_dispatch(g, a, c.dispatch, c.queue_bpc, err) != TW_OK) {
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                set_tuning_fields(g, saved);
                return err.code;
            }
            hipEventRecord(e1, g->stream);
            TW_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            TW_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep == 1 || (rep > 1 && ms < ms_min)) ms_min = ms;
        }
        if (first || ms_min < best_ms) {
            best_ms = ms_min;
            pick = c;
            first = false;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    set_tuning_fields(g, pick);
    if (best) {
        best[0] = pick.dispatch;
        best[1] = pick.queue_bpc;
    }
    return TW_OK;
}

tw_tuning get_tuning(const tw_graph* g) {
    return tw_tuning{g->auto_dispatch ? g->auto_dispatch : TW_DISPATCH_FULL_WALK, g->auto_bpc,
                     g->coop_regroup, g->coop_wave_min, (int32_t)g->coop_panel, g->coop_sync};
}

void set_tuning_fields(tw_graph* g, const tw_tuning& t) {
    g->auto_dispatch = t.dispatch;
    g->auto_bpc = t.queue_bpc;
    g->coop_regroup = t.coop_regroup;
    g->coop_wave_min = t.coop_wave_min;
    g->coop_panel = (uint32_t)t.coop_panel;
    g->coop_sync = t.coop_sync;
}

tw_status set_tuning(tw_graph* g, const tw_tuning* t, Error& err) {
    if (!t || t->dispatch < TW_DISPATCH_FULL_WALK || t->dispatch > TW_DISPATCH_QUEUE ||
        t->queue_bpc < 0 || t->coop_regroup < 0 || t->coop_regroup > 1 || t->coop_wave_min < 1 ||
        t->coop_wave_min > 64 || t->coop_panel < 64 || t->coop_panel > 8192 ||
        t->coop_panel % 64 != 0 || t->coop_sync < 1 || t->coop_sync > 64) {
        err = Error{TW_EINVAL, "set_tuning: dispatch FULL_WALK..QUEUE, queue_bpc >= 0, regroup 0 or "
                               "1, wave_min 1..64, panel 64..8192 in steps of 64, sync 1..64"};
        return err.code;
    }
    set_tuning_fields(g, *t);
    return TW_OK;
}

}  // namespace tw
