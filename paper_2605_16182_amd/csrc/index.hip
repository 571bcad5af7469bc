// Streaming ingest, window eviction and the dual-index rebuild
// (Tempest, Sec. "Dual-Index Organization" and "Streaming Ingestion and
// Window Management").
//
// Layout in HBM (structure of arrays, all indices uint32):
//   timestamp view (the edge store):   e_src[m] e_dst[m] e_ts[m]
//   its timestamp groups:              gg_ts[Gg] gg_off[Gg+1]
//   node-and-timestamp view:           n_dst[m] n_ts[m]  (sorted by src, ts,
//                                      timestamp-view position)
//   its (node, timestamp) groups:      ng_ts[Gn] ng_off[Gn+1]
//   node table:                        rec[V] (32-byte NodeRec)
//
// One ingest: stage (validate, mirror, min/max) -> late drop -> stable radix
// sort of the batch by timestamp -> merge-path merge after the surviving
// window (old records first on equal timestamps) -> rebuild of the groups,
// the node view (stable radix sort by source) and the node table.
#include <algorithm>

#include "tw_internal.h"

namespace tw {
namespace {

constexpr int T = 256;

inline dim3 grid_for(int64_t n, int per_thread = 1) {
    int64_t b = ceil_div(std::max<int64_t>(n, 1), (int64_t)T * per_thread);
    return dim3((unsigned)b);
}

// int64 <-> order-preserving uint64
__device__ __host__ inline uint64_t ord(int64_t x) { return (uint64_t)x ^ 0x8000000000000000ull; }
__device__ __host__ inline int64_t unord(uint64_t x) { return (int64_t)(x ^ 0x8000000000000000ull); }

// scalars[0] = min ts (ordered), scalars[1] = max ts (ordered). Grid-stride
// over the batch so that only one pair of atomics per block reaches memory.
__global__ void k_stage(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                        const int64_t* __restrict__ ts, int64_t n, int32_t V, int directed,
                        int32_t* __restrict__ b_src, int32_t* __restrict__ b_dst,
                        int64_t* __restrict__ b_ts, uint32_t* err,
                        unsigned long long* scalars, uint32_t* unsorted) {
    __shared__ unsigned long long smin[T], smax[T];
    unsigned long long lo = ~0ull, hi = 0ull;
    bool bad = false, down = false;
    const int64_t stride = (int64_t)gridDim.x * T;
    for (int64_t i = (int64_t)blockIdx.x * T + threadIdx.x; i < n; i += stride) {
        int32_t u = src[i], v = dst[i];
        int64_t t = ts[i];
        bad |= (u < 0 || u >= V || v < 0 || v >= V);
        down |= (i > 0 && ts[i - 1] > t);
        unsigned long long o = ord(t);
        lo = o < lo ? o : lo;
        hi = o > hi ? o : hi;
        if (directed) {
            b_src[i] = u; b_dst[i] = v; b_ts[i] = t;
        } else {
            b_src[2 * i] = u; b_dst[2 * i] = v; b_ts[2 * i] = t;
            b_src[2 * i + 1] = v; b_dst[2 * i + 1] = u; b_ts[2 * i + 1] = t;
        }
    }
    if (bad) atomicOr(err, 1u);
    if (down) atomicOr(unsorted, 1u);
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int off = T / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&scalars[0], smin[0]);
        atomicMax(&scalars[1], smax[0]);
    }
}

__global__ void k_init_minmax(unsigned long long* scalars, uint32_t* err, uint32_t* unsorted) {
    scalars[0] = ~0ull;
    scalars[1] = 0ull;
    *err = 0u;
    *unsorted = 0u;
}

// first index of the sorted ts[0..n) with ts >= cut, and ts at that index
__global__ void k_sorted_cut(const int64_t* __restrict__ ts, int64_t n, int64_t cut,
                             uint32_t* pos, int64_t* first_ts) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (ts[mid] < cut) lo = mid + 1; else hi = mid;
    }
    *pos = (uint32_t)lo;
    *first_ts = lo < n ? ts[lo] : INT64_MAX;
}

// keep flag of staged records for the late-edge drop
__global__ void k_keep_flags(const int64_t* __restrict__ ts, int64_t n, int64_t cut,
                             uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) flags[i] = ts[i] >= cut ? 1u : 0u;
}

// sort keys (timestamp minus base) and staged indices of kept records
__global__ void k_make_keys(const int64_t* __restrict__ ts, int64_t n, int64_t base,
                            const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n) return;
    if (flags && !flags[i]) return;
    uint32_t o = pos ? pos[i] : (uint32_t)i;
    keys[o] = (uint64_t)(ts[i] - base);
    vals[o] = (uint32_t)i;
}

__global__ void k_gather_batch(const uint32_t* __restrict__ vals, int64_t n,
                               const int32_t* __restrict__ s_src, const int32_t* __restrict__ s_dst,
                               const int64_t* __restrict__ s_ts, int32_t* __restrict__ o_src,
                               int32_t* __restrict__ o_dst, int64_t* __restrict__ o_ts) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n) return;
    uint32_t j = vals[i];
    o_src[i] = s_src[j];
    o_dst[i] = s_dst[j];
    o_ts[i] = s_ts[j];
}

// number of entries of ts[0..n) below cut, into *out
__global__ void k_lower_bound(const int64_t* __restrict__ ts, int64_t n, int64_t cut,
                              uint32_t* out) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (ts[mid] < cut) lo = mid + 1; else hi = mid;
    }
    *out = (uint32_t)lo;
}

// Merge-path merge of A = old window (from a_begin) and B = sorted batch.
// Each thread produces MP_ITEMS consecutive outputs; on equal timestamps A
// goes first, which keeps older records before newer ones.
constexpr int MP_ITEMS = 8;
__global__ void k_merge(const int32_t* __restrict__ a_src, const int32_t* __restrict__ a_dst,
                        const int64_t* __restrict__ a_ts, int64_t na,
                        const int32_t* __restrict__ b_src, const int32_t* __restrict__ b_dst,
                        const int64_t* __restrict__ b_ts, int64_t nb, int32_t* __restrict__ o_src,
                        int32_t* __restrict__ o_dst, int64_t* __restrict__ o_ts) {
    int64_t d = ((int64_t)blockIdx.x * T + threadIdx.x) * MP_ITEMS;
    int64_t total = na + nb;
    if (d >= total) return;
    // i = how many A records precede output slot d
    int64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a_ts[mid] <= b_ts[d - 1 - mid]) lo = mid + 1; else hi = mid;
    }
    int64_t i = lo, j = d - lo;
    int64_t end = d + MP_ITEMS < total ? d + MP_ITEMS : total;
    for (int64_t o = d; o < end; ++o) {
        bool take_a = i < na && (j >= nb || a_ts[i] <= b_ts[j]);
        if (take_a) {
            o_src[o] = a_src[i]; o_dst[o] = a_dst[i]; o_ts[o] = a_ts[i]; ++i;
        } else {
            o_src[o] = b_src[j]; o_dst[o] = b_dst[j]; o_ts[o] = b_ts[j]; ++j;
        }
    }
}

// group-start flags of the timestamp view
__global__ void k_ts_group_flags(const int64_t* __restrict__ ts, int64_t m,
                                 uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m) flags[i] = (i == 0 || ts[i] != ts[i - 1]) ? 1u : 0u;
}

__global__ void k_ts_group_scatter(const int64_t* __restrict__ ts, int64_t m,
                                   const uint32_t* __restrict__ flags,
                                   const uint32_t* __restrict__ gidx, int64_t* __restrict__ g_ts,
                                   uint32_t* __restrict__ g_off, const uint32_t* G) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m && flags[i]) {
        g_ts[gidx[i]] = ts[i];
        g_off[gidx[i]] = (uint32_t)i;
    }
    if (i == 0) g_off[*G] = (uint32_t)m;
}

// (node, timestamp) groups of the node view, with the node of each group
__global__ void k_node_group_scatter(const int64_t* __restrict__ ts,
                                     const uint32_t* __restrict__ n_src, int64_t m,
                                     const uint32_t* __restrict__ flags,
                                     const uint32_t* __restrict__ gidx, int64_t* __restrict__ g_ts,
                                     uint32_t* __restrict__ g_off, uint32_t* __restrict__ g_node,
                                     const uint32_t* G) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m && flags[i]) {
        uint32_t k = gidx[i];
        g_ts[k] = ts[i];
        g_off[k] = (uint32_t)i;
        g_node[k] = n_src[i];
    }
    if (i == 0) g_off[*G] = (uint32_t)m;
}

// levels K and total entries of the fence of a node with G groups
__device__ __forceinline__ void fence_shape(uint32_t G, uint32_t* levels, uint32_t* size) {
    uint32_t K = 0, total = 0;
    if (G > (uint32_t)FENCE_FAN) {
        uint64_t n = G;
        do {
            n = (n + FENCE_FAN - 1) / FENCE_FAN;
            ++K;
            total += (uint32_t)((n + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN);
        } while (n > (uint64_t)FENCE_FAN);
    }
    *levels = K;
    *size = total;
}

__global__ void k_node_group_flags(const uint32_t* __restrict__ n_src,
                                   const int64_t* __restrict__ n_ts, int64_t m,
                                   uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m)
        flags[i] = (i == 0 || n_src[i] != n_src[i - 1] || n_ts[i] != n_ts[i - 1]) ? 1u : 0u;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) p[i] = v;
}

// Per node present in the node view: first edge and one past its last edge.
__global__ void k_run_bounds(const uint32_t* __restrict__ n_src, int64_t m,
                             uint32_t* __restrict__ first, uint32_t* __restrict__ end) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= m) return;
    uint32_t u = n_src[i];
    if (i == 0 || n_src[i - 1] != u) first[u] = (uint32_t)i;
    if (i == m - 1 || n_src[i + 1] != u) end[u] = (uint32_t)(i + 1);
}

// Edge and group counts per node (in place over first / end); the exclusive
// scans of these counts are the node offsets. gidx is the exclusive scan of
// the (node, timestamp) group flags, so gidx[j] counts groups starting before
// edge j, and Gn stands for gidx[m].
__global__ void k_node_counts(uint32_t* __restrict__ first_to_ecnt,
                              uint32_t* __restrict__ end_to_gcnt, int32_t V, int64_t m,
                              const uint32_t* __restrict__ gidx, const uint32_t* Gn) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v > V) return;
    if (v == V) {
        first_to_ecnt[v] = 0;
        end_to_gcnt[v] = 0;
        return;
    }
    uint32_t f = first_to_ecnt[v], e = end_to_gcnt[v];
    uint32_t ge = (int64_t)e >= m ? *Gn : gidx[e];
    uint32_t gc = e > f ? ge - gidx[f] : 0;
    first_to_ecnt[v] = e - f;
    end_to_gcnt[v] = gc;
}

// node records; fence sizes of every node into fsize[v] (fsize[V] = 0)
__global__ void k_node_records(const uint32_t* __restrict__ node_e,
                               const uint32_t* __restrict__ node_g, int32_t V,
                               const int64_t* __restrict__ ng_ts, NodeRec* __restrict__ rec,
                               uint32_t* __restrict__ fsize) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v > V) return;
    if (v == V) {
        fsize[v] = 0;
        return;
    }
    NodeRec r;
    r.gb = node_g[v];
    r.ge = node_g[v + 1];
    r.eb = node_e[v];
    r.ee = node_e[v + 1];
    uint32_t size;
    fence_shape(r.ge - r.gb, &r.levels, &size);
    r.fence_off = 0;
    r.t_last = r.gb < r.ge ? ng_ts[r.ge - 1] : INT64_MIN;
    rec[v] = r;
    fsize[v] = size;
}

__global__ void k_fence_offsets(const uint32_t* __restrict__ foff, int32_t V,
                                NodeRec* __restrict__ rec) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v < V) rec[v].fence_off = foff[v];
}

__global__ void k_fill_i64(int64_t* __restrict__ p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) p[i] = v;
}

// Each group p whose position inside its node is a multiple of FENCE_FAN^k
// writes its timestamp into level k of the node's fence.
__global__ void k_fence_fill(const int64_t* __restrict__ ng_ts, const uint32_t* __restrict__ ng_node,
                             int64_t Gn, const NodeRec* __restrict__ rec,
                             int64_t* __restrict__ fence) {
    int64_t p = (int64_t)blockIdx.x * T + threadIdx.x;
    if (p >= Gn) return;
    const NodeRec r = rec[ng_node[p]];
    if (r.levels == 0) return;
    const uint64_t rel = (uint64_t)((uint32_t)p - r.gb);
    if (rel & (FENCE_FAN - 1)) return;
    const uint32_t G = r.ge - r.gb;
    uint64_t nk[9];
    uint64_t n = G;
    for (uint32_t k = 1; k <= r.levels; ++k) {
        n = (n + FENCE_FAN - 1) / FENCE_FAN;
        nk[k] = n;
    }
    uint64_t off = r.fence_off;  // level K first
    const int64_t t = ng_ts[p];
    for (uint32_t k = r.levels; k >= 1; --k) {
        const uint32_t sh = FENCE_LOG * k;
        if ((rel & ((1ull << sh) - 1)) == 0) fence[off + (rel >> sh)] = t;
        off += (nk[k] + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN;
    }
}

__global__ void k_adj_keys(const uint32_t* __restrict__ n_src, const int32_t* __restrict__ n_dst,
                           int64_t m, uint64_t* __restrict__ keys) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m) keys[i] = ((uint64_t)n_src[i] << 32) | (uint32_t)n_dst[i];
}

__global__ void k_adj_extract(const uint64_t* __restrict__ keys, int64_t m,
                              int32_t* __restrict__ adj) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m) adj[i] = (int32_t)(uint32_t)keys[i];
}

__global__ void k_widen(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i];
}

__global__ void k_export_nodes(const NodeRec* __restrict__ rec, int32_t V, int64_t m, int64_t Gn,
                               int64_t* __restrict__ ebeg, int64_t* __restrict__ gbeg) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v > V) return;
    if (ebeg) ebeg[v] = v < V ? (int64_t)rec[v].eb : m;
    if (gbeg) gbeg[v] = v < V ? (int64_t)rec[v].gb : Gn;
}

// sizes and timestamp range after a rebuild: out = {Gg, Gn, t_min, t_max}
__global__ void k_summary(const int64_t* __restrict__ ts, int64_t m, const uint32_t* G,
                          int64_t* out) {
    out[0] = G[0];
    out[1] = G[1];
    out[2] = m > 0 ? ts[0] : 0;
    out[3] = m > 0 ? ts[m - 1] : 0;
}

// Rebuild everything derived from the timestamp view e_* (m records).
tw_status rebuild_views(tw_graph* g, Error& err) {
    hipStream_t s = g->stream;
    const int64_t m = g->m, V = g->V;
    // device scalars: bytes 16..23 hold Gg, Gn, bytes 24..31 the fence length;
    // bytes 32..63 the summary
    uint32_t* sc = g->scal.as<uint32_t>() + 2;  // sc[2] = Gg, sc[3] = Gn
    uint32_t* fence_total = g->scal.as<uint32_t>() + 7;
    TW_HIP(ensure(g->flags, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->idx, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->gg_ts, sizeof(int64_t) * (m + 1)));
    TW_HIP(ensure(g->gg_off, sizeof(uint32_t) * (m + 2)));
    TW_HIP(ensure(g->n_dst, sizeof(int32_t) * (m + 1)));
    TW_HIP(ensure(g->n_ts, sizeof(int64_t) * (m + 1)));
    TW_HIP(ensure(g->n_src, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->ng_ts, sizeof(int64_t) * (m + 1)));
    TW_HIP(ensure(g->ng_off, sizeof(uint32_t) * (m + 2)));
    TW_HIP(ensure(g->ng_node, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->rec, sizeof(NodeRec) * V));
    TW_HIP(ensure(g->b_vals, sizeof(uint32_t) * (3 * (V + 1) + 1)));
    uint32_t* flags = g->flags.as<uint32_t>();
    uint32_t* gidx = g->idx.as<uint32_t>();

    // global timestamp groups
    hipLaunchKernelGGL(k_ts_group_flags, grid_for(m), dim3(T), 0, s, g->e_ts.as<int64_t>(), m, flags);
    TW_HIP(scan_exclusive_u32(flags, gidx, m, sc + 2, g->ws, s));
    hipLaunchKernelGGL(k_ts_group_scatter, grid_for(m), dim3(T), 0, s, g->e_ts.as<int64_t>(), m,
                       flags, gidx, g->gg_ts.as<int64_t>(), g->gg_off.as<uint32_t>(), sc + 2);

    // node view: stable sort of the timestamp view by source, carrying the
    // destination and timestamp as payload
    uint32_t* keys = g->n_src.as<uint32_t>();
    TW_HIP(radix_sort_u32_kv(reinterpret_cast<const uint32_t*>(g->e_src.p),
                             reinterpret_cast<const uint32_t*>(g->e_dst.p),
                             reinterpret_cast<const uint64_t*>(g->e_ts.p), keys,
                             reinterpret_cast<uint32_t*>(g->n_dst.p),
                             reinterpret_cast<uint64_t*>(g->n_ts.p), m, 0,
                             bits_for((uint64_t)(V - 1)), g->ws, s));

    // (node, timestamp) groups
    hipLaunchKernelGGL(k_node_group_flags, grid_for(m), dim3(T), 0, s, keys, g->n_ts.as<int64_t>(),
                       m, flags);
    TW_HIP(scan_exclusive_u32(flags, gidx, m, sc + 3, g->ws, s));
    hipLaunchKernelGGL(k_node_group_scatter, grid_for(m), dim3(T), 0, s, g->n_ts.as<int64_t>(),
                       keys, m, flags, gidx, g->ng_ts.as<int64_t>(), g->ng_off.as<uint32_t>(),
                       g->ng_node.as<uint32_t>(), sc + 3);

    // node table: per-node edge / group counts, then their exclusive scans
    uint32_t* node_e = g->b_vals.as<uint32_t>();  // V+1 entries each
    uint32_t* node_g = node_e + (V + 1);
    uint32_t* fsize = node_g + (V + 1);
    hipLaunchKernelGGL(k_fill_u32, grid_for(2 * (V + 1)), dim3(T), 0, s, node_e, 2 * (V + 1), 0u);
    hipLaunchKernelGGL(k_run_bounds, grid_for(m), dim3(T), 0, s, keys, m, node_e, node_g);
    hipLaunchKernelGGL(k_node_counts, grid_for(V + 1), dim3(T), 0, s, node_e, node_g,
                       (int32_t)V, m, gidx, sc + 3);
    TW_HIP(scan_exclusive_u32(node_e, node_e, V + 1, nullptr, g->ws, s));
    TW_HIP(scan_exclusive_u32(node_g, node_g, V + 1, nullptr, g->ws, s));
    hipLaunchKernelGGL(k_node_records, grid_for(V + 1), dim3(T), 0, s, node_e, node_g, (int32_t)V,
                       g->ng_ts.as<int64_t>(), g->rec.as<NodeRec>(), fsize);
    TW_HIP(scan_exclusive_u32(fsize, fsize, V + 1, fence_total, g->ws, s));
    hipLaunchKernelGGL(k_fence_offsets, grid_for(V), dim3(T), 0, s, fsize, (int32_t)V,
                       g->rec.as<NodeRec>());
    TW_HIP(hipGetLastError());

    int64_t* summary = g->scal.as<int64_t>() + 4;  // bytes 32..63
    hipLaunchKernelGGL(k_summary, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>(), m, sc + 2,
                       summary);
    TW_HIP(hipGetLastError());
    int64_t host_sum[4];
    uint32_t host_fence = 0;
    TW_HIP(hipMemcpyAsync(host_sum, summary, sizeof(host_sum), hipMemcpyDeviceToHost, s));
    TW_HIP(hipMemcpyAsync(&host_fence, fence_total, sizeof(host_fence), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    g->Gg = host_sum[0];
    g->Gn = host_sum[1];
    g->t_min = host_sum[2];
    g->t_max = host_sum[3];

    // fence levels of nodes with many groups
    g->fence_len = host_fence;
    TW_HIP(ensure(g->fence, sizeof(int64_t) * (host_fence + FENCE_FAN)));
    if (host_fence > 0) {
        hipLaunchKernelGGL(k_fill_i64, grid_for(host_fence), dim3(T), 0, s, g->fence.as<int64_t>(),
                           (int64_t)host_fence, INT64_MAX);
        hipLaunchKernelGGL(k_fence_fill, grid_for(g->Gn), dim3(T), 0, s, g->ng_ts.as<int64_t>(),
                           g->ng_node.as<uint32_t>(), g->Gn, g->rec.as<NodeRec>(),
                           g->fence.as<int64_t>());
        TW_HIP(hipGetLastError());
    }
    g->adj_ready = false;
    return TW_OK;
}

tw_status ensure_common(tw_graph* g, Error& err) {
    TW_HIP(ensure(g->err, sizeof(uint32_t) * 4));
    TW_HIP(ensure(g->scal, sizeof(uint64_t) * 16));
    return TW_OK;
}

}  // namespace

tw_status ingest(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                 int64_t n, tw_ingest_info* info, Error& err) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    const int64_t B = g->directed ? n : 2 * n;  // staged records
    if (g->m + B > (int64_t)UINT32_MAX - 2) {
        err = Error{TW_EINVAL, "window would exceed 2^32 - 2 records"};
        return err.code;
    }
    // reserve everything this ingest may need before touching the window
    TW_HIP(ensure(g->b_src, sizeof(int32_t) * (B + 1)));
    TW_HIP(ensure(g->b_dst, sizeof(int32_t) * (B + 1)));
    TW_HIP(ensure(g->b_ts, sizeof(int64_t) * (B + 1)));
    const int64_t m_max = g->m + B;
    TW_HIP(ensure(g->a_src, sizeof(int32_t) * (m_max + 1)));
    TW_HIP(ensure(g->a_dst, sizeof(int32_t) * (m_max + 1)));
    TW_HIP(ensure(g->a_ts, sizeof(int64_t) * (m_max + 1)));

    unsigned long long* mm = g->scal.as<unsigned long long>();  // [0] min, [1] max
    uint32_t* errf = g->err.as<uint32_t>();
    uint32_t* unsorted = g->scal.as<uint32_t>() + 6;
    hipLaunchKernelGGL(k_init_minmax, dim3(1), dim3(1), 0, s, mm, errf + 1, unsorted);
    int32_t* s_src = g->b_src.as<int32_t>();
    int32_t* s_dst = g->b_dst.as<int32_t>();
    int64_t* s_ts = g->b_ts.as<int64_t>();
    if (n > 0)
        hipLaunchKernelGGL(k_stage, dim3((unsigned)std::min<int64_t>(ceil_div(n, T), 2048)),
                           dim3(T), 0, s, src, dst, ts, n, g->V, g->directed ? 1 : 0, s_src, s_dst,
                           s_ts, errf + 1, mm, unsorted);
    TW_HIP(hipGetLastError());
    unsigned long long hmm[2];
    uint32_t herr = 0, hunsorted = 0;
    TW_HIP(hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s));
    TW_HIP(hipMemcpyAsync(&herr, errf + 1, sizeof(herr), hipMemcpyDeviceToHost, s));
    TW_HIP(hipMemcpyAsync(&hunsorted, unsorted, sizeof(hunsorted), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    if (herr) {
        err = Error{TW_ERANGE, "ingest_batch: node id outside [0, num_nodes)"};
        return err.code;
    }
    int64_t bmin = 0, bmax = 0;
    if (n > 0) {
        bmin = unord(hmm[0]);
        bmax = unord(hmm[1]);
        g->t_now = g->has_time ? std::max(g->t_now, bmax) : bmax;
        g->has_time = true;
    }
    const bool sorted = hunsorted == 0;

    // window cut, late drop and eviction counts
    const bool windowed = g->window > 0 && g->has_time;
    int64_t cut = INT64_MIN;
    if (windowed) cut = (g->t_now < INT64_MIN + g->window) ? INT64_MIN : g->t_now - g->window;
    uint32_t* sc = g->scal.as<uint32_t>() + 24;          // [0] kept / cut position, [1] evicted
    int64_t* first_kept = g->scal.as<int64_t>() + 13;    // bytes 104..111
    const bool drop = windowed && B > 0 && bmin < cut;
    const bool evicting = windowed && g->m > 0 && g->t_min < cut;
    int64_t kept = B, evicted = 0, batch_first = bmin, drop_lo = 0;
    int64_t key_base = drop ? cut : bmin;
    uint64_t* keys = nullptr;
    uint32_t* vals = nullptr;
    if (drop && sorted) {
        // late records of a sorted batch are a prefix
        hipLaunchKernelGGL(k_sorted_cut, dim3(1), dim3(1), 0, s, s_ts, B, cut, sc, first_kept);
    } else if (!sorted && B > 0) {
        TW_HIP(ensure(g->b_keys, sizeof(uint64_t) * (B + 1)));
        TW_HIP(ensure(g->b_vals, sizeof(uint32_t) * (B + 1)));
        keys = g->b_keys.as<uint64_t>();
        vals = g->b_vals.as<uint32_t>();
        if (drop) {
            TW_HIP(ensure(g->b_flags, sizeof(uint32_t) * (B + 1)));
            TW_HIP(ensure(g->idx, sizeof(uint32_t) * (B + 1)));
            uint32_t* fl = g->b_flags.as<uint32_t>();
            uint32_t* pos = g->idx.as<uint32_t>();
            hipLaunchKernelGGL(k_keep_flags, grid_for(B), dim3(T), 0, s, s_ts, B, cut, fl);
            TW_HIP(scan_exclusive_u32(fl, pos, B, sc, g->ws, s));
            hipLaunchKernelGGL(k_make_keys, grid_for(B), dim3(T), 0, s, s_ts, B, key_base, fl,
                               pos, keys, vals);
        } else {
            hipLaunchKernelGGL(k_make_keys, grid_for(B), dim3(T), 0, s, s_ts, B, key_base, nullptr,
                               nullptr, keys, vals);
        }
    }
    if (evicting)
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>(), g->m, cut,
                           sc + 1);
    TW_HIP(hipGetLastError());
    if (drop || evicting) {
        uint32_t h2[2] = {0, 0};
        int64_t hf = INT64_MAX;
        TW_HIP(hipMemcpyAsync(h2, sc, sizeof(h2), hipMemcpyDeviceToHost, s));
        TW_HIP(hipMemcpyAsync(&hf, first_kept, sizeof(hf), hipMemcpyDeviceToHost, s));
        TW_HIP(hipStreamSynchronize(s));
        if (drop && sorted) {
            drop_lo = h2[0];
            kept = B - drop_lo;
            batch_first = hf;
        } else if (drop) {
            kept = h2[0];
            batch_first = cut;  // a lower bound of the kept records
        }
        if (evicting) evicted = h2[1];
    }

    // the kept batch records in timestamp order (stable)
    const int32_t* q_src = s_src + drop_lo;
    const int32_t* q_dst = s_dst + drop_lo;
    const int64_t* q_ts = s_ts + drop_lo;
    if (!sorted && kept > 0) {
        int kb = bits_for((uint64_t)(bmax - key_base));
        TW_HIP(radix_sort_u64(keys, vals, kept, 0, kb, g->ws, s));
        TW_HIP(ensure(g->n_src, sizeof(uint32_t) * (kept + 1)));
        TW_HIP(ensure(g->flags, sizeof(uint32_t) * (kept + 1)));
        TW_HIP(ensure(g->b_flags, sizeof(int64_t) * (kept + 1)));
        int32_t* o_src = reinterpret_cast<int32_t*>(g->n_src.as<uint32_t>());
        int32_t* o_dst = reinterpret_cast<int32_t*>(g->flags.as<uint32_t>());
        int64_t* o_ts = reinterpret_cast<int64_t*>(g->b_flags.as<uint32_t>());
        hipLaunchKernelGGL(k_gather_batch, grid_for(kept), dim3(T), 0, s, vals, kept, s_src, s_dst,
                           s_ts, o_src, o_dst, o_ts);
        q_src = o_src;
        q_dst = o_dst;
        q_ts = o_ts;
    }

    // merge the surviving window with the batch into the alternate buffers;
    // a batch that starts at or after the window's last timestamp is appended
    const int64_t na = g->m - evicted;
    const int64_t m_new = na + kept;
    const bool append = na == 0 || kept == 0 || batch_first >= g->t_max;
    if (append) {
        if (na > 0) {
            TW_HIP(hipMemcpyAsync(g->a_src.p, g->e_src.as<int32_t>() + evicted, 4 * na,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->a_dst.p, g->e_dst.as<int32_t>() + evicted, 4 * na,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->a_ts.p, g->e_ts.as<int64_t>() + evicted, 8 * na,
                                  hipMemcpyDeviceToDevice, s));
        }
        if (kept > 0) {
            TW_HIP(hipMemcpyAsync(g->a_src.as<int32_t>() + na, q_src, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->a_dst.as<int32_t>() + na, q_dst, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->a_ts.as<int64_t>() + na, q_ts, 8 * kept,
                                  hipMemcpyDeviceToDevice, s));
        }
    } else {
        hipLaunchKernelGGL(k_merge, grid_for(m_new, MP_ITEMS), dim3(T), 0, s,
                           g->e_src.as<int32_t>() + evicted, g->e_dst.as<int32_t>() + evicted,
                           g->e_ts.as<int64_t>() + evicted, na, q_src, q_dst, q_ts, kept,
                           g->a_src.as<int32_t>(), g->a_dst.as<int32_t>(), g->a_ts.as<int64_t>());
    }
    TW_HIP(hipGetLastError());
    std::swap(g->e_src, g->a_src);
    std::swap(g->e_dst, g->a_dst);
    std::swap(g->e_ts, g->a_ts);
    g->m = m_new;
    if (rebuild_views(g, err) != TW_OK) return err.code;

    g->last.accepted = kept;
    g->last.dropped_late = B - kept;
    g->last.evicted = evicted;
    g->last.active_edges = g->m;
    g->last.t_min = g->t_min;
    g->last.t_max = g->t_max;
    if (info) *info = g->last;
    return TW_OK;
}

tw_status evict_before(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    int64_t ev = 0;
    if (g->m > 0 && g->t_min < cutoff) {
        uint32_t* sc = g->scal.as<uint32_t>() + 24;
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>(), g->m,
                           cutoff, sc + 1);
        uint32_t h = 0;
        TW_HIP(hipMemcpyAsync(&h, sc + 1, sizeof(h), hipMemcpyDeviceToHost, s));
        TW_HIP(hipStreamSynchronize(s));
        ev = h;
    }
    if (ev > 0) {
        int64_t keep = g->m - ev;
        TW_HIP(ensure(g->a_src, sizeof(int32_t) * (keep + 1)));
        TW_HIP(ensure(g->a_dst, sizeof(int32_t) * (keep + 1)));
        TW_HIP(ensure(g->a_ts, sizeof(int64_t) * (keep + 1)));
        TW_HIP(hipMemcpyAsync(g->a_src.p, g->e_src.as<int32_t>() + ev, sizeof(int32_t) * keep,
                              hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->a_dst.p, g->e_dst.as<int32_t>() + ev, sizeof(int32_t) * keep,
                              hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->a_ts.p, g->e_ts.as<int64_t>() + ev, sizeof(int64_t) * keep,
                              hipMemcpyDeviceToDevice, s));
        std::swap(g->e_src, g->a_src);
        std::swap(g->e_dst, g->a_dst);
        std::swap(g->e_ts, g->a_ts);
        g->m = keep;
        if (rebuild_views(g, err) != TW_OK) return err.code;
    }
    g->last.accepted = 0;
    g->last.dropped_late = 0;
    g->last.evicted = ev;
    g->last.active_edges = g->m;
    g->last.t_min = g->t_min;
    g->last.t_max = g->t_max;
    if (n_evicted) *n_evicted = ev;
    return TW_OK;
}

tw_status init_empty(tw_graph* g, Error& err) {
    if (ensure_common(g, err) != TW_OK) return err.code;
    return rebuild_views(g, err);
}

tw_status build_adjacency(tw_graph* g, Error& err) {
    if (g->adj_ready) return TW_OK;
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    TW_HIP(ensure(g->adj, sizeof(int32_t) * (m + 1)));
    TW_HIP(ensure(g->b_keys, sizeof(uint64_t) * (m + 1)));
    uint64_t* keys = g->b_keys.as<uint64_t>();
    hipLaunchKernelGGL(k_adj_keys, grid_for(m), dim3(T), 0, s, g->n_src.as<uint32_t>(),
                       g->n_dst.as<int32_t>(), m, keys);
    int vb = bits_for((uint64_t)(g->V - 1));
    TW_HIP(radix_sort_u64(keys, nullptr, m, 0, vb, g->ws, s));
    TW_HIP(radix_sort_u64(keys, nullptr, m, 32, 32 + vb, g->ws, s));
    hipLaunchKernelGGL(k_adj_extract, grid_for(m), dim3(T), 0, s, keys, m, g->adj.as<int32_t>());
    TW_HIP(hipGetLastError());
    g->adj_ready = true;
    return TW_OK;
}

tw_status export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                       int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                       int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg, Error& err) {
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    auto cp = [&](void* d, const void* sp, size_t bytes) -> hipError_t {
        if (!d || bytes == 0) return hipSuccess;
        return hipMemcpyAsync(d, sp, bytes, hipMemcpyDeviceToDevice, s);
    };
    TW_HIP(cp(src, g->e_src.p, sizeof(int32_t) * m));
    TW_HIP(cp(dst, g->e_dst.p, sizeof(int32_t) * m));
    TW_HIP(cp(ts, g->e_ts.p, sizeof(int64_t) * m));
    TW_HIP(cp(g_ts, g->gg_ts.p, sizeof(int64_t) * g->Gg));
    TW_HIP(cp(n_dst, g->n_dst.p, sizeof(int32_t) * m));
    TW_HIP(cp(n_ts, g->n_ts.p, sizeof(int64_t) * m));
    TW_HIP(cp(n_gts, g->ng_ts.p, sizeof(int64_t) * g->Gn));
    if (g_off && g->gg_off.p)
        hipLaunchKernelGGL(k_widen, grid_for(g->Gg + 1), dim3(T), 0, s, g->gg_off.as<uint32_t>(),
                           g->Gg + 1, g_off);
    else if (g_off)
        TW_HIP(hipMemsetAsync(g_off, 0, sizeof(int64_t), s));
    if (n_goff && g->ng_off.p)
        hipLaunchKernelGGL(k_widen, grid_for(g->Gn + 1), dim3(T), 0, s, g->ng_off.as<uint32_t>(),
                           g->Gn + 1, n_goff);
    else if (n_goff)
        TW_HIP(hipMemsetAsync(n_goff, 0, sizeof(int64_t), s));
    if ((n_ebeg || n_gbeg) && g->rec.p)
        hipLaunchKernelGGL(k_export_nodes, grid_for(g->V + 1), dim3(T), 0, s,
                           g->rec.as<NodeRec>(), g->V, m, g->Gn, n_ebeg, n_gbeg);
    else {
        if (n_ebeg) TW_HIP(hipMemsetAsync(n_ebeg, 0, sizeof(int64_t) * (g->V + 1), s));
        if (n_gbeg) TW_HIP(hipMemsetAsync(n_gbeg, 0, sizeof(int64_t) * (g->V + 1), s));
    }
    TW_HIP(hipGetLastError());
    TW_HIP(hipStreamSynchronize(s));
    return TW_OK;
}

}  // namespace tw
