// Streaming ingest, window eviction and the dual-index rebuild
// (Tempest, Sec. "Dual-Index Organization" and "Streaming Ingestion and
// Window Management").
//
// Layout in HBM (structure of arrays, all positions uint32):
//   timestamp view (the edge store):   e_src e_dst e_ts, the window at
//                                      [e_base, e_base + m) of buffers with
//                                      room to append
//   its timestamp groups:              gg_ts gg_off at [gg_base, gg_base + Gg],
//                                      offsets are edge-store positions
//   node-and-timestamp view:           n_src n_dst n_ts [m] (sorted by source,
//                                      timestamp, arrival)
//   its (node, timestamp) groups:      ng_ts ng_off [Gn]
//   node table:                        rec[V] (32-byte NodeRec), fence levels
//
// One ingest: stage (validate, mirror, min/max, sortedness) -> late drop ->
// (unsorted batch only) stable radix sort by timestamp -> timestamp view:
// evicting moves e_base, a batch that starts at or after the window's last
// timestamp is appended in place and its groups appended, any other batch is
// merged (merge path, older records first on equal timestamps) and the groups
// rebuilt -> node view: the batch is sorted by source and every node's
// surviving run is merged with its batch run -> (node, timestamp) groups,
// node table and fence from the node view.
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

// groups of the timestamp view; offsets are positions in the edge-store
// buffer (pos_base is the buffer position of ts[0])
__global__ void k_ts_group_scatter(const int64_t* __restrict__ ts, int64_t m,
                                   const uint32_t* __restrict__ flags,
                                   const uint32_t* __restrict__ gidx, int64_t* __restrict__ g_ts,
                                   uint32_t* __restrict__ g_off, const uint32_t* G,
                                   uint32_t pos_base) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < m && flags[i]) {
        g_ts[gidx[i]] = ts[i];
        g_off[gidx[i]] = pos_base + (uint32_t)i;
    }
    if (i == 0) g_off[*G] = pos_base + (uint32_t)m;
}

// group-start flags of a batch appended after a window whose last timestamp
// is last_ts (has_last = 0: empty window)
__global__ void k_append_group_flags(const int64_t* __restrict__ ts, int64_t n, int64_t last_ts,
                                     int has_last, uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0) ? (!has_last || ts[0] != last_ts) : (ts[i] != ts[i - 1]);
}

// Surviving old edges to their merged positions: before them within the node
// go the batch edges with a strictly smaller timestamp (older edges first on
// equal timestamps).
__global__ void k_merge_old(const uint32_t* __restrict__ n_src, const int32_t* __restrict__ n_dst,
                            const int64_t* __restrict__ n_ts, int64_t m_old,
                            const uint4* __restrict__ plan, const uint32_t* __restrict__ neb,
                            const int64_t* __restrict__ bs_ts, uint32_t* __restrict__ o_src,
                            int32_t* __restrict__ o_dst, int64_t* __restrict__ o_ts,
                            uint32_t* __restrict__ o_flag) {
    int64_t j = (int64_t)blockIdx.x * T + threadIdx.x;
    if (j >= m_old) return;
    const uint32_t v = n_src[j];
    const uint4 p = plan[v];
    if ((uint32_t)j < p.x) return;  // evicted
    const int64_t t = n_ts[j];
    uint32_t c = 0;
    if (p.z < p.w && bs_ts[p.z] < t) {
        uint32_t lo = p.z, hi = p.w;
        while (lo < hi) {
            uint32_t mid = lo + ((hi - lo) >> 1);
            if (bs_ts[mid] < t) lo = mid + 1; else hi = mid;
        }
        c = lo - p.z;
    }
    const uint32_t d = neb[v] + ((uint32_t)j - p.x) + c;
    o_src[d] = v;
    o_dst[d] = n_dst[j];
    o_ts[d] = t;
    // a surviving old edge starts a (node, timestamp) group unless the old
    // edge before it has the same timestamp (no batch edge can sit between
    // equal old timestamps, since older edges go first on ties)
    o_flag[d] = ((uint32_t)j == p.x || n_ts[j - 1] != t) ? 1u : 0u;
}

// Batch edges (sorted by source, stable) to their merged positions: before
// them go the surviving old edges of the node with a timestamp <= theirs.
__global__ void k_merge_new(const uint32_t* __restrict__ bs_src, const int32_t* __restrict__ bs_dst,
                            const int64_t* __restrict__ bs_ts, int64_t nb,
                            const uint4* __restrict__ plan, const uint32_t* __restrict__ neb,
                            const int64_t* __restrict__ n_ts, uint32_t* __restrict__ o_src,
                            int32_t* __restrict__ o_dst, int64_t* __restrict__ o_ts,
                            uint32_t* __restrict__ o_flag) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= nb) return;
    const uint32_t v = bs_src[i];
    const uint4 p = plan[v];
    const int64_t y = bs_ts[i];
    uint32_t c = 0;
    if (p.x < p.y) {
        if (n_ts[p.y - 1] <= y) {
            c = p.y - p.x;
        } else {
            uint32_t lo = p.x, hi = p.y;
            while (lo < hi) {
                uint32_t mid = lo + ((hi - lo) >> 1);
                if (n_ts[mid] <= y) lo = mid + 1; else hi = mid;
            }
            c = lo - p.x;
        }
    }
    const uint32_t d = neb[v] + ((uint32_t)i - p.z) + c;
    o_src[d] = v;
    o_dst[d] = bs_dst[i];
    o_ts[d] = y;
    // the merged predecessor: the last surviving old edge with timestamp <= y
    // when it comes after the previous batch edge of the node (old edges
    // with a timestamp equal to that batch edge's come before it), else the
    // previous batch edge; none for the node's first edge
    uint32_t flag = 1;
    const bool has_prev_b = (uint32_t)i > p.z;
    if (c > 0 && (!has_prev_b || n_ts[p.x + c - 1] > bs_ts[i - 1]))
        flag = n_ts[p.x + c - 1] != y;
    else if (has_prev_b)
        flag = bs_ts[i - 1] != y;
    o_flag[d] = flag;
}

// (node, timestamp) groups of the node view, with the node of each group


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

__global__ void k_fill_i64(int64_t* __restrict__ p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) p[i] = v;
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

__global__ void k_widen2(const uint2* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i].x;
}

__global__ void k_widen(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out,
                        int64_t minus) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i] - minus;
}

// ---------------------------------------------------------- active nodes
//
// The node table is maintained over the nodes that have edges (the active
// nodes, kept as a sorted list); every other node holds the empty record.
// Each ingest forms the union of the active list with the batch's source
// runs, merges per union node, and writes records only for union nodes.

__device__ __forceinline__ NodeRec empty_rec() {
    NodeRec r;
    r.gb = r.ge = r.eb = r.ee = 0;
    r.fence_off = r.levels = 0;
    r.t_last = INT64_MIN;
    return r;
}

__global__ void k_fill_empty_rec(NodeRec* __restrict__ rec, int64_t V) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v < V) rec[v] = empty_rec();
}

// flags[i] = 1 where a new source starts in the source-sorted src[0..n)
__global__ void k_run_start_flags(const uint32_t* __restrict__ src, int64_t n,
                                  uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || src[i] != src[i - 1]) ? 1u : 0u;
}

// Union items: the old active nodes (payload ~0) after the batch's source
// runs (payload bf << 32 | be), so that a stable sort keeps a node's old
// item first. rpos = exclusive scan of the run-start flags.
__global__ void k_items_old(const uint32_t* __restrict__ act, int64_t A, int64_t at,
                            uint32_t* __restrict__ keys, uint64_t* __restrict__ pay) {
    int64_t k = (int64_t)blockIdx.x * T + threadIdx.x;
    if (k < A) {
        keys[at + k] = act[k];
        pay[at + k] = ~0ull;
    }
}

__global__ void k_items_batch(const uint32_t* __restrict__ bsrc, int64_t n,
                              const uint32_t* __restrict__ flags, const uint32_t* __restrict__ rpos,
                              uint32_t* __restrict__ keys, uint64_t* __restrict__ pay) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = bsrc[i];
    uint32_t* halves = reinterpret_cast<uint32_t*>(pay);  // [2r] = be, [2r+1] = bf
    if (flags[i]) {
        const uint32_t r = rpos[i];
        keys[r] = v;
        halves[2 * r + 1] = (uint32_t)i;
    }
    if (i == n - 1 || bsrc[i + 1] != v) halves[2 * (rpos[i] + flags[i] - 1)] = (uint32_t)(i + 1);
}

// Per union node (first item of each key): the merge plan {ob, oe, bf, be}
// (surviving old run [ob, oe) after evicting edges older than cut, batch run
// [bf, be)) and its merged size.
__global__ void k_union_plan(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ pay,
                             int64_t n, const uint32_t* __restrict__ uflags,
                             const uint32_t* __restrict__ upos, const NodeRec* __restrict__ rec,
                             const int64_t* __restrict__ n_ts, int evicting, int64_t cut,
                             uint4* __restrict__ plan, uint32_t* __restrict__ u_node,
                             uint32_t* __restrict__ u_cnt) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n || !uflags[i]) return;
    const uint32_t v = keys[i];
    bool has_old = false;
    uint32_t bf = 0, be = 0;
    for (int64_t j = i; j < n && j < i + 2 && keys[j] == v; ++j) {
        const uint64_t p = pay[j];
        if (p == ~0ull) {
            has_old = true;
        } else {
            bf = (uint32_t)(p >> 32);
            be = (uint32_t)p;
        }
    }
    uint32_t ob = 0, oe = 0;
    if (has_old) {
        const NodeRec r = rec[v];
        ob = r.eb;
        oe = r.ee;
        if (evicting && ob < oe && n_ts[ob] < cut) {
            uint32_t lo = ob, hi = oe;
            while (lo < hi) {
                uint32_t mid = lo + ((hi - lo) >> 1);
                if (n_ts[mid] < cut) lo = mid + 1; else hi = mid;
            }
            ob = lo;
        }
    }
    plan[v] = make_uint4(ob, oe, bf, be);
    const uint32_t u = upos[i];
    u_node[u] = v;
    u_cnt[u] = (oe - ob) + (be - bf);
}

__global__ void k_union_offsets(const uint32_t* __restrict__ u_node,
                                const uint32_t* __restrict__ u_neb, int64_t U,
                                uint32_t* __restrict__ neb_v) {
    int64_t u = (int64_t)blockIdx.x * T + threadIdx.x;
    if (u < U) neb_v[u_node[u]] = u_neb[u];
}

// union nodes left without edges get the empty record; flags the others
__global__ void k_union_active(const uint32_t* __restrict__ u_node,
                               const uint32_t* __restrict__ u_cnt, int64_t U,
                               NodeRec* __restrict__ rec, uint32_t* __restrict__ aflags) {
    int64_t u = (int64_t)blockIdx.x * T + threadIdx.x;
    if (u >= U) return;
    const bool a = u_cnt[u] > 0;
    if (!a) rec[u_node[u]] = empty_rec();
    aflags[u] = a ? 1u : 0u;
}

// the new active list with each node's first edge and edge count
__global__ void k_active_compact(const uint32_t* __restrict__ aflags,
                                 const uint32_t* __restrict__ apos, int64_t U,
                                 const uint32_t* __restrict__ u_node,
                                 const uint32_t* __restrict__ u_neb,
                                 const uint32_t* __restrict__ u_cnt, uint32_t* __restrict__ act,
                                 uint32_t* __restrict__ a_eb, uint32_t* __restrict__ a_cnt) {
    int64_t u = (int64_t)blockIdx.x * T + threadIdx.x;
    if (u < U && aflags[u]) {
        const uint32_t k = apos[u];
        act[k] = u_node[u];
        a_eb[k] = u_neb[u];
        a_cnt[k] = u_cnt[u];
    }
}

// group range and fence size of every active node: its first edge and its
// end are group starts, found by binary search in the group offsets
__device__ __forceinline__ uint32_t find_group(const uint2* __restrict__ g_od, uint32_t n,
                                               uint32_t e) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (g_od[mid].x < e) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_active_groups(const uint32_t* __restrict__ a_eb,
                                const uint32_t* __restrict__ a_cnt, int64_t A, int64_t m,
                                const uint2* __restrict__ g_off, const uint32_t* Gn,
                                uint32_t* __restrict__ a_gb, uint32_t* __restrict__ a_ge,
                                uint32_t* __restrict__ fsize) {
    int64_t k = (int64_t)blockIdx.x * T + threadIdx.x;
    if (k >= A) return;
    const uint32_t G = *Gn;
    const uint32_t eb = a_eb[k], ee = eb + a_cnt[k];
    const uint32_t gb = find_group(g_off, G, eb);
    const uint32_t ge = (int64_t)ee >= m ? G : find_group(g_off, G, ee);
    a_gb[k] = gb;
    a_ge[k] = ge;
    fsize[k] = fence_geometry(gb, ge).size;
}

// Fence entries [j0, j1) (stride) of a node whose fence body starts at
// group a0 and has `body` groups.
__device__ __forceinline__ void fence_entries(const int64_t* __restrict__ ng_ts, uint32_t a0,
                                              uint32_t body, uint32_t levels, uint32_t j0,
                                              uint32_t j1, uint32_t stride,
                                              int64_t* __restrict__ out) {
    // level k (stored from K down to 1) holds ng_ts[a0 + i * FAN^k], i < n_k,
    // padded with INT64_MAX to a multiple of FENCE_FAN
    uint64_t nk[FENCE_MAX_LEVELS + 1];
    uint64_t n = body;
    if (levels > (uint32_t)FENCE_MAX_LEVELS) return;  // cannot happen for 32-bit groups
    for (uint32_t k = 1; k <= levels; ++k) {
        n = (n + FENCE_FAN - 1) / FENCE_FAN;
        nk[k] = n;
    }
    for (uint32_t j = j0; j < j1; j += stride) {
        uint64_t off = 0;
        int k = (int)levels;
        for (; k >= 1; --k) {
            const uint64_t len = (nk[k] + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN;
            if (j < off + len) break;
            off += len;
        }
        const uint64_t i = j - off;
        out[j] = i < nk[k] ? ng_ts[a0 + (i << (FENCE_LOG * k))] : INT64_MAX;
    }
}

__global__ void k_active_records(const uint32_t* __restrict__ act,
                                 const uint32_t* __restrict__ a_eb,
                                 const uint32_t* __restrict__ a_cnt,
                                 const uint32_t* __restrict__ a_gb,
                                 const uint32_t* __restrict__ a_ge,
                                 const uint32_t* __restrict__ foff, int64_t A,
                                 const int64_t* __restrict__ ng_ts, NodeRec* __restrict__ rec) {
    int64_t k = (int64_t)blockIdx.x * T + threadIdx.x;
    if (k >= A) return;
    NodeRec r;
    r.eb = a_eb[k];
    r.ee = r.eb + a_cnt[k];
    r.gb = a_gb[k];
    r.ge = a_ge[k];
    r.levels = fence_geometry(r.gb, r.ge).levels;
    r.fence_off = foff[k];
    r.t_last = ng_ts[r.ge - 1];
    rec[act[k]] = r;
}

// Fence entry j of the concatenated fences of the active nodes: its node is
// the last active node whose fence starts at or before j.
__global__ void k_fence_fill(const uint32_t* __restrict__ foff, int64_t A, int64_t total,
                             const uint32_t* __restrict__ act, const NodeRec* __restrict__ rec,
                             const int64_t* __restrict__ ng_ts, int64_t* __restrict__ fence) {
    int64_t j = (int64_t)blockIdx.x * T + threadIdx.x;
    if (j >= total) return;
    int64_t lo = 0, hi = A;  // first node whose fence starts after j
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)foff[mid] <= j) lo = mid + 1; else hi = mid;
    }
    const uint32_t k = (uint32_t)(lo - 1);
    const NodeRec r = rec[act[k]];
    const FenceGeom f = fence_geometry(r.gb, r.ge);
    const uint32_t rel = (uint32_t)(j - foff[k]);
    fence_entries(ng_ts, f.a0, r.ge - f.a0, f.levels, rel, rel + 1, 1, fence + foff[k]);
}

// CSR-style export of the node table: an empty node starts where the next
// active node starts (or at the end)
__global__ void k_export_nodes(const NodeRec* __restrict__ rec, const uint32_t* __restrict__ act,
                               int64_t A, int32_t V, int64_t m, int64_t Gn,
                               int64_t* __restrict__ ebeg, int64_t* __restrict__ gbeg) {
    int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v > V) return;
    int64_t e = m, gg = Gn;
    if (v < V && rec[v].ee > rec[v].eb) {
        e = rec[v].eb;
        gg = rec[v].gb;
    } else if (v < V) {
        int64_t lo = 0, hi = A;  // first active node > v
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)act[mid] <= v) lo = mid + 1; else hi = mid;
        }
        if (lo < A) {
            e = rec[act[lo]].eb;
            gg = rec[act[lo]].gb;
        }
    }
    if (ebeg) ebeg[v] = e;
    if (gbeg) gbeg[v] = gg;
}

__global__ void k_window_summary(const int64_t* __restrict__ ts, int64_t m, int64_t* out) {
    out[0] = m > 0 ? ts[0] : 0;
    out[1] = m > 0 ? ts[m - 1] : 0;
}

uint32_t* u32_slot(tw_graph* g, int k) { return g->scal.as<uint32_t>() + k; }
int64_t* i64_slot(tw_graph* g, int k) { return g->scal.as<int64_t>() + k; }

tw_status ensure_common(tw_graph* g, Error& err) {
    if (!g->err.p) {
        // device error flags start cleared
        TW_HIP(ensure(g->err, sizeof(uint32_t) * 4));
        TW_HIP(hipMemsetAsync(g->err.p, 0, sizeof(uint32_t) * 4, g->stream));
    }
    TW_HIP(ensure(g->scal, SCALAR_BYTES));
    return TW_OK;
}

// Capacity of the edge-store buffers for a window of `need` records; growing
// copies the window to the front of the new buffers (e_base = 0).
tw_status reserve_window(tw_graph* g, int64_t need, Error& err) {
    if (need <= g->e_cap) return TW_OK;
    int64_t cap = std::max<int64_t>(need, 2 * g->e_cap);
    cap = std::max<int64_t>(cap, need + need / 2 + 1024);
    cap = std::min<int64_t>(cap, (int64_t)UINT32_MAX - 1);
    TW_HIP(ensure(g->a_src, sizeof(int32_t) * cap));
    TW_HIP(ensure(g->a_dst, sizeof(int32_t) * cap));
    TW_HIP(ensure(g->a_ts, sizeof(int64_t) * cap));
    hipStream_t s = g->stream;
    if (g->m > 0) {
        TW_HIP(hipMemcpyAsync(g->a_src.p, g->e_src.as<int32_t>() + g->e_base, 4 * g->m,
                              hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->a_dst.p, g->e_dst.as<int32_t>() + g->e_base, 4 * g->m,
                              hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->a_ts.p, g->e_ts.as<int64_t>() + g->e_base, 8 * g->m,
                              hipMemcpyDeviceToDevice, s));
    }
    std::swap(g->e_src, g->a_src);
    std::swap(g->e_dst, g->a_dst);
    std::swap(g->e_ts, g->a_ts);
    TW_HIP(ensure(g->a_src, sizeof(int32_t) * cap));
    TW_HIP(ensure(g->a_dst, sizeof(int32_t) * cap));
    TW_HIP(ensure(g->a_ts, sizeof(int64_t) * cap));
    TW_HIP(ensure(g->gg_ts, sizeof(int64_t) * (cap + 2)));
    TW_HIP(ensure(g->gg_off, sizeof(uint32_t) * (cap + 2)));
    g->e_base = 0;
    g->e_cap = cap;
    return TW_OK;
}

// Global timestamp groups of the whole window, from scratch (gg_base = 0).
// The count lands in the GROUPS slot.
tw_status build_ts_groups(tw_graph* g, Error& err) {
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    const int64_t* ts = g->e_ts.as<int64_t>() + g->e_base;
    uint32_t* G = u32_slot(g, SLOT_U32_GROUPS);
    TW_HIP(group_starts(nullptr, ts, m, (uint32_t)g->e_base, g->gg_ts.as<int64_t>(),
                        g->gg_off.as<uint32_t>(), nullptr, nullptr, G, g->ws, s));
    g->gg_base = 0;
    return TW_OK;
}

// Merge the node view with `kept` batch records (timestamp order) after
// removing every node's edges older than `cut` (when evicting). The batch is
// sorted by source (stable); the union of the active nodes and the batch's
// sources gets per-node plans and offsets (a scan over the union only); each
// node's surviving run and batch run are merged by timestamp, older first on
// ties, into the alternate arrays. Leaves the new active list in act0 with
// each node's first edge and edge count.
tw_status merge_node_view(tw_graph* g, const int32_t* q_src, const int32_t* q_dst,
                          const int64_t* q_ts, int64_t kept, int64_t m_old, int64_t m_new,
                          bool evicting, int64_t cut, Error& err) {
    hipStream_t s = g->stream;
    const int64_t V = g->V, A_old = g->A;
    TW_HIP(ensure(g->bs_src, sizeof(uint32_t) * (kept + 1)));
    TW_HIP(ensure(g->bs_dst, sizeof(int32_t) * (kept + 1)));
    TW_HIP(ensure(g->bs_ts, sizeof(int64_t) * (kept + 1)));
    TW_HIP(ensure(g->an_src, sizeof(uint32_t) * (m_new + 1)));
    TW_HIP(ensure(g->an_dst, sizeof(int32_t) * (m_new + 1)));
    TW_HIP(ensure(g->an_ts, sizeof(int64_t) * (m_new + 1)));
    TW_HIP(ensure(g->plan, sizeof(uint4) * (V + 1)));
    TW_HIP(ensure(g->neb_v, sizeof(uint32_t) * (V + 1)));
    TW_HIP(ensure(g->flags, sizeof(uint32_t) * (kept + 1)));
    TW_HIP(ensure(g->idx, sizeof(uint32_t) * (kept + 1)));
    uint32_t* bsrc = g->bs_src.as<uint32_t>();
    int32_t* bdst = g->bs_dst.as<int32_t>();
    int64_t* bts = g->bs_ts.as<int64_t>();
    TW_HIP(radix_sort_u32_kv(reinterpret_cast<const uint32_t*>(q_src),
                             reinterpret_cast<const uint32_t*>(q_dst),
                             reinterpret_cast<const uint64_t*>(q_ts), bsrc,
                             reinterpret_cast<uint32_t*>(bdst), reinterpret_cast<uint64_t*>(bts),
                             kept, 0, bits_for((uint64_t)(V - 1)), g->ws, s));

    // the batch's source runs
    uint32_t* rflags = g->flags.as<uint32_t>();
    uint32_t* rpos = g->idx.as<uint32_t>();
    uint32_t* sc_runs = u32_slot(g, SLOT_U32_RUNS);
    hipLaunchKernelGGL(k_run_start_flags, grid_for(kept), dim3(T), 0, s, bsrc, kept, rflags);
    TW_HIP(scan_exclusive_u32(rflags, rpos, kept, sc_runs, g->ws, s));
    uint32_t R = 0;
    TW_HIP(hipMemcpyAsync(&R, sc_runs, sizeof(R), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));

    // union items: batch runs, then the old active nodes; sort by node (stable)
    const int64_t n_items = (int64_t)R + A_old;
    TW_HIP(ensure(g->it_keys, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->it_pay, sizeof(uint64_t) * (n_items + 1)));
    TW_HIP(ensure(g->it_skeys, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->it_spay, sizeof(uint64_t) * (n_items + 1)));
    hipLaunchKernelGGL(k_items_batch, grid_for(kept), dim3(T), 0, s, bsrc, kept, rflags, rpos,
                       g->it_keys.as<uint32_t>(), g->it_pay.as<uint64_t>());
    hipLaunchKernelGGL(k_items_old, grid_for(A_old), dim3(T), 0, s, g->act0.as<uint32_t>(), A_old,
                       (int64_t)R, g->it_keys.as<uint32_t>(), g->it_pay.as<uint64_t>());
    TW_HIP(radix_sort_u32_kv(g->it_keys.as<uint32_t>(), nullptr, g->it_pay.as<uint64_t>(),
                             g->it_skeys.as<uint32_t>(), nullptr, g->it_spay.as<uint64_t>(),
                             n_items, 0, bits_for((uint64_t)(V - 1)), g->ws, s));

    // union nodes: plans, merged sizes, offsets
    TW_HIP(ensure(g->u_flags, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->u_pos, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->u_node, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->u_cnt, sizeof(uint32_t) * (n_items + 1)));
    TW_HIP(ensure(g->u_neb, sizeof(uint32_t) * (n_items + 1)));
    uint32_t* uflags = g->u_flags.as<uint32_t>();
    uint32_t* upos = g->u_pos.as<uint32_t>();
    uint32_t* sc_u = u32_slot(g, SLOT_U32_UNION);
    hipLaunchKernelGGL(k_run_start_flags, grid_for(n_items), dim3(T), 0, s,
                       g->it_skeys.as<uint32_t>(), n_items, uflags);
    TW_HIP(scan_exclusive_u32(uflags, upos, n_items, sc_u, g->ws, s));
    hipLaunchKernelGGL(k_union_plan, grid_for(n_items), dim3(T), 0, s, g->it_skeys.as<uint32_t>(),
                       g->it_spay.as<uint64_t>(), n_items, uflags, upos, g->rec.as<NodeRec>(),
                       g->n_ts.as<int64_t>(), evicting ? 1 : 0, cut, g->plan.as<uint4>(),
                       g->u_node.as<uint32_t>(), g->u_cnt.as<uint32_t>());
    uint32_t U = 0;
    TW_HIP(hipMemcpyAsync(&U, sc_u, sizeof(U), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    TW_HIP(scan_exclusive_u32(g->u_cnt.as<uint32_t>(), g->u_neb.as<uint32_t>(), U, nullptr, g->ws,
                              s));
    hipLaunchKernelGGL(k_union_offsets, grid_for(U), dim3(T), 0, s, g->u_node.as<uint32_t>(),
                       g->u_neb.as<uint32_t>(), (int64_t)U, g->neb_v.as<uint32_t>());

    // merge
    TW_HIP(ensure(g->gflags, sizeof(uint32_t) * (m_new + 1)));
    hipLaunchKernelGGL(k_merge_old, grid_for(m_old), dim3(T), 0, s, g->n_src.as<uint32_t>(),
                       g->n_dst.as<int32_t>(), g->n_ts.as<int64_t>(), m_old, g->plan.as<uint4>(),
                       g->neb_v.as<uint32_t>(), bts, g->an_src.as<uint32_t>(),
                       g->an_dst.as<int32_t>(), g->an_ts.as<int64_t>(), g->gflags.as<uint32_t>());
    hipLaunchKernelGGL(k_merge_new, grid_for(kept), dim3(T), 0, s, bsrc, bdst, bts, kept,
                       g->plan.as<uint4>(), g->neb_v.as<uint32_t>(), g->n_ts.as<int64_t>(),
                       g->an_src.as<uint32_t>(), g->an_dst.as<int32_t>(), g->an_ts.as<int64_t>(),
                       g->gflags.as<uint32_t>());
    TW_HIP(hipGetLastError());
    std::swap(g->n_src, g->an_src);
    std::swap(g->n_dst, g->an_dst);
    std::swap(g->n_ts, g->an_ts);

    // the new active list; nodes left without edges get the empty record
    TW_HIP(ensure(g->act1, sizeof(uint32_t) * (U + 1)));
    TW_HIP(ensure(g->a_eb, sizeof(uint32_t) * (U + 1)));
    TW_HIP(ensure(g->a_cnt, sizeof(uint32_t) * (U + 1)));
    uint32_t* sc_a = u32_slot(g, SLOT_U32_ACTIVE);
    hipLaunchKernelGGL(k_union_active, grid_for(U), dim3(T), 0, s, g->u_node.as<uint32_t>(),
                       g->u_cnt.as<uint32_t>(), (int64_t)U, g->rec.as<NodeRec>(), uflags);
    TW_HIP(scan_exclusive_u32(uflags, upos, U, sc_a, g->ws, s));
    hipLaunchKernelGGL(k_active_compact, grid_for(U), dim3(T), 0, s, uflags, upos, (int64_t)U,
                       g->u_node.as<uint32_t>(), g->u_neb.as<uint32_t>(), g->u_cnt.as<uint32_t>(),
                       g->act1.as<uint32_t>(), g->a_eb.as<uint32_t>(), g->a_cnt.as<uint32_t>());
    TW_HIP(hipGetLastError());
    std::swap(g->act0, g->act1);
    uint32_t A = 0;
    TW_HIP(hipMemcpyAsync(&A, sc_a, sizeof(A), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    g->A = A;
    (void)m_new;
    return TW_OK;
}

// Groups, node records and fences of the active nodes; then one
// synchronisation reads the counts. Gg is taken from the GROUPS slot when
// gg_full, else it is gg_old - gg_evicted + GROUPS (appended groups).
tw_status finish_index(tw_graph* g, bool gg_full, int64_t gg_old, int64_t gg_evicted,
                       Error& err) {
    hipStream_t s = g->stream;
    const int64_t m = g->m, A = g->A;
    TW_HIP(ensure(g->flags, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->idx, sizeof(uint32_t) * (m + 1)));
    TW_HIP(ensure(g->ng_ts, sizeof(int64_t) * (m + 1)));
    TW_HIP(ensure(g->ngo, sizeof(uint2) * (m + 2)));
    TW_HIP(ensure(g->a_gb, sizeof(uint32_t) * (A + 1)));
    TW_HIP(ensure(g->a_foff, sizeof(uint32_t) * (A + 1)));
    TW_HIP(ensure(g->gflags, sizeof(uint32_t) * (m + 1)));
    uint32_t* flags = g->gflags.as<uint32_t>();  // group starts, written by the merge
    uint32_t* Gn = u32_slot(g, SLOT_U32_GN);
    uint32_t* fence_total = u32_slot(g, SLOT_U32_FENCE);
    TW_HIP(ensure(g->a_ge, sizeof(uint32_t) * (A + 1)));

    // (node, timestamp) groups
    TW_HIP(group_starts(flags, g->n_ts.as<int64_t>(), m, 0u, g->ng_ts.as<int64_t>(), nullptr,
                        g->ngo.as<uint2>(), g->n_dst.as<int32_t>(), Gn, g->ws, s));

    // group ranges, fence sizes and offsets of the active nodes
    hipLaunchKernelGGL(k_active_groups, grid_for(A), dim3(T), 0, s, g->a_eb.as<uint32_t>(),
                       g->a_cnt.as<uint32_t>(), A, m, g->ngo.as<uint2>(), Gn,
                       g->a_gb.as<uint32_t>(), g->a_ge.as<uint32_t>(), g->a_foff.as<uint32_t>());
    TW_HIP(scan_exclusive_u32(g->a_foff.as<uint32_t>(), g->a_foff.as<uint32_t>(), A, fence_total,
                              g->ws, s));
    int64_t* summary = i64_slot(g, SLOT_I64_SUMMARY);
    hipLaunchKernelGGL(k_window_summary, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>() + g->e_base,
                       m, summary);
    TW_HIP(hipGetLastError());

    uint32_t host_u32[4];  // GROUPS, GN, UNSORTED, FENCE
    int64_t host_sum[2];
    TW_HIP(hipMemcpyAsync(host_u32, u32_slot(g, SLOT_U32_GROUPS), sizeof(host_u32),
                          hipMemcpyDeviceToHost, s));
    TW_HIP(hipMemcpyAsync(host_sum, summary, sizeof(host_sum), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    g->Gg = gg_full ? (int64_t)host_u32[0] : gg_old - gg_evicted + (int64_t)host_u32[0];
    g->Gn = host_u32[1];
    g->t_min = host_sum[0];
    g->t_max = host_sum[1];
    g->fence_len = host_u32[3];
    TW_HIP(ensure(g->fence, sizeof(int64_t) * (g->fence_len + FENCE_FAN)));

    // records, then the fences
    hipLaunchKernelGGL(k_active_records, grid_for(A), dim3(T), 0, s, g->act0.as<uint32_t>(),
                       g->a_eb.as<uint32_t>(), g->a_cnt.as<uint32_t>(), g->a_gb.as<uint32_t>(),
                       g->a_ge.as<uint32_t>(), g->a_foff.as<uint32_t>(), A,
                       g->ng_ts.as<int64_t>(), g->rec.as<NodeRec>());
    if (g->fence_len > 0)
        hipLaunchKernelGGL(k_fence_fill, grid_for(g->fence_len), dim3(T), 0, s,
                           g->a_foff.as<uint32_t>(), A, g->fence_len, g->act0.as<uint32_t>(),
                           g->rec.as<NodeRec>(), g->ng_ts.as<int64_t>(), g->fence.as<int64_t>());
    TW_HIP(hipGetLastError());
    g->adj_ready = false;
    return TW_OK;
}

}  // namespace

tw_status ingest(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                 int64_t n, tw_ingest_info* info, Error& err) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    const int64_t B = g->directed ? n : 2 * n;  // staged records
    if (g->m + B > (int64_t)UINT32_MAX - 2) {
        err = Error{TW_EINVAL, "window would exceed 2^32 - 2 records"};
        return err.code;
    }
    TW_HIP(ensure(g->b_src, sizeof(int32_t) * (B + 1)));
    TW_HIP(ensure(g->b_dst, sizeof(int32_t) * (B + 1)));
    TW_HIP(ensure(g->b_ts, sizeof(int64_t) * (B + 1)));

    unsigned long long* mm = reinterpret_cast<unsigned long long*>(i64_slot(g, SLOT_I64_MINMAX));
    uint32_t* errf = g->err.as<uint32_t>();
    uint32_t* unsorted = u32_slot(g, SLOT_U32_UNSORTED);
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
    uint32_t* sc_kept = u32_slot(g, SLOT_U32_KEPT);
    uint32_t* sc_ev = u32_slot(g, SLOT_U32_EVICTED);
    uint32_t* sc_gev = u32_slot(g, SLOT_U32_GG_EVICTED);
    int64_t* first_kept = i64_slot(g, SLOT_I64_FIRST_KEPT);
    const bool drop = windowed && B > 0 && bmin < cut;
    const bool evicting = windowed && g->m > 0 && g->t_min < cut;
    int64_t kept = B, evicted = 0, gg_evicted = 0, batch_first = bmin, drop_lo = 0;
    const int64_t key_base = drop ? cut : bmin;
    uint64_t* keys = nullptr;
    uint32_t* vals = nullptr;
    if (drop && sorted) {
        // late records of a sorted batch are a prefix
        hipLaunchKernelGGL(k_sorted_cut, dim3(1), dim3(1), 0, s, s_ts, B, cut, sc_kept,
                           first_kept);
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
            TW_HIP(scan_exclusive_u32(fl, pos, B, sc_kept, g->ws, s));
            hipLaunchKernelGGL(k_make_keys, grid_for(B), dim3(T), 0, s, s_ts, B, key_base, fl,
                               pos, keys, vals);
        } else {
            hipLaunchKernelGGL(k_make_keys, grid_for(B), dim3(T), 0, s, s_ts, B, key_base, nullptr,
                               nullptr, keys, vals);
        }
    }
    if (evicting) {
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>() + g->e_base,
                           g->m, cut, sc_ev);
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s,
                           g->gg_ts.as<int64_t>() + g->gg_base, g->Gg, cut, sc_gev);
    }
    TW_HIP(hipGetLastError());
    if (drop || evicting) {
        uint32_t h2[2] = {0, 0}, hg = 0;
        int64_t hf = INT64_MAX;
        TW_HIP(hipMemcpyAsync(h2, sc_kept, sizeof(h2), hipMemcpyDeviceToHost, s));
        TW_HIP(hipMemcpyAsync(&hg, sc_gev, sizeof(hg), hipMemcpyDeviceToHost, s));
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
        if (evicting) {
            evicted = h2[1];
            gg_evicted = hg;
        }
    }

    // the kept batch records in timestamp order (stable)
    const int32_t* q_src = s_src + drop_lo;
    const int32_t* q_dst = s_dst + drop_lo;
    const int64_t* q_ts = s_ts + drop_lo;
    if (!sorted && kept > 0) {
        int kb = bits_for((uint64_t)(bmax - key_base));
        TW_HIP(radix_sort_u64(keys, vals, kept, 0, kb, g->ws, s));
        TW_HIP(ensure(g->q_src, sizeof(int32_t) * (kept + 1)));
        TW_HIP(ensure(g->q_dst, sizeof(int32_t) * (kept + 1)));
        TW_HIP(ensure(g->q_ts, sizeof(int64_t) * (kept + 1)));
        hipLaunchKernelGGL(k_gather_batch, grid_for(kept), dim3(T), 0, s, vals, kept, s_src, s_dst,
                           s_ts, g->q_src.as<int32_t>(), g->q_dst.as<int32_t>(),
                           g->q_ts.as<int64_t>());
        q_src = g->q_src.as<int32_t>();
        q_dst = g->q_dst.as<int32_t>();
        q_ts = g->q_ts.as<int64_t>();
    }

    // timestamp view: a batch that starts at or after the window's last
    // timestamp is appended in place (eviction only moves e_base); any other
    // batch is merged (merge path, older records first on equal timestamps)
    const int64_t m_old = g->m;
    const int64_t na = m_old - evicted;
    const int64_t m_new = na + kept;
    const bool append = na == 0 || kept == 0 || batch_first >= g->t_max;
    const int64_t last_ts = g->t_max;
    const int64_t gg_old = g->Gg;
    bool gg_full = false;
    if (append) {
        g->e_base += evicted;
        g->gg_base += gg_evicted;
        if (na == 0) {
            g->e_base = 0;
            g->gg_base = 0;
        }
        g->m = na;
        if (g->e_base + m_new > g->e_cap) {
            if (m_new <= g->e_cap && g->m > 0) {
                // compact to the front of the alternate buffers
                TW_HIP(hipMemcpyAsync(g->a_src.p, g->e_src.as<int32_t>() + g->e_base, 4 * na,
                                      hipMemcpyDeviceToDevice, s));
                TW_HIP(hipMemcpyAsync(g->a_dst.p, g->e_dst.as<int32_t>() + g->e_base, 4 * na,
                                      hipMemcpyDeviceToDevice, s));
                TW_HIP(hipMemcpyAsync(g->a_ts.p, g->e_ts.as<int64_t>() + g->e_base, 8 * na,
                                      hipMemcpyDeviceToDevice, s));
                std::swap(g->e_src, g->a_src);
                std::swap(g->e_dst, g->a_dst);
                std::swap(g->e_ts, g->a_ts);
                g->e_base = 0;
            } else if (reserve_window(g, m_new, err) != TW_OK) {
                return err.code;
            }
            gg_full = true;
        }
        if (kept > 0) {
            const int64_t at = g->e_base + na;
            TW_HIP(hipMemcpyAsync(g->e_src.as<int32_t>() + at, q_src, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->e_dst.as<int32_t>() + at, q_dst, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->e_ts.as<int64_t>() + at, q_ts, 8 * kept,
                                  hipMemcpyDeviceToDevice, s));
        }
        g->m = m_new;
        if (gg_full || na == 0) {
            gg_full = true;
            if (build_ts_groups(g, err) != TW_OK) return err.code;
        } else if (kept > 0) {
            TW_HIP(ensure(g->flags, sizeof(uint32_t) * (kept + 1)));
            uint32_t* fl = g->flags.as<uint32_t>();
            uint32_t* G = u32_slot(g, SLOT_U32_GROUPS);
            const int64_t gpos = g->gg_base + (gg_old - gg_evicted);
            hipLaunchKernelGGL(k_append_group_flags, grid_for(kept), dim3(T), 0, s, q_ts, kept,
                               last_ts, 1, fl);
            TW_HIP(group_starts(fl, q_ts, kept, (uint32_t)(g->e_base + na),
                                g->gg_ts.as<int64_t>() + gpos, g->gg_off.as<uint32_t>() + gpos,
                                nullptr, nullptr, G, g->ws, s));
        } else {
            // eviction only: the groups keep their offsets
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(T), 0, s, u32_slot(g, SLOT_U32_GROUPS), 1,
                               0u);
        }
    } else {
        if (reserve_window(g, m_new, err) != TW_OK) return err.code;
        const int64_t from = g->e_base + evicted;
        hipLaunchKernelGGL(k_merge, grid_for(m_new, MP_ITEMS), dim3(T), 0, s,
                           g->e_src.as<int32_t>() + from, g->e_dst.as<int32_t>() + from,
                           g->e_ts.as<int64_t>() + from, na, q_src, q_dst, q_ts, kept,
                           g->a_src.as<int32_t>(), g->a_dst.as<int32_t>(), g->a_ts.as<int64_t>());
        TW_HIP(hipGetLastError());
        std::swap(g->e_src, g->a_src);
        std::swap(g->e_dst, g->a_dst);
        std::swap(g->e_ts, g->a_ts);
        g->e_base = 0;
        g->m = m_new;
        gg_full = true;
        if (build_ts_groups(g, err) != TW_OK) return err.code;
    }

    // node view: per-node merge of the surviving runs with the batch
    if (merge_node_view(g, q_src, q_dst, q_ts, kept, m_old, m_new, evicting, cut, err) != TW_OK)
        return err.code;
    if (finish_index(g, gg_full, gg_old, gg_evicted, err) != TW_OK) return err.code;

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
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    int64_t ev = 0, gev = 0;
    if (g->m > 0 && g->t_min < cutoff) {
        uint32_t* sc_ev = u32_slot(g, SLOT_U32_EVICTED);
        uint32_t* sc_gev = u32_slot(g, SLOT_U32_GG_EVICTED);
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>() + g->e_base,
                           g->m, cutoff, sc_ev);
        hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1), 0, s,
                           g->gg_ts.as<int64_t>() + g->gg_base, g->Gg, cutoff, sc_gev);
        uint32_t h[2] = {0, 0};
        TW_HIP(hipMemcpyAsync(&h[0], sc_ev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TW_HIP(hipMemcpyAsync(&h[1], sc_gev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TW_HIP(hipStreamSynchronize(s));
        ev = h[0];
        gev = h[1];
    }
    if (ev > 0) {
        const int64_t m_old = g->m, gg_old = g->Gg;
        g->e_base += ev;
        g->gg_base += gev;
        g->m = m_old - ev;
        bool gg_full = false;
        if (g->m == 0) {
            g->e_base = 0;
            gg_full = true;
            if (build_ts_groups(g, err) != TW_OK) return err.code;
        } else {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(T), 0, s, u32_slot(g, SLOT_U32_GROUPS), 1,
                               0u);
        }
        if (merge_node_view(g, nullptr, nullptr, nullptr, 0, m_old, g->m, true, cutoff, err) !=
            TW_OK)
            return err.code;
        if (finish_index(g, gg_full, gg_old, gev, err) != TW_OK) return err.code;
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
    if (reserve_window(g, 1024, err) != TW_OK) return err.code;
    TW_HIP(ensure(g->n_src, sizeof(uint32_t) * 2));
    TW_HIP(ensure(g->n_dst, sizeof(int32_t) * 2));
    TW_HIP(ensure(g->n_ts, sizeof(int64_t) * 2));
    g->m = 0;
    g->A = 0;
    TW_HIP(ensure(g->rec, sizeof(NodeRec) * g->V));
    TW_HIP(ensure(g->act0, sizeof(uint32_t) * 2));
    hipLaunchKernelGGL(k_fill_empty_rec, grid_for(g->V), dim3(T), 0, g->stream,
                       g->rec.as<NodeRec>(), (int64_t)g->V);
    if (build_ts_groups(g, err) != TW_OK) return err.code;
    return finish_index(g, true, 0, 0, err);
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
    TW_HIP(cp(src, g->e_src.as<int32_t>() + g->e_base, sizeof(int32_t) * m));
    TW_HIP(cp(dst, g->e_dst.as<int32_t>() + g->e_base, sizeof(int32_t) * m));
    TW_HIP(cp(ts, g->e_ts.as<int64_t>() + g->e_base, sizeof(int64_t) * m));
    TW_HIP(cp(g_ts, g->gg_ts.as<int64_t>() + g->gg_base, sizeof(int64_t) * g->Gg));
    TW_HIP(cp(n_dst, g->n_dst.p, sizeof(int32_t) * m));
    TW_HIP(cp(n_ts, g->n_ts.p, sizeof(int64_t) * m));
    TW_HIP(cp(n_gts, g->ng_ts.p, sizeof(int64_t) * g->Gn));
    if (g_off)
        hipLaunchKernelGGL(k_widen, grid_for(g->Gg + 1), dim3(T), 0, s,
                           g->gg_off.as<uint32_t>() + g->gg_base, g->Gg + 1, g_off, g->e_base);
    if (n_goff)
        hipLaunchKernelGGL(k_widen2, grid_for(g->Gn + 1), dim3(T), 0, s, g->ngo.as<uint2>(),
                           g->Gn + 1, n_goff);
    if (n_ebeg || n_gbeg)
        hipLaunchKernelGGL(k_export_nodes, grid_for(g->V + 1), dim3(T), 0, s,
                           g->rec.as<NodeRec>(), g->act0.as<uint32_t>(), g->A, g->V, m, g->Gn,
                           n_ebeg, n_gbeg);
    TW_HIP(hipGetLastError());
    TW_HIP(hipStreamSynchronize(s));
    return TW_OK;
}

}  // namespace tw
