// Internal declarations of the MI355X temporal-walk library: graph state,
// device buffers and the primitives shared between the ingest and walk
// translation units. Not part of the public ABI (include/tw.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "tw.h"

namespace tw {

constexpr int64_t TS_NONE = INT64_MIN;

// One record per node, 32 bytes so a hop reads all of it with one
// contiguous load: the node's range of (node, timestamp) groups [gb, ge),
// its edge range [eb, ee) in the node view, where its fence levels start in
// the fence array and how many there are, and the last group timestamp
// (t_last lets a hop that cannot continue stop without searching).
struct alignas(32) NodeRec {
    uint32_t gb, ge, eb, ee;
    uint32_t fence_off, levels;
    int64_t t_last;
};

// Fence index. A node's groups [gb, ge) split into a head [gb, a0), where
// a0 is the first group index that is a multiple of FENCE_FAN, and a body
// [a0, ge). When the body has more than FENCE_FAN groups, fence level k
// (k = 1..K) holds the timestamps of groups a0 + i FENCE_FAN^k, padded to a
// multiple of FENCE_FAN entries with INT64_MAX, stored top level (K) first;
// K is the smallest level with at most FENCE_FAN entries. A search reads one
// FENCE_FAN-entry window (one aligned 128-byte line) per level and one
// aligned window of the group timestamps.
constexpr int FENCE_FAN = 8;
constexpr int FENCE_LOG = 3;

// most levels a fence can have: group indices are 32-bit
constexpr int FENCE_MAX_LEVELS = (32 + FENCE_LOG - 1) / FENCE_LOG + 1;
static_assert((1 << FENCE_LOG) == FENCE_FAN, "FENCE_FAN must be 2^FENCE_LOG");

struct FenceGeom {
    uint32_t a0;      // first aligned group of the body
    uint32_t levels;  // K (0: no fence, the node is scanned directly)
    uint32_t size;    // fence entries
};

__host__ __device__ inline FenceGeom fence_geometry(uint32_t gb, uint32_t ge) {
    FenceGeom f;
    f.a0 = (gb + FENCE_FAN - 1) & ~(uint32_t)(FENCE_FAN - 1);
    f.levels = 0;
    f.size = 0;
    const uint64_t body = ge > f.a0 ? (uint64_t)(ge - f.a0) : 0;
    if (body > (uint64_t)FENCE_FAN) {
        uint64_t n = body;
        do {
            n = (n + FENCE_FAN - 1) / FENCE_FAN;
            ++f.levels;
            f.size += (uint32_t)((n + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN);
        } while (n > (uint64_t)FENCE_FAN);
    }
    return f;
}

// Slots of the graph's device scalar buffer (256 bytes): u32 indices
// (SLOT_U32_*) and int64 indices (SLOT_I64_*).
constexpr int SLOT_I64_MINMAX = 0;     // batch min / max timestamp (ordered u64) in [0], [1]
constexpr int SLOT_U32_GROUPS = 4;     // groups counted by the last timestamp-group scan
constexpr int SLOT_U32_GN = 5;         // node-timestamp groups
constexpr int SLOT_U32_UNSORTED = 6;   // batch not in timestamp order
constexpr int SLOT_U32_FENCE = 7;      // fence entries
constexpr int SLOT_I64_SUMMARY = 4;    // [4] t_min, [5] t_max of the window
constexpr int SLOT_U32_KEPT = 24;      // kept batch records / late-prefix length
constexpr int SLOT_U32_EVICTED = 25;   // evicted window records
constexpr int SLOT_I64_FIRST_KEPT = 13;
constexpr int SLOT_U32_N_LIVE = 28;    // live walks (cooperative dispatch)
constexpr int SLOT_U32_GG_EVICTED = 29;
constexpr int SLOT_U32_RUNS = 30;      // source runs of the batch
constexpr int SLOT_U32_UNION = 31;     // union of active nodes and batch sources
constexpr int SLOT_U32_ACTIVE = 32;    // active nodes
constexpr int SLOT_U32_BIG = 33;       // queued large fences
constexpr int SCALAR_BYTES = 256;

// A grow-only device allocation.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Error carried up to the C ABI.
struct Error {
    tw_status code;
    std::string msg;
};

hipError_t ensure(DevBuf& b, size_t bytes);  // keeps contents only if no growth
void release(DevBuf& b);

// Scratch space reused by the primitives.
struct Workspace {
    DevBuf scan_part;   // scan partial sums
    DevBuf hist;        // radix histograms
    DevBuf keys_alt, vals_alt, v64_alt;
    DevBuf misc;        // small scalars
};

// -------------------------------------------------------------- primitives

// out[i] = sum_{j<i} in[i]; total (device scalar, nullable) = sum of all.
// n may be 0. in and out may alias.
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                              Workspace& ws, hipStream_t s);

// Groups of a sequence: the k-th position i that starts a group (flags[i]
// != 0, or with flags null, ts[i] != ts[i-1]) gives g_ts[k] = ts[i] and
// g_off[k] = pos_base + i; g_off[total] = pos_base + n; total (device) = the
// number of groups. n may be 0.
// With g_od non-null, g_od[k] = {pos_base + i, dst[i]} replaces g_off.
hipError_t group_starts(const uint32_t* flags, const int64_t* ts, int64_t n, uint32_t pos_base,
                        int64_t* g_ts, uint32_t* g_off, uint2* g_od, const int32_t* dst,
                        uint32_t* total, Workspace& ws, hipStream_t s);

// Stable LSD radix sort of (keys, vals) by bits [bit_lo, bit_hi) of the key.
// vals may be null. Result ends in keys / vals. The alternate buffers come
// from the workspace.
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bit_lo, int bit_hi,
                          Workspace& ws, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bit_lo, int bit_hi,
                          Workspace& ws, hipStream_t s);
// Stable sort of (kin, vin, win) by bits [bit_lo, bit_hi) of kin into
// (kout, vout, wout), carrying a 32-bit and a 64-bit payload (either may be
// null). The inputs are only read; no pass writes into them unless they are
// the outputs.
hipError_t radix_sort_u32_kv(const uint32_t* kin, const uint32_t* vin, const uint64_t* win,
                             uint32_t* kout, uint32_t* vout, uint64_t* wout, int64_t n, int bit_lo,
                             int bit_hi, Workspace& ws, hipStream_t s);

// Bits needed to represent values in [0, x].
inline int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace tw

// --------------------------------------------------------------- graph

struct tw_graph {
    int32_t V = 0;
    bool directed = true;
    int64_t window = 0;
    hipStream_t stream = nullptr;
    int device = 0;

    bool has_time = false;
    int64_t t_now = 0;

    // host mirrors of the index sizes. The window occupies positions
    // [e_base, e_base + m) of the edge-store buffers (capacity e_cap); its
    // timestamp groups occupy [gg_base, gg_base + Gg) of gg_ts / gg_off, whose
    // offsets are edge-store buffer positions.
    int64_t m = 0, Gg = 0, Gn = 0;
    int64_t e_base = 0, e_cap = 0, gg_base = 0;
    int64_t t_min = 0, t_max = 0;
    tw_ingest_info last{};

    // timestamp view (the edge store) and its alternate for merges
    tw::DevBuf e_src, e_dst, e_ts, a_src, a_dst, a_ts;
    tw::DevBuf gg_ts, gg_off;          // global timestamp groups
    tw::DevBuf n_dst, n_ts;            // node-and-timestamp view
    tw::DevBuf an_src, an_dst, an_ts;  // its alternate for the merge
    tw::DevBuf bs_src, bs_dst, bs_ts;  // batch sorted by source
    tw::DevBuf q_src, q_dst, q_ts;     // batch sorted by timestamp (unsorted input)
    tw::DevBuf plan, neb_v;            // per-node merge plan / merged offset (union nodes)
    tw::DevBuf act0, act1;             // sorted active nodes (current, scratch)
    int64_t A = 0;                     // active nodes
    tw::DevBuf a_eb, a_cnt, a_gb, a_ge, a_foff;   // per active node
    tw::DevBuf gflags;                 // (node, timestamp) group starts of the node view
    tw::DevBuf it_keys, it_pay, it_skeys, it_spay;  // union items
    tw::DevBuf u_flags, u_pos, u_node, u_cnt, u_neb;  // union nodes
    tw::DevBuf ng_ts, ngo;             // its (node, timestamp) groups: timestamps,
                                       // {first edge, destination of the first edge}
    tw::DevBuf n_src;                  // source of each node-view edge (build temp)
    tw::DevBuf fence;                  // fence levels of nodes with many groups
    int64_t fence_len = 0;
    tw::DevBuf rec;                    // NodeRec[V]
    tw::DevBuf adj;                    // per-node dst sorted ascending (node2vec)
    bool adj_ready = false;

    // cooperative dispatch: per-walk state, live list, sort buffers
    tw::DevBuf c_node0, c_walk0, c_t0, c_node1, c_walk1, c_t1, c_node2, c_walk2, c_t2;
    tw::DevBuf c_prev, c_flags, c_pos;
    uint32_t coop_panel = 4096;        // LDS panel entries per workgroup

    // batch staging
    tw::DevBuf b_src, b_dst, b_ts, b_keys, b_vals, b_flags;
    tw::DevBuf flags, idx;             // per-edge temporaries
    tw::DevBuf err;                    // device error flags (uint32)
    tw::DevBuf scal;                   // device scalars
    tw::Workspace ws;
};

namespace tw {

// index.hip
tw_status ingest(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                 int64_t n, tw_ingest_info* info, Error& err);
tw_status evict_before(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err);
tw_status build_adjacency(tw_graph* g, Error& err);
tw_status init_empty(tw_graph* g, Error& err);  // empty index for a graph never ingested
tw_status export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                       int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                       int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg, Error& err);

// walk.hip
tw_status sample_walks(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                       int32_t* len, Error& err);

}  // namespace tw

#define TW_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = tw::Error{e_ == hipErrorOutOfMemory ? TW_ENOMEM : TW_EDEVICE,       \
                            std::string(#call) + ": " + hipGetErrorString(e_)};       \
            return err.code;                                                          \
        }                                                                             \
    } while (0)
