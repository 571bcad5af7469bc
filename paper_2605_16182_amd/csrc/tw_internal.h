// Internal declarations of the MI355X temporal-walk library: graph state,
// device buffers and the primitives shared between the ingest and walk
// translation units. Not part of the public ABI (include/tw.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cmath>
#include <string>
#include <vector>

#include "tw.h"

namespace tw {

constexpr int64_t TS_NONE = INT64_MIN;

// One (node, timestamp) group of the node view, 16 bytes: the timestamp,
// the pool position of the group's first edge and that edge's destination,
// with the sign bit set when the group holds that edge only (a pick of a
// one-edge group needs neither the next record nor an edge load).
struct alignas(16) GroupRec {
    int64_t ts;
    uint32_t first;
    int32_t dst;
};

// One record per node, 48 bytes, read at the start of every hop (three
// independent 16-byte loads). A node's edges
// and groups live in a segment of the edge and group pools: the live groups
// are [gb, ge), the live edges end at ee (they start at the first edge of
// group gb). g0 is the segment's first group (a multiple of FENCE_FAN), the
// origin of the node's fence; fence_off is where the fence starts in the
// fence pool; lv = levels in use | (capacity code << 8) | (key shift << 16),
// the segment holding FENCE_FAN << code groups. t_last is the last live
// timestamp (INT64_MIN for a node without edges), so a hop that cannot
// continue stops after this load. kbase is the fence's key base (the
// segment's first group timestamp): with the shift here, a search needs no
// load before its first fence window.
struct alignas(16) NodeRec {
    uint32_t gb, ge, g0, ee;
    uint32_t fence_off, lv;
    int64_t t_last;
    int64_t kbase;
    int64_t pad;
};
static_assert(sizeof(NodeRec) == 48, "three 16-byte loads");
__host__ __device__ inline uint32_t rec_levels(uint32_t lv) { return lv & 0xffu; }
__host__ __device__ inline uint32_t rec_code(uint32_t lv) { return (lv >> 8) & 0xffu; }
__host__ __device__ inline uint32_t rec_shift(uint32_t lv) { return (lv >> 16) & 0xffu; }

// Fence index with 32-bit keys. A segment of capacity C > FENCE_FAN groups
// has a fence of levels k = 0..K(C) (key base and shift are in the node
// record): level k
// holds the keys of groups g0 + i FENCE_FAN^k, i < ceil(C / FENCE_FAN^k),
// padded to a multiple of FENCE_FAN words; key(g) = (ts(g) - base) >> shift,
// and unwritten entries hold UINT32_MAX. Ingest keeps every key of a segment
// below UINT32_MAX (a batch that would not fit rewrites the segment with a
// new base and shift). Keys are monotone in the timestamp; where a key equals
// the query's, the group's own timestamp decides. A search over the groups
// [g0, ge) starts at level K(ge - g0), the smallest level with at most
// FENCE_FAN entries in use, and reads one FENCE_FAN-word window (32 bytes,
// two 16-byte loads) per level down to level 0. Groups evicted from the
// front of the segment stay in place until the segment is rewritten; their
// timestamps precede every live one. Segments of at most FENCE_FAN groups
// have no fence: their few groups are counted directly.
constexpr int FENCE_FAN = 8;
constexpr int FENCE_LOG = 3;

// most levels a fence can have: group indices are 32-bit
constexpr int FENCE_MAX_LEVELS = (32 + FENCE_LOG - 1) / FENCE_LOG + 1;
static_assert((1 << FENCE_LOG) == FENCE_FAN, "FENCE_FAN must be 2^FENCE_LOG");

// levels above level 0 needed for n groups: 0 when n <= FENCE_FAN
__host__ __device__ inline int fence_levels(uint64_t n) {
    int k = 0;
    while (n > (uint64_t)FENCE_FAN) {
        n = (n + FENCE_FAN - 1) >> FENCE_LOG;
        ++k;
    }
    return k;
}

// words stored for level k (k >= 0) of a segment of cap groups
__host__ __device__ inline uint32_t fence_level_len(uint64_t cap, int k) {
    const uint64_t n = (cap + (1ull << (FENCE_LOG * k)) - 1) >> (FENCE_LOG * k);
    return (uint32_t)((n + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN);
}

// total fence words of a segment of cap groups (0: no fence)
__host__ __device__ inline uint32_t fence_cap(uint64_t cap) {
    if (cap <= (uint64_t)FENCE_FAN) return 0;
    uint32_t s = 0;
    const int K = fence_levels(cap);
    for (int k = 0; k <= K; ++k) s += fence_level_len(cap, k);
    return s;
}

// word offset of level k inside a segment's fence
__host__ __device__ inline uint32_t fence_level_off(uint64_t cap, int k) {
    uint32_t off = 0;
    for (int j = 0; j < k; ++j) off += fence_level_len(cap, j);
    return off;
}

// key shift for a segment whose keys must reach span (keep a 4x margin for
// later appends before a rewrite)
__host__ __device__ inline uint32_t fence_shift(uint64_t span) {
    uint32_t s = 0;
    while ((span >> s) >= (1ull << 30)) ++s;
    return s;
}

// Workgroups of a launch go to the chip's 8 XCDs in turn (workgroup i to
// XCD i mod 8), each XCD with its own L2. Tile index of workgroup bid among
// nb such that every XCD takes one contiguous range of tiles: neighbouring
// tiles then share an L2, and partial cache lines at the ends of their
// output runs merge there before they are written back.
constexpr uint32_t NUM_XCD = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nb) {
    const uint32_t x = bid % NUM_XCD, q = bid / NUM_XCD;
    const uint32_t per = nb / NUM_XCD, rem = nb % NUM_XCD;
    return x * per + (x < rem ? x : rem) + q;
}

__host__ __device__ inline uint64_t seg_groups(uint32_t code) {
    return (uint64_t)FENCE_FAN << code;
}

// node2vec adjacency: an open-addressing table (linear probing) of the
// window's (source, destination) pairs, each with its record count; a pair
// whose count fell to 0 keeps its slot until the table is rebuilt.
struct __align__(16) AdjSlot {
    uint64_t key;  // source << 32 | destination, or ADJ_EMPTY
    uint32_t cnt;
    uint32_t pad;
};
constexpr uint64_t ADJ_EMPTY = ~0ull;

__host__ __device__ inline uint64_t adj_key(int32_t src, int32_t dst) {
    return ((uint64_t)(uint32_t)src << 32) | (uint32_t)dst;
}

// the SplitMix64 output mix (Steele, Lea, Flood, OOPSLA 2014)
__host__ __device__ inline uint64_t adj_hash(uint64_t k) {
    k = (k ^ (k >> 30)) * 0xBF58476D1CE4E5B9ull;
    k = (k ^ (k >> 27)) * 0x94D049BB133111EBull;
    return k ^ (k >> 31);
}

// Slots of the graph's device scalar buffer (256 bytes): u32 indices
// (SLOT_U32_*) and int64 indices (SLOT_I64_*, byte offset 8 k).
constexpr int SLOT_I64_MINMAX = 0;     // batch min / max timestamp (ordered u64) in [0], [1]
constexpr int SLOT_U32_GROUPS = 4;     // groups counted by the last timestamp-group scan
constexpr int SLOT_U32_UNSORTED = 6;   // batch not in timestamp order
constexpr int SLOT_I64_SUMMARY = 4;    // [4] t_min, [5] t_max of the window
constexpr int SLOT_I64_GG = 6;         // global timestamp groups of the window
constexpr int SLOT_I64_WIN = 7;        // [7] e_base, [8] m, [9] gg_base of the timestamp view
constexpr int SLOT_U32_KEPT = 24;      // kept batch records / late-prefix length
constexpr int SLOT_U32_EVICTED = 25;   // evicted window records
constexpr int SLOT_I64_FIRST_KEPT = 13;
constexpr int SLOT_U32_N_LIVE = 28;    // live walks (cooperative dispatch)
constexpr int SLOT_U32_GG_EVICTED = 29;
constexpr int SLOT_U32_RUNS = 30;      // source runs of the batch (node-view jobs)
constexpr int SLOT_U32_EV_NODES = 31;  // nodes touched only by eviction
constexpr int SLOT_U32_ACTIVE = 32;    // other active nodes (full rewrite)
constexpr int SLOT_U32_OUT = 33;       // node-view edges written by the jobs
constexpr int SLOT_U32_REQ_E = 34;     // edge slots requested by new segments
constexpr int SLOT_U32_REQ_G = 35;     // group slots requested
constexpr int SLOT_U32_REQ_F = 36;     // fence entries requested
constexpr int SLOT_U32_FENCE_W = 37;   // fence entries written by the jobs
constexpr int SLOT_U32_GN = 38;        // node-view groups (counted on demand)
constexpr int SLOT_U32_EXP_E = 39;     // export: edges
constexpr int SLOT_U32_W_GROUPS = 40;  // live groups counted by the weight build
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

// Room for `bytes` in b, growing it in the order of stream s (contents are
// kept only if it does not grow; a failed growth leaves b unchanged).
hipError_t ensure(DevBuf& b, size_t bytes, hipStream_t s);
// Returns b's block to the device pool after the work enqueued on s.
void release(DevBuf& b, hipStream_t s);

// Scratch space reused by the primitives.
struct Workspace {
    DevBuf scan_part;   // scan partial sums
    DevBuf hist;        // radix histograms
    DevBuf keys_alt, vals_alt, v64_alt;
    DevBuf tiles;       // per-tile counts of the two-pass compaction
};

// -------------------------------------------------------------- primitives

// out[i] = sum_{j<i} in[i]; total (device scalar, nullable) = sum of all.
// n may be 0. in and out may alias.
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                              Workspace& ws, hipStream_t s);

// The same scan with caller-provided room for its partial sums (at least
// scan_parts_u32(n) words at part): it allocates nothing.
int64_t scan_parts_u32(int64_t n);
hipError_t scan_exclusive_u32_into(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                   uint32_t* part, hipStream_t s);

// Four exclusive u32 scans of n elements at once (in[k] and out[k] may
// alias); total[k] (device, nullable) receives the sum of array k.
// n_dev (nullable): the arrays hold n_dev[0] + n_dev[1] elements, counted on
// the device and at most n
hipError_t scan_exclusive_u32x4(const uint32_t* const in[4], uint32_t* const out[4],
                                uint32_t* const total[4], int64_t n, Workspace& ws,
                                hipStream_t s, const uint32_t* n_dev = nullptr);

// out[i] = sum_{j<i} in[j] in 64 bits (in >= 0); total (nullable) = the sum.
hipError_t scan_exclusive_i32_to_u64(const int32_t* in, uint64_t* out, int64_t n, uint64_t* total,
                                     Workspace& ws, hipStream_t s);

// Groups of a sequence of timestamps: the k-th position i that starts a group
// (ts[i] != ts[i-1]; position 0 always, or with has_last, when ts[0] !=
// last_ts, the timestamp before the sequence) gives g_off[k] = pos_base + i;
// g_off[total] = pos_base + n; total (device) = the number of groups. A
// group's timestamp is that of its first position. n may be 0. counted
// (nullable) already holds the group starts of every tile of GS_TILE
// positions (k_stage_count), for the same has_last and last_ts.
constexpr int GS_TILE = 4096;
hipError_t group_starts(int has_last, int64_t last_ts, const int64_t* ts, int64_t n,
                        uint32_t pos_base, uint32_t* g_off, uint32_t* total, Workspace& ws,
                        hipStream_t s, DevBuf* counted = nullptr);

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
// The same sort with the 32-bit and 64-bit payloads leaving packed as one:
// pout[i] = (win - base) << 32 | vin (win - base must fit 32 bits). Fewer
// bytes move in every pass after the first.
hipError_t radix_sort_u32_pack(const uint32_t* kin, const uint32_t* vin, const uint64_t* win,
                               uint64_t base, uint32_t* kout, uint64_t* pout, int64_t n,
                               int bit_lo, int bit_hi, Workspace& ws, hipStream_t s);

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
    // set while an ingest or eviction changes the index in place; still set
    // after one that failed midway, which leaves the graph unusable
    bool broken = false;

    // host mirrors of the index sizes. The window occupies positions
    // [e_base, e_base + m) of the edge-store buffers (capacity e_cap); its
    // timestamp groups occupy [gg_base, gg_base + Gg] of gg_off: edge-store
    // buffer positions of each group's first record (and the end); a group's
    // timestamp is that record's, and t_min / t_max are the window's first
    // and last timestamps.
    int64_t m = 0, Gg = 0;
    int64_t e_base = 0, e_cap = 0, gg_base = 0;
    int64_t t_min = 0, t_max = 0;
    // Gg, t_min and t_max of an update are computed on the device (scalar
    // slots SLOT_I64_GG, SLOT_I64_SUMMARY) and reach these mirrors with the
    // next read-back of the slots (sum_stale until then); t_min_lb is a
    // host-known lower bound of the window's first timestamp meanwhile
    bool sum_stale = false;
    int64_t t_min_lb = INT64_MIN;
    tw_ingest_info last{};

    // timestamp view (the edge store) and its alternate for merges
    tw::DevBuf e_src, e_dst, e_ts, a_src, a_dst, a_ts;
    tw::DevBuf gg_off;                 // global timestamp groups
    tw::DevBuf gs_tiles;               // group starts per tile of a staged batch

    // node view: per-node segments of the edge pool (n_dst, n_ts), the
    // group pool (ng, GroupRec) and the fence pool (fence). New segments are
    // taken from the top of each pool; when a pool is full every active node
    // is rewritten into the alternate pools (an_*), which then swap in.
    tw::DevBuf n_dst, n_ts, ng, fence;  // fence: uint32 words
    tw::DevBuf an_dst, an_ts, ang, afence;
    int64_t pe_top = 0, pe_cap = 0, pg_top = 0, pg_cap = 0, pf_top = 0, pf_cap = 0;
    uint32_t pool_gen = 1;             // segments of older generations are void
    tw::DevBuf rec;                    // NodeRec[V]
    tw::DevBuf seg;                    // SegRec[V] (ingest only)
    tw::DevBuf touched;                // u32[V]: epoch of the last ingest that touched v
    uint32_t epoch = 0;
    // node-view jobs (one per touched node) and their temporaries
    tw::DevBuf bs_src, bs_dst, bs_ts;  // batch sorted by source
    bool bs_packed = false;            // bs_ts holds (ts - bs_base) << 32 | dst
    int64_t bs_base = 0;
    tw::DevBuf q_src, q_dst, q_ts;     // batch sorted by timestamp (unsorted input)
    tw::DevBuf c_node, c_bf, c_be;     // job candidates: node, batch run
    tw::DevBuf jobs, j_cnt, j_off, j_re, j_rg, j_rf, j_fw;
    tw::DevBuf o_flag, o_rank;         // per written edge: group start, rank
    tw::DevBuf o_tf, f_tf;             // first job of every tile of written edges, fence words
    int64_t T = 0;         // at most this many jobs collected for the next update; their
                           // count is on the device (SLOT_U32_RUNS + SLOT_U32_EV_NODES)
    int64_t jobs_last = 0; // jobs of the last update (sizes the next plan's launches)
    // counters of the last update: jobs, edges written, edge slots of new
    // segments, whether every active node was rewritten
    int64_t st_jobs = 0, st_written = 0, st_new_slots = 0, st_full = 0;
    // node2vec: the pair table (adj_mask + 1 slots, a power of two), valid
    // for the current window while adj_ready; adj_used bounds the slots
    // holding a key (the pairs inserted since the build, with repeats)
    tw::DevBuf adj_tab;
    uint64_t adj_mask = 0;
    int64_t adj_used = 0;
    bool adj_ready = false;
    // weight-based picker: cumulative group weights (group pool slots) for
    // the time scale w_scale, valid while w_ready
    tw::DevBuf cw, w_tiles;
    bool w_ready = false;
    double w_scale = 0.0;
    // the time scale whose weights every ingest and eviction rebuilds (NaN:
    // none; the first weight-based walk after a change builds them)
    double ingest_weight_tau = NAN;
    // backward walks of a directed graph: the in-view, a graph fed every
    // batch with source and destination swapped (null until first needed)
    tw_graph* rev = nullptr;

    // cooperative dispatch: per-walk state, live list, sort buffers
    tw::DevBuf c_node0, c_walk0, c_t0, c_node1, c_walk1, c_t1, c_node2, c_walk2, c_t2;
    tw::DevBuf c_prev, c_flags, c_pos;
    // tunables of the cooperative dispatch (tw_autotune sets them): LDS
    // panel entries per workgroup, lanes of a wavefront at one node that
    // engage the wavefront tier, regroup per step (0: stable sort by node,
    // 1: none), steps between read-backs of the live count
    uint32_t coop_panel = 4096;
    int coop_wave_min = 64;
    int coop_regroup = 0;
    int coop_sync = 1;
    // queue dispatch: slice counters; compute units; the dispatch AUTO runs
    // (0: full-walk until tw_autotune chooses) and the queue's workgroups per CU
    tw::DevBuf wq;
    int cu_count = 0, queue_bpc_max = 0;
    int auto_dispatch = 0;
    int auto_bpc = 0;

    // batch staging
    tw::DevBuf b_src, b_dst, b_ts, b_keys, b_vals, b_flags;
    tw::DevBuf flags, idx;             // per-edge temporaries
    tw::DevBuf v_flags, v_pos;         // per-node temporaries
    tw::DevBuf err;                    // device error flags (uint32)
    tw::DevBuf scal;                   // device scalars
    void* h_scal = nullptr;            // pinned host copy: scal, then the 4 error flags
    tw::Workspace ws;

    // every device allocation of the graph
    std::vector<tw::DevBuf*> buffers() {
        return {&e_src, &e_dst, &e_ts, &a_src, &a_dst, &a_ts, &gg_off, &gs_tiles,
                &n_dst, &n_ts, &ng, &fence, &an_dst, &an_ts, &ang, &afence,
                &rec, &seg, &touched, &bs_src, &bs_dst, &bs_ts, &q_src, &q_dst, &q_ts,
                &c_node, &c_bf, &c_be, &jobs, &j_cnt, &j_off, &j_re, &j_rg, &j_rf, &j_fw,
                &o_flag, &o_rank, &o_tf, &f_tf, &adj_tab,
                &c_node0, &c_walk0, &c_t0, &c_node1, &c_walk1, &c_t1, &c_node2, &c_walk2,
                &c_t2, &c_prev, &c_flags, &c_pos, &wq,
                &b_src, &b_dst, &b_ts, &b_keys, &b_vals, &b_flags, &flags, &idx, &v_flags,
                &v_pos, &err, &scal, &ws.scan_part, &ws.hist, &ws.keys_alt, &ws.vals_alt,
                &ws.v64_alt, &ws.tiles, &cw, &w_tiles};
    }
};

namespace tw {

// index.hip
// Copy the device scalar slots (with flags: also the device error flags) to
// the graph's pinned host copy and wait for the graph's stream.
tw_status pull_scalars(tw_graph* g, bool flags, Error& err);
// the window summary on the host: a read-back of the slots when it is stale
tw_status refresh_summary(tw_graph* g, Error& err);
inline uint32_t host_u32(const tw_graph* g, int k) {
    return static_cast<const uint32_t*>(g->h_scal)[k];
}
inline int64_t host_i64(const tw_graph* g, int k) {
    return static_cast<const int64_t*>(g->h_scal)[k];
}
inline const uint32_t* host_flags(const tw_graph* g) {
    return static_cast<const uint32_t*>(g->h_scal) + SCALAR_BYTES / 4;
}

// nodeview.hip
// Sort the kept batch (timestamp order) by source and list the node-view
// jobs: the batch's source nodes, then the nodes that lose edges to the
// eviction of window positions [ev_from, ev_from + ev_n) of the timestamp
// view, which must still hold the evicted records.
// [ts_lo, ts_hi] bounds the kept records' timestamps.
tw_status nv_collect(tw_graph* g, const int32_t* q_src, const int32_t* q_dst, const int64_t* q_ts,
                     int64_t kept, int64_t ts_lo, int64_t ts_hi, int64_t ev_from, int64_t ev_n,
                     Error& err);
// Apply the collected jobs: evict edges older than cut (when evicting),
// append or rewrite every job node's run, its groups, fence and record.
tw_status nv_apply(tw_graph* g, bool evicting, int64_t cut, Error& err);
// Empty node view (every record empty, pools reset).
tw_status nv_reset(tw_graph* g, Error& err);
// Distinct (node, timestamp) groups of the window. Synchronises.
tw_status nv_group_count(tw_graph* g, int64_t* gn, Error& err);
// The node view in its canonical contiguous form (any pointer may be null).
tw_status nv_export(tw_graph* g, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts, int64_t* n_goff,
                    int64_t* n_ebeg, int64_t* n_gbeg, Error& err);

// index.hip
tw_status ingest(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                 int64_t n, tw_ingest_info* info, Error& err);
// An ingest in two parts. ingest_prepare stages, validates, sorts the batch
// and collects the node-view jobs: it writes only ingest buffers and the
// free tail of the window buffers, so walks over the current index may run
// meanwhile. ingest_apply then changes the index in place (nothing else may
// change it in between; walks must not run during it).
struct IngestPlan {
    enum { IN_TAIL = 0, IN_ALT = 1, IN_BUF = 2 };  // where the batch was staged
    int64_t n = 0, B = 0;
    int place = IN_BUF;
    int32_t* s_src = nullptr;
    int32_t* s_dst = nullptr;
    int64_t* s_ts = nullptr;
    const int32_t* q_src = nullptr;  // kept records in timestamp order
    const int32_t* q_dst = nullptr;
    const int64_t* q_ts = nullptr;
    bool staged_counts = false;
    int stage_has_last = 0;
    int64_t bmin = 0, t_now = 0;
    bool has_time = false, sorted = true, evicting = false, evict_all = false;
    int64_t cut = 0, kept = 0, evicted = 0, gg_evicted = 0, batch_first = 0, drop_lo = 0;
    int64_t m_old = 0, e_base = 0;  // the window the plan was made against
    uint32_t epoch = 0;
};
// walk_flags: report (and clear) the error flags earlier walks left on the
// graph, read back with the batch's counts, instead of ingesting
tw_status ingest_prepare(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                         int64_t n, IngestPlan& P, Error& err, bool walk_flags = false);
tw_status ingest_apply(tw_graph* g, const IngestPlan& P, tw_ingest_info* info, Error& err);
tw_status evict_before(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err);
// ingest / evict_before on the graph and on its in-view (when it has one).
// before_apply (nullable): the graph's stream waits for it between planning
// the batch and changing the index.
tw_status ingest_views(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                       int64_t n, tw_ingest_info* info, Error& err,
                       hipEvent_t before_apply = nullptr, bool walk_flags = false);
tw_status evict_views(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err);
// adjacency.hip: the node2vec pair table of the window, built when first
// needed; adj_update keeps it current at an ingest or eviction (the evicted
// window records counted down, the kept batch records up) or drops it when
// it would fill past three quarters (the next node2vec walk rebuilds it)
tw_status build_adjacency(tw_graph* g, Error& err);
tw_status adj_update(tw_graph* g, const int32_t* ev_src, const int32_t* ev_dst, int64_t ev_n,
                     const int32_t* add_src, const int32_t* add_dst, int64_t add_n, Error& err);
// The graph whose node view holds the in-edges (backward walks): g itself
// when undirected, else g->rev, created from g's window on first use and
// fed every later ingest and eviction.
tw_status backward_view(tw_graph* g, tw_graph** out, Error& err);
// Releases a graph's device and pinned memory (and its in-view's).
void release_graph(tw_graph* g);
// weights.hip: cumulative group weights of the node view for the
// weight-based picker at time scale tau (tau <= 0: 1); a no-op while built.
tw_status build_weights(tw_graph* g, double tau, Error& err);
tw_status init_empty(tw_graph* g, Error& err);  // empty index for a graph never ingested
tw_status export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                       int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                       int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg, Error& err);

// walk.hip
tw_status sample_walks(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                       int32_t* len, Error& err);
tw_status sample_walks_batch(tw_graph* g, const tw_batch_params* p, int32_t* nodes, int64_t* ts,
                             int32_t* len, Error& err);
tw_status row_offsets(tw_graph* g, const int32_t* max_len, int64_t n, int64_t* row,
                      int64_t* total, Error& err);
tw_status autotune(tw_graph* g, const tw_walk_params* p, int64_t sample, int32_t* nodes,
                   int64_t* ts, int32_t* len, int32_t best[2], Error& err);
tw_tuning get_tuning(const tw_graph* g);
void set_tuning_fields(tw_graph* g, const tw_tuning& t);
tw_status set_tuning(tw_graph* g, const tw_tuning* t, Error& err);
// allocation-free walks: set-up once per device (device current), the call
tw_status noalloc_setup(int device, Error& err);
int64_t noalloc_scratch_bytes();
tw_status sample_walks_noalloc(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                               int32_t* len, Error& err);

// One request of a serving launch: count walks of max_len nodes written to
// rows of width max_len at nodes / ts, lengths at len (validated by the
// caller).
struct ServeReq {
    int64_t count;
    int32_t max_len;
    tw_bias hop, start;
    int32_t start_mode;
    const int32_t* start_nodes;
    uint64_t seed, base;
    int32_t* nodes;
    int64_t* ts;
    int32_t* len;
};
// Parameter checks of a walk request (as tw_sample_walks makes them).
tw_status check_walk_params(const tw_walk_params* p, Error& err);
// Device table bytes for n requests (d_table / h_table hold that much; the
// host table should be pinned and must stay untouched until the launch's
// copy has run).
size_t serve_table_bytes(int n);
// Enqueue the padding and the walks of n requests (1..1024) in one launch;
// *d_hops accumulates the launch's hops; request r's error words are
// d_err[2 r] (a start node out of range) and d_err[2 r + 1] (node2vec
// trial-cap hits), which the caller clears before the launch (d_err holds
// at least 4 words). One large forward request runs the full-walk kernel.
// rev: backward requests (g is the in-view). Weight-based requests of one
// launch share one time scale (tau).
tw_status serve_launch(tw_graph* g, const ServeReq* reqs, int n, void* d_table, void* h_table,
                       unsigned long long* d_hops, uint32_t* d_err, bool rev, Error& err);

// serve.hip
tw_status server_create(tw_graph* g, const tw_server_config* cfg, tw_server** out, Error& err);
tw_status server_submit(tw_server* s, const tw_walk_params* p, uint64_t* id, Error& err);
tw_status server_ingest(tw_server* s, const int32_t* src, const int32_t* dst, const int64_t* ts,
                        int64_t n, uint64_t* id, Error& err);
tw_status server_wait(tw_server* s, uint64_t id, int64_t timeout_us, tw_request_result* out,
                      Error& err);
tw_status server_release(tw_server* s, uint64_t id, Error& err);
tw_status server_copy_out(tw_server* s, uint64_t id, int32_t* nodes, int64_t* ts, int32_t* len,
                          Error& err);
tw_status server_stats(tw_server* s, tw_server_counters* out, Error& err);
tw_status server_destroy(tw_server* s, Error& err);

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
