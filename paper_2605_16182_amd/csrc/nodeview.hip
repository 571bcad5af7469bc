// Incremental node-and-timestamp view (Tempest, Sec. "Dual-Index
// Organization"; maintained under the window of Sec. "Streaming Ingestion
// and Window Management").
//
// Every node's edges (sorted by timestamp, then arrival), its (node,
// timestamp) groups and its fence live in one segment of the edge, group and
// fence pools. An ingest touches only the nodes that receive batch edges or
// lose edges to eviction; each such node is a job:
//   * evict: the node's first live group moves past the evicted groups;
//   * append: the batch run starts at or after the node's last timestamp and
//     fits the segment's free tail, so it is written in place, extending the
//     last group when it shares its timestamp;
//   * rewrite: the surviving run merged with the batch run (older first on
//     equal timestamps) goes to a new segment with slack.
// Only new groups add fence entries. When a pool has no room for the new
// segments, every active node is rewritten into fresh pools.
#include <algorithm>
#include <type_traits>

#include "compact.h"
#include "tw_internal.h"
#include "walk_device.h"

namespace tw {
namespace {

constexpr int T = 256;
constexpr int NV_ITEMS = 8;       // job outputs per thread (lane-strided)
constexpr int NV_TILE = T * NV_ITEMS;
constexpr int FENCE_GRID = 2048;  // grid-stride launch for the fence entries

inline dim3 grid_for(int64_t n, int items = 1) {
    return dim3((unsigned)std::max<int64_t>(ceil_div(std::max<int64_t>(n, 1), (int64_t)T * items), 1));
}

// A node's allocation, used by ingest only. gen tags the pool generation the
// segment belongs to; segments of older generations are void.
struct alignas(32) SegRec {
    uint32_t e0, ecap, g0, gcode;
    uint32_t f0, gen, pad0, pad1;
};

enum : uint32_t { JOB_EVICT = 0, JOB_APPEND = 1, JOB_REWRITE = 2 };

// Fields are grouped in 16-byte words by the kernels that read them per
// output (a job's outputs read the same words from consecutive lanes): the
// run's place (every output), the writer's targets, the fence keys.
struct alignas(16) Job {
    uint32_t kind, merge, ob, oe;    // kind; runs interleave; surviving old edges
    uint32_t bf, e_at, g_at, oge;    // batch run start; first written edge / new group; old end
    uint32_t gcode, f0, g0, kshift;  // the segment after the job and its fence key shift
    int64_t kbase;                   // fence key base of the segment after the job
    int64_t t_last;                  // last surviving old timestamp (INT64_MIN: none)
    uint32_t v, fresh, ogb, be;      // node; needs a new segment; surviving old groups; run end
    uint32_t e0, ecap, pad0, pad1;   // the segment after the job
};
static_assert(sizeof(Job) == 96, "six 16-byte words");

__device__ __forceinline__ NodeRec empty_rec() {
    NodeRec r;
    r.gb = r.ge = r.g0 = r.ee = 0;
    r.fence_off = r.lv = 0;
    r.t_last = INT64_MIN;
    r.kbase = r.pad = 0;
    return r;
}

// Edge slots of a new segment holding n edges: twice n plus 4. A node whose
// window slides (appends at the tail, evictions at the head) then finds,
// when its tail is full, its live run past the first half of the segment,
// and rewrites it to the segment's start without a new segment (the two
// ranges are disjoint).
__device__ __forceinline__ uint32_t edge_cap(uint32_t n) {
    const uint64_t c = 2 * (uint64_t)n + 4;
    return (uint32_t)std::min<uint64_t>(c, UINT32_MAX - 1);
}

// capacity code of a group segment for n groups: FENCE_FAN << code >= 2 n
__device__ __forceinline__ uint32_t group_code(uint64_t n) {
    const uint64_t want = 2 * n;
    uint32_t c = 0;
    while (seg_groups(c) < want) ++c;
    return c;
}

// last index j in [0, n) with off[j] <= t (off ascending, off[0] <= t)
__device__ __forceinline__ uint32_t job_of(const uint32_t* __restrict__ off, uint32_t n,
                                           uint64_t t) {
    uint32_t lo = 0, hi = n;  // first index with off > t
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((uint64_t)off[mid] <= t) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

__global__ void k_empty_rec(NodeRec* __restrict__ rec, int64_t V) {
    const int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v < V) rec[v] = empty_rec();
}

__global__ void k_copy_u32(const uint32_t* __restrict__ from, uint32_t* __restrict__ to) {
    *to = *from;
}

// to[n] = *from, n = n_dev[0] + n_dev[1] capped at cap
__global__ void k_copy_u32_at(const uint32_t* __restrict__ from, uint32_t* __restrict__ to,
                              const uint32_t* __restrict__ n_dev, int64_t cap) {
    const int64_t n = (int64_t)n_dev[0] + (int64_t)n_dev[1];
    to[n < cap ? n : cap] = *from;
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ----------------------------------------------------------- job lists

// One job per source run of the source-sorted batch, flagged at the run's
// last record (job k: records [c_bf[k], c_be[k])); marks the node touched.
struct RunEndOp {
    const uint32_t* src;
    int64_t n;
    uint32_t epoch;
    uint32_t* touched;
    uint32_t *c_node, *c_bf, *c_be;
    static constexpr bool kHoist = true;
    __device__ bool flag(int64_t i) const {
        const uint32_t a = src[i], b = src[i + 1 < n ? i + 1 : i];  // no branch around loads
        return i + 1 == n || a != b;
    }
    __device__ void emit(int64_t i, uint32_t k) const {
        const uint32_t v = src[i];
        c_node[k] = v;
        c_be[k] = (uint32_t)(i + 1);
        if (k == 0) c_bf[0] = 0;
        if (i + 1 < n) c_bf[k + 1] = (uint32_t)(i + 1);
        touched[v] = epoch;
    }
    __device__ void end(int64_t, uint32_t) const {}
};

// flags[i] = 1 for exactly one evicted position of every source node that is
// not a batch node yet (the first to claim the node's mark)
__global__ void k_evict_marks(const int32_t* __restrict__ e_src, int64_t n, uint32_t epoch,
                              uint32_t* __restrict__ touched, uint32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = (uint32_t)e_src[i];
    uint32_t f = 0;
    if (touched[v] != epoch && atomicExch(&touched[v], epoch) != epoch) f = 1;
    flags[i] = f;
}

// jobs at base0 + base1 + pos[i] for flagged positions, node = nodes[i]
// (identity when nodes is null), no batch run
__global__ void k_flag_jobs(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                            int64_t n, const int32_t* __restrict__ nodes,
                            const uint32_t* __restrict__ base0, const uint32_t* __restrict__ base1,
                            uint32_t* __restrict__ c_node, uint32_t* __restrict__ c_bf,
                            uint32_t* __restrict__ c_be) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t j = *base0 + (base1 ? *base1 : 0u) + pos[i];
    c_node[j] = nodes ? (uint32_t)nodes[i] : (uint32_t)i;
    c_bf[j] = 0;
    c_be[j] = 0;
}

// One eviction-only job per flagged position (flags from k_evict_marks),
// after the batch's jobs (their count in *runs): no batch run.
struct EvictJobOp {
    const uint32_t* flags;
    const int32_t* nodes;
    const uint32_t* runs;
    uint32_t *c_node, *c_bf, *c_be;
    static constexpr bool kHoist = true;
    __device__ bool flag(int64_t i) const { return flags[i] != 0; }
    __device__ void emit(int64_t i, uint32_t k) const {
        const uint32_t j = *runs + k;
        c_node[j] = (uint32_t)nodes[i];
        c_bf[j] = 0;
        c_be[j] = 0;
    }
    __device__ void end(int64_t, uint32_t) const {}
};

// nodes with live edges that no job covers yet
__global__ void k_active_flags(const NodeRec* __restrict__ rec, int64_t V,
                               const uint32_t* __restrict__ touched, uint32_t epoch,
                               uint32_t* __restrict__ flags) {
    const int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v < V) {
        const NodeRec r = rec[v];
        flags[v] = (r.ge > r.gb && touched[v] != epoch) ? 1u : 0u;
    }
}

// ------------------------------------------------------------- jobs

struct Elem {
    int32_t dst;
    int64_t ts;
};

// The source-sorted batch: (dst, ts) arrays, or one packed word per record,
// (ts - base) << 32 | dst, when the batch's time span fits 32 bits (ts then
// holds the words).
struct BatchRuns {
    const int32_t* dst;
    const int64_t* ts;
    int64_t base;
    int packed;

    __device__ __forceinline__ int64_t t(uint32_t i) const {
        return packed ? base + (int64_t)((uint64_t)ts[i] >> 32) : ts[i];
    }
    __device__ __forceinline__ Elem elem(uint32_t i) const {
        if (packed) {
            const uint64_t w = (uint64_t)ts[i];
            return Elem{(int32_t)(uint32_t)w, base + (int64_t)(w >> 32)};
        }
        return Elem{dst[i], ts[i]};
    }
};

BatchRuns batch_runs(const tw_graph* g) {
    return BatchRuns{g->bs_dst.as<int32_t>(), g->bs_ts.as<int64_t>(), g->bs_base,
                     g->bs_packed ? 1 : 0};
}

// Plan of every job: eviction of the node's groups older than cut, then the
// kind, the written edge count and the slots a new segment needs.
// nj jobs, or, with nj_dev, nj_dev[0] + nj_dev[1] of them (counted on the
// device, at most nj)
__global__ void k_job_setup(const uint32_t* __restrict__ c_node, const uint32_t* __restrict__ c_bf,
                            const uint32_t* __restrict__ c_be, int64_t nj,
                            const uint32_t* __restrict__ nj_dev,
                            const NodeRec* __restrict__ rec, const SegRec* __restrict__ seg,
                            const GroupRec* __restrict__ ng, const uint32_t* __restrict__ fence,
                            const BatchRuns b,
                            int evicting, int64_t cut, int rewrite_all, uint32_t gen,
                            Job* __restrict__ jobs, uint32_t* __restrict__ cnt,
                            uint32_t* __restrict__ req_e, uint32_t* __restrict__ req_g,
                            uint32_t* __restrict__ req_f) {
    const int64_t j = (int64_t)blockIdx.x * T + threadIdx.x;
    if (nj_dev) {
        const int64_t c = (int64_t)nj_dev[0] + (int64_t)nj_dev[1];
        if (c < nj) nj = c;
    }
    if (j >= nj) return;
    Job J{};
    J.v = c_node[j];
    J.bf = c_bf[j];
    J.be = c_be[j];
    const NodeRec r = rec[J.v];
    uint32_t gb = r.gb;
    const uint32_t ge = r.ge;
    // the first group at or after cut: through the node's fence (a hub's
    // eviction then costs a few window reads, not a binary search over its
    // groups); everything goes when the last timestamp precedes cut
    if (evicting && gb < ge && ng[gb].ts < cut)
        gb = r.t_last < cut ? ge : fence_search(ng, fence, r, cut - 1, nullptr, 0, 0);
    J.ogb = gb;
    J.oge = ge;
    J.oe = r.ee;
    J.ob = gb < ge ? ng[gb].first : r.ee;
    const uint32_t ne = J.oe - J.ob;
    J.t_last = ne ? r.t_last : INT64_MIN;
    const uint32_t k = J.be - J.bf;
    const SegRec sg = seg[J.v];
    const bool has_seg = sg.gen == gen && sg.ecap > 0;
    J.kind = JOB_EVICT;
    J.e0 = sg.e0;
    J.ecap = sg.ecap;
    J.g0 = sg.g0;
    J.gcode = sg.gcode;
    J.f0 = sg.f0;
    uint32_t c = 0, re = 0, rg = 0, rf = 0;
    if ((k > 0 || rewrite_all) && ne + k > 0) {
        const bool after = ne == 0 || k == 0 || b.t(J.bf) >= J.t_last;
        // an append keeps the segment's key base and shift: its last
        // timestamp must still have a key below UINT32_MAX
        bool keys_fit = true;
        if (has_seg && ne > 0 && k > 0 && fence_cap(seg_groups(sg.gcode)) > 0) {
            J.kbase = r.kbase;
            J.kshift = rec_shift(r.lv);
            const int64_t t_end = b.t(J.be - 1);
            keys_fit = t_end >= J.kbase &&
                       ((uint64_t)(t_end - J.kbase) >> J.kshift) < 0xFFFFFFFFull;
        }
        if (!rewrite_all && has_seg && ne > 0 && after && keys_fit &&
            (uint64_t)J.oe + k <= (uint64_t)sg.e0 + sg.ecap &&
            (uint64_t)ge + k <= (uint64_t)sg.g0 + seg_groups(sg.gcode)) {
            J.kind = JOB_APPEND;
            J.e_at = J.oe;
            J.g_at = ge;
            c = k;
        } else if (!rewrite_all && has_seg &&
                   (ne == 0 ? k <= sg.ecap && (uint64_t)k <= seg_groups(sg.gcode)
                            : (uint64_t)sg.e0 + ne + k <= J.ob &&
                                  (uint64_t)sg.g0 + (ge - gb) + k <= gb)) {
            // nothing survives and the batch run fits the node's own segment,
            // or the merged run fits before the surviving run there: rewrite
            // it at the segment's start (source and destination are disjoint)
            J.kind = JOB_REWRITE;
            J.merge = (ne > 0 && k > 0 && !after) ? 1u : 0u;
            J.e_at = sg.e0;
            J.g_at = sg.g0;
            c = ne + k;
        } else {
            J.kind = JOB_REWRITE;
            J.fresh = 1;
            J.merge = (ne > 0 && k > 0 && !after) ? 1u : 0u;
            J.ecap = edge_cap(ne + k);
            J.gcode = group_code((uint64_t)(ge - gb) + k);
            re = J.ecap;
            rg = (uint32_t)seg_groups(J.gcode);
            rf = fence_cap(rg);
            c = ne + k;
        }
        if (J.kind == JOB_REWRITE) {
            // keys of the rewritten run: base its first timestamp, the shift
            // for its span (both runs are sorted by timestamp)
            int64_t lo = INT64_MAX, hi = INT64_MIN;
            if (ne > 0) {
                lo = ng[gb].ts;
                hi = r.t_last;
            }
            if (k > 0) {
                lo = std::min(lo, b.t(J.bf));
                hi = std::max(hi, b.t(J.be - 1));
            }
            J.kbase = lo;
            J.kshift = fence_shift((uint64_t)(hi - lo));
        }
    }
    jobs[j] = J;
    cnt[j] = c;
    req_e[j] = re;
    req_g[j] = rg;
    req_f[j] = rf;
}

// new segments at the pool tops plus the scanned requests
__global__ void k_job_place(Job* __restrict__ jobs, int64_t nj, const uint32_t* __restrict__ e_off,
                            const uint32_t* __restrict__ g_off, const uint32_t* __restrict__ f_off,
                            uint32_t e_top, uint32_t g_top, uint32_t f_top) {
    const int64_t j = (int64_t)blockIdx.x * T + threadIdx.x;
    if (j >= nj) return;
    Job J = jobs[j];
    if (!J.fresh) return;
    J.e0 = e_top + e_off[j];
    J.g0 = g_top + g_off[j];
    J.f0 = f_top + f_off[j];
    J.e_at = J.e0;
    J.g_at = J.g0;
    jobs[j] = J;
}


// Element i of a merging job's run (stable merge of the surviving old run
// and the batch run, old first on equal timestamps): returns true when it is
// old element *k, else batch element *k.
__device__ __forceinline__ bool merge_pick(const Job& J, uint32_t i,
                                           const int64_t* __restrict__ ots,
                                           const BatchRuns& bt, uint32_t* k) {
    const uint32_t na = J.oe - J.ob, nb = J.be - J.bf;
    // a = old elements among the first i outputs
    uint32_t lo = i > nb ? i - nb : 0, hi = i < na ? i : na;
    while (lo < hi) {
        const uint32_t a = lo + ((hi - lo) >> 1);
        if (ots[J.ob + a] <= bt.t(J.bf + (i - a - 1))) lo = a + 1; else hi = a;
    }
    const uint32_t a = lo, b = i - lo;
    if (a < na && (b >= nb || ots[J.ob + a] <= bt.t(J.bf + b))) {
        *k = a;
        return true;
    }
    *k = b;
    return false;
}

// element i of job J's written run
__device__ __forceinline__ Elem job_elem(const Job& J, uint32_t i, const int32_t* __restrict__ odst,
                                         const int64_t* __restrict__ ots,
                                         const BatchRuns& bt) {
    if (J.kind == JOB_APPEND) return bt.elem(J.bf + i);
    const uint32_t na = J.oe - J.ob;
    if (!J.merge) {
        if (i < na) return Elem{odst[J.ob + i], ots[J.ob + i]};
        return bt.elem(J.bf + i - na);
    }
    uint32_t k;
    if (merge_pick(J, i, ots, bt, &k)) return Elem{odst[J.ob + k], ots[J.ob + k]};
    return bt.elem(J.bf + k);
}

// timestamp of element i of job J's written run
__device__ __forceinline__ int64_t job_ts(const Job& J, uint32_t i, const int64_t* __restrict__ ots,
                                          const BatchRuns& bt) {
    if (J.kind == JOB_APPEND) return bt.t(J.bf + i);
    const uint32_t na = J.oe - J.ob;
    if (!J.merge) return i < na ? ots[J.ob + i] : bt.t(J.bf + i - na);
    uint32_t k;
    return merge_pick(J, i, ots, bt, &k) ? ots[J.ob + k] : bt.t(J.bf + k);
}

// last j in [lo, hi] with off[j] <= t (off[lo] <= t)
__device__ __forceinline__ uint32_t job_in(const uint32_t* __restrict__ off, uint32_t lo,
                                           uint32_t hi, uint64_t t) {
    uint32_t a = lo + 1, b = hi + 1;
    while (a < b) {
        const uint32_t mid = a + ((b - a) >> 1);
        if ((uint64_t)off[mid] <= t) a = mid + 1; else b = mid;
    }
    return a - 1;
}

// First job of every tile of NV_TILE outputs (the job holding the tile's
// first output), one thread per tile; tf[nt] = nj - 1 closes the last range.
__global__ void k_tile_first(const uint32_t* __restrict__ off, int64_t nj, int64_t nt,
                             uint32_t* __restrict__ tf) {
    const int64_t b = (int64_t)blockIdx.x * T + threadIdx.x;
    if (b > nt) return;
    tf[b] = b == nt ? (uint32_t)(nj - 1) : job_of(off, (uint32_t)nj, (uint64_t)b * NV_TILE);
}

// The jobs that may cover a tile of NV_TILE consecutive outputs (or entries):
// the tile's items go to consecutive lanes, so reads and writes of the
// per-node runs coalesce. Their offsets off[j0 .. j1 + 1] are staged in LDS
// when they fit (the job lookups of the tile then stay in LDS).
constexpr int OFF_LDS = 2 * NV_TILE + 2;

struct TileJobs {
    uint32_t j0, j1;
    bool staged;

    __device__ TileJobs(const uint32_t* __restrict__ tf, uint32_t tile,
                        const uint32_t* __restrict__ off, uint32_t* soff) {
        j0 = tf[tile];
        j1 = tf[tile + 1];
        const uint32_t cnt = j1 - j0 + 2;
        staged = cnt <= (uint32_t)OFF_LDS;
        if (staged)
            for (uint32_t i = threadIdx.x; i < cnt; i += T) soff[i] = off[j0 + i];
        __syncthreads();
    }
    // The job holding output t of the tile. S = staged (uniform over the
    // workgroup): the kernels run their rounds in one code path per case, so
    // that a lookup is an LDS read or a global read, never a generic one.
    template <bool S>
    __device__ uint32_t job(const uint32_t* __restrict__ off, const uint32_t* soff,
                            uint64_t t) const {
        if constexpr (!S) {
            return job_in(off, j0, j1, t);
        } else {
            uint32_t a = 1, b = j1 - j0 + 1;  // last k with soff[k] <= t (soff[0] <= t)
            while (a < b) {
                const uint32_t mid = a + ((b - a) >> 1);
                if ((uint64_t)soff[mid] <= t) a = mid + 1; else b = mid;
            }
            return j0 + a - 1;
        }
    }
    // off[j] for a job j of the tile's range, or j1 + 1
    template <bool S>
    __device__ uint32_t start(const uint32_t* __restrict__ off, const uint32_t* soff,
                              uint32_t j) const {
        if constexpr (S) return soff[j - j0];
        else return off[j];
    }
};

// Group starts of the job outputs as a bitmap (bit t & 63 of word t >> 6
// marks output t; each round of a wavefront covers one word) and the number
// of group starts in every tile of NV_TILE outputs.
__global__ void __launch_bounds__(T) k_job_flags(const Job* __restrict__ jobs,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ tf,
                                                 int64_t total, const int64_t* __restrict__ ots,
                                                 const BatchRuns bt, uint64_t* __restrict__ bm,
                                                 uint32_t* __restrict__ tcnt) {
    __shared__ uint32_t soff[OFF_LDS];
    __shared__ uint32_t wsum[T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)tile * NV_TILE;
    const TileJobs tj(tf, tile, off, soff);
    // M: 0 = job lookups in global memory, 1 = in LDS, 2 = the tile lies in
    // one job (a hub's run), read once as uniform loads
    auto rounds = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        constexpr bool S = M == 1;
        uint32_t c = 0;
        for (int u = 0; u < NV_ITEMS; ++u) {
            const int64_t t0 = base + (int64_t)u * T + wave * 64;  // the word's first output
            const int64_t t = t0 + lane;
            bool start = false;
            if (t < total) {
                const uint32_t j = M == 2 ? tj.j0 : tj.template job<S>(off, soff, (uint64_t)t);
                const Job J = jobs[j];
                const uint32_t jb = M == 2 ? off[tj.j0] : tj.template start<S>(off, soff, j);
                const uint32_t i = (uint32_t)(t - jb);
                const int64_t x = job_ts(J, i, ots, bt);
                if (i == 0) start = J.kind != JOB_APPEND || x != J.t_last;
                else start = x != job_ts(J, i - 1, ots, bt);
            }
            const uint64_t b = __ballot(start);
            if (lane == 0 && t0 < total) bm[t0 >> 6] = b;
            c += (uint32_t)__popcll(b);
        }
        return c;
    };
    const uint32_t c = tj.j0 == tj.j1 ? rounds(std::integral_constant<int, 2>{})
                       : tj.staged   ? rounds(std::integral_constant<int, 1>{})
                                     : rounds(std::integral_constant<int, 0>{});
    if (lane == 0) wsum[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) sum += wsum[w];
        tcnt[tile] = sum;
    }
}

__device__ __forceinline__ uint64_t below(int b) { return b == 0 ? 0ull : (~0ull >> (64 - b)); }

// group starts among the outputs before p (pref: each word's first rank;
// total outputs, total_groups = all group starts)
__device__ __forceinline__ uint32_t out_rank(const uint64_t* __restrict__ bm,
                                             const uint32_t* __restrict__ pref, int64_t total,
                                             uint32_t total_groups, int64_t p) {
    if (p >= total) return total_groups;
    return pref[p >> 6] + (uint32_t)__popcll(bm[p >> 6] & below((int)(p & 63)));
}

// Every job output's edge, and the group record and level-0 fence key of
// each group start. A group's index in its job is its rank among the group
// starts minus the rank at the job's first output: ranks inside the tile come
// from its bitmap words (in LDS) and the scanned tile counts (toff); a job
// that began in an earlier tile is the only one of its tile, so its first
// rank is that tile's offset plus the bits before it. Stores each word's first
// rank in pref for k_job_finish.
__global__ void __launch_bounds__(T) k_job_write(const Job* __restrict__ jobs,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ tf,
                                                 int64_t total, const int32_t* __restrict__ odst,
                                                 const int64_t* __restrict__ ots,
                                                 const BatchRuns bt,
                                                 const uint64_t* __restrict__ bm,
                                                 const uint32_t* __restrict__ toff,
                                                 uint32_t* __restrict__ pref,
                                                 int32_t* __restrict__ ndst,
                                                 int64_t* __restrict__ nts,
                                                 GroupRec* __restrict__ ngd,
                                                 uint32_t* __restrict__ fence) {
    constexpr int WORDS = NV_TILE / 64;
    static_assert(WORDS <= 64, "one wavefront scans a tile's words");
    __shared__ uint32_t soff[OFF_LDS];
    __shared__ uint64_t sbm[WORDS];
    __shared__ uint32_t spre[WORDS];
    __shared__ uint32_t k_first;  // rank at the first output of a job begun earlier
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)tile * NV_TILE;
    const int64_t last = std::min<int64_t>(base + NV_TILE, total) - 1;
    const TileJobs tj(tf, tile, off, soff);
    if (wave == 0) {
        const int64_t nw = ((last - base) >> 6) + 1;
        const uint64_t wb = lane < nw ? bm[(base >> 6) + lane] : 0ull;
        const uint32_t c = (uint32_t)__popcll(wb);
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        const uint32_t p0 = toff[tile] + inc - c;
        if (lane < WORDS) {
            sbm[lane] = wb;
            spre[lane] = p0;
        }
        if (lane < nw) pref[(base >> 6) + lane] = p0;
    } else if (wave == 1) {
        const int64_t s0 = tj.staged ? tj.start<true>(off, soff, tj.j0)
                                     : tj.start<false>(off, soff, tj.j0);
        if (s0 < base) {
            const int64_t a = s0 / NV_TILE;
            const int64_t q = s0 >> 6, wd = ((a * NV_TILE) >> 6) + lane;
            uint32_t c = 0;
            if (wd < q) c = (uint32_t)__popcll(bm[wd]);
            else if (wd == q) c = (uint32_t)__popcll(bm[q] & below((int)(s0 & 63)));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            if (lane == 0) k_first = toff[a] + c;
        }
    }
    __syncthreads();
    // M: 0 = job lookups in global memory, 1 = in LDS, 2 = the tile lies in
    // one job (a hub's run), read once as uniform loads
    auto rounds = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        constexpr bool S = M == 1;
        for (int u = 0; u < NV_ITEMS; ++u) {
            const int64_t t = base + (int64_t)u * T + threadIdx.x;
            if (t >= total) break;
            const uint32_t j = M == 2 ? tj.j0 : tj.template job<S>(off, soff, (uint64_t)t);
            const Job J = jobs[j];
            const uint32_t jb = M == 2 ? off[tj.j0] : tj.template start<S>(off, soff, j);
            const uint32_t i = (uint32_t)(t - jb);
            const Elem e = job_elem(J, i, odst, ots, bt);
            const uint32_t pos = J.e_at + i;
            ndst[pos] = e.dst;
            nts[pos] = e.ts;
            const int lt = (int)(t - base);
            const uint64_t word = sbm[lt >> 6];
            const bool starts = (word >> (lt & 63)) & 1ull;
            if (i == 0 && J.kind == JOB_APPEND && !starts) {
                // the first new edge joins the node's last group: no longer a
                // one-edge group
                int32_t* d = &ngd[J.oge - 1].dst;
                *d = *d & 0x7fffffff;
            }
            if (starts) {
                // a one-edge group: the job's next output starts a group, or
                // there is none
                bool single =
                    (uint64_t)t + 1 >= (uint64_t)(M == 2 ? off[tj.j0 + 1]
                                                         : tj.template start<S>(off, soff, j + 1));
                if (!single) {
                    const int ln = lt + 1;
                    uint64_t nw;
                    if (ln < NV_TILE) {
                        nw = sbm[ln >> 6];
                    } else {  // the next tile's first word, read as two halves so
                              // that the two reads stay an LDS and a global one
                        const uint32_t* h =
                            reinterpret_cast<const uint32_t*>(bm + ((uint64_t)(t + 1) >> 6));
                        nw = (uint64_t)h[0] | ((uint64_t)h[1] << 32);
                    }
                    single = (nw >> (ln & 63)) & 1ull;
                }
                const uint32_t rk = spre[lt >> 6] + (uint32_t)__popcll(word & below(lt & 63));
                uint32_t kj;
                if ((int64_t)jb >= base) {
                    const int lb = (int)(jb - base);
                    kj = spre[lb >> 6] + (uint32_t)__popcll(sbm[lb >> 6] & below(lb & 63));
                } else {
                    kj = k_first;
                }
                GroupRec g;
                g.ts = e.ts;
                g.first = pos;
                g.dst = single ? (int32_t)((uint32_t)e.dst | 0x80000000u) : e.dst;
                const uint32_t gi = J.g_at + (rk - kj);
                ngd[gi] = g;
                // the group's fence keys (segments of more than FENCE_FAN groups
                // have a fence): level 0 holds every group's, level k that of
                // every FENCE_FAN^k-th group
                if (J.gcode > 0) {
                    const uint32_t rel = gi - J.g0;
                    const uint32_t key = (uint32_t)((uint64_t)(e.ts - J.kbase) >> J.kshift);
                    const uint64_t cap = seg_groups(J.gcode);
                    uint32_t* f = fence + J.f0;
                    f[rel] = key;
                    const int K = fence_levels(cap);
                    uint64_t off = 0;
                    for (int k = 1; k <= K && (rel & ((1u << (FENCE_LOG * k)) - 1u)) == 0; ++k) {
                        off += fence_level_len(cap, k - 1);
                        f[off + (rel >> (FENCE_LOG * k))] = key;
                    }
                }
            }
        }
    };
    if (tj.j0 == tj.j1) rounds(std::integral_constant<int, 2>{});
    else if (tj.staged) rounds(std::integral_constant<int, 1>{});
    else rounds(std::integral_constant<int, 0>{});
}

// Level k of a segment with n groups in use holds the keys of its entries
// [0, level_count(n, k)) and UINT32_MAX up to the next multiple of FENCE_FAN
// (every 8-entry window a search can reach); entries past that are never read.
__device__ __forceinline__ uint64_t level_count(uint64_t n, int k) {
    return (n + (1ull << (FENCE_LOG * k)) - 1) >> (FENCE_LOG * k);
}

__device__ __forceinline__ uint64_t pad_fan(uint64_t c) {
    return (c + FENCE_FAN - 1) & ~(uint64_t)(FENCE_FAN - 1);
}

// Fence words a rewrite of a segment of cap groups with n in use leaves to
// k_job_fence: the padding of every level (k_job_write stores the keys with
// the group records).
__device__ __forceinline__ uint32_t rewrite_words(uint64_t cap, uint64_t n) {
    if (fence_cap(cap) == 0) return 0;
    uint64_t w = 0;
    const int K = fence_levels(cap);
    for (int k = 0; k <= K; ++k) w += pad_fan(level_count(n, k)) - level_count(n, k);
    return (uint32_t)w;
}

// What an append from n0 to n1 groups in use writes at level k: keys of the
// entries [key0, key0 + nkeys) (k_job_write, with the new groups' records),
// UINT32_MAX at [pad0, pad0 + npad) (k_job_fence).
struct LevelWrite {
    uint64_t key0, nkeys, pad0, npad;
};

__device__ __forceinline__ LevelWrite append_level(uint64_t n0, uint64_t n1, int k) {
    const uint64_t c0 = level_count(n0, k), c1 = level_count(n1, k);
    const uint64_t p0 = c1 > pad_fan(c0) ? c1 : pad_fan(c0), p1 = pad_fan(c1);
    return LevelWrite{c0, c1 - c0, p0, p1 > p0 ? p1 - p0 : 0};
}

// New node records (and segments) of the jobs, and the fence entries each
// job writes: all of a new or restarted segment's fence, or the entries of
// an append's new groups.
__global__ void k_job_finish(const Job* __restrict__ jobs, const uint32_t* __restrict__ off,
                             int64_t nj, const uint64_t* __restrict__ bm,
                             const uint32_t* __restrict__ pref, int64_t total,
                             const uint32_t* __restrict__ total_groups,
                             const GroupRec* __restrict__ ngd, NodeRec* __restrict__ rec,
                             SegRec* __restrict__ seg, uint32_t gen, uint32_t* __restrict__ fw) {
    const int64_t j = (int64_t)blockIdx.x * T + threadIdx.x;
    if (j >= nj) return;
    const Job J = jobs[j];
    const uint32_t tg = *total_groups;
    const uint32_t newg = out_rank(bm, pref, total, tg, off[j + 1]) - out_rank(bm, pref, total, tg, off[j]);
    const uint32_t written = off[j + 1] - off[j];
    NodeRec r = rec[J.v];
    uint32_t f = 0;
    if (J.kind == JOB_EVICT) {
        r.gb = J.ogb;
        if (r.gb >= r.ge) r = empty_rec();
    } else {
        const uint64_t cap = seg_groups(J.gcode);
        if (J.kind == JOB_APPEND) {
            r.gb = J.ogb;
            r.ge = J.oge + newg;
            r.ee = J.oe + written;
            if (fence_cap(cap) > 0) {
                const int K = fence_levels(cap);
                for (int k = 0; k <= K; ++k)
                    f += (uint32_t)append_level(J.oge - J.g0, r.ge - J.g0, k).npad;
            }
        } else {
            r.gb = J.g0;
            r.ge = J.g0 + newg;
            r.ee = J.e_at + written;
            f = rewrite_words(cap, newg);
            if (J.fresh) {
                SegRec s;
                s.e0 = J.e0;
                s.ecap = J.ecap;
                s.g0 = J.g0;
                s.gcode = J.gcode;
                s.f0 = J.f0;
                s.gen = gen;
                s.pad0 = s.pad1 = 0;
                seg[J.v] = s;
            }
        }
        r.g0 = J.g0;
        r.fence_off = J.f0;
        r.lv = (uint32_t)fence_levels(r.ge - J.g0) | (J.gcode << 8) | (J.kshift << 16);
        r.kbase = J.kbase;
        r.t_last = ngd[r.ge - 1].ts;
    }
    rec[J.v] = r;
    fw[j] = f;
}

// Fence word u of job J (u counts the words the job writes): the padding
// that a rewritten segment needs on every level, or that an append's new
// groups move. k_job_write stores every level's keys with the group
// records, so only padding is left here.
__device__ __forceinline__ void fence_entry(const Job& J, uint32_t ge,
                                            uint32_t* __restrict__ fence, uint64_t u) {
    const uint64_t cap = seg_groups(J.gcode);
    uint32_t* f = fence + J.f0;
    const uint64_t n = ge - J.g0;
    const int K = fence_levels(cap);
    uint64_t off = 0;
    for (int k = 0; k <= K; ++k) {
        uint64_t pad0, npad;
        if (J.kind == JOB_REWRITE) {
            pad0 = level_count(n, k);
            npad = pad_fan(pad0) - pad0;
        } else {
            const LevelWrite lw = append_level(J.oge - J.g0, n, k);
            pad0 = lw.pad0;
            npad = lw.npad;
        }
        if (u < npad) {
            f[off + pad0 + u] = 0xFFFFFFFFu;
            return;
        }
        u -= npad;
        off += fence_level_len(cap, k);
    }
}

// First job of every tile of the fence entries (total = foff[nj], on the
// device), as k_tile_first; grid-stride.
__global__ void k_tile_first_dev(const uint32_t* __restrict__ foff, int64_t nj,
                                 uint32_t* __restrict__ tf) {
    const uint64_t nt = ((uint64_t)foff[nj] + NV_TILE - 1) / NV_TILE;
    for (uint64_t b = (uint64_t)blockIdx.x * T + threadIdx.x; b <= nt;
         b += (uint64_t)gridDim.x * T)
        tf[b] = b == nt ? (uint32_t)(nj - 1) : job_of(foff, (uint32_t)nj, b * NV_TILE);
}

// the fence entries of the jobs (total = foff[nj]), tiles of NV_TILE
// entries, grid-stride
__global__ void __launch_bounds__(T) k_job_fence(const Job* __restrict__ jobs,
                                                 const uint32_t* __restrict__ foff,
                                                 const uint32_t* __restrict__ tf, int64_t nj,
                                                 const NodeRec* __restrict__ rec,
                                                 uint32_t* __restrict__ fence) {
    __shared__ uint32_t soff[OFF_LDS];
    const uint64_t total = foff[nj];
    for (uint64_t tile = blockIdx.x; tile * NV_TILE < total; tile += gridDim.x) {
        __syncthreads();  // the previous tile's offsets are no longer read
        const uint64_t base = tile * NV_TILE;
        const TileJobs tj(tf, (uint32_t)tile, foff, soff);
        auto rounds = [&](auto staged) {
            constexpr bool S = decltype(staged)::value;
            for (int u = 0; u < NV_ITEMS; ++u) {
                const uint64_t t = base + (uint64_t)u * T + threadIdx.x;
                if (t >= total) break;
                const uint32_t j = tj.template job<S>(foff, soff, t);
                const Job J = jobs[j];
                fence_entry(J, rec[J.v].ge, fence, t - tj.template start<S>(foff, soff, j));
            }
        };
        if (tj.staged) rounds(std::true_type{});
        else rounds(std::false_type{});
    }
}

// ------------------------------------------------------------- export

__global__ void k_node_counts(const NodeRec* __restrict__ rec, const GroupRec* __restrict__ ng,
                              int64_t V, uint32_t* __restrict__ ecnt, uint32_t* __restrict__ gcnt) {
    const int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v >= V) return;
    const NodeRec r = rec[v];
    const bool live = r.ge > r.gb;
    if (ecnt) ecnt[v] = live ? r.ee - ng[r.gb].first : 0u;
    if (gcnt) gcnt[v] = live ? r.ge - r.gb : 0u;
}

__global__ void k_widen_u32(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) out[i] = in[i];
}

// output edge p of the contiguous node view
__global__ void k_export_edges(const uint32_t* __restrict__ ebeg, int64_t V, int64_t m,
                               const NodeRec* __restrict__ rec, const GroupRec* __restrict__ ng,
                               const int32_t* __restrict__ pdst, const int64_t* __restrict__ pts,
                               int32_t* __restrict__ n_dst, int64_t* __restrict__ n_ts) {
    const int64_t p = (int64_t)blockIdx.x * T + threadIdx.x;
    if (p >= m) return;
    const uint32_t v = job_of(ebeg, (uint32_t)(V + 1), (uint64_t)p);
    const NodeRec r = rec[v];
    const uint32_t e = ng[r.gb].first + (uint32_t)(p - ebeg[v]);
    if (n_dst) n_dst[p] = pdst[e];
    if (n_ts) n_ts[p] = pts[e];
}

// output group q: its timestamp and the contiguous position of its first edge
__global__ void k_export_groups(const uint32_t* __restrict__ gbeg, const uint32_t* __restrict__ ebeg,
                                int64_t V, int64_t G, const NodeRec* __restrict__ rec,
                                const GroupRec* __restrict__ ng, int64_t* __restrict__ n_gts,
                                int64_t* __restrict__ n_goff, int64_t m) {
    const int64_t q = (int64_t)blockIdx.x * T + threadIdx.x;
    if (q > G) return;
    if (q == G) {
        if (n_goff) n_goff[G] = m;
        return;
    }
    const uint32_t v = job_of(gbeg, (uint32_t)(V + 1), (uint64_t)q);
    const NodeRec r = rec[v];
    const GroupRec g = ng[r.gb + (uint32_t)(q - gbeg[v])];
    if (n_gts) n_gts[q] = g.ts;
    if (n_goff) n_goff[q] = (int64_t)ebeg[v] + (g.first - ng[r.gb].first);
}

uint32_t* slot(tw_graph* g, int k) { return g->scal.as<uint32_t>() + k; }

// scan of n job values into out (n + 1 entries: out[n] = total); the total
// also lands in *total_slot when given
hipError_t scan_jobs(const uint32_t* in, uint32_t* out, int64_t n, Workspace& ws, hipStream_t s) {
    return scan_exclusive_u32(in, out, n, out + n, ws, s);
}

tw_status run_jobs(tw_graph* g, int64_t nj, bool counted, bool evicting, int64_t cut,
                   bool rewrite_all, Error& err);

}  // namespace

tw_status nv_reset(tw_graph* g, Error& err) {
    const int64_t V = g->V;
    TW_HIP(ensure(g->rec, sizeof(NodeRec) * V, g->stream));
    if (!g->seg.p) {
        // generation 0 marks every segment void (pool_gen starts above 0)
        TW_HIP(ensure(g->seg, sizeof(SegRec) * V, g->stream));
        const int64_t words = V * (int64_t)(sizeof(SegRec) / sizeof(uint32_t));
        hipLaunchKernelGGL(k_zero_u32, grid_for(words), dim3(T), 0, g->stream,
                           g->seg.as<uint32_t>(), words);
    }
    if (!g->touched.p) {
        TW_HIP(ensure(g->touched, sizeof(uint32_t) * V, g->stream));
        hipLaunchKernelGGL(k_zero_u32, grid_for(V), dim3(T), 0, g->stream,
                           g->touched.as<uint32_t>(), V);
    }
    hipLaunchKernelGGL(k_empty_rec, grid_for(V), dim3(T), 0, g->stream, g->rec.as<NodeRec>(), V);
    TW_HIP(hipGetLastError());
    g->pe_top = g->pg_top = g->pf_top = 0;
    g->st_jobs = g->st_written = g->st_new_slots = g->st_full = 0;
    ++g->pool_gen;  // every segment is void
    g->T = 0;
    g->w_ready = false;
    return TW_OK;
}

tw_status nv_collect(tw_graph* g, const int32_t* q_src, const int32_t* q_dst, const int64_t* q_ts,
                     int64_t kept, int64_t ts_lo, int64_t ts_hi, int64_t ev_from, int64_t ev_n,
                     Error& err) {
    hipStream_t s = g->stream;
    if (++g->epoch == 0) {  // wrapped: clear the marks
        hipLaunchKernelGGL(k_zero_u32, grid_for(g->V), dim3(T), 0, s, g->touched.as<uint32_t>(),
                           (int64_t)g->V);
        g->epoch = 1;
    }
    // a node is one job at most, so V + 1 entries hold any job list (also
    // the full rewrite's, which appends to this one)
    const int64_t cand = (int64_t)g->V + 1;
    TW_HIP(ensure(g->c_node, sizeof(uint32_t) * cand, g->stream));
    TW_HIP(ensure(g->c_bf, sizeof(uint32_t) * cand, g->stream));
    TW_HIP(ensure(g->c_be, sizeof(uint32_t) * cand, g->stream));
    const int64_t nf = std::max(kept, ev_n);
    TW_HIP(ensure(g->flags, sizeof(uint32_t) * (nf + 1), g->stream));
    TW_HIP(ensure(g->idx, sizeof(uint32_t) * (nf + 1), g->stream));
    uint32_t* flags = g->flags.as<uint32_t>();
    uint32_t* pos = g->idx.as<uint32_t>();
    uint32_t* sl_runs = slot(g, SLOT_U32_RUNS);
    uint32_t* sl_ev = slot(g, SLOT_U32_EV_NODES);
    // a batch whose timestamps span less than 2^32 travels through the sort
    // as one packed word per record instead of 12 bytes
    g->bs_packed = kept > 0 && ts_hi >= ts_lo && (uint64_t)ts_hi - (uint64_t)ts_lo < (1ull << 32);
    g->bs_base = g->bs_packed ? ts_lo : 0;
    TW_HIP(ensure(g->bs_src, sizeof(uint32_t) * (kept + 1), g->stream));
    if (!g->bs_packed) TW_HIP(ensure(g->bs_dst, sizeof(int32_t) * (kept + 1), g->stream));
    TW_HIP(ensure(g->bs_ts, sizeof(int64_t) * (kept + 1), g->stream));
    if (kept > 0) {
        uint32_t* bsrc = g->bs_src.as<uint32_t>();
        const int vbits = bits_for((uint64_t)(g->V - 1));
        if (g->bs_packed)
            TW_HIP(radix_sort_u32_pack(reinterpret_cast<const uint32_t*>(q_src),
                                       reinterpret_cast<const uint32_t*>(q_dst),
                                       reinterpret_cast<const uint64_t*>(q_ts), (uint64_t)ts_lo,
                                       bsrc, g->bs_ts.as<uint64_t>(), kept, 0, vbits, g->ws, s));
        else
            TW_HIP(radix_sort_u32_kv(reinterpret_cast<const uint32_t*>(q_src),
                                     reinterpret_cast<const uint32_t*>(q_dst),
                                     reinterpret_cast<const uint64_t*>(q_ts), bsrc,
                                     g->bs_dst.as<uint32_t>(), g->bs_ts.as<uint64_t>(), kept, 0,
                                     vbits, g->ws, s));
        const RunEndOp op{bsrc,
                          kept,
                          g->epoch,
                          g->touched.as<uint32_t>(),
                          g->c_node.as<uint32_t>(),
                          g->c_bf.as<uint32_t>(),
                          g->c_be.as<uint32_t>()};
        TW_HIP(compact(op, kept, sl_runs, g->ws.tiles, g->ws, s));
    } else {
        TW_HIP(scan_exclusive_u32(nullptr, nullptr, 0, sl_runs, g->ws, s));
    }
    if (ev_n > 0) {
        const int32_t* esrc = g->e_src.as<int32_t>() + ev_from;
        hipLaunchKernelGGL(k_evict_marks, grid_for(ev_n), dim3(T), 0, s, esrc, ev_n, g->epoch,
                           g->touched.as<uint32_t>(), flags);
        const EvictJobOp op{flags,
                            esrc,
                            sl_runs,
                            g->c_node.as<uint32_t>(),
                            g->c_bf.as<uint32_t>(),
                            g->c_be.as<uint32_t>()};
        TW_HIP(compact(op, ev_n, sl_ev, g->ws.tiles, g->ws, s));
    } else {
        TW_HIP(scan_exclusive_u32(nullptr, nullptr, 0, sl_ev, g->ws, s));
    }
    TW_HIP(hipGetLastError());
    // the job count stays on the device (the plan reads it back with its
    // totals); a node is one job at most
    g->T = std::min<int64_t>(kept + ev_n, (int64_t)g->V + 1);
    return TW_OK;
}

namespace {

tw_status ensure_jobs(tw_graph* g, int64_t nj, Error& err) {
    TW_HIP(ensure(g->jobs, sizeof(Job) * (nj + 1), g->stream));
    DevBuf* b[] = {&g->j_cnt, &g->j_off, &g->j_re, &g->j_rg, &g->j_rf, &g->j_fw};
    for (DevBuf* p : b) TW_HIP(ensure(*p, sizeof(uint32_t) * (nj + 2), g->stream));
    return TW_OK;
}

// Plan the jobs and scan their outputs and requests; returns the totals
// {written edges, edge slots, group slots, fence entries}. counted: nj is a
// bound and the count is on the device (SLOT_U32_RUNS + SLOT_U32_EV_NODES):
// the launches cover a capacity (twice the last update's jobs, at least 1M,
// at most nj), read the count on the device and it comes back with the
// totals in one read-back, which sets nj; a count above the capacity is
// planned again. Synchronises.
tw_status plan_jobs(tw_graph* g, int64_t& nj, bool counted, bool evicting, int64_t cut,
                    bool rewrite_all, uint32_t gen, uint64_t tot[4], Error& err) {
    hipStream_t s = g->stream;
    const uint32_t* nj_dev = counted ? slot(g, SLOT_U32_RUNS) : nullptr;  // [0] runs, [1] nodes
    static_assert(SLOT_U32_EV_NODES == SLOT_U32_RUNS + 1, "the job count is two adjacent words");
    const int64_t cap =
        counted ? std::min<int64_t>(nj, std::max<int64_t>(2 * g->jobs_last, 1 << 20)) : nj;
    if (ensure_jobs(g, cap, err) != TW_OK) return err.code;
    hipLaunchKernelGGL(k_job_setup, grid_for(cap), dim3(T), 0, s, g->c_node.as<uint32_t>(),
                       g->c_bf.as<uint32_t>(), g->c_be.as<uint32_t>(), cap, nj_dev,
                       g->rec.as<NodeRec>(),
                       g->seg.as<SegRec>(), g->ng.as<GroupRec>(), g->fence.as<uint32_t>(),
                       batch_runs(g), evicting ? 1 : 0, cut, rewrite_all ? 1 : 0, gen, g->jobs.as<Job>(),
                       g->j_cnt.as<uint32_t>(), g->j_re.as<uint32_t>(), g->j_rg.as<uint32_t>(),
                       g->j_rf.as<uint32_t>());
    TW_HIP(hipGetLastError());
    // output counts into offsets (total also at j_off[nj]); requests scanned
    // in place: j_re / j_rg / j_rf become offsets
    uint32_t* sl = slot(g, SLOT_U32_REQ_E);
    uint32_t* j_off = g->j_off.as<uint32_t>();
    const uint32_t* in4[4] = {g->j_cnt.as<uint32_t>(), g->j_re.as<uint32_t>(),
                              g->j_rg.as<uint32_t>(), g->j_rf.as<uint32_t>()};
    uint32_t* const out4[4] = {j_off, g->j_re.as<uint32_t>(), g->j_rg.as<uint32_t>(),
                               g->j_rf.as<uint32_t>()};
    uint32_t* const tot4[4] = {slot(g, SLOT_U32_OUT), sl, sl + 1, sl + 2};
    TW_HIP(scan_exclusive_u32x4(in4, out4, tot4, cap, g->ws, s, nj_dev));
    if (counted)
        hipLaunchKernelGGL(k_copy_u32_at, dim3(1), dim3(1), 0, s, slot(g, SLOT_U32_OUT), j_off,
                           nj_dev, cap);
    else
        hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s, slot(g, SLOT_U32_OUT), j_off + nj);
    TW_HIP(hipGetLastError());
    if (pull_scalars(g, false, err) != TW_OK) return err.code;
    if (counted) {
        const int64_t n = (int64_t)host_u32(g, SLOT_U32_RUNS) + host_u32(g, SLOT_U32_EV_NODES);
        if (n > nj) {
            err = Error{TW_EDEVICE, "node view: more jobs than the batch can make"};
            return err.code;
        }
        nj = n;
        if (n > cap) return plan_jobs(g, nj, false, evicting, cut, rewrite_all, gen, tot, err);
    }
    tot[0] = host_u32(g, SLOT_U32_OUT);
    for (int i = 0; i < 3; ++i) tot[1 + i] = host_u32(g, SLOT_U32_REQ_E + i);
    g->jobs_last = nj;
    return TW_OK;
}

// Run planned jobs: reads runs from the source pools (sdst, sts, sng),
// writes into the destination pools (the same ones unless rewriting all).
tw_status execute_jobs(tw_graph* g, int64_t nj, uint64_t out, const int32_t* sdst,
                       const int64_t* sts, int32_t* ddst, int64_t* dts, GroupRec* dng,
                       uint32_t* dfence, uint32_t gen, Error& err) {
    hipStream_t s = g->stream;
    Job* jobs = g->jobs.as<Job>();
    const uint32_t* off = g->j_off.as<uint32_t>();
    // group-start bitmap and per-word ranks (o_flag), tile counts scanned in
    // place (o_rank, total at [nt])
    const int64_t words = ceil_div((int64_t)out, 64), nt = ceil_div((int64_t)out, NV_TILE);
    TW_HIP(ensure(g->o_flag, sizeof(uint64_t) * (words + 1) + sizeof(uint32_t) * (words + 1), g->stream));
    TW_HIP(ensure(g->o_rank, sizeof(uint32_t) * (nt + 1), g->stream));
    TW_HIP(ensure(g->o_tf, sizeof(uint32_t) * (nt + 1), g->stream));
    uint64_t* bm = g->o_flag.as<uint64_t>();
    uint32_t* pref = reinterpret_cast<uint32_t*>(bm + words + 1);
    uint32_t* tcnt = g->o_rank.as<uint32_t>();
    uint32_t* tf = g->o_tf.as<uint32_t>();
    if (out > 0) {
        hipLaunchKernelGGL(k_tile_first, grid_for(nt + 1), dim3(T), 0, s, off, nj, nt, tf);
        hipLaunchKernelGGL(k_job_flags, dim3((unsigned)nt), dim3(T), 0, s, jobs, off, tf,
                           (int64_t)out, sts, batch_runs(g), bm, tcnt);
    }
    TW_HIP(scan_exclusive_u32(tcnt, tcnt, nt, tcnt + nt, g->ws, s));
    if (out > 0)
        hipLaunchKernelGGL(k_job_write, dim3((unsigned)nt), dim3(T), 0, s, jobs, off, tf,
                           (int64_t)out, sdst, sts, batch_runs(g), bm, tcnt, pref, ddst, dts, dng,
                           dfence);
    hipLaunchKernelGGL(k_job_finish, grid_for(nj), dim3(T), 0, s, jobs, off, nj, bm, pref,
                       (int64_t)out, tcnt + nt, dng, g->rec.as<NodeRec>(), g->seg.as<SegRec>(),
                       gen, g->j_fw.as<uint32_t>());
    TW_HIP(scan_jobs(g->j_fw.as<uint32_t>(), g->j_fw.as<uint32_t>(), nj, g->ws, s));
    if (nj > 0) {
        // every fence word a job writes is a distinct word of the pool
        const uint64_t fcap = (dfence == g->fence.as<uint32_t>() ? g->fence.bytes
                                                                  : g->afence.bytes) /
                              sizeof(uint32_t);
        TW_HIP(ensure(g->f_tf, sizeof(uint32_t) * (fcap / NV_TILE + 2), g->stream));
        hipLaunchKernelGGL(k_tile_first_dev, dim3(FENCE_GRID / 8), dim3(T), 0, s,
                           g->j_fw.as<uint32_t>(), nj, g->f_tf.as<uint32_t>());
        hipLaunchKernelGGL(k_job_fence, dim3(FENCE_GRID), dim3(T), 0, s, jobs,
                           g->j_fw.as<uint32_t>(), g->f_tf.as<uint32_t>(), nj,
                           g->rec.as<NodeRec>(), dfence);
    }
    TW_HIP(hipGetLastError());
    return TW_OK;
}

// counted: nj bounds the jobs, whose count is on the device (plan_jobs)
tw_status run_jobs(tw_graph* g, int64_t nj, bool counted, bool evicting, int64_t cut,
                   bool rewrite_all, Error& err) {
    hipStream_t s = g->stream;
    uint64_t tot[4];
    const uint32_t gen = rewrite_all ? g->pool_gen + 1 : g->pool_gen;
    if (plan_jobs(g, nj, counted, evicting, cut, rewrite_all, gen, tot, err) != TW_OK)
        return err.code;
    if (nj == 0) return TW_OK;
    g->st_jobs = nj;
    g->st_written = (int64_t)tot[0];
    g->st_new_slots = (int64_t)tot[1];
    g->st_full = rewrite_all ? 1 : 0;
    if (!rewrite_all) {
        if (g->pe_top + (int64_t)tot[1] > g->pe_cap || g->pg_top + (int64_t)tot[2] > g->pg_cap ||
            g->pf_top + (int64_t)tot[3] > g->pf_cap) {
            // no room: list every other active node and rewrite all of them
            const int64_t V = g->V;
            TW_HIP(ensure(g->v_flags, sizeof(uint32_t) * (V + 1), g->stream));
            TW_HIP(ensure(g->v_pos, sizeof(uint32_t) * (V + 1), g->stream));
            uint32_t* sl_act = slot(g, SLOT_U32_ACTIVE);
            hipLaunchKernelGGL(k_active_flags, grid_for(V), dim3(T), 0, s, g->rec.as<NodeRec>(), V,
                               g->touched.as<uint32_t>(), g->epoch, g->v_flags.as<uint32_t>());
            TW_HIP(scan_exclusive_u32(g->v_flags.as<uint32_t>(), g->v_pos.as<uint32_t>(), V,
                                      sl_act, g->ws, s));
            if (pull_scalars(g, false, err) != TW_OK) return err.code;
            const uint32_t na = host_u32(g, SLOT_U32_ACTIVE);
            const int64_t all = nj + na;  // <= V: the lists hold V + 1 entries
            hipLaunchKernelGGL(k_flag_jobs, grid_for(V), dim3(T), 0, s, g->v_flags.as<uint32_t>(),
                               g->v_pos.as<uint32_t>(), V, nullptr, slot(g, SLOT_U32_RUNS),
                               slot(g, SLOT_U32_EV_NODES), g->c_node.as<uint32_t>(),
                               g->c_bf.as<uint32_t>(), g->c_be.as<uint32_t>());
            TW_HIP(hipGetLastError());
            return run_jobs(g, all, false, evicting, cut, true, err);
        }
        hipLaunchKernelGGL(k_job_place, grid_for(nj), dim3(T), 0, s, g->jobs.as<Job>(), nj,
                           g->j_re.as<uint32_t>(), g->j_rg.as<uint32_t>(), g->j_rf.as<uint32_t>(),
                           (uint32_t)g->pe_top, (uint32_t)g->pg_top, (uint32_t)g->pf_top);
        if (execute_jobs(g, nj, tot[0], g->n_dst.as<int32_t>(), g->n_ts.as<int64_t>(),
                         g->n_dst.as<int32_t>(), g->n_ts.as<int64_t>(), g->ng.as<GroupRec>(),
                         g->fence.as<uint32_t>(), gen, err) != TW_OK)
            return err.code;
        g->pe_top += (int64_t)tot[1];
        g->pg_top += (int64_t)tot[2];
        g->pf_top += (int64_t)tot[3];
        return TW_OK;
    }
    // fresh pools with room for as much again
    const int64_t lim = (int64_t)UINT32_MAX - 1;
    const int64_t ce = std::min<int64_t>(std::max<int64_t>(2 * (int64_t)tot[1], 1024), lim);
    const int64_t cg = std::min<int64_t>(std::max<int64_t>(2 * (int64_t)tot[2], 1024), lim);
    const int64_t cf = std::min<int64_t>(std::max<int64_t>(2 * (int64_t)tot[3], 1024), lim);
    if ((int64_t)tot[1] > lim / 2 || (int64_t)tot[2] > lim / 2 || (int64_t)tot[3] > lim / 2) {
        err = Error{TW_ENOMEM, "node view: pools would exceed 2^32 slots"};
        return err.code;
    }
    TW_HIP(ensure(g->an_dst, sizeof(int32_t) * ce, g->stream));
    TW_HIP(ensure(g->an_ts, sizeof(int64_t) * ce, g->stream));
    TW_HIP(ensure(g->ang, sizeof(GroupRec) * cg, g->stream));
    TW_HIP(ensure(g->afence, sizeof(uint32_t) * cf, g->stream));
    hipLaunchKernelGGL(k_job_place, grid_for(nj), dim3(T), 0, s, g->jobs.as<Job>(), nj,
                       g->j_re.as<uint32_t>(), g->j_rg.as<uint32_t>(), g->j_rf.as<uint32_t>(), 0u,
                       0u, 0u);
    if (execute_jobs(g, nj, tot[0], g->n_dst.as<int32_t>(), g->n_ts.as<int64_t>(),
                     g->an_dst.as<int32_t>(), g->an_ts.as<int64_t>(), g->ang.as<GroupRec>(),
                     g->afence.as<uint32_t>(), gen, err) != TW_OK)
        return err.code;
    std::swap(g->n_dst, g->an_dst);
    std::swap(g->n_ts, g->an_ts);
    std::swap(g->ng, g->ang);
    std::swap(g->fence, g->afence);
    g->pe_cap = (int64_t)(g->n_dst.bytes / sizeof(int32_t));
    g->pe_cap = std::min<int64_t>(g->pe_cap, (int64_t)(g->n_ts.bytes / sizeof(int64_t)));
    g->pg_cap = (int64_t)(g->ng.bytes / sizeof(GroupRec));
    g->pf_cap = (int64_t)(g->fence.bytes / sizeof(uint32_t));
    g->pe_cap = std::min(g->pe_cap, lim);
    g->pg_cap = std::min(g->pg_cap, lim);
    g->pf_cap = std::min(g->pf_cap, lim);
    g->pe_top = (int64_t)tot[1];
    g->pg_top = (int64_t)tot[2];
    g->pf_top = (int64_t)tot[3];
    g->pool_gen = gen;
    return TW_OK;
}

}  // namespace

tw_status nv_apply(tw_graph* g, bool evicting, int64_t cut, Error& err) {
    g->st_jobs = g->st_written = g->st_new_slots = g->st_full = 0;
    if (g->T == 0) return TW_OK;
    if (run_jobs(g, g->T, true, evicting, cut, false, err) != TW_OK) return err.code;
    g->w_ready = false;
    return TW_OK;
}

tw_status nv_group_count(tw_graph* g, int64_t* gn, Error& err) {
    hipStream_t s = g->stream;
    const int64_t V = g->V;
    TW_HIP(ensure(g->v_flags, sizeof(uint32_t) * (V + 1), g->stream));
    TW_HIP(ensure(g->v_pos, sizeof(uint32_t) * (V + 1), g->stream));
    hipLaunchKernelGGL(k_node_counts, grid_for(V), dim3(T), 0, s, g->rec.as<NodeRec>(),
                       g->ng.as<GroupRec>(), V, nullptr, g->v_flags.as<uint32_t>());
    uint32_t* sl = slot(g, SLOT_U32_GN);
    TW_HIP(scan_exclusive_u32(g->v_flags.as<uint32_t>(), g->v_pos.as<uint32_t>(), V, sl, g->ws, s));
    if (pull_scalars(g, false, err) != TW_OK) return err.code;
    *gn = host_u32(g, SLOT_U32_GN);
    return TW_OK;
}

tw_status nv_export(tw_graph* g, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts, int64_t* n_goff,
                    int64_t* n_ebeg, int64_t* n_gbeg, Error& err) {
    hipStream_t s = g->stream;
    const int64_t V = g->V, m = g->m;
    TW_HIP(ensure(g->v_flags, sizeof(uint32_t) * (V + 1), g->stream));
    TW_HIP(ensure(g->v_pos, sizeof(uint32_t) * (V + 1), g->stream));
    TW_HIP(ensure(g->idx, sizeof(uint32_t) * (V + 2), g->stream));
    TW_HIP(ensure(g->flags, sizeof(uint32_t) * (V + 2), g->stream));
    uint32_t* ecnt = g->v_flags.as<uint32_t>();
    uint32_t* gcnt = g->v_pos.as<uint32_t>();
    uint32_t* ebeg = g->idx.as<uint32_t>();
    uint32_t* gbeg = g->flags.as<uint32_t>();
    hipLaunchKernelGGL(k_node_counts, grid_for(V), dim3(T), 0, s, g->rec.as<NodeRec>(),
                       g->ng.as<GroupRec>(), V, ecnt, gcnt);
    TW_HIP(scan_exclusive_u32(ecnt, ebeg, V, ebeg + V, g->ws, s));
    TW_HIP(scan_exclusive_u32(gcnt, gbeg, V, gbeg + V, g->ws, s));
    uint32_t G = 0;
    TW_HIP(hipMemcpyAsync(&G, gbeg + V, sizeof(G), hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    if (n_ebeg) hipLaunchKernelGGL(k_widen_u32, grid_for(V + 1), dim3(T), 0, s, ebeg, V + 1, n_ebeg);
    if (n_gbeg) hipLaunchKernelGGL(k_widen_u32, grid_for(V + 1), dim3(T), 0, s, gbeg, V + 1, n_gbeg);
    if ((n_dst || n_ts) && m > 0)
        hipLaunchKernelGGL(k_export_edges, grid_for(m), dim3(T), 0, s, ebeg, V, m,
                           g->rec.as<NodeRec>(), g->ng.as<GroupRec>(), g->n_dst.as<int32_t>(),
                           g->n_ts.as<int64_t>(), n_dst, n_ts);
    if (n_gts || n_goff)
        hipLaunchKernelGGL(k_export_groups, grid_for((int64_t)G + 1), dim3(T), 0, s, gbeg, ebeg, V,
                           (int64_t)G, g->rec.as<NodeRec>(), g->ng.as<GroupRec>(), n_gts, n_goff, m);
    TW_HIP(hipGetLastError());
    return TW_OK;
}

}  // namespace tw
