// Streaming ingest, window eviction and the timestamp-grouped view
// (Tempest, Sec. "Dual-Index Organization" and "Streaming Ingestion and
// Window Management"); the node-and-timestamp view is maintained by
// nodeview.hip.
//
// Layout in HBM (structure of arrays, all positions uint32):
//   timestamp view (the edge store):   e_src e_dst e_ts, the window at
//                                      [e_base, e_base + m) of buffers with
//                                      room to append
//   its timestamp groups:              gg_off at [gg_base, gg_base + Gg],
//                                      edge-store positions of each group's
//                                      first record (its timestamp is that
//                                      record's), then the end
//
// One ingest: stage (validate, mirror, min/max, sortedness) -> late drop and
// eviction counts -> (unsorted batch only) stable radix sort by timestamp ->
// node-view jobs collected (the batch sorted by source; the sources of the
// evicted records) -> timestamp view: evicting moves e_base, a batch that
// starts at or after the window's last timestamp is appended in place and
// its groups appended, any other batch is merged (merge path, older records
// first on equal timestamps) and the groups rebuilt -> node-view jobs applied.
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

// k_stage for a directed batch, one workgroup per tile of GS_TILE records,
// also counting each tile's timestamp group starts into
// gcnt[tile] (a record whose timestamp differs from the one before it; the
// first record compared with last_ts when has_last): the counting pass of
// the group starts' compaction when the batch is appended as staged.
__global__ void __launch_bounds__(T)
k_stage_count(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
              const int64_t* __restrict__ ts, int64_t n, int32_t V, int32_t* __restrict__ b_src,
              int32_t* __restrict__ b_dst, int64_t* __restrict__ b_ts, uint32_t* err,
              unsigned long long* scalars, uint32_t* unsorted, int has_last,
              const int64_t* last_ts_p, uint32_t* __restrict__ gcnt) {
    __shared__ unsigned long long smin[T], smax[T];
    __shared__ uint32_t wsum[T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long lo = ~0ull, hi = 0ull;
    bool bad = false, down = false;
    {
        const int64_t tile = blockIdx.x;
        uint32_t c = 0;
        for (int r = 0; r < GS_TILE / T; ++r) {
            const int64_t i = tile * GS_TILE + r * T + threadIdx.x;
            bool start = false;
            if (i < n) {
                const int32_t u = src[i], v = dst[i];
                const int64_t t = ts[i];
                bad |= (u < 0 || u >= V || v < 0 || v >= V);
                if (i > 0) {
                    const int64_t tp = ts[i - 1];
                    down |= tp > t;
                    start = t != tp;
                } else {
                    start = !has_last || t != *last_ts_p;
                }
                const unsigned long long o = ord(t);
                lo = o < lo ? o : lo;
                hi = o > hi ? o : hi;
                b_src[i] = u;
                b_dst[i] = v;
                b_ts[i] = t;
            }
            c += (uint32_t)__popcll(__ballot(start));
        }
        if (lane == 0) wsum[wave] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t sum = 0;
#pragma unroll
            for (int w = 0; w < T / 64; ++w) sum += wsum[w];
            gcnt[tile] = sum;
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

// timestamps of the global groups (their first records')
__global__ void k_group_ts(const int64_t* __restrict__ e_ts, const uint32_t* __restrict__ gg_off,
                           int64_t Gg, int64_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * T + threadIdx.x;
    if (k < Gg) out[k] = e_ts[gg_off[k]];
}

// The first index of [0, n) where a monotone predicate (true, then false)
// is false, searched by one wavefront: each round the 64 lanes probe 64
// evenly spaced positions of the remaining range at once and keep the part
// between the last true and the first false probe, so a search over 2^28
// records takes 5 dependent loads instead of 28. Every lane returns it.
template <typename P>
__device__ int64_t wave_lower_bound(int64_t n, P pred) {
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t pos = lo + (int64_t)lane * step;
        const uint64_t yes = __ballot(pos < hi && pred(pos));
        const int64_t k = __popcll(yes);  // probes 0 .. k - 1 hold
        if (k == 0) return lo;
        const int64_t last = lo + (k - 1) * step;
        const int64_t next = lo + k * step;
        lo = last + 1;
        hi = next < hi ? next : hi;
    }
    return lo;
}

// Evicted prefix of the window (records with ts < cut: ev) and of its
// global groups (groups whose first record is evicted: the groups end at
// record boundaries of equal timestamps, so these are the groups that start
// before w_base + ev). One wavefront; lane 0 writes.
__device__ void evicted_prefix(const int64_t* __restrict__ w_ts, int64_t m, int64_t cut,
                               const uint32_t* __restrict__ gg_off, int64_t Gg, int64_t w_base,
                               uint32_t* sc_ev, uint32_t* sc_gev) {
    const int64_t ev = wave_lower_bound(m, [&](int64_t i) { return w_ts[i] < cut; });
    const uint64_t end = (uint64_t)(w_base + ev);
    const int64_t gev =
        wave_lower_bound(Gg, [&](int64_t i) { return (uint64_t)gg_off[i] < end; });
    if ((threadIdx.x & 63) == 0) {
        *sc_ev = (uint32_t)ev;
        *sc_gev = (uint32_t)gev;
    }
}

// Gg from the window summary slot (written by the last update); one wavefront
__global__ void k_evict_counts(const int64_t* __restrict__ w_ts, int64_t m, int64_t cut,
                               const uint32_t* __restrict__ gg_off, const int64_t* gg_p,
                               int64_t w_base, uint32_t* sc_ev, uint32_t* sc_gev) {
    evicted_prefix(w_ts, m, cut, gg_off, *gg_p, w_base, sc_ev, sc_gev);
}

// The window cut of an ingest from the staged batch's range (the same
// arithmetic as the host's once it reads the range back), and the searches
// it needs, each by the whole wavefront: the late prefix of a sorted batch
// (its length and first kept timestamp), the evicted prefix of the window
// and of its global groups. Each writes its default (no late record,
// nothing evicted) when its condition does not hold, so one read-back serves
// the whole decision.
__global__ void k_cut_counts(const unsigned long long* __restrict__ mm,
                             const uint32_t* __restrict__ unsorted, int has_time, int64_t t_now,
                             int64_t window, const int64_t* __restrict__ b_ts, int64_t B,
                             const int64_t* __restrict__ w_ts, int64_t m,
                             const int64_t* summary, const uint32_t* __restrict__ gg_off,
                             const int64_t* gg_p, int64_t w_base,
                             uint32_t* sc_kept, int64_t* first_kept, uint32_t* sc_ev,
                             uint32_t* sc_gev) {
    const int64_t bmin = unord(mm[0]), bmax = unord(mm[1]);
    const int64_t now = B > 0 ? (has_time ? (t_now > bmax ? t_now : bmax) : bmax) : t_now;
    const bool timed = has_time || B > 0;
    const bool windowed = window > 0 && timed;
    const int64_t cut = !windowed ? INT64_MIN
                        : (now < INT64_MIN + window ? INT64_MIN : now - window);
    const bool lane0 = threadIdx.x == 0;
    if (windowed && B > 0 && bmin < cut && *unsorted == 0u) {
        const int64_t lo = wave_lower_bound(B, [&](int64_t i) { return b_ts[i] < cut; });
        if (lane0) {
            *sc_kept = (uint32_t)lo;
            *first_kept = lo < B ? b_ts[lo] : INT64_MAX;
        }
    } else if (lane0) {
        *sc_kept = 0u;
        *first_kept = bmin;
    }
    if (windowed && m > 0 && summary[0] < cut) {
        evicted_prefix(w_ts, m, cut, gg_off, *gg_p, w_base, sc_ev, sc_gev);
    } else if (lane0) {
        *sc_ev = 0u;
        *sc_gev = 0u;
    }
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

// group-start flags of a batch appended after a window whose last timestamp
// is last_ts (has_last = 0: empty window)
__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_widen(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out,
                        int64_t minus) {
    int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i] - minus;
}

// the window's first and last timestamps and its global group count: the
// groups just counted (all of them when gg_full, else those appended after
// the gg_kept surviving ones); and where the window lies in the timestamp
// view (win: e_base, m, gg_base), so that a walk launch recorded in a HIP
// graph reads the current window when it is replayed
__global__ void k_window_summary(const int64_t* __restrict__ ts, int64_t m, int64_t* out,
                                 int gg_full, int64_t gg_kept, const uint32_t* groups,
                                 int64_t* gg_out, int64_t e_base, int64_t gg_base,
                                 int64_t* win) {
    out[0] = m > 0 ? ts[0] : 0;
    out[1] = m > 0 ? ts[m - 1] : 0;
    *gg_out = gg_full ? (int64_t)*groups : gg_kept + (int64_t)*groups;
    win[0] = e_base;
    win[1] = m;
    win[2] = gg_base;
}

uint32_t* u32_slot(tw_graph* g, int k) { return g->scal.as<uint32_t>() + k; }
int64_t* i64_slot(tw_graph* g, int k) { return g->scal.as<int64_t>() + k; }

tw_status ensure_common(tw_graph* g, Error& err) {
    if (!g->err.p) {
        // device error flags start cleared
        TW_HIP(ensure(g->err, sizeof(uint32_t) * 4, g->stream));
        TW_HIP(hipMemsetAsync(g->err.p, 0, sizeof(uint32_t) * 4, g->stream));
    }
    TW_HIP(ensure(g->scal, SCALAR_BYTES, g->stream));
    if (!g->h_scal) TW_HIP(hipHostMalloc(&g->h_scal, SCALAR_BYTES + 16, hipHostMallocDefault));
    return TW_OK;
}

// Moves the window to the front of edge-store buffers of at least `cap`
// records (e_base = 0). The capacity recorded is what every buffer of the
// timestamp view holds, so the allocator's rounding is not wasted. The global
// groups must be rebuilt afterwards.
tw_status grow_window(tw_graph* g, int64_t cap, Error& err) {
    cap = std::min<int64_t>(cap, (int64_t)UINT32_MAX - 1);
    TW_HIP(ensure(g->a_src, sizeof(int32_t) * cap, g->stream));
    TW_HIP(ensure(g->a_dst, sizeof(int32_t) * cap, g->stream));
    TW_HIP(ensure(g->a_ts, sizeof(int64_t) * cap, g->stream));
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
    TW_HIP(ensure(g->a_src, sizeof(int32_t) * cap, g->stream));
    TW_HIP(ensure(g->a_dst, sizeof(int32_t) * cap, g->stream));
    TW_HIP(ensure(g->a_ts, sizeof(int64_t) * cap, g->stream));
    TW_HIP(ensure(g->gg_off, sizeof(uint32_t) * (cap + 2), g->stream));
    int64_t held = (int64_t)UINT32_MAX - 1;
    for (const DevBuf* b : {&g->e_src, &g->e_dst, &g->a_src, &g->a_dst})
        held = std::min<int64_t>(held, (int64_t)(b->bytes / 4));
    for (const DevBuf* b : {&g->e_ts, &g->a_ts})
        held = std::min<int64_t>(held, (int64_t)(b->bytes / 8));
    held = std::min<int64_t>(held, (int64_t)(g->gg_off.bytes / 4) - 2);
    g->e_base = 0;
    g->e_cap = held;
    return TW_OK;
}

// Capacity of the edge-store buffers for a window of `need` records; growing
// copies the window to the front of the new buffers (e_base = 0).
tw_status reserve_window(tw_graph* g, int64_t need, Error& err) {
    if (need <= g->e_cap) return TW_OK;
    int64_t cap = std::max<int64_t>(need, 2 * g->e_cap);
    cap = std::max<int64_t>(cap, need + need / 2 + 1024);
    return grow_window(g, cap, err);
}

// Whether the device has room to grow the timestamp view to `cap` records
// (edge store, its alternates and the global groups: 44 bytes a record),
// keeping 1 GiB free.
bool window_growth_fits(tw_graph* g, int64_t cap) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const int64_t extra = std::max<int64_t>(cap - g->e_cap, 0) * 44;
    return (int64_t)free_b > extra + (1ll << 30);
}

// Global timestamp groups of the whole window, from scratch (gg_base = 0).
// The count lands in the GROUPS slot. counted (nullable): the window's group
// starts per tile, already counted (with no timestamp before the window).
tw_status build_ts_groups(tw_graph* g, Error& err, DevBuf* counted = nullptr) {
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    const int64_t* ts = g->e_ts.as<int64_t>() + g->e_base;
    uint32_t* G = u32_slot(g, SLOT_U32_GROUPS);
    TW_HIP(group_starts(0, 0, ts, m, (uint32_t)g->e_base, g->gg_off.as<uint32_t>(), G, g->ws,
                        s, counted));
    g->gg_base = 0;
    return TW_OK;
}

// Window timestamp range and global group count after an update, computed
// on the device: Gg is the GROUPS slot when gg_full, else gg_old -
// gg_evicted + GROUPS (appended groups). No synchronisation: the host
// mirrors follow with the next read-back of the slots.
tw_status finish_ts(tw_graph* g, bool gg_full, int64_t gg_old, int64_t gg_evicted, Error& err) {
    hipStream_t s = g->stream;
    hipLaunchKernelGGL(k_window_summary, dim3(1), dim3(1), 0, s, g->e_ts.as<int64_t>() + g->e_base,
                       g->m, i64_slot(g, SLOT_I64_SUMMARY), gg_full ? 1 : 0,
                       gg_old - gg_evicted, u32_slot(g, SLOT_U32_GROUPS),
                       i64_slot(g, SLOT_I64_GG), g->e_base, g->gg_base,
                       i64_slot(g, SLOT_I64_WIN));
    TW_HIP(hipGetLastError());
    g->sum_stale = true;
    return TW_OK;
}

}  // namespace

tw_status ingest_prepare(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                         int64_t n, IngestPlan& P, Error& err, bool walk_flags) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    const int64_t B = g->directed ? n : 2 * n;  // staged records
    if (g->m + B > (int64_t)UINT32_MAX - 2) {
        err = Error{TW_EINVAL, "window would exceed 2^32 - 2 records"};
        return err.code;
    }
    // Staging place of the batch: the free tail of the window buffers, else
    // the alternate buffers, else the staging buffers. A sorted batch staged
    // in the tail is appended where it lies; one staged in the alternates
    // becomes the window by a swap when nothing of the old window survives.
    int place = IngestPlan::IN_BUF;
    int32_t *s_src, *s_dst;
    int64_t* s_ts;
    if (B > 0 && g->e_base + g->m + B <= g->e_cap) {
        place = IngestPlan::IN_TAIL;
        const int64_t at = g->e_base + g->m;
        s_src = g->e_src.as<int32_t>() + at;
        s_dst = g->e_dst.as<int32_t>() + at;
        s_ts = g->e_ts.as<int64_t>() + at;
    } else if (B > 0 && B <= g->e_cap) {
        place = IngestPlan::IN_ALT;
        s_src = g->a_src.as<int32_t>();
        s_dst = g->a_dst.as<int32_t>();
        s_ts = g->a_ts.as<int64_t>();
    } else {
        TW_HIP(ensure(g->b_src, sizeof(int32_t) * (B + 1), g->stream));
        TW_HIP(ensure(g->b_dst, sizeof(int32_t) * (B + 1), g->stream));
        TW_HIP(ensure(g->b_ts, sizeof(int64_t) * (B + 1), g->stream));
        s_src = g->b_src.as<int32_t>();
        s_dst = g->b_dst.as<int32_t>();
        s_ts = g->b_ts.as<int64_t>();
    }

    unsigned long long* mm = reinterpret_cast<unsigned long long*>(i64_slot(g, SLOT_I64_MINMAX));
    uint32_t* errf = g->err.as<uint32_t>();
    uint32_t* unsorted = u32_slot(g, SLOT_U32_UNSORTED);
    hipLaunchKernelGGL(k_init_minmax, dim3(1), dim3(1), 0, s, mm, errf + 1, unsorted);
    // a directed batch also gets the group starts of its tiles, for the case
    // where it is appended as staged (the window's last timestamp before it)
    const bool staged_counts = g->directed && n > 0;
    const int stage_has_last = g->m > 0 ? 1 : 0;
    if (staged_counts) {
        const int64_t ntiles = ceil_div(n, (int64_t)GS_TILE);
        TW_HIP(ensure(g->gs_tiles, sizeof(uint32_t) * (ntiles + 1), g->stream));
        hipLaunchKernelGGL(k_stage_count, dim3((unsigned)ntiles), dim3(T), 0, s, src, dst, ts, n,
                           g->V, s_src, s_dst, s_ts, errf + 1, mm, unsorted, stage_has_last,
                           i64_slot(g, SLOT_I64_SUMMARY) + 1, g->gs_tiles.as<uint32_t>());
    } else if (n > 0) {
        hipLaunchKernelGGL(k_stage, dim3((unsigned)std::min<int64_t>(ceil_div(n, T), 2048)),
                           dim3(T), 0, s, src, dst, ts, n, g->V, g->directed ? 1 : 0, s_src, s_dst,
                           s_ts, errf + 1, mm, unsorted);
    }
    // the window's cut and its searches run on the device before the first
    // read-back (results for the cases that need them; defaults otherwise)
    uint32_t* sc_kept = u32_slot(g, SLOT_U32_KEPT);
    uint32_t* sc_ev = u32_slot(g, SLOT_U32_EVICTED);
    uint32_t* sc_gev = u32_slot(g, SLOT_U32_GG_EVICTED);
    int64_t* first_kept = i64_slot(g, SLOT_I64_FIRST_KEPT);
    if (g->window > 0)
        hipLaunchKernelGGL(k_cut_counts, dim3(1), dim3(64), 0, s, mm, unsorted,
                           g->has_time ? 1 : 0, g->t_now, g->window, s_ts, B,
                           g->e_ts.as<int64_t>() + g->e_base, g->m,
                           i64_slot(g, SLOT_I64_SUMMARY), g->gg_off.as<uint32_t>() + g->gg_base,
                           i64_slot(g, SLOT_I64_GG), g->e_base, sc_kept, first_kept, sc_ev,
                           sc_gev);
    TW_HIP(hipGetLastError());
    if (pull_scalars(g, true, err) != TW_OK) return err.code;
    const uint64_t hmm[2] = {(uint64_t)host_i64(g, SLOT_I64_MINMAX),
                             (uint64_t)host_i64(g, SLOT_I64_MINMAX + 1)};
    const uint32_t herr = host_flags(g)[1], hunsorted = host_u32(g, SLOT_U32_UNSORTED);
    if (walk_flags && (host_flags(g)[0] || host_flags(g)[3])) {
        // errors of earlier walks, read back with this batch's counts: they
        // are reported (and cleared) instead of ingesting
        const bool range = host_flags(g)[0] != 0;
        uint32_t* d = g->err.as<uint32_t>();
        TW_HIP(hipMemsetAsync(d, 0, sizeof(uint32_t), s));
        TW_HIP(hipMemsetAsync(d + 3, 0, sizeof(uint32_t), s));
        TW_HIP(hipStreamSynchronize(s));
        err = range ? Error{TW_ERANGE, "a walk start node was outside [0, num_nodes)"}
                    : Error{TW_EINVAL,
                            "a batched walk had a length limit, bias index or row out of range"};
        return err.code;
    }
    if (herr) {
        err = Error{TW_ERANGE, "ingest_batch: node id outside [0, num_nodes)"};
        return err.code;
    }
    // the clock advances only when the ingest completes
    int64_t bmin = 0, bmax = 0, t_now = g->t_now;
    bool has_time = g->has_time;
    if (n > 0) {
        bmin = unord(hmm[0]);
        bmax = unord(hmm[1]);
        t_now = has_time ? std::max(t_now, bmax) : bmax;
        has_time = true;
    }
    const bool sorted = hunsorted == 0;

    // window cut, late drop and eviction counts
    const bool windowed = g->window > 0 && has_time;
    int64_t cut = INT64_MIN;
    if (windowed) cut = (t_now < INT64_MIN + g->window) ? INT64_MIN : t_now - g->window;
    const bool drop = windowed && B > 0 && bmin < cut;
    const bool evicting = windowed && g->m > 0 && g->t_min < cut;
    int64_t kept = B, evicted = 0, gg_evicted = 0, batch_first = bmin, drop_lo = 0;
    const int64_t key_base = drop ? cut : bmin;
    uint64_t* keys = nullptr;
    uint32_t* vals = nullptr;
    if (drop && sorted) {
        // late records of a sorted batch are a prefix (its length came back)
        drop_lo = host_u32(g, SLOT_U32_KEPT);
        kept = B - drop_lo;
        batch_first = host_i64(g, SLOT_I64_FIRST_KEPT);
    } else if (!sorted && B > 0) {
        TW_HIP(ensure(g->b_keys, sizeof(uint64_t) * (B + 1), g->stream));
        TW_HIP(ensure(g->b_vals, sizeof(uint32_t) * (B + 1), g->stream));
        keys = g->b_keys.as<uint64_t>();
        vals = g->b_vals.as<uint32_t>();
        if (drop) {
            TW_HIP(ensure(g->b_flags, sizeof(uint32_t) * (B + 1), g->stream));
            TW_HIP(ensure(g->idx, sizeof(uint32_t) * (B + 1), g->stream));
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
        evicted = host_u32(g, SLOT_U32_EVICTED);
        gg_evicted = host_u32(g, SLOT_U32_GG_EVICTED);
    }
    TW_HIP(hipGetLastError());
    if (drop && !sorted) {
        if (pull_scalars(g, false, err) != TW_OK) return err.code;
        kept = host_u32(g, SLOT_U32_KEPT);
        batch_first = cut;  // a lower bound of the kept records
    }

    // the kept batch records in timestamp order (stable)
    const int32_t* q_src = s_src + drop_lo;
    const int32_t* q_dst = s_dst + drop_lo;
    const int64_t* q_ts = s_ts + drop_lo;
    if (!sorted && kept > 0) {
        int kb = bits_for((uint64_t)(bmax - key_base));
        TW_HIP(radix_sort_u64(keys, vals, kept, 0, kb, g->ws, s));
        TW_HIP(ensure(g->q_src, sizeof(int32_t) * (kept + 1), g->stream));
        TW_HIP(ensure(g->q_dst, sizeof(int32_t) * (kept + 1), g->stream));
        TW_HIP(ensure(g->q_ts, sizeof(int64_t) * (kept + 1), g->stream));
        hipLaunchKernelGGL(k_gather_batch, grid_for(kept), dim3(T), 0, s, vals, kept, s_src, s_dst,
                           s_ts, g->q_src.as<int32_t>(), g->q_dst.as<int32_t>(),
                           g->q_ts.as<int64_t>());
        q_src = g->q_src.as<int32_t>();
        q_dst = g->q_dst.as<int32_t>();
        q_ts = g->q_ts.as<int64_t>();
    }

    // node-view jobs, while the evicted records are still in the window
    // buffers (none when the whole window goes: the node view is emptied)
    const bool evict_all = evicting && evicted == g->m;
    if (nv_collect(g, q_src, q_dst, q_ts, kept, bmin, bmax, evict_all ? 0 : g->e_base,
                   evict_all ? 0 : evicted, err) != TW_OK)
        return err.code;
    P = IngestPlan{};
    P.n = n;
    P.B = B;
    P.place = place;
    P.s_src = s_src;
    P.s_dst = s_dst;
    P.s_ts = s_ts;
    P.q_src = q_src;
    P.q_dst = q_dst;
    P.q_ts = q_ts;
    P.staged_counts = staged_counts;
    P.stage_has_last = stage_has_last;
    P.bmin = bmin;
    P.t_now = t_now;
    P.has_time = has_time;
    P.sorted = sorted;
    P.evicting = evicting;
    P.evict_all = evict_all;
    P.cut = cut;
    P.kept = kept;
    P.evicted = evicted;
    P.gg_evicted = gg_evicted;
    P.batch_first = batch_first;
    P.drop_lo = drop_lo;
    P.m_old = g->m;
    P.e_base = g->e_base;
    P.epoch = g->epoch;
    return TW_OK;
}

tw_status ingest_apply(tw_graph* g, const IngestPlan& P, tw_ingest_info* info, Error& err) {
    hipStream_t s = g->stream;
    if (P.m_old != g->m || P.e_base != g->e_base || P.epoch != g->epoch) {
        err = Error{TW_EINVAL, "ingest: the index changed between planning and applying a batch"};
        return err.code;
    }
    const int64_t B = P.B, kept = P.kept, evicted = P.evicted, gg_evicted = P.gg_evicted;
    const int64_t batch_first = P.batch_first, drop_lo = P.drop_lo, cut = P.cut;
    const bool sorted = P.sorted, evicting = P.evicting, staged_counts = P.staged_counts;
    const int stage_has_last = P.stage_has_last;
    const int place = P.place;
    const int32_t* q_src = P.q_src;
    const int32_t* q_dst = P.q_dst;
    const int64_t* q_ts = P.q_ts;
    // From here on the index changes in place: a failure before the end
    // leaves the graph marked unusable (every later call refuses it).
    g->broken = true;
    const int64_t m_old = g->m;
    // the node2vec pairs: the evicted prefix of the window down, the kept
    // batch records up (both still where the plan found them)
    if (adj_update(g, g->e_src.as<int32_t>() + g->e_base, g->e_dst.as<int32_t>() + g->e_base,
                   evicted, q_src, q_dst, kept, err) != TW_OK)
        return err.code;
    if (P.evict_all) {
        const int64_t jobs = g->T;  // the batch's jobs, collected by the plan
        if (nv_reset(g, err) != TW_OK) return err.code;
        g->T = jobs;
    }

    // timestamp view: a batch that starts at or after the window's last
    // timestamp is appended in place (eviction only moves e_base); any other
    // batch is merged (merge path, older records first on equal timestamps)
    const int64_t na = m_old - evicted;
    const int64_t m_new = na + kept;
    const bool append = na == 0 || kept == 0 || batch_first >= g->t_max;
    const int64_t last_ts = g->t_max;
    const int64_t gg_old = g->Gg;
    bool gg_full = false;
    // A sorted batch still lies where it was staged. In the window tail it
    // stays there when appended after the surviving records (no late prefix
    // in between) or when it is the whole new window, and a merge only reads
    // it; in the alternates it stays when it is the whole new window. In any
    // other case the update would move it over itself or overwrite it, so it
    // is copied to the staging buffers first.
    const bool q_tail = sorted && kept > 0 && place == IngestPlan::IN_TAIL;
    const bool q_alt = sorted && kept > 0 && place == IngestPlan::IN_ALT;
    const bool keep_tail = q_tail && (!append || na == 0 || drop_lo == 0);
    const bool keep_alt = q_alt && append && na == 0;
    if ((q_tail && !keep_tail) || (q_alt && !keep_alt)) {
        TW_HIP(ensure(g->b_src, sizeof(int32_t) * (kept + 1), g->stream));
        TW_HIP(ensure(g->b_dst, sizeof(int32_t) * (kept + 1), g->stream));
        TW_HIP(ensure(g->b_ts, sizeof(int64_t) * (kept + 1), g->stream));
        TW_HIP(hipMemcpyAsync(g->b_src.p, q_src, 4 * kept, hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->b_dst.p, q_dst, 4 * kept, hipMemcpyDeviceToDevice, s));
        TW_HIP(hipMemcpyAsync(g->b_ts.p, q_ts, 8 * kept, hipMemcpyDeviceToDevice, s));
        q_src = g->b_src.as<int32_t>();
        q_dst = g->b_dst.as<int32_t>();
        q_ts = g->b_ts.as<int64_t>();
    }
    if (append) {
        g->e_base += evicted;
        g->gg_base += gg_evicted;
        if (na == 0) {
            g->e_base = 0;
            g->gg_base = 0;
            if (keep_tail) {
                g->e_base = q_src - g->e_src.as<int32_t>();
            } else if (keep_alt) {
                std::swap(g->e_src, g->a_src);
                std::swap(g->e_dst, g->a_dst);
                std::swap(g->e_ts, g->a_ts);
                g->e_base = drop_lo;
            }
        }
        // the batch already lies at e_base + na (and fits: it was staged
        // inside the buffers' capacity)
        const bool placed = keep_tail || keep_alt;
        g->m = na;
        if (!placed && g->e_base + m_new > g->e_cap) {
            // After a move to the front, the free tail should take about as
            // many records as the window holds, so that a record is moved
            // about once while it is in the window: a tighter buffer grows
            // instead (when the device has room), which moves it as well.
            const int64_t roomy = 2 * m_new + kept;
            const bool grow = roomy > g->e_cap && window_growth_fits(g, roomy);
            if (grow) {
                if (grow_window(g, roomy, err) != TW_OK) return err.code;
            } else if (m_new <= g->e_cap && g->m > 0) {
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
        if (kept > 0 && !placed) {
            const int64_t at = g->e_base + na;
            TW_HIP(hipMemcpyAsync(g->e_src.as<int32_t>() + at, q_src, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->e_dst.as<int32_t>() + at, q_dst, 4 * kept,
                                  hipMemcpyDeviceToDevice, s));
            TW_HIP(hipMemcpyAsync(g->e_ts.as<int64_t>() + at, q_ts, 8 * kept,
                                  hipMemcpyDeviceToDevice, s));
        }
        g->m = m_new;
        // the stage counted the group starts of the batch as staged: they
        // serve when the whole batch is kept in order and compared with the
        // same predecessor (the window's last timestamp, or none)
        const bool as_staged = staged_counts && sorted && drop_lo == 0 && kept == B;
        if (gg_full || na == 0) {
            // the window is the batch alone when nothing of the old one survives
            const bool use = as_staged && na == 0 && stage_has_last == 0;
            gg_full = true;
            if (build_ts_groups(g, err, use ? &g->gs_tiles : nullptr) != TW_OK) return err.code;
        } else if (kept > 0) {
            const bool use = as_staged && stage_has_last == 1;
            uint32_t* G = u32_slot(g, SLOT_U32_GROUPS);
            const int64_t gpos = g->gg_base + (gg_old - gg_evicted);
            TW_HIP(group_starts(1, last_ts, q_ts, kept, (uint32_t)(g->e_base + na),
                                g->gg_off.as<uint32_t>() + gpos, G, g->ws, s,
                                use ? &g->gs_tiles : nullptr));
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

    if (nv_apply(g, evicting && evicted < m_old, cut, err) != TW_OK) return err.code;
    if (finish_ts(g, gg_full, gg_old, gg_evicted, err) != TW_OK) return err.code;

    g->t_now = P.t_now;
    g->has_time = P.has_time;
    // every window record is at or after the cut now
    if (P.cut > g->t_min_lb) g->t_min_lb = P.cut;
    g->broken = false;
    g->last.accepted = kept;
    g->last.dropped_late = B - kept;
    g->last.evicted = evicted;
    g->last.active_edges = g->m;
    if (info) {
        // the caller asked for the window's range: read the summary back
        if (refresh_summary(g, err) != TW_OK) return err.code;
        g->last.t_min = g->t_min;
        g->last.t_max = g->t_max;
        *info = g->last;
    }
    return TW_OK;
}

tw_status ingest(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                 int64_t n, tw_ingest_info* info, Error& err) {
    IngestPlan P;
    if (ingest_prepare(g, src, dst, ts, n, P, err) != TW_OK) return err.code;
    return ingest_apply(g, P, info, err);
}

tw_status evict_before(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    int64_t ev = 0, gev = 0;
    if (g->m > 0 && cutoff > (g->sum_stale ? g->t_min_lb : g->t_min)) {
        uint32_t* sc_ev = u32_slot(g, SLOT_U32_EVICTED);
        uint32_t* sc_gev = u32_slot(g, SLOT_U32_GG_EVICTED);
        hipLaunchKernelGGL(k_evict_counts, dim3(1), dim3(64), 0, s,
                           g->e_ts.as<int64_t>() + g->e_base, g->m, cutoff,
                           g->gg_off.as<uint32_t>() + g->gg_base, i64_slot(g, SLOT_I64_GG),
                           g->e_base, sc_ev, sc_gev);
        if (pull_scalars(g, false, err) != TW_OK) return err.code;
        ev = host_u32(g, SLOT_U32_EVICTED);
        gev = host_u32(g, SLOT_U32_GG_EVICTED);
    }
    if (ev > 0) {
        const int64_t m_old = g->m, gg_old = g->Gg;
        g->broken = true;  // cleared when the eviction completes
        if (adj_update(g, g->e_src.as<int32_t>() + g->e_base, g->e_dst.as<int32_t>() + g->e_base,
                       ev, nullptr, nullptr, 0, err) != TW_OK)
            return err.code;
        if (ev == m_old) {
            if (nv_reset(g, err) != TW_OK) return err.code;
        } else if (nv_collect(g, nullptr, nullptr, nullptr, 0, 0, 0, g->e_base, ev, err) !=
                   TW_OK) {
            return err.code;
        }
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
            if (nv_apply(g, true, cutoff, err) != TW_OK) return err.code;
        }
        if (finish_ts(g, gg_full, gg_old, gev, err) != TW_OK) return err.code;
        g->broken = false;
    }
    if (cutoff > g->t_min_lb) g->t_min_lb = cutoff;
    g->last.accepted = 0;
    g->last.dropped_late = 0;
    g->last.evicted = ev;
    g->last.active_edges = g->m;
    if (n_evicted) *n_evicted = ev;
    return TW_OK;
}

tw_status backward_view(tw_graph* g, tw_graph** out, Error& err) {
    if (!g->directed) {
        *out = g;
        return TW_OK;
    }
    if (!g->rev) {
        if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
        tw_graph* r = new tw_graph();
        r->V = g->V;
        r->directed = true;
        r->window = g->window;
        r->stream = g->stream;
        r->device = g->device;
        // the same clock: late drops and cuts of later batches agree
        r->t_now = g->t_now;
        r->has_time = g->has_time;
        g->rev = r;
        // the window's records, source and destination swapped, in one batch
        // (in canonical order, so ties keep their arrival order)
        if (g->m > 0 &&
            ingest(r, g->e_dst.as<int32_t>() + g->e_base, g->e_src.as<int32_t>() + g->e_base,
                   g->e_ts.as<int64_t>() + g->e_base, g->m, nullptr, err) != TW_OK) {
            release_graph(r);
            g->rev = nullptr;
            return err.code;
        }
    }
    *out = g->rev;
    return TW_OK;
}

void release_graph(tw_graph* g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    release_graph(g->rev);
    for (DevBuf* b : g->buffers()) release(*b, g->stream);
    (void)hipStreamSynchronize(g->stream);
    if (g->h_scal) (void)hipHostFree(g->h_scal);
    delete g;
}

// The weight-based picker's cumulative weights, rebuilt with the index
// when the graph asks for them at ingest. A failed build leaves them to the
// next weight-based walk, which builds them itself.
static void ingest_weights(tw_graph* g) {
    if (std::isnan(g->ingest_weight_tau) || g->m == 0) return;
    Error e{TW_OK, ""};
    if (build_weights(g, g->ingest_weight_tau, e) != TW_OK) {
        (void)hipGetLastError();
        g->w_ready = false;
    }
}

tw_status ingest_views(tw_graph* g, const int32_t* src, const int32_t* dst, const int64_t* ts,
                       int64_t n, tw_ingest_info* info, Error& err, hipEvent_t before_apply,
                       bool walk_flags) {
    IngestPlan P;
    if (ingest_prepare(g, src, dst, ts, n, P, err, walk_flags) != TW_OK) return err.code;
    // the index changes only after the event: work it marks (walks over the
    // current index) may run while the batch is planned
    if (before_apply) TW_HIP(hipStreamWaitEvent(g->stream, before_apply, 0));
    if (ingest_apply(g, P, info, err) != TW_OK) return err.code;
    ingest_weights(g);
    if (g->rev) {
        // the in-view takes the batch with source and destination swapped;
        // if that fails it is dropped and rebuilt from the window on the next
        // backward walk, so the graph stays consistent either way
        Error e{TW_OK, ""};
        if (ingest(g->rev, dst, src, ts, n, nullptr, e) != TW_OK) {
            release_graph(g->rev);
            g->rev = nullptr;
        }
    }
    return TW_OK;
}

tw_status evict_views(tw_graph* g, int64_t cutoff, int64_t* n_evicted, Error& err) {
    if (evict_before(g, cutoff, n_evicted, err) != TW_OK) return err.code;
    ingest_weights(g);
    if (g->rev) {
        Error e{TW_OK, ""};
        if (evict_before(g->rev, cutoff, nullptr, e) != TW_OK) {
            release_graph(g->rev);
            g->rev = nullptr;
        }
    }
    return TW_OK;
}

tw_status pull_scalars(tw_graph* g, bool flags, Error& err) {
    hipStream_t s = g->stream;
    if (ensure_common(g, err) != TW_OK) return err.code;
    TW_HIP(hipMemcpyAsync(g->h_scal, g->scal.p, SCALAR_BYTES, hipMemcpyDeviceToHost, s));
    if (flags)
        TW_HIP(hipMemcpyAsync(static_cast<char*>(g->h_scal) + SCALAR_BYTES, g->err.p, 16,
                              hipMemcpyDeviceToHost, s));
    TW_HIP(hipStreamSynchronize(s));
    if (g->sum_stale) {
        // the slots of the last finished update came back too
        g->t_min = host_i64(g, SLOT_I64_SUMMARY);
        g->t_max = host_i64(g, SLOT_I64_SUMMARY + 1);
        g->Gg = host_i64(g, SLOT_I64_GG);
        g->sum_stale = false;
    }
    return TW_OK;
}

tw_status refresh_summary(tw_graph* g, Error& err) {
    if (!g->sum_stale) return TW_OK;
    return pull_scalars(g, false, err);
}

tw_status init_empty(tw_graph* g, Error& err) {
    if (ensure_common(g, err) != TW_OK) return err.code;
    if (reserve_window(g, 1024, err) != TW_OK) return err.code;
    g->m = 0;
    if (nv_reset(g, err) != TW_OK) return err.code;
    if (build_ts_groups(g, err) != TW_OK) return err.code;
    return finish_ts(g, true, 0, 0, err);
}

tw_status export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                       int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                       int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg, Error& err) {
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    if (refresh_summary(g, err) != TW_OK) return err.code;
    auto cp = [&](void* d, const void* sp, size_t bytes) -> hipError_t {
        if (!d || bytes == 0) return hipSuccess;
        return hipMemcpyAsync(d, sp, bytes, hipMemcpyDeviceToDevice, s);
    };
    TW_HIP(cp(src, g->e_src.as<int32_t>() + g->e_base, sizeof(int32_t) * m));
    TW_HIP(cp(dst, g->e_dst.as<int32_t>() + g->e_base, sizeof(int32_t) * m));
    TW_HIP(cp(ts, g->e_ts.as<int64_t>() + g->e_base, sizeof(int64_t) * m));
    if (g_ts && g->Gg > 0)
        hipLaunchKernelGGL(k_group_ts, grid_for(g->Gg), dim3(T), 0, s, g->e_ts.as<int64_t>(),
                           g->gg_off.as<uint32_t>() + g->gg_base, g->Gg, g_ts);
    if (g_off)
        hipLaunchKernelGGL(k_widen, grid_for(g->Gg + 1), dim3(T), 0, s,
                           g->gg_off.as<uint32_t>() + g->gg_base, g->Gg + 1, g_off, g->e_base);
    TW_HIP(hipGetLastError());
    if (nv_export(g, n_dst, n_ts, n_gts, n_goff, n_ebeg, n_gbeg, err) != TW_OK) return err.code;
    TW_HIP(hipStreamSynchronize(s));
    return TW_OK;
}

}  // namespace tw
