// Device-side pieces of a hop: counter-based RNG, the closed-form pickers
// and the causal-neighbourhood search (Tempest, Sec. "Dual-Index
// Organization" and "Temporal Bias Sampling").
#pragma once

#include "tw_internal.h"

namespace tw {

// Four 64-bit words of Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11,
// "Parallel random numbers: as easy as 1, 2, 3") for counter
// (walk, hop, trial, 0) and key (seed, 0).
struct Draw {
    uint64_t x0, x1, x2, x3;
};

__device__ __forceinline__ Draw philox(uint64_t walk, uint64_t hop, uint64_t trial, uint64_t seed) {
    uint64_t c0 = walk, c1 = hop, c2 = trial, c3 = 0;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t hi0 = __umul64hi(m0, c0), lo0 = m0 * c0;
        uint64_t hi1 = __umul64hi(m1, c2), lo1 = m1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    return Draw{c0, c1, c2, c3};
}

// floor(x * n / 2^64): Eq. (1) with u = x / 2^64
__device__ __forceinline__ uint64_t scale_u64(uint64_t x, uint64_t n) { return __umul64hi(x, n); }

// (2 (x>>12) + 1) 2^-53, in (0, 1)
__device__ __forceinline__ double unit_open(uint64_t x) {
    return (double)(2 * (x >> 12) + 1) * 0x1.0p-53;
}
// (x>>11) 2^-53, in [0, 1)
__device__ __forceinline__ double unit_closed_open(uint64_t x) {
    return (double)(x >> 11) * 0x1.0p-53;
}

// Eq. (2) over n >= 1 groups with u = (x>>11) / 2^53. The square root is
// taken in FP64; the index is then fixed up against the exact integer
// condition i(i+1) 2^53 <= a n(n+1), so the result is exact.
__device__ __forceinline__ uint32_t pick_linear(uint32_t n, uint64_t x) {
    const uint64_t a = x >> 11;
    const uint64_t nn1 = (uint64_t)n * ((uint64_t)n + 1);
    const uint64_t ahi = __umul64hi(a, nn1), alo = a * nn1;
    auto le = [&](uint64_t i) {
        uint64_t ii1 = i * (i + 1);
        uint64_t hi = ii1 >> 11, lo = ii1 << 53;
        return hi < ahi || (hi == ahi && lo <= alo);
    };
    double u = (double)a * 0x1.0p-53;
    double r = (sqrt(1.0 + 4.0 * u * (double)nn1) - 1.0) * 0.5;
    int64_t i = (int64_t)r;
    if (i < 0) i = 0;
    if (i > (int64_t)n - 1) i = (int64_t)n - 1;
    while (i + 1 < (int64_t)n && le((uint64_t)i + 1)) ++i;
    while (i > 0 && !le((uint64_t)i)) --i;
    return (uint32_t)i;
}

// lambda of Eq. (3) for n groups spanning [t_first, t_last]
__device__ __forceinline__ double exp_lambda(int64_t t_first, int64_t t_last, uint32_t n,
                                             double tau) {
    if (tau <= 0.0 || n <= 1) return 1.0;
    return (double)(t_last - t_first) / ((double)(n - 1) * tau);
}

// Eq. (3) as the exact inverse CDF of P(i) ~ exp(lambda i), i in [0, n)
__device__ __forceinline__ uint32_t pick_exponential(uint32_t n, double lam, uint64_t x) {
    if (n <= 1) return 0;
    double u = unit_open(x);
    double ln = lam * (double)n;
    double xi;
    if (ln <= 1.0)
        xi = log1p(u * expm1(ln)) / lam;
    else
        xi = (double)n + log(u + (1.0 - u) * exp(-ln)) / lam;
    double f = floor(xi);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(n - 1)) return n - 1;
    return (uint32_t)f;
}

// count of the groups [lo, hi) (timestamps ascending) whose timestamp is
// <= t: a few are counted directly, longer ranges by binary search
__device__ __forceinline__ uint32_t count_le(const GroupRec* __restrict__ ng, uint32_t lo,
                                             uint32_t hi, int64_t t) {
    if (hi - lo <= 4) {
        uint32_t c = 0;
        for (uint32_t j = lo; j < hi; ++j) c += (ng[j].ts <= t);
        return c;
    }
    uint32_t a = lo, b = hi;
    while (a < b) {
        const uint32_t mid = a + ((b - a) >> 1);
        if (ng[mid].ts <= t) a = mid + 1; else b = mid;
    }
    return a - lo;
}

// Entries of one 8-word key window <= the query, exactly: keys below q
// count, keys equal to q are decided by their group's timestamp (group
// index g0 + (lo + i) * step for entry i).
__device__ __forceinline__ uint32_t window_count(const uint32_t* win, uint32_t q, int64_t t,
                                                 const GroupRec* __restrict__ ng, uint64_t gbase,
                                                 uint64_t step) {
    const uint4 a = reinterpret_cast<const uint4*>(win)[0];
    const uint4 b = reinterpret_cast<const uint4*>(win)[1];
    const uint32_t k[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t lt = 0, le = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        lt += k[j] < q;
        le += k[j] <= q;
    }
    for (uint32_t j = lt; j < le; ++j) lt += ng[gbase + j * step].ts <= t;
    return lt;
}

// Gamma lookup (Sec. "Dual-Index Organization": the node's first timestamp
// group strictly after t) through the node's fence: with the key base and
// shift from the node record, one 8-word key window per level from the top
// level in use down to level 0. Requires t < r.t_last, so the result is below r.ge.
// Returns the absolute group index. panel (nullable) holds fence words
// [panel_base, panel_base + panel_len) in LDS; windows inside it are read
// from there.
__device__ __forceinline__ uint32_t fence_search(const GroupRec* __restrict__ ng,
                                                 const uint32_t* __restrict__ fence,
                                                 const NodeRec& r, int64_t t,
                                                 const uint32_t* panel, uint64_t panel_base,
                                                 uint32_t panel_len) {
    const int K = (int)rec_levels(r.lv);
    if (K == 0) return r.gb + count_le(ng, r.gb, r.ge, t);
    const int64_t base = r.kbase;
    if (t < base) return r.gb;  // every group of the segment is later
    const uint32_t q = (uint32_t)((uint64_t)(t - base) >> rec_shift(r.lv));
    const uint64_t cap = seg_groups(rec_code(r.lv));
    int k = K;
    uint64_t lo = 0;
    // A deep fence starts lower: at level k0, whose entries are 8^k0 groups
    // apart with 8^k0 about sqrt(n) / 4, the window around the entry that
    // t's place between the segment's first and last timestamps predicts.
    // When that window brackets t (a key <= t, and one > t or the level's
    // end), the descent goes on from there; otherwise from the top.
    const uint32_t n = r.ge - r.g0;
    const int k0 = (31 - __clz(n) + 2) / 6;
    if (k0 + 1 < K) {
        const uint64_t cnt = (n + (1ull << (FENCE_LOG * k0)) - 1) >> (FENCE_LOG * k0);
        const double fr = (double)(t - base) / (double)(r.t_last - base);
        const uint64_t e = (uint64_t)(fr * (double)cnt);
        uint64_t lo0 = e >= 4 ? (e - 4) & ~3ull : 0;  // 16-byte aligned
        const uint64_t top = ((cnt + FENCE_FAN - 1) & ~(uint64_t)(FENCE_FAN - 1)) - FENCE_FAN;
        if (lo0 > top) lo0 = top;
        const uint64_t at = r.fence_off + fence_level_off(cap, k0) + lo0;
        const uint32_t* win = at >= panel_base && at + FENCE_FAN <= panel_base + panel_len
                                  ? panel + (at - panel_base)
                                  : fence + at;
        const uint32_t c = window_count(win, q, t, ng, r.g0 + (lo0 << (FENCE_LOG * k0)),
                                        1ull << (FENCE_LOG * k0));
        if (c >= 1 && (c < FENCE_FAN || lo0 + FENCE_FAN >= cnt)) {
            if (k0 == 0) {
                const uint32_t res = r.g0 + (uint32_t)lo0 + c;
                return res < r.gb ? r.gb : res;
            }
            k = k0 - 1;
            lo = (lo0 + c - 1) * FENCE_FAN;
        }
    }
    uint64_t off = fence_level_off(cap, k);
    for (; k >= 0; --k) {
        const uint64_t at = r.fence_off + off + lo;
        const uint32_t* win = at >= panel_base && at + FENCE_FAN <= panel_base + panel_len
                                  ? panel + (at - panel_base)
                                  : fence + at;
        const uint32_t c =
            window_count(win, q, t, ng, r.g0 + (lo << (FENCE_LOG * k)), 1ull << (FENCE_LOG * k));
        if (k == 0) {
            const uint32_t res = r.g0 + (uint32_t)lo + c;
            return res < r.gb ? r.gb : res;
        }
        // c == 0 only at the top level: t precedes the segment's first group
        if (c == 0) return r.gb;
        lo = (lo + c - 1) * FENCE_FAN;
        off -= fence_level_len(cap, k - 1);
    }
    return r.gb;  // not reached
}

// Does the window hold an edge src -> dst (node2vec's adjacency test)? One
// probe sequence of the pair table: the pair's slot (its count > 0 while
// records of the pair are in the window) or an empty slot first.
__device__ __forceinline__ bool adj_has(const AdjSlot* __restrict__ tab, uint64_t mask,
                                        int32_t src, int32_t dst) {
    const uint64_t k = adj_key(src, dst);
    uint64_t j = adj_hash(k) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe, j = (j + 1) & mask) {
        const AdjSlot e = tab[j];
        if (e.key == k) return e.cnt > 0;
        if (e.key == ADJ_EMPTY) return false;
    }
    return false;
}

// The group index picked among n groups by a linear or exponential bias.
__device__ __forceinline__ uint32_t pick_group(uint32_t n, int kind, double tau, int64_t t_first,
                                               int64_t t_last, uint64_t x) {
    if (kind == TW_LINEAR) return pick_linear(n, x);
    return pick_exponential(n, exp_lambda(t_first, t_last, n, tau), x);
}

// Does a pick of this kind read its first candidate's timestamp?
__device__ __forceinline__ bool reads_first_ts(int kind) {
    return kind == TW_EXPONENTIAL || kind == TW_NODE2VEC;
}

// Timestamp of group g of node record r. Level 0 of a fence starts it and
// keys every group of the segment, so with unshifted keys the timestamp is
// the key base plus g's level-0 key: a word of the window a search ending
// near g has just read, where g's group record is another line.
__device__ __forceinline__ int64_t group_ts(const GroupRec* __restrict__ ng,
                                           const uint32_t* __restrict__ fence, const NodeRec& r,
                                           uint32_t g) {
    if (rec_levels(r.lv) > 0 && rec_shift(r.lv) == 0)
        return r.kbase + (int64_t)fence[(uint64_t)r.fence_off + (g - r.g0)];
    return ng[g].ts;
}

// A pick in the node view among the groups [gc, ge) of a node whose edges
// end at `end`: uniform over the edges, or biased over the groups and then
// uniform inside the group. A group record carries the destination of the
// group's first edge, so a one-edge group needs no edge load.
struct Pick {
    int32_t dst;
    int64_t t;
};

// rev: a backward walk lists the candidates in reverse, so every index i
// among n (the edge, the group, the edge inside the group) becomes n - 1 - i.
// t_first and t_last are the timestamps of the first and the last candidate
// group, gc and ge - 1 (t_first is read by the exponential picker only).
__device__ __forceinline__ Pick pick_node(const GroupRec* __restrict__ ng,
                                          const int32_t* __restrict__ n_dst,
                                          const int64_t* __restrict__ n_ts, uint32_t gc,
                                          uint32_t ge, uint32_t end, int kind, double tau,
                                          int64_t t_first, int64_t t_last, const Draw& d,
                                          bool rev = false) {
    if (kind == TW_UNIFORM) {
        const uint32_t c = ng[gc].first;
        const uint32_t i = (uint32_t)scale_u64(d.x0, end - c);
        const uint32_t e = rev ? end - 1 - i : c + i;
        return Pick{n_dst[e], n_ts[e]};
    }
    const uint32_t n = ge - gc;
    const uint32_t i = pick_group(n, kind, tau, n > 1 ? t_first : 0, t_last, d.x0);
    const uint32_t k = rev ? ge - 1 - i : gc + i;
    const GroupRec a = ng[k];
    if (a.dst < 0) return Pick{a.dst & 0x7fffffff, a.ts};  // a one-edge group
    const uint32_t size = (k + 1 < ge ? ng[k + 1].first : end) - a.first;
    const uint32_t j = (uint32_t)scale_u64(d.x1, size);
    return Pick{n_dst[a.first + (rev ? size - 1 - j : j)], a.ts};
}

// The weight-based pick (Sec. "Temporal Bias Sampling") among groups
// [gc, ge) of a node whose live groups start at gb and whose edges end at
// end: cw holds the node's cumulative group weights (weights exp((ts -
// t_last) / sc) per edge). r = u times the candidates' total weight; the
// group is the first whose cumulative weight reaches the candidates' prefix
// plus r (the last candidate when rounding leaves none), and the edge inside
// it the one whose share of the group's weight r falls in (every edge of a
// group weighs the same), so one draw selects the edge, as the edge-by-edge
// inversion does. t_first is the timestamp of group gc.
//
// The search starts at a predicted group: with evenly spaced timestamps the
// group weights grow by a constant factor, and the closed-form exponential
// picker with the rate that spacing gives returns the group sought. From
// there a galloping search (steps 1, 2, 4, ... toward the answer, then
// bisection of the last step) finds the first group reaching the target, in
// a few reads near the prediction instead of log2(candidates) dependent
// reads. Cumulative weights do not decrease except by rounding where the
// build's parallel scan joins two partial sums, so the result is the one a
// bisection of all candidates gives unless the target lies within that
// rounding of a boundary (inside the picks' boundary tolerance).
__device__ __forceinline__ Pick pick_weight(const GroupRec* __restrict__ ng,
                                            const int32_t* __restrict__ n_dst,
                                            const double* __restrict__ cw, uint32_t gb,
                                            uint32_t gc, uint32_t ge, uint32_t end, double sc,
                                            int64_t t_first, int64_t t_last, const Draw& d) {
    const double prefix = gc > gb ? cw[gc - 1] : 0.0;
    const double target = prefix + unit_open(d.x0) * (cw[ge - 1] - prefix);
    // reaches(g): group g is at or past the answer (always true for the last)
    const uint32_t last = ge - 1;
    auto reaches = [&](uint32_t g) { return g == last || cw[g] >= target; };
    uint32_t lo = gc, hi = last;
    const uint32_t n = ge - gc;
    if (n > 8) {
        const uint32_t p = gc + pick_exponential(n, exp_lambda(t_first, t_last, n, sc), d.x0);
        uint64_t step = 1;  // 64-bit: it may pass 2^31 before a gallop ends
        if (reaches(p)) {
            hi = p;
            while (hi > gc) {
                const uint32_t q = hi - gc > step ? hi - (uint32_t)step : gc;
                if (!reaches(q)) {
                    lo = q + 1;
                    break;
                }
                hi = q;
                step <<= 1;
            }
        } else {
            lo = p + 1;
            while (true) {
                const uint32_t q = last - lo > step ? lo + (uint32_t)step : last;
                if (reaches(q)) {
                    hi = q;
                    break;
                }
                lo = q + 1;
                step <<= 1;
            }
        }
    }
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (reaches(mid)) hi = mid; else lo = mid + 1;
    }
    const GroupRec a = ng[lo];
    if (a.dst < 0) return Pick{a.dst & 0x7fffffff, a.ts};  // a one-edge group
    const uint32_t size = (lo + 1 < ge ? ng[lo + 1].first : end) - a.first;
    const double below = lo > gb ? cw[lo - 1] : 0.0;
    const double w = exp((double)(a.ts - t_last) / sc);
    double j = ceil((target - below) / w) - 1.0;
    j = j < 0.0 ? 0.0 : (j > (double)(size - 1) ? (double)(size - 1) : j);
    return Pick{n_dst[a.first + (uint32_t)j], a.ts};
}

// The edge-store position picked among the window's Gg timestamp groups.
__device__ __forceinline__ uint32_t pick_global(const uint32_t* __restrict__ gg_off, uint32_t Gg,
                                                int64_t t_first, int64_t t_last, int kind,
                                                double tau, const Draw& d, bool rev = false) {
    const uint32_t i = pick_group(Gg, kind, tau, Gg > 1 ? t_first : 0, t_last, d.x0);
    const uint32_t k = rev ? Gg - 1 - i : i;
    const uint32_t b0 = gg_off[k], b1 = gg_off[k + 1];
    const uint32_t j = (uint32_t)scale_u64(d.x1, b1 - b0);
    return rev ? b1 - 1 - j : b0 + j;
}

}  // namespace tw
