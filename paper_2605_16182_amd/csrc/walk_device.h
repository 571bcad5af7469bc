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

// first index in [lo, hi) with ts[index] > t (hi when none)
__device__ __forceinline__ uint32_t upper_bound_ts(const int64_t* __restrict__ ts, uint32_t lo,
                                                   uint32_t hi, int64_t t) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (ts[mid] <= t) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Gamma lookup (Sec. "Dual-Index Organization": the first timestamp group of
// the node strictly after t) through the node's fence: one FENCE_FAN-entry
// window per level, each a single 128-byte line, then one window of the
// node's own group timestamps. Requires t < r.t_last, so the result is
// below r.ge. Returns the absolute group index.
// panel (nullable) holds the first panel_len entries of the node's fence
// (its top levels) in LDS; windows inside it are read from there.
__device__ __forceinline__ uint32_t fence_search(const int64_t* __restrict__ gts,
                                                 const int64_t* __restrict__ fence,
                                                 const NodeRec& r, int64_t t,
                                                 const int64_t* panel, uint32_t panel_len) {
    const uint32_t G = r.ge - r.gb;
    uint64_t lo = 0;
    if (r.levels > 0) {
        uint64_t off = r.fence_off;
        for (int k = (int)r.levels; k >= 1; --k) {
            const uint64_t rel = off - r.fence_off + lo;
            const longlong2* win = reinterpret_cast<const longlong2*>(
                rel + FENCE_FAN <= panel_len ? panel + rel : fence + off + lo);
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < FENCE_FAN / 2; ++j) {
                const longlong2 v = win[j];
                c += (v.x <= t) + (v.y <= t);
            }
            if (c == 0) return r.gb;  // only possible at the top level: t precedes the node
            lo = (lo + c - 1) * FENCE_FAN;
            const uint32_t sh = FENCE_LOG * (uint32_t)k;
            const uint64_t nk = ((uint64_t)G + (1ull << sh) - 1) >> sh;
            off += (nk + FENCE_FAN - 1) / FENCE_FAN * FENCE_FAN;
        }
    }
    const int64_t* base = gts + r.gb + lo;
    uint32_t c = 0;
    if (lo + FENCE_FAN <= G) {
#pragma unroll
        for (int j = 0; j < FENCE_FAN; ++j) c += (base[j] <= t);
    } else {
        const uint32_t rem = (uint32_t)(G - lo);
        for (uint32_t j = 0; j < rem; ++j) c += (base[j] <= t);
    }
    return r.gb + (uint32_t)lo + c;
}

// levels K and total entries of the fence of a node with G groups
__device__ __forceinline__ void fence_shape_dev(uint32_t G, uint32_t* levels, uint32_t* size) {
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

// is w among the sorted values adj[lo, hi)?
__device__ __forceinline__ bool sorted_contains(const int32_t* __restrict__ adj, uint32_t lo,
                                                uint32_t hi, int32_t w) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        int32_t v = adj[mid];
        if (v == w) return true;
        if (v < w) lo = mid + 1; else hi = mid;
    }
    return false;
}

// One biased or uniform pick among groups [gc, ge) of (gts, goff), where
// goff[ge] == end. Returns the edge index and its timestamp.
struct Pick {
    uint32_t e;
    int64_t t;
};

__device__ __forceinline__ Pick pick_in_groups(const int64_t* __restrict__ gts,
                                               const uint32_t* __restrict__ goff,
                                               const int64_t* __restrict__ ets, uint32_t gc,
                                               uint32_t ge, uint32_t end, int kind, double tau,
                                               int64_t t_last, const Draw& d) {
    if (kind == TW_UNIFORM) {
        uint32_t c = goff[gc];
        uint32_t e = c + (uint32_t)scale_u64(d.x0, end - c);
        return Pick{e, ets[e]};
    }
    uint32_t n = ge - gc, i;
    if (kind == TW_LINEAR) {
        i = pick_linear(n, d.x0);
    } else {
        double lam = exp_lambda(n > 1 ? gts[gc] : 0, t_last, n, tau);
        i = pick_exponential(n, lam, d.x0);
    }
    uint32_t k = gc + i;
    uint32_t b0 = goff[k], b1 = goff[k + 1];
    return Pick{b0 + (uint32_t)scale_u64(d.x1, b1 - b0), gts[k]};
}

}  // namespace tw
