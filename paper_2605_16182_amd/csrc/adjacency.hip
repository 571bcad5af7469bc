// node2vec's adjacency test (Tempest, Sec. "Temporal Bias Sampling"): the
// return and in-out weights need to know whether the window holds an edge
// prev -> w at any timestamp. The window's (source, destination) pairs live
// in an open-addressing hash table with a record count per pair, built on
// the first node2vec walk and then kept current by every ingest and
// eviction: the evicted window records count their pairs down, the kept
// batch records count theirs up, so an update costs O(batch), not
// O(window). A lookup is one 16-byte slot read for most pairs.
#include <algorithm>

#include "tw_internal.h"

namespace tw {

namespace {

constexpr int AT = 256;  // threads per workgroup

__global__ void __launch_bounds__(AT) k_adj_clear(AdjSlot* __restrict__ tab, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * AT + threadIdx.x;
    if (i < n) tab[i] = AdjSlot{ADJ_EMPTY, 0u, 0u};
}

// +1 for each pair (src[i], dst[i]): claim the first empty slot of the probe
// sequence or count on the pair's slot. The table never fills (the host
// keeps it at most three quarters full), so the probe ends.
__global__ void __launch_bounds__(AT) k_adj_add(AdjSlot* __restrict__ tab, uint64_t mask,
                                                 const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = adj_key(src[i], dst[i]);
    uint64_t j = adj_hash(k) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe, j = (j + 1) & mask) {
        const uint64_t cur = tab[j].key;
        if (cur == k) {
            atomicAdd(&tab[j].cnt, 1u);
            return;
        }
        if (cur == ADJ_EMPTY) {
            // a stale read only costs a failed claim: the exchange decides
            const unsigned long long prev =
                atomicCAS(reinterpret_cast<unsigned long long*>(&tab[j].key),
                          (unsigned long long)ADJ_EMPTY, (unsigned long long)k);
            if (prev == ADJ_EMPTY || prev == k) {
                atomicAdd(&tab[j].cnt, 1u);
                return;
            }
        }
    }
}

// -1 for each pair: every pair counted down was counted up before (it is a
// window record), so its slot is on the probe sequence before any empty slot
__global__ void __launch_bounds__(AT) k_adj_sub(AdjSlot* __restrict__ tab, uint64_t mask,
                                                 const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = adj_key(src[i], dst[i]);
    uint64_t j = adj_hash(k) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe, j = (j + 1) & mask) {
        const uint64_t cur = tab[j].key;
        if (cur == k) {
            atomicSub(&tab[j].cnt, 1u);
            return;
        }
        if (cur == ADJ_EMPTY) return;
    }
}

dim3 grid_of(int64_t n) { return dim3((unsigned)std::max<int64_t>((n + AT - 1) / AT, 1)); }

// slots for a table holding m pairs at most half full (a power of two)
uint64_t adj_capacity(int64_t m) {
    uint64_t cap = 1024;
    while (cap < 2 * (uint64_t)std::max<int64_t>(m, 1)) cap <<= 1;
    return cap;
}

constexpr uint64_t ADJ_MAX_SLOTS = 1ull << 31;

}  // namespace

tw_status build_adjacency(tw_graph* g, Error& err) {
    if (g->adj_ready) return TW_OK;
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    const uint64_t cap = adj_capacity(m);
    if (cap > ADJ_MAX_SLOTS) {
        err = Error{TW_ENOMEM, "node2vec adjacency: the window has too many records"};
        return err.code;
    }
    TW_HIP(ensure(g->adj_tab, sizeof(AdjSlot) * cap, s));
    hipLaunchKernelGGL(k_adj_clear, grid_of((int64_t)cap), dim3(AT), 0, s,
                       g->adj_tab.as<AdjSlot>(), cap);
    if (m > 0)
        hipLaunchKernelGGL(k_adj_add, grid_of(m), dim3(AT), 0, s, g->adj_tab.as<AdjSlot>(),
                           cap - 1, g->e_src.as<int32_t>() + g->e_base,
                           g->e_dst.as<int32_t>() + g->e_base, m);
    TW_HIP(hipGetLastError());
    g->adj_mask = cap - 1;
    g->adj_used = m;
    g->adj_ready = true;
    return TW_OK;
}

tw_status adj_update(tw_graph* g, const int32_t* ev_src, const int32_t* ev_dst, int64_t ev_n,
                     const int32_t* add_src, const int32_t* add_dst, int64_t add_n, Error& err) {
    if (!g->adj_ready) return TW_OK;
    const uint64_t cap = g->adj_mask + 1;
    if ((uint64_t)(g->adj_used + add_n) > cap / 4 * 3) {
        // too full (counting every insert since the build): rebuild when needed
        g->adj_ready = false;
        return TW_OK;
    }
    hipStream_t s = g->stream;
    AdjSlot* tab = g->adj_tab.as<AdjSlot>();
    if (ev_n > 0)
        hipLaunchKernelGGL(k_adj_sub, grid_of(ev_n), dim3(AT), 0, s, tab, g->adj_mask, ev_src,
                           ev_dst, ev_n);
    if (add_n > 0)
        hipLaunchKernelGGL(k_adj_add, grid_of(add_n), dim3(AT), 0, s, tab, g->adj_mask, add_src,
                           add_dst, add_n);
    TW_HIP(hipGetLastError());
    g->adj_used += add_n;
    return TW_OK;
}

}  // namespace tw
