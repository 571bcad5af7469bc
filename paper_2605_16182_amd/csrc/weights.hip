// Cumulative group weights of the node view for the weight-based picker
// (Tempest, Sec. "Temporal Bias Sampling": each candidate edge weighs
// exp(t - t_min), and a draw is inverted through the cumulative weights of
// the candidate set Gamma_t(v)).
//
// For a node v with live groups [gb, ge) and last timestamp t_last:
//   cw[g] = sum over j in [gb, g] of size_j * exp((ts_j - t_last) / tau)
// (inclusive, in the group pool's slots). A hop's candidate set is a suffix
// [gc, ge) of the live groups; its cumulative weights are cw[g] - cw[gc - 1]
// times the factor exp((t_last - t_min) / tau), common to every candidate,
// which cancels from the inversion. Weights relative to t_last are at most
// the group size, so none overflows. Built on demand for one tau (tau <= 0:
// 1) and kept until the node view changes.
//
// Layout of the build: the live groups of all nodes, node by node, are the
// items [0, G) (item f of node v is group gb(v) + f - off[v], off = the
// exclusive scan of the live group counts). A segmented inclusive scan over
// the items (a segment per node) runs in three passes: per tile the combined
// (head, sum) pair, a single-workgroup scan of the tile pairs, and per tile
// the scan with the carry of the tiles before it.
#include <algorithm>
#include <cmath>

#include "tw_internal.h"

namespace tw {
namespace {

constexpr int T = 256;
constexpr int W_ITEMS = 16;            // consecutive items per thread
constexpr int W_TILE = T * W_ITEMS;    // items per tile
// LDS position of tile item k: one pad word after every W_ITEMS items, so
// that a thread's W_ITEMS consecutive items (the scan's reads) and lanes'
// consecutive items (the loads' writes) fall in distinct banks
constexpr int W_LDS = W_TILE + W_TILE / W_ITEMS;
__device__ __forceinline__ int lds_at(int k) { return k + k / W_ITEMS; }

// (head, sum): a segment head inside the range, and the sum since the last
// head (the whole sum when there is none)
struct Seg {
    uint32_t head;
    double sum;
};

__device__ __forceinline__ Seg seg_add(Seg a, Seg b) {
    return Seg{a.head | b.head, b.head ? b.sum : a.sum + b.sum};
}

__global__ void k_w_counts(const NodeRec* __restrict__ rec, int64_t V, uint32_t* __restrict__ cnt) {
    const int64_t v = (int64_t)blockIdx.x * T + threadIdx.x;
    if (v < V) cnt[v] = rec[v].ge - rec[v].gb;
}

// the node owning item f: the largest v in [lo, hi] with off[v] <= f
__device__ __forceinline__ uint32_t node_of(const uint32_t* __restrict__ off, uint32_t lo,
                                            uint32_t hi, uint32_t f) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// exclusive prefix maximum of one value per thread over the workgroup
__device__ uint32_t block_max_excl(uint32_t x) {
    __shared__ uint32_t wmax[T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc = y > inc ? y : inc;
    }
    if (lane == 63) wmax[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int k = 0; k < T / 64; ++k)
        if (k < wave) before = wmax[k] > before ? wmax[k] : before;
    uint32_t ex = __shfl_up(inc, 1, 64);
    if (lane == 0) ex = 0;
    __syncthreads();
    return ex > before ? ex : before;
}

// Weights of a tile's items into LDS (lane-strided, so the group records
// are read in order), a segment head (a node's first item) as a negative
// weight (-0.0 for a zero weight), and the items' group slots into slot. The
// owning node of every item comes from LDS: each non-empty node of the
// tile's node range marks its first item with its id, and a prefix maximum
// over the tile (node ids grow with the items) carries it to the node's
// other items, with the node of the tile's first item as the start.
__device__ void tile_weights(const uint32_t* __restrict__ off, int64_t V, uint32_t G,
                             const NodeRec* __restrict__ rec, const GroupRec* __restrict__ ng,
                             double inv_sc, uint32_t base, double* w, uint32_t* slot,
                             uint32_t* vr) {
    const uint32_t last = std::min<uint32_t>(base + W_TILE, G) - 1;
    if (threadIdx.x == 0) {
        vr[0] = node_of(off, 0, (uint32_t)V - 1, base);
        vr[1] = node_of(off, vr[0], (uint32_t)V - 1, last);
    }
    for (int k = threadIdx.x; k < W_TILE; k += T) slot[lds_at(k)] = 0;
    __syncthreads();
    // nodes after vr[0] start inside the tile (vr[0] is the last node whose
    // first item is at or before base); only a non-empty node marks its start
    for (uint32_t v = vr[0] + 1 + threadIdx.x; v <= vr[1]; v += T) {
        const uint32_t next = (int64_t)v + 1 < V ? off[v + 1] : G;
        if (off[v] < next) slot[lds_at((int)(off[v] - base))] = v;
    }
    __syncthreads();
    {
        const int k0 = threadIdx.x * W_ITEMS;
        uint32_t m = threadIdx.x == 0 ? vr[0] : 0u;
#pragma unroll
        for (int k = 0; k < W_ITEMS; ++k) {
            const uint32_t x = slot[lds_at(k0 + k)];
            m = x > m ? x : m;
        }
        uint32_t run = block_max_excl(m);
        if (threadIdx.x == 0) run = vr[0];
#pragma unroll
        for (int k = 0; k < W_ITEMS; ++k) {
            const uint32_t x = slot[lds_at(k0 + k)];
            run = x > run ? x : run;
            slot[lds_at(k0 + k)] = run;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < W_TILE; k += T) {
        const uint32_t f = base + (uint32_t)k;
        if (f >= G) {
            w[lds_at(k)] = 0.0;
            continue;
        }
        const uint32_t v = slot[lds_at(k)];
        const NodeRec r = rec[v];
        const uint32_t g = r.gb + (f - off[v]);
        const GroupRec a = ng[g];
        const uint32_t next = g + 1 < r.ge ? ng[g + 1].first : r.ee;
        const double wt = (double)(next - a.first) * exp((double)(a.ts - r.t_last) * inv_sc);
        w[lds_at(k)] = f == off[v] ? -wt : wt;
        slot[lds_at(k)] = g;
    }
    __syncthreads();
}

// exclusive scan of one Seg per thread over the workgroup; returns this
// thread's prefix and the workgroup total in *all
__device__ Seg block_seg_excl(Seg s, Seg* all) {
    __shared__ uint32_t wh[T / 64];
    __shared__ double wsum[T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Seg inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        Seg y;
        y.head = __shfl_up(inc.head, o, 64);
        y.sum = __shfl_up(inc.sum, o, 64);
        if (lane >= o) inc = seg_add(y, inc);
    }
    if (lane == 63) {
        wh[wave] = inc.head;
        wsum[wave] = inc.sum;
    }
    __syncthreads();
    Seg before{0, 0.0}, tot{0, 0.0};
#pragma unroll
    for (int k = 0; k < T / 64; ++k) {
        const Seg x{wh[k], wsum[k]};
        if (k < wave) before = seg_add(before, x);
        tot = seg_add(tot, x);
    }
    __syncthreads();
    // this thread's exclusive prefix: the waves before, then the lanes before
    Seg lane_ex;
    lane_ex.head = __shfl_up(inc.head, 1, 64);
    lane_ex.sum = __shfl_up(inc.sum, 1, 64);
    if (lane == 0) lane_ex = Seg{0, 0.0};
    *all = tot;
    return seg_add(before, lane_ex);
}

// Pass 1: every tile's combined pair. Only the items from the tile's last
// segment head on contribute to its sum; that head is the first item of the
// node owning the tile's last item, when it lies inside the tile.
__global__ void __launch_bounds__(T)
k_w_tiles(const uint32_t* __restrict__ off, int64_t V, const uint32_t* __restrict__ Gp,
          const NodeRec* __restrict__ rec, const GroupRec* __restrict__ ng, double inv_sc,
          uint32_t* __restrict__ t_head, double* __restrict__ t_sum) {
    __shared__ double wsum[T / 64];
    const uint32_t G = *Gp;
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * (uint32_t)W_TILE;
    if (base >= G) return;
    const uint32_t last = std::min<uint32_t>(base + W_TILE, G) - 1;
    const uint32_t v = node_of(off, 0, (uint32_t)V - 1, last);  // uniform over the block
    const uint32_t from = std::max(base, off[v]);
    const NodeRec r = rec[v];
    double s = 0.0;
    for (uint32_t f = from + threadIdx.x; f <= last; f += T) {
        const uint32_t g = r.gb + (f - off[v]);
        const GroupRec a = ng[g];
        const uint32_t next = g + 1 < r.ge ? ng[g + 1].first : r.ee;
        s += (double)(next - a.first) * exp((double)(a.ts - r.t_last) * inv_sc);
    }
    // the block's total (the order of this sum is the build's own)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
#pragma unroll
        for (int k = 0; k < T / 64; ++k) tot += wsum[k];
        t_head[tile] = off[v] >= base;
        t_sum[tile] = tot;
    }
}

// Pass 3: the scan, with carry[t] the combination of the tiles before t,
// into cw at the items' group slots.
__global__ void __launch_bounds__(T)
k_w_scan(const uint32_t* __restrict__ off, int64_t V, const uint32_t* __restrict__ Gp,
         const NodeRec* __restrict__ rec, const GroupRec* __restrict__ ng, double inv_sc,
         const uint32_t* __restrict__ c_head, const double* __restrict__ c_sum,
         double* __restrict__ cw) {
    __shared__ double w[W_LDS];
    __shared__ uint32_t slot[W_LDS];
    __shared__ uint32_t vr[2];
    const uint32_t G = *Gp;
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * (uint32_t)W_TILE;
    if (base >= G) return;  // the grid is sized for an upper bound of G
    tile_weights(off, V, G, rec, ng, inv_sc, base, w, slot, vr);
    // this thread's items [i0, i0 + W_ITEMS) in order
    const int i0 = threadIdx.x * W_ITEMS;
    auto item = [&](int i) {
        const double x = w[lds_at(i)];
        return Seg{signbit(x) ? 1u : 0u, fabs(x)};
    };
    Seg mine{0, 0.0};
    for (int k = 0; k < W_ITEMS; ++k) mine = seg_add(mine, item(i0 + k));
    Seg all;
    Seg pre = seg_add(Seg{c_head[tile], c_sum[tile]}, block_seg_excl(mine, &all));
    for (int k = 0; k < W_ITEMS; ++k) {
        const int i = i0 + k;
        pre = seg_add(pre, item(i));
        if (base + (uint32_t)i < G) cw[slot[lds_at(i)]] = pre.sum;
    }
}

// Pass 2: exclusive scan of the nt tile pairs by one workgroup.
__global__ void __launch_bounds__(T)
k_w_carry(const uint32_t* __restrict__ Gp, const uint32_t* __restrict__ t_head,
          const double* __restrict__ t_sum, uint32_t* __restrict__ c_head,
          double* __restrict__ c_sum) {
    const uint32_t G = *Gp;
    const uint32_t nt = (G + W_TILE - 1) / W_TILE;
    const uint32_t per = (nt + T - 1) / T;
    const uint32_t b = threadIdx.x * per, e = std::min<uint32_t>(b + per, nt);
    Seg mine{0, 0.0};
    for (uint32_t t = b; t < e; ++t) mine = seg_add(mine, Seg{t_head[t], t_sum[t]});
    Seg all;
    Seg pre = block_seg_excl(mine, &all);
    for (uint32_t t = b; t < e; ++t) {
        c_head[t] = pre.head;
        c_sum[t] = pre.sum;
        pre = seg_add(pre, Seg{t_head[t], t_sum[t]});
    }
}

}  // namespace

tw_status build_weights(tw_graph* g, double tau, Error& err) {
    const double sc = tau > 0.0 ? tau : 1.0;
    if (g->w_ready && g->w_scale == sc) return TW_OK;
    hipStream_t s = g->stream;
    const int64_t V = g->V;
    TW_HIP(ensure(g->v_flags, sizeof(uint32_t) * (V + 1), g->stream));
    TW_HIP(ensure(g->v_pos, sizeof(uint32_t) * (V + 1), g->stream));
    uint32_t* cnt = g->v_flags.as<uint32_t>();
    uint32_t* off = g->v_pos.as<uint32_t>();
    uint32_t* Gd = g->scal.as<uint32_t>() + SLOT_U32_W_GROUPS;
    hipLaunchKernelGGL(k_w_counts, dim3((unsigned)ceil_div(V, T)), dim3(T), 0, s,
                       g->rec.as<NodeRec>(), V, cnt);
    TW_HIP(scan_exclusive_u32(cnt, off, V, Gd, g->ws, s));
    // the grid covers every live group: at most the group pool's top
    const int64_t nt = std::max<int64_t>(ceil_div(std::max<int64_t>(g->pg_top, 1), W_TILE), 1);
    if (nt > (int64_t)T * 4096) {
        err = Error{TW_ENOMEM, "weight build: too many groups"};
        return err.code;
    }
    TW_HIP(ensure(g->cw, sizeof(double) * std::max<int64_t>(g->pg_cap, 1), g->stream));
    TW_HIP(ensure(g->w_tiles, (sizeof(uint32_t) + sizeof(double)) * 2 * nt, g->stream));
    uint32_t* t_head = g->w_tiles.as<uint32_t>();
    uint32_t* c_head = t_head + nt;
    double* t_sum = reinterpret_cast<double*>(c_head + nt);  // 8 nt bytes in: aligned
    double* c_sum = t_sum + nt;
    const double inv_sc = 1.0 / sc;
    hipLaunchKernelGGL(k_w_tiles, dim3((unsigned)nt), dim3(T), 0, s, off, V, Gd,
                       g->rec.as<NodeRec>(), g->ng.as<GroupRec>(), inv_sc, t_head, t_sum);
    hipLaunchKernelGGL(k_w_carry, dim3(1), dim3(T), 0, s, Gd, t_head, t_sum, c_head, c_sum);
    hipLaunchKernelGGL(k_w_scan, dim3((unsigned)nt), dim3(T), 0, s, off, V, Gd,
                       g->rec.as<NodeRec>(), g->ng.as<GroupRec>(), inv_sc, c_head, c_sum,
                       g->cw.as<double>());
    TW_HIP(hipGetLastError());
    g->w_ready = true;
    g->w_scale = sc;
    return TW_OK;
}

}  // namespace tw
