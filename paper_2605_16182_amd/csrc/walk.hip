// Walk sampling (Tempest, Sec. "Temporal Bias Sampling" and "The Full-Walk
// Baseline"). A walk is keyed by (seed, walk id); hop h, trial r draws
// Philox4x64-10 at counter (id, h, r, 0), so every dispatch produces the
// same walks.
#include <algorithm>
#include <cmath>

#include "walk_device.h"

namespace tw {
namespace {

struct WalkArgs {
    // timestamp view and its groups
    const int32_t* e_src;
    const int32_t* e_dst;
    const int64_t* e_ts;
    const int64_t* gg_ts;
    const uint32_t* gg_off;
    uint32_t m, Gg;
    // node view
    const int32_t* n_dst;
    const int64_t* n_ts;
    const int64_t* ng_ts;
    const uint32_t* ng_off;
    const NodeRec* rec;
    const int64_t* fence;
    const int32_t* adj;
    int32_t V;
    // parameters
    int64_t num_walks;
    int32_t L;
    int32_t hop_kind, start_kind, start_mode;
    double hop_tau, start_tau, inv_p, inv_q, beta_max;
    const int32_t* start_nodes;
    uint64_t seed, base;
    // outputs
    int32_t* nodes;
    int64_t* ts;
    int32_t* len;
    uint32_t* err;  // [0] start node out of range, [2] node2vec trial cap hits
};

constexpr int WALK_THREADS = 256;
constexpr uint32_t N2V_MAX_TRIALS = 4096;

// One full walk per thread: the full-walk baseline.
__global__ void __launch_bounds__(WALK_THREADS) k_walk_full(const WalkArgs a) {
    const int64_t w = (int64_t)blockIdx.x * WALK_THREADS + threadIdx.x;
    if (w >= a.num_walks) return;
    const uint64_t id = a.base + (uint64_t)w;
    const int32_t L = a.L;
    int32_t* out_n = a.nodes + w * L;
    int64_t* out_t = a.ts + w * L;
    int32_t len = 0, cur = 0, prev = 0;
    int64_t tcur = 0;

    const Draw d0 = philox(id, 0, 0, a.seed);
    if (a.start_mode == TW_START_EDGE) {
        if (a.m == 0) goto done;
        uint32_t e;
        if (a.start_kind == TW_UNIFORM) {
            e = (uint32_t)scale_u64(d0.x0, a.m);
        } else {
            Pick p = pick_in_groups(a.gg_ts, a.gg_off, a.e_ts, 0, a.Gg, a.m, a.start_kind,
                                    a.start_tau, a.gg_ts[a.Gg - 1], d0);
            e = p.e;
        }
        const int32_t s = a.e_src[e], t_dst = a.e_dst[e];
        const int64_t t = a.e_ts[e];
        out_n[0] = s;
        out_t[0] = TS_NONE;
        len = 1;
        if (L == 1) goto done;
        out_n[1] = t_dst;
        out_t[1] = t;
        len = 2;
        prev = s;
        cur = t_dst;
        tcur = t;
    } else {
        const int32_t v0 = a.start_nodes[w];
        if (v0 < 0 || v0 >= a.V) {
            atomicOr(&a.err[0], 1u);
            goto done;
        }
        out_n[0] = v0;
        out_t[0] = TS_NONE;
        len = 1;
        if (L == 1) goto done;
        const NodeRec r = a.rec[v0];
        if (r.gb == r.ge) goto done;
        Pick p = pick_in_groups(a.ng_ts, a.ng_off, a.n_ts, r.gb, r.ge, r.ee, a.start_kind,
                                a.start_tau, r.t_last, d0);
        const int32_t nx = a.n_dst[p.e];
        out_n[1] = nx;
        out_t[1] = p.t;
        len = 2;
        prev = v0;
        cur = nx;
        tcur = p.t;
    }

    for (uint64_t hop = 1; len < L; ++hop) {
        const NodeRec r = a.rec[cur];
        if (tcur >= r.t_last) break;  // Gamma_t(cur) is empty
        const uint32_t gc = fence_search(a.ng_ts, a.fence, r, tcur);
        Pick p;
        if (a.hop_kind == TW_NODE2VEC) {
            const NodeRec rp = a.rec[prev];
            bool accepted = false;
            for (uint32_t trial = 0; trial < N2V_MAX_TRIALS; ++trial) {
                const Draw d = philox(id, hop, trial, a.seed);
                p = pick_in_groups(a.ng_ts, a.ng_off, a.n_ts, gc, r.ge, r.ee, TW_EXPONENTIAL,
                                   a.hop_tau, r.t_last, d);
                const int32_t wnode = a.n_dst[p.e];
                double beta;
                if (wnode == prev) beta = a.inv_p;
                else if (sorted_contains(a.adj, rp.eb, rp.ee, wnode)) beta = 1.0;
                else beta = a.inv_q;
                if (unit_closed_open(d.x2) * a.beta_max < beta) {
                    accepted = true;
                    break;
                }
            }
            if (!accepted) {
                atomicAdd(&a.err[2], 1u);
                break;
            }
        } else {
            const Draw d = philox(id, hop, 0, a.seed);
            p = pick_in_groups(a.ng_ts, a.ng_off, a.n_ts, gc, r.ge, r.ee, a.hop_kind, a.hop_tau,
                               r.t_last, d);
        }
        const int32_t nx = a.n_dst[p.e];
        out_n[len] = nx;
        out_t[len] = p.t;
        ++len;
        prev = cur;
        cur = nx;
        tcur = p.t;
    }
done:
    for (int32_t j = len; j < L; ++j) {
        out_n[j] = -1;
        out_t[j] = TS_NONE;
    }
    a.len[w] = len;
}

bool valid_tau(double t) { return std::isfinite(t); }

}  // namespace

tw_status sample_walks(tw_graph* g, const tw_walk_params* p, int32_t* nodes, int64_t* ts,
                       int32_t* len, Error& err) {
    if (!p || p->num_walks < 0 || p->max_len < 1) {
        err = Error{TW_EINVAL, "sample_walks: need num_walks >= 0 and max_len >= 1"};
        return err.code;
    }
    const tw_bias& hb = p->hop_bias;
    const tw_bias& sb = p->start_bias;
    if (hb.kind < TW_UNIFORM || hb.kind > TW_NODE2VEC || sb.kind < TW_UNIFORM ||
        sb.kind > TW_EXPONENTIAL || !valid_tau(hb.tau) || !valid_tau(sb.tau)) {
        err = Error{TW_EINVAL, "sample_walks: bad bias kind or tau (start bias cannot be node2vec)"};
        return err.code;
    }
    if (hb.kind == TW_NODE2VEC && !(hb.p > 0.0 && hb.q > 0.0 && std::isfinite(hb.p) &&
                                    std::isfinite(hb.q))) {
        err = Error{TW_EINVAL, "sample_walks: node2vec needs p > 0 and q > 0"};
        return err.code;
    }
    if (p->start_mode != TW_START_EDGE && p->start_mode != TW_START_NODE) {
        err = Error{TW_EINVAL, "sample_walks: bad start mode"};
        return err.code;
    }
    if (p->start_mode == TW_START_NODE && !p->d_start_nodes && p->num_walks > 0) {
        err = Error{TW_EINVAL, "sample_walks: start mode NODE needs d_start_nodes"};
        return err.code;
    }
    if (p->dispatch < TW_DISPATCH_AUTO || p->dispatch > TW_DISPATCH_COOP) {
        err = Error{TW_EINVAL, "sample_walks: bad dispatch"};
        return err.code;
    }
    if (p->num_walks == 0) return TW_OK;
    if (!nodes || !ts || !len) {
        err = Error{TW_EINVAL, "sample_walks: null output"};
        return err.code;
    }
    TW_HIP(ensure(g->err, sizeof(uint32_t) * 4));
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    if (hb.kind == TW_NODE2VEC && g->m > 0) {
        if (build_adjacency(g, err) != TW_OK) return err.code;
    }
    WalkArgs a{};
    a.e_src = g->e_src.as<int32_t>();
    a.e_dst = g->e_dst.as<int32_t>();
    a.e_ts = g->e_ts.as<int64_t>();
    a.gg_ts = g->gg_ts.as<int64_t>();
    a.gg_off = g->gg_off.as<uint32_t>();
    a.m = (uint32_t)g->m;
    a.Gg = (uint32_t)g->Gg;
    a.n_dst = g->n_dst.as<int32_t>();
    a.n_ts = g->n_ts.as<int64_t>();
    a.ng_ts = g->ng_ts.as<int64_t>();
    a.ng_off = g->ng_off.as<uint32_t>();
    a.rec = g->rec.as<NodeRec>();
    a.fence = g->fence.as<int64_t>();
    a.adj = g->adj.as<int32_t>();
    a.V = g->V;
    a.num_walks = p->num_walks;
    a.L = p->max_len;
    a.hop_kind = hb.kind;
    a.start_kind = sb.kind;
    a.start_mode = p->start_mode;
    a.hop_tau = hb.tau;
    a.start_tau = sb.tau;
    a.inv_p = hb.kind == TW_NODE2VEC ? 1.0 / hb.p : 1.0;
    a.inv_q = hb.kind == TW_NODE2VEC ? 1.0 / hb.q : 1.0;
    a.beta_max = std::max(std::max(a.inv_p, 1.0), a.inv_q);
    a.start_nodes = p->d_start_nodes;
    a.seed = p->seed;
    a.base = p->walk_id_base;
    a.nodes = nodes;
    a.ts = ts;
    a.len = len;
    a.err = g->err.as<uint32_t>();
    int64_t blocks = ceil_div(p->num_walks, WALK_THREADS);
    hipLaunchKernelGGL(k_walk_full, dim3((unsigned)blocks), dim3(WALK_THREADS), 0, g->stream, a);
    TW_HIP(hipGetLastError());
    return TW_OK;
}

}  // namespace tw
