/*
 * tw_oracle — plain, slow, obviously-correct CPU oracle for streaming
 * temporal random walks (Tempest, arxiv 2605.16182).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or constant generator with the GPU library; the two meet
 * only at the seeded inputs produced by the `synth` module.
 *
 * What it computes, and where the paper defines it:
 *   - active window W(t) = {e : t - Delta <= t_e <= t}, late edges dropped at
 *     merge time, batch sorted by timestamp before merge
 *     (Sec. "Streaming Ingestion and Window Management");
 *   - the dual index: the timestamp-grouped view (edges in global timestamp
 *     order plus one offset per distinct-timestamp group) and the
 *     node-and-timestamp-grouped view (edges grouped by source, timestamp
 *     ascending within a node, with node offsets and node-timestamp-group
 *     offsets) (Sec. "Dual-Index Organization");
 *   - the causal neighbourhood Gamma_t(v) = out-edges of v with t' > t,
 *     located by a binary search over v's timestamp groups
 *     (Sec. "Design Constraints" and "Dual-Index Organization");
 *   - the index-based closed-form pickers, Eqs. (1)-(3), and temporal
 *     node2vec by rejection on the exponential proposal with acceptance
 *     beta / max(1/p, 1, 1/q) (Sec. "Temporal Bias Sampling");
 *   - the weight-based exponential picker, the paper's default sampler:
 *     each candidate edge e_i of Gamma_t(v) weighs exp(t_i - t_min), the
 *     cumulative array W over the candidates in order, and a draw u picks
 *     the smallest k with W[k] >= u W[n-1] (Sec. "Temporal Bias Sampling");
 *   - ties on timestamps broken uniformly at random (Sec. "Design
 *     Constraints");
 *   - backward walks over Gamma-_t(v) = in-edges of v with t' < t, the
 *     backward case the paper defines by analogy (Sec. "Design
 *     Constraints").
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - canonical order: timestamp ascending, ties in arrival order (older
 *     batch first, then input position; an undirected edge (u,v,t) is
 *     stored as (u,v,t) then (v,u,t));
 *   - uniform picks range over edges; linear and exponential picks range
 *     over distinct-timestamp groups, later groups weighted more, then a
 *     uniform edge inside the group;
 *   - Eq. (3) is read as the exact inverse CDF of P(i) ~ exp(lambda*i) on
 *     i = 0..n-1, with lambda = (t_last - t_first) / ((n-1) * tau), or
 *     lambda = 1 when tau <= 0;
 *   - weight-based picker: weights exp((t_i - t_min) / tau) with tau in
 *     timestamp units (tau <= 0: tau = 1, the printed form), evaluated as
 *     exp((t_i - t_last) / tau) with t_last the candidates' last timestamp:
 *     the common factor exp((t_last - t_min) / tau) cancels from u W[n-1]
 *     and W[k], the law is unchanged and no weight overflows; u is the open
 *     uniform U_open(x0); W is summed edge by edge in candidate order;
 *   - backward walks run on the in-view (the node view of the graph fed the
 *     batches with source and destination swapped; an undirected graph is
 *     its own in-view) and are forward walks over the candidates listed in
 *     reverse canonical order: every pick index i over n candidates (edges,
 *     groups, the edge inside a group, the start edge or group of the whole
 *     window) becomes n - 1 - i. Without equal timestamps this is a forward
 *     walk on the graph with reversed edges and negated timestamps. The
 *     weight-based picker is forward only;
 *   - node2vec: beta = 1/p when the candidate is the previous node, 1 when
 *     the active window holds an edge prev -> candidate, else 1/q;
 *   - max_len counts nodes; the first pick is RNG hop 0;
 *   - RNG: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
 *     (seed, 0), counter (walk id, hop, trial, 0); U(x) = (x>>11)*2^-53,
 *     U_open(x) = (2*(x>>12)+1)*2^-53, integer scaling floor(x*n/2^64).
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef unsigned __int128 u128;

const int64_t TS_NONE = std::numeric_limits<int64_t>::min();

enum { ST_OK = 0, ST_EINVAL = 1, ST_ERANGE = 4 };
enum { K_UNIFORM = 0, K_LINEAR = 1, K_EXPONENTIAL = 2, K_NODE2VEC = 3, K_WEIGHT = 4 };
enum { START_EDGE = 0, START_NODE = 1 };

struct Edge {
    int32_t src, dst;
    int64_t ts;
};

/* ---------------------------------------------------------------- Philox */

void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        u128 p0 = (u128)0xD2E7470EE14C6C93ULL * c0;
        u128 p1 = (u128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

struct Draw {
    uint64_t x[4];
};

Draw draw(uint64_t seed, uint64_t walk_id, uint64_t hop, uint64_t trial) {
    uint64_t ctr[4] = {walk_id, hop, trial, 0};
    uint64_t key[2] = {seed, 0};
    Draw d;
    philox4x64_10(ctr, key, d.x);
    return d;
}

double unit_closed_open(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
double unit_open(uint64_t x) { return (double)(2 * (x >> 12) + 1) * 0x1.0p-53; }
uint64_t scale(uint64_t x, uint64_t n) { return (uint64_t)(((u128)x * n) >> 64); }

/* --------------------------------------------------------------- pickers */

/* Eq. (1): uniform index in [0, n) */
int64_t pick_uniform(int64_t n, uint64_t x) { return (int64_t)scale(x, (uint64_t)n); }

/*
 * Eq. (2) evaluated exactly: with a = x>>11 and u = a / 2^53, Eq. (2) returns
 * the largest i with i(i+1) <= u n (n+1), i.e. i(i+1) 2^53 <= a n (n+1).
 * That gives P(i) = 2(i+1) / (n(n+1)). Found here by bisection on integers.
 */
int64_t pick_linear(int64_t n, uint64_t x) {
    u128 a = x >> 11;
    u128 rhs = a * ((u128)n * (u128)(n + 1));
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        u128 lhs = ((u128)mid * (u128)(mid + 1)) << 53;
        if (lhs <= rhs) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* CDF of the discrete exponential law at integer boundary k: P(i < k) */
double exp_cdf(int64_t n, double lam, int64_t k) {
    double ln = lam * (double)n;
    if (ln <= 1.0) return std::expm1(lam * (double)k) / std::expm1(ln);
    double en = std::exp(-ln);
    return (std::exp(lam * (double)(k - n)) - en) / (1.0 - en);
}

/*
 * Eq. (3) as the exact inverse CDF of P(i) ~ exp(lam i), i in [0, n):
 * x = log(1 + u (e^{lam n} - 1)) / lam, i = floor(x). Written in the form
 * log1p(u expm1(lam n)) / lam when lam n <= 1 and as
 * n + log(u + (1 - u) e^{-lam n}) / lam otherwise.
 */
int64_t pick_exponential(int64_t n, double lam, uint64_t x, double* margin) {
    if (n <= 1) {
        if (margin) *margin = INFINITY;
        return 0;
    }
    double u = unit_open(x);
    double ln = lam * (double)n;
    double xi;
    if (ln <= 1.0)
        xi = std::log1p(u * std::expm1(ln)) / lam;
    else
        xi = (double)n + std::log(u + (1.0 - u) * std::exp(-ln)) / lam;
    int64_t i = (int64_t)std::floor(xi);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    if (margin) {
        double lo = u - exp_cdf(n, lam, i);
        double hi = exp_cdf(n, lam, i + 1) - u;
        *margin = std::min(std::fabs(lo), std::fabs(hi));
    }
    return i;
}

/*
 * The weight-based picker over n candidate edges with timestamps ts[0..n)
 * (ascending): weights exp((ts[i] - ts[n-1]) / tau), cumulative sums W
 * edge by edge, r = u W[n-1] with u = U_open(x); returns the smallest k with
 * W[k] >= r. margin: the distance of u from the nearest boundary W[k] /
 * W[n-1] around the picked index (0 and 1 are not boundaries: u lies
 * strictly between them).
 */
int64_t pick_weight(const int64_t* ts, int64_t n, double tau, uint64_t x, double* margin) {
    const double sc = tau > 0.0 ? tau : 1.0;
    std::vector<double> W((size_t)n);
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        acc += std::exp((double)(ts[i] - ts[n - 1]) / sc);
        W[(size_t)i] = acc;
    }
    const double u = unit_open(x);
    const double r = u * W[(size_t)(n - 1)];
    int64_t lo = 0, hi = n - 1;  // smallest k with W[k] >= r
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (W[(size_t)mid] >= r) hi = mid; else lo = mid + 1;
    }
    if (margin) {  // interior boundaries only: u is never 0 or 1
        const double tot = W[(size_t)(n - 1)];
        *margin = INFINITY;
        if (lo > 0) *margin = std::fabs(u - W[(size_t)(lo - 1)] / tot);
        if (lo < n - 1) *margin = std::min(*margin, std::fabs(W[(size_t)lo] / tot - u));
    }
    return lo;
}

/* lambda of the exponential law over groups with first/last timestamps */
double exp_lambda(int64_t t_first, int64_t t_last, int64_t n, double tau) {
    if (tau <= 0.0) return 1.0;
    if (n <= 1) return 1.0;
    return (double)(t_last - t_first) / ((double)(n - 1) * tau);
}

/* ----------------------------------------------------------------- graph */

struct Graph {
    int32_t V = 0;
    bool directed = true;
    int64_t window = 0;
    bool has_time = false;
    int64_t t_now = 0;
    std::vector<Edge> active; /* canonical order: the timestamp view */

    bool dirty = true;
    std::vector<int64_t> g_ts, g_off;      /* global timestamp groups */
    std::vector<Edge> nview;               /* stable sort of active by src */
    std::vector<int64_t> n_gts, n_goff;    /* (src, ts) groups of nview */
    std::vector<int64_t> n_ebeg, n_gbeg;   /* node table, V + 1 entries */
    bool adj_ready = false;
    std::vector<std::vector<int32_t>> adj; /* per node: sorted out-neighbours */
};

int64_t evict(Graph& g, int64_t cut) {
    int64_t before = (int64_t)g.active.size();
    std::vector<Edge> kept;
    for (const Edge& e : g.active)
        if (e.ts >= cut) kept.push_back(e);
    g.active.swap(kept);
    int64_t removed = before - (int64_t)g.active.size();
    if (removed) { g.dirty = true; g.adj_ready = false; }
    return removed;
}

void rebuild(Graph& g) {
    if (!g.dirty) return;
    const std::vector<Edge>& a = g.active;
    int64_t m = (int64_t)a.size();

    g.g_ts.clear();
    g.g_off.clear();
    for (int64_t i = 0; i < m; ++i) {
        if (i == 0 || a[i].ts != a[i - 1].ts) {
            g.g_ts.push_back(a[i].ts);
            g.g_off.push_back(i);
        }
    }
    g.g_off.push_back(m);

    g.nview = a;
    std::stable_sort(g.nview.begin(), g.nview.end(),
                     [](const Edge& x, const Edge& y) { return x.src < y.src; });

    g.n_gts.clear();
    g.n_goff.clear();
    for (int64_t i = 0; i < m; ++i) {
        const Edge& e = g.nview[i];
        if (i == 0 || e.src != g.nview[i - 1].src || e.ts != g.nview[i - 1].ts) {
            g.n_gts.push_back(e.ts);
            g.n_goff.push_back(i);
        }
    }
    int64_t gn = (int64_t)g.n_gts.size();
    g.n_goff.push_back(m);

    g.n_ebeg.assign((size_t)g.V + 1, m);
    g.n_gbeg.assign((size_t)g.V + 1, gn);
    /* first edge / first group of each node; nodes without edges take the
       next node's start */
    for (int64_t i = m - 1; i >= 0; --i) g.n_ebeg[g.nview[i].src] = i;
    for (int64_t k = gn - 1; k >= 0; --k) g.n_gbeg[g.nview[g.n_goff[k]].src] = k;
    for (int64_t v = g.V - 1; v >= 0; --v) {
        if (g.n_ebeg[v] > g.n_ebeg[v + 1]) g.n_ebeg[v] = g.n_ebeg[v + 1];
        if (g.n_gbeg[v] > g.n_gbeg[v + 1]) g.n_gbeg[v] = g.n_gbeg[v + 1];
    }
    g.dirty = false;
}

void build_adjacency(Graph& g) {
    rebuild(g);
    if (g.adj_ready) return;
    g.adj.assign((size_t)g.V, std::vector<int32_t>());
    for (const Edge& e : g.active) g.adj[e.src].push_back(e.dst);
    for (auto& l : g.adj) std::sort(l.begin(), l.end());
    g.adj_ready = true;
}

bool has_edge(const Graph& g, int32_t u, int32_t w) {
    const std::vector<int32_t>& l = g.adj[u];
    return std::binary_search(l.begin(), l.end(), w);
}

/* --------------------------------------------------------------- walking */

struct Bias {
    int32_t kind;
    double tau, p, q;
};

struct Params {
    int32_t max_len;
    Bias hop, start;
    int32_t start_mode;
    uint64_t seed, walk_id_base;
    bool backward;
};

struct WalkStats {
    int64_t cap_hits = 0, trials = 0;
};

/*
 * One biased pick over groups [gc, ge) of (gts, goff): returns the edge
 * index. Linear and exponential choose a group, then a uniform edge in it.
 * rev: the candidates are listed in reverse order (a backward walk), so each
 * index i among n becomes n - 1 - i.
 */
int64_t pick_in_groups(const std::vector<int64_t>& gts, const std::vector<int64_t>& goff,
                       int64_t gc, int64_t ge, int32_t kind, double tau, const Draw& d,
                       double* margin, bool rev = false) {
    if (margin) *margin = INFINITY;
    if (kind == K_UNIFORM) {
        int64_t c = goff[gc], b = goff[ge];
        int64_t i = pick_uniform(b - c, d.x[0]);
        return rev ? b - 1 - i : c + i;
    }
    if (kind == K_WEIGHT) {
        // the candidates edge by edge, each with its group's timestamp
        const int64_t c = goff[gc], b = goff[ge];
        std::vector<int64_t> ets((size_t)(b - c));
        for (int64_t k = gc; k < ge; ++k)
            for (int64_t e = goff[k]; e < goff[k + 1]; ++e) ets[(size_t)(e - c)] = gts[k];
        return c + pick_weight(ets.data(), b - c, tau, d.x[0], margin);
    }
    int64_t n = ge - gc, i;
    if (kind == K_LINEAR) {
        i = pick_linear(n, d.x[0]);
    } else {
        double lam = exp_lambda(gts[gc], gts[ge - 1], n, tau);
        i = pick_exponential(n, lam, d.x[0], margin);
    }
    int64_t k = rev ? ge - 1 - i : gc + i;
    int64_t size = goff[k + 1] - goff[k];
    int64_t j = pick_uniform(size, d.x[1]);
    return rev ? goff[k + 1] - 1 - j : goff[k] + j;
}

/* returns 0, or ST_ERANGE for a start node outside [0, V) */
int walk_one(const Graph& g, const Params& P, uint64_t walk_id, int32_t start_node,
             int32_t* nodes, int64_t* ts, int32_t* len_out, double* margin, WalkStats& st) {
    const int32_t L = P.max_len;
    for (int32_t j = 0; j < L; ++j) {
        nodes[j] = -1;
        ts[j] = TS_NONE;
        if (margin) margin[j] = INFINITY;
    }
    *len_out = 0;
    int64_t m = (int64_t)g.active.size();
    int32_t len = 0, cur, prev;
    int64_t tcur;
    Draw d0 = draw(P.seed, walk_id, 0, 0);
    double mg = INFINITY;

    if (P.start_mode == START_EDGE) {
        if (m == 0) return ST_OK;
        int64_t e = pick_in_groups(g.g_ts, g.g_off, 0, (int64_t)g.g_ts.size(), P.start.kind,
                                   P.start.tau, d0, &mg, P.backward);
        const Edge& se = g.active[e];
        nodes[0] = se.src;
        if (margin) margin[0] = mg;
        len = 1;
        if (L == 1) { *len_out = len; return ST_OK; }
        nodes[1] = se.dst;
        ts[1] = se.ts;
        if (margin) margin[1] = mg;
        len = 2;
        prev = se.src;
        cur = se.dst;
        tcur = se.ts;
    } else {
        if (start_node < 0 || start_node >= g.V) return ST_ERANGE;
        nodes[0] = start_node;
        len = 1;
        if (L == 1) { *len_out = len; return ST_OK; }
        int64_t gb = g.n_gbeg[start_node], ge = g.n_gbeg[start_node + 1];
        if (gb == ge) { *len_out = len; return ST_OK; }
        int64_t e = pick_in_groups(g.n_gts, g.n_goff, gb, ge, P.start.kind, P.start.tau, d0, &mg,
                                   P.backward);
        nodes[1] = g.nview[e].dst;
        ts[1] = g.nview[e].ts;
        if (margin) margin[1] = mg;
        len = 2;
        prev = start_node;
        cur = g.nview[e].dst;
        tcur = g.nview[e].ts;
    }

    for (uint64_t hop = 1; len < L; ++hop) {
        int64_t gb = g.n_gbeg[cur], ge = g.n_gbeg[cur + 1];
        int64_t gc;
        if (!P.backward) {
            /* Gamma_t(cur): the first group with timestamp strictly after tcur */
            gc = std::upper_bound(g.n_gts.begin() + gb, g.n_gts.begin() + ge, tcur) -
                 g.n_gts.begin();
            if (gc == ge) break;
        } else {
            /* Gamma-_t(cur): the groups [gb, ge) before the first one at or after tcur */
            ge = std::lower_bound(g.n_gts.begin() + gb, g.n_gts.begin() + ge, tcur) -
                 g.n_gts.begin();
            gc = gb;
            if (gc == ge) break;
        }
        int64_t e;
        if (P.hop.kind == K_NODE2VEC) {
            double beta_max = std::max(std::max(1.0 / P.hop.p, 1.0), 1.0 / P.hop.q);
            bool accepted = false;
            double worst = INFINITY;
            e = -1;
            for (uint64_t trial = 0; trial < 4096; ++trial) {
                Draw d = draw(P.seed, walk_id, hop, trial);
                double tm;
                int64_t cand = pick_in_groups(g.n_gts, g.n_goff, gc, ge, K_EXPONENTIAL,
                                              P.hop.tau, d, &tm, P.backward);
                worst = std::min(worst, tm);
                int32_t w = g.nview[cand].dst;
                double beta;
                if (w == prev) beta = 1.0 / P.hop.p;
                else if (has_edge(g, prev, w)) beta = 1.0;
                else beta = 1.0 / P.hop.q;
                st.trials++;
                if (unit_closed_open(d.x[2]) * beta_max < beta) {
                    e = cand;
                    accepted = true;
                    break;
                }
            }
            mg = worst;
            if (!accepted) {
                st.cap_hits++;
                break;
            }
        } else {
            Draw d = draw(P.seed, walk_id, hop, 0);
            e = pick_in_groups(g.n_gts, g.n_goff, gc, ge, P.hop.kind, P.hop.tau, d, &mg,
                               P.backward);
        }
        nodes[len] = g.nview[e].dst;
        ts[len] = g.nview[e].ts;
        if (margin) margin[len] = mg;
        ++len;
        prev = cur;
        cur = g.nview[e].dst;
        tcur = g.nview[e].ts;
    }
    *len_out = len;
    return ST_OK;
}

}  // namespace

/* ================================================================ C ABI */

extern "C" {

void oracle_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
    philox4x64_10(ctr, key, out);
}

int64_t oracle_pick_uniform(int64_t n, uint64_t x) { return pick_uniform(n, x); }
int64_t oracle_pick_linear(int64_t n, uint64_t x) { return pick_linear(n, x); }
int64_t oracle_pick_exponential(int64_t n, double lam, uint64_t x, double* margin) {
    return pick_exponential(n, lam, x, margin);
}
int64_t oracle_pick_weight(const int64_t* ts, int64_t n, double tau, uint64_t x, double* margin) {
    return pick_weight(ts, n, tau, x, margin);
}
double oracle_exp_lambda(int64_t t_first, int64_t t_last, int64_t n, double tau) {
    return exp_lambda(t_first, t_last, n, tau);
}
double oracle_unit_open(uint64_t x) { return unit_open(x); }

void* oracle_create(int32_t num_nodes, int32_t directed, int64_t window) {
    if (num_nodes < 0) return nullptr;
    Graph* g = new Graph();
    g->V = num_nodes;
    g->directed = directed != 0;
    g->window = window;
    return g;
}

void oracle_destroy(void* h) { delete static_cast<Graph*>(h); }

/* info[6] = accepted, dropped_late, evicted, active_edges, t_min, t_max */
int oracle_ingest(void* h, const int32_t* src, const int32_t* dst, const int64_t* ts, int64_t n,
                  int64_t* info) {
    Graph& g = *static_cast<Graph*>(h);
    if (n < 0) return ST_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (src[i] < 0 || src[i] >= g.V || dst[i] < 0 || dst[i] >= g.V) return ST_ERANGE;

    std::vector<Edge> batch;
    for (int64_t i = 0; i < n; ++i) {
        batch.push_back(Edge{src[i], dst[i], ts[i]});
        if (!g.directed) batch.push_back(Edge{dst[i], src[i], ts[i]});
    }
    for (const Edge& e : batch) {
        if (!g.has_time || e.ts > g.t_now) g.t_now = e.ts;
        g.has_time = true;
    }
    int64_t dropped = 0, evicted = 0;
    if (g.window > 0 && g.has_time) {
        int64_t cut = g.t_now - g.window; /* window keeps ts >= t_now - Delta */
        std::vector<Edge> kept;
        for (const Edge& e : batch)
            if (e.ts >= cut) kept.push_back(e);
        dropped = (int64_t)batch.size() - (int64_t)kept.size();
        batch.swap(kept);
        evicted = evict(g, cut);
    }
    std::stable_sort(batch.begin(), batch.end(),
                     [](const Edge& x, const Edge& y) { return x.ts < y.ts; });
    std::vector<Edge> merged;
    merged.reserve(g.active.size() + batch.size());
    /* std::merge takes from the first range on ties: old edges first */
    std::merge(g.active.begin(), g.active.end(), batch.begin(), batch.end(),
               std::back_inserter(merged),
               [](const Edge& x, const Edge& y) { return x.ts < y.ts; });
    g.active.swap(merged);
    if (!batch.empty()) { g.dirty = true; g.adj_ready = false; }
    if (info) {
        info[0] = (int64_t)batch.size();
        info[1] = dropped;
        info[2] = evicted;
        info[3] = (int64_t)g.active.size();
        info[4] = g.active.empty() ? 0 : g.active.front().ts;
        info[5] = g.active.empty() ? 0 : g.active.back().ts;
    }
    return ST_OK;
}

int64_t oracle_evict_before(void* h, int64_t cutoff) {
    return evict(*static_cast<Graph*>(h), cutoff);
}

/* sizes[4] = active edges, global groups, node groups, nodes */
void oracle_sizes(void* h, int64_t* sizes) {
    Graph& g = *static_cast<Graph*>(h);
    rebuild(g);
    sizes[0] = (int64_t)g.active.size();
    sizes[1] = (int64_t)g.g_ts.size();
    sizes[2] = (int64_t)g.n_gts.size();
    sizes[3] = g.V;
}

/* copy the views out; any pointer may be null */
void oracle_views(void* h, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                  int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                  int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg) {
    Graph& g = *static_cast<Graph*>(h);
    rebuild(g);
    int64_t m = (int64_t)g.active.size();
    for (int64_t i = 0; i < m; ++i) {
        if (src) src[i] = g.active[i].src;
        if (dst) dst[i] = g.active[i].dst;
        if (ts) ts[i] = g.active[i].ts;
        if (n_dst) n_dst[i] = g.nview[i].dst;
        if (n_ts) n_ts[i] = g.nview[i].ts;
    }
    for (size_t k = 0; k < g.g_ts.size(); ++k) if (g_ts) g_ts[k] = g.g_ts[k];
    for (size_t k = 0; k < g.g_off.size(); ++k) if (g_off) g_off[k] = g.g_off[k];
    for (size_t k = 0; k < g.n_gts.size(); ++k) if (n_gts) n_gts[k] = g.n_gts[k];
    for (size_t k = 0; k < g.n_goff.size(); ++k) if (n_goff) n_goff[k] = g.n_goff[k];
    for (size_t k = 0; k < g.n_ebeg.size(); ++k) {
        if (n_ebeg) n_ebeg[k] = g.n_ebeg[k];
        if (n_gbeg) n_gbeg[k] = g.n_gbeg[k];
    }
}

/*
 * Walks for the ids listed in walk_idx (walk_idx == null: ids 0..n_out-1).
 * Row r of the outputs belongs to walk index walk_idx[r]; its RNG id is
 * walk_id_base + walk_idx[r]. NODE mode reads start_nodes[walk_idx[r]].
 * margin (nullable, n_out * max_len): for each output node, the distance of
 * the pick's uniform draw from the nearest CDF boundary of the exponential
 * or weight-based law (infinity for exact integer picks). stats[2] = node2vec trial-cap hits,
 * node2vec trials. backward: a backward walk on this graph, which must be
 * the in-view (see the header). Returns ST_OK, ST_EINVAL or ST_ERANGE (some
 * start node out of range; those walks have length 0).
 */
int oracle_sample_walks(void* h, int32_t max_len, int32_t hop_kind, double hop_tau, double p,
                        double q, int32_t start_kind, double start_tau, int32_t start_mode,
                        const int32_t* start_nodes, uint64_t seed, uint64_t walk_id_base,
                        const int64_t* walk_idx, int64_t n_out, int32_t* nodes, int64_t* ts,
                        int32_t* len, double* margin, int64_t* stats, int32_t nthreads,
                        int32_t backward) {
    Graph& g = *static_cast<Graph*>(h);
    if (max_len < 1 || n_out < 0) return ST_EINVAL;
    if (hop_kind < K_UNIFORM || hop_kind > K_WEIGHT) return ST_EINVAL;
    if (backward && hop_kind == K_WEIGHT) return ST_EINVAL;
    if (start_kind < K_UNIFORM || start_kind > K_EXPONENTIAL) return ST_EINVAL;
    if (hop_kind == K_NODE2VEC && !(p > 0.0 && q > 0.0)) return ST_EINVAL;
    if (start_mode == START_NODE && !start_nodes) return ST_EINVAL;
    if (start_mode != START_NODE && start_mode != START_EDGE) return ST_EINVAL;
    rebuild(g);
    if (hop_kind == K_NODE2VEC) build_adjacency(g);

    Params P;
    P.max_len = max_len;
    P.hop = Bias{hop_kind, hop_tau, p, q};
    P.start = Bias{start_kind, start_tau, 1.0, 1.0};
    P.start_mode = start_mode;
    P.seed = seed;
    P.walk_id_base = walk_id_base;
    P.backward = backward != 0;

    int64_t cap_hits = 0, trials = 0;
    int status = ST_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cap_hits, trials)
    for (int64_t r = 0; r < n_out; ++r) {
        int64_t w = walk_idx ? walk_idx[r] : r;
        WalkStats st;
        int32_t sn = start_mode == START_NODE ? start_nodes[w] : 0;
        int rc = walk_one(g, P, walk_id_base + (uint64_t)w, sn, nodes + r * max_len,
                          ts + r * max_len, len + r, margin ? margin + r * max_len : nullptr, st);
        cap_hits += st.cap_hits;
        trials += st.trials;
        if (rc != ST_OK) {
#pragma omp critical
            status = rc;
        }
    }
    if (stats) {
        stats[0] = cap_hits;
        stats[1] = trials;
    }
    return status;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

}  // extern "C"
