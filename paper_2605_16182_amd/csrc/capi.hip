// The C ABI declared in include/tw.h: argument checks, error reporting and
// dispatch to the ingest and walk code. No exception crosses this layer.
#include <new>
#include <string>

#include <cstring>

#include "tw_internal.h"

namespace {

thread_local std::string g_last_error;

tw_status fail(tw_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

tw_status report(tw_status code, const tw::Error& e) {
    if (code != TW_OK) g_last_error = e.msg;
    return code;
}

template <typename F>
tw_status guarded(const char* what, F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(TW_ENOMEM, std::string(what) + ": host allocation failed");
    } catch (...) {
        return fail(TW_EDEVICE, std::string(what) + ": unexpected exception");
    }
}

// pending device-side errors from walks: flag 0, a start node out of range;
// flag 3, a batched walk with a length limit, bias index or row out of range
tw_status check_flags_of(tw_graph* g) {
    if (!g->err.p || !g->h_scal) return TW_OK;
    // the flags land in the pinned host copy, after the scalar slots
    uint32_t* f = static_cast<uint32_t*>(g->h_scal) + tw::SCALAR_BYTES / 4;
    if (hipMemcpyAsync(f, g->err.p, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, g->stream) !=
            hipSuccess ||
        hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(TW_EDEVICE, "reading device error flags failed");
    if (f[0] || f[3]) {
        uint32_t* d = static_cast<uint32_t*>(g->err.p);
        hipMemsetAsync(d, 0, sizeof(uint32_t), g->stream);
        hipMemsetAsync(d + 3, 0, sizeof(uint32_t), g->stream);
        hipStreamSynchronize(g->stream);
        if (f[0]) return fail(TW_ERANGE, "a walk start node was outside [0, num_nodes)");
        return fail(TW_EINVAL, "a batched walk had a length limit, bias index or row out of range");
    }
    return TW_OK;
}

// the graph's flags, then its in-view's (backward walks run there)
tw_status check_device_flags(tw_graph* g) {
    tw_status st = check_flags_of(g);
    if (st == TW_OK && g->rev) st = check_flags_of(g->rev);
    return st;
}

// A graph whose last ingest or eviction failed midway holds a partly
// updated index: every later call that reads or changes it is refused.
tw_status refuse_broken(const tw_graph* g, const char* what) {
    if (!g->broken) return TW_OK;
    return fail(TW_EDEVICE, std::string(what) +
                                ": the graph is unusable (an ingest or eviction failed midway, "
                                "out of device memory); destroy it");
}

}  // namespace

extern "C" {

tw_status tw_create(const tw_config* cfg, tw_graph** out) {
    return guarded("tw_create", [&]() -> tw_status {
        if (!cfg || !out) return fail(TW_EINVAL, "tw_create: null argument");
        if (cfg->num_nodes < 1) return fail(TW_EINVAL, "tw_create: num_nodes must be >= 1");
        tw_graph* g = new tw_graph();
        g->V = cfg->num_nodes;
        g->directed = cfg->directed != 0;
        g->window = cfg->window;
        g->stream = static_cast<hipStream_t>(cfg->hip_stream);
        if (hipGetDevice(&g->device) != hipSuccess) {
            delete g;
            return fail(TW_EDEVICE, "tw_create: no HIP device");
        }
        // the device array of tw_sample_walks_noalloc, with the device current
        tw::Error e{TW_OK, ""};
        if (tw::noalloc_setup(g->device, e) != TW_OK) {
            delete g;
            return report(e.code, e);
        }
        *out = g;
        return TW_OK;
    });
}

tw_status tw_destroy(tw_graph* g) {
    if (!g) return TW_OK;
    return guarded("tw_destroy", [&]() -> tw_status {
        tw::release_graph(g);
        return TW_OK;
    });
}

tw_status tw_set_stream(tw_graph* g, void* hip_stream) {
    if (!g) return fail(TW_EINVAL, "tw_set_stream: null graph");
    if (hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(TW_EDEVICE, "tw_set_stream: synchronising the old stream failed");
    g->stream = static_cast<hipStream_t>(hip_stream);
    if (g->rev) g->rev->stream = g->stream;
    return TW_OK;
}

tw_status tw_ingest_batch(tw_graph* g, const int32_t* d_src, const int32_t* d_dst,
                          const int64_t* d_ts, int64_t n, tw_ingest_info* info) {
    if (!g) return fail(TW_EINVAL, "tw_ingest_batch: null graph");
    if (n < 0 || (n > 0 && (!d_src || !d_dst || !d_ts)))
        return fail(TW_EINVAL, "tw_ingest_batch: need n >= 0 and non-null arrays");
    return guarded("tw_ingest_batch", [&]() -> tw_status {
        tw_status st = refuse_broken(g, "tw_ingest_batch");
        // the graph's own flags come back with the batch's first read-back;
        // the in-view's (backward walks) are read here
        if (st == TW_OK && g->rev) st = check_flags_of(g->rev);
        if (st != TW_OK) return st;
        tw::Error e{TW_OK, ""};
        return report(tw::ingest_views(g, d_src, d_dst, d_ts, n, info, e, nullptr, true), e);
    });
}

tw_status tw_evict_before(tw_graph* g, int64_t t_cutoff, int64_t* n_evicted) {
    if (!g) return fail(TW_EINVAL, "tw_evict_before: null graph");
    return guarded("tw_evict_before", [&]() -> tw_status {
        tw_status st = refuse_broken(g, "tw_evict_before");
        if (st != TW_OK) return st;
        // nothing to evict: no device work and no synchronisation (with the
        // window summary still on the device, its host-known lower bound)
        if (g->m == 0 || t_cutoff <= (g->sum_stale ? g->t_min_lb : g->t_min)) {
            g->last.accepted = 0;
            g->last.dropped_late = 0;
            g->last.evicted = 0;
            if (n_evicted) *n_evicted = 0;
            return TW_OK;
        }
        st = check_device_flags(g);
        if (st != TW_OK) return st;
        tw::Error e{TW_OK, ""};
        return report(tw::evict_views(g, t_cutoff, n_evicted, e), e);
    });
}

tw_status tw_set_ingest_weights(tw_graph* g, double tau) {
    if (!g) return fail(TW_EINVAL, "tw_set_ingest_weights: null graph");
    if (std::isinf(tau)) return fail(TW_EINVAL, "tw_set_ingest_weights: tau must be finite or NaN");
    g->ingest_weight_tau = tau;
    return TW_OK;
}

tw_status tw_get_tuning(const tw_graph* g, tw_tuning* out) {
    if (!g || !out) return fail(TW_EINVAL, "tw_get_tuning: null argument");
    *out = tw::get_tuning(g);
    return TW_OK;
}

tw_status tw_set_tuning(tw_graph* g, const tw_tuning* t) {
    if (!g) return fail(TW_EINVAL, "tw_set_tuning: null graph");
    tw::Error e{TW_OK, ""};
    return report(tw::set_tuning(g, t, e), e);
}

tw_status tw_sample_walks(tw_graph* g, const tw_walk_params* params, int32_t* d_nodes,
                          int64_t* d_ts, int32_t* d_len) {
    if (!g) return fail(TW_EINVAL, "tw_sample_walks: null graph");
    return guarded("tw_sample_walks", [&]() -> tw_status {
        if (refuse_broken(g, "tw_sample_walks") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        return report(tw::sample_walks(g, params, d_nodes, d_ts, d_len, e), e);
    });
}

tw_status tw_sample_walks_noalloc(tw_graph* g, const tw_walk_params* params, int32_t* d_nodes,
                                  int64_t* d_ts, int32_t* d_len) {
    if (!g) return fail(TW_EINVAL, "tw_sample_walks_noalloc: null graph");
    return guarded("tw_sample_walks_noalloc", [&]() -> tw_status {
        if (refuse_broken(g, "tw_sample_walks_noalloc") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        return report(tw::sample_walks_noalloc(g, params, d_nodes, d_ts, d_len, e), e);
    });
}

tw_status tw_sample_walks_batch(tw_graph* g, const tw_batch_params* params, int32_t* d_nodes,
                                int64_t* d_ts, int32_t* d_len) {
    if (!g) return fail(TW_EINVAL, "tw_sample_walks_batch: null graph");
    return guarded("tw_sample_walks_batch", [&]() -> tw_status {
        if (refuse_broken(g, "tw_sample_walks_batch") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        return report(tw::sample_walks_batch(g, params, d_nodes, d_ts, d_len, e), e);
    });
}

tw_status tw_row_offsets(tw_graph* g, const int32_t* d_max_len, int64_t n, int64_t* d_row,
                         int64_t* total) {
    if (!g) return fail(TW_EINVAL, "tw_row_offsets: null graph");
    return guarded("tw_row_offsets", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::row_offsets(g, d_max_len, n, d_row, total, e), e);
    });
}

tw_status tw_autotune(tw_graph* g, const tw_walk_params* params, int64_t sample_walks,
                      int32_t* d_nodes, int64_t* d_ts, int32_t* d_len, int32_t best[2]) {
    if (!g) return fail(TW_EINVAL, "tw_autotune: null graph");
    return guarded("tw_autotune", [&]() -> tw_status {
        if (refuse_broken(g, "tw_autotune") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        return report(tw::autotune(g, params, sample_walks, d_nodes, d_ts, d_len, best, e), e);
    });
}

tw_status tw_server_create(tw_graph* g, const tw_server_config* cfg, tw_server** out) {
    return guarded("tw_server_create", [&]() -> tw_status {
        if (g && refuse_broken(g, "tw_server_create") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        return report(tw::server_create(g, cfg, out, e), e);
    });
}

tw_status tw_server_submit(tw_server* s, const tw_walk_params* req, uint64_t* id) {
    if (!s) return fail(TW_EINVAL, "tw_server_submit: null server");
    return guarded("tw_server_submit", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_submit(s, req, id, e), e);
    });
}

tw_status tw_server_ingest(tw_server* s, const int32_t* d_src, const int32_t* d_dst,
                           const int64_t* d_ts, int64_t n, uint64_t* id) {
    if (!s) return fail(TW_EINVAL, "tw_server_ingest: null server");
    return guarded("tw_server_ingest", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_ingest(s, d_src, d_dst, d_ts, n, id, e), e);
    });
}

tw_status tw_server_wait(tw_server* s, uint64_t id, int64_t timeout_us, tw_request_result* out) {
    if (!s) return fail(TW_EINVAL, "tw_server_wait: null server");
    return guarded("tw_server_wait", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_wait(s, id, timeout_us, out, e), e);
    });
}

tw_status tw_server_release(tw_server* s, uint64_t id) {
    if (!s) return fail(TW_EINVAL, "tw_server_release: null server");
    return guarded("tw_server_release", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_release(s, id, e), e);
    });
}

tw_status tw_server_copy_out(tw_server* s, uint64_t id, int32_t* d_nodes, int64_t* d_ts,
                             int32_t* d_len) {
    if (!s) return fail(TW_EINVAL, "tw_server_copy_out: null server");
    return guarded("tw_server_copy_out", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_copy_out(s, id, d_nodes, d_ts, d_len, e), e);
    });
}

tw_status tw_server_stats(tw_server* s, tw_server_counters* out) {
    if (!s) return fail(TW_EINVAL, "tw_server_stats: null server");
    return guarded("tw_server_stats", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_stats(s, out, e), e);
    });
}

tw_status tw_server_destroy(tw_server* s) {
    if (!s) return TW_OK;
    return guarded("tw_server_destroy", [&]() -> tw_status {
        tw::Error e{TW_OK, ""};
        return report(tw::server_destroy(s, e), e);
    });
}

tw_status tw_sync(tw_graph* g) {
    if (!g) return fail(TW_EINVAL, "tw_sync: null graph");
    if (hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(TW_EDEVICE, "tw_sync: stream synchronisation failed");
    return check_device_flags(g);
}

tw_status tw_stats(tw_graph* g, tw_ingest_info* info) {
    if (!g || !info) return fail(TW_EINVAL, "tw_stats: null argument");
    tw_status st = tw_sync(g);
    tw::Error e{TW_OK, ""};
    if (st == TW_OK && tw::refresh_summary(g, e) != TW_OK) st = report(e.code, e);
    *info = g->last;
    info->active_edges = g->m;
    info->t_min = g->t_min;
    info->t_max = g->t_max;
    return st;
}

tw_status tw_view_sizes(tw_graph* g, int64_t out[4]) {
    if (!g || !out) return fail(TW_EINVAL, "tw_view_sizes: null argument");
    if (hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(TW_EDEVICE, "tw_view_sizes: stream synchronisation failed");
    return guarded("tw_view_sizes", [&]() -> tw_status {
        if (refuse_broken(g, "tw_view_sizes") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        if (!g->rec.p && tw::init_empty(g, e) != TW_OK) return report(e.code, e);
        int64_t gn = 0;
        if (tw::nv_group_count(g, &gn, e) != TW_OK) return report(e.code, e);
        if (tw::refresh_summary(g, e) != TW_OK) return report(e.code, e);
        out[0] = g->m;
        out[1] = g->Gg;
        out[2] = gn;
        out[3] = g->V;
        return TW_OK;
    });
}

tw_status tw_export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                          int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                          int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg) {
    if (!g) return fail(TW_EINVAL, "tw_export_views: null graph");
    return guarded("tw_export_views", [&]() -> tw_status {
        if (refuse_broken(g, "tw_export_views") != TW_OK) return TW_EDEVICE;
        tw::Error e{TW_OK, ""};
        if (!g->rec.p && tw::init_empty(g, e) != TW_OK) return report(e.code, e);
        return report(tw::export_views(g, src, dst, ts, g_ts, g_off, n_dst, n_ts, n_gts, n_goff,
                                       n_ebeg, n_gbeg, e),
                      e);
    });
}

tw_status tw_last_update(const tw_graph* g, int64_t out[4]) {
    if (!g || !out) return fail(TW_EINVAL, "tw_last_update: null argument");
    out[0] = g->last.accepted;
    out[1] = g->last.dropped_late;
    out[2] = g->last.evicted;
    out[3] = g->m;
    return TW_OK;
}

namespace {

// FNV-1a over the words that decide what a recorded walk launch reads
uint64_t layout_of(const tw_graph* g) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
        for (int k = 0; k < 8; ++k) {
            h ^= (x >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (const tw::DevBuf* b : const_cast<tw_graph*>(g)->buffers())
        mix(reinterpret_cast<uintptr_t>(b->p));
    mix(g->adj_ready ? 1u : 0u);
    mix(g->adj_mask);
    mix(g->w_ready ? 1u : 0u);
    uint64_t ws;
    std::memcpy(&ws, &g->w_scale, sizeof ws);
    mix(ws);
    mix(g->rev ? layout_of(g->rev) : 0u);
    return h;
}

}  // namespace

tw_status tw_walk_layout(const tw_graph* g, uint64_t* out) {
    if (!g || !out) return fail(TW_EINVAL, "tw_walk_layout: null argument");
    *out = layout_of(g);
    return TW_OK;
}

tw_status tw_index_stats(const tw_graph* g, int64_t out[8]) {
    if (!g || !out) return fail(TW_EINVAL, "tw_index_stats: null argument");
    out[0] = g->st_jobs;
    out[1] = g->st_written;
    out[2] = g->st_new_slots;
    out[3] = g->st_full;
    out[4] = g->pe_top;
    out[5] = g->pg_top;
    out[6] = g->pf_top;
    out[7] = g->pe_cap;
    return TW_OK;
}

int64_t tw_device_bytes(const tw_graph* g) {
    if (!g) return 0;

    int64_t total = 0;
    for (const tw::DevBuf* b : const_cast<tw_graph*>(g)->buffers()) total += (int64_t)b->bytes;
    return total + (g->rev ? tw_device_bytes(g->rev) : 0);
}

const char* tw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
