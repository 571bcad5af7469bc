// Serving loop: continuous batching of walk requests interleaved with
// ingestion (the request loop of the C ABI's tw_server_* calls).
//
// Submissions (walk requests and ingest batches) enter one FIFO. A worker
// thread owns the graph: it applies an ingest batch when it reaches the
// front, and packs the consecutive requests at the front into one serving
// launch (walk.hip, k_walk_serve) once their outputs fit in the arena, while
// earlier launches may still run (continuous batching, up to max_inflight
// launches enqueued). A request therefore sees exactly the batches submitted
// before it. Completion is observed through one HIP event per launch;
// latency runs from submission to the worker seeing that event.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "tw_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t ALIGN = 256;
constexpr int MAX_INFLIGHT = 8;
constexpr int MAX_REQ_PER_LAUNCH = 1024;

size_t round_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    // offset, or SIZE_MAX when no free range is large enough
    size_t alloc(size_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

enum { ST_QUEUED = 0, ST_RUNNING = 1, ST_DONE = 2 };

struct Item {
    bool ingest = false;
    int state = ST_QUEUED;
    tw_status status = TW_OK;
    // request
    tw_walk_params p{};
    size_t off = SIZE_MAX, bytes = 0;
    int32_t* nodes = nullptr;
    int64_t* ts = nullptr;
    int32_t* len = nullptr;
    // ingest
    const int32_t* src = nullptr;
    const int32_t* dst = nullptr;
    const int64_t* its = nullptr;
    int64_t n = 0;
    tw_ingest_info info{};
    int64_t cap_hits = 0;  // node2vec walks that ended at the trial cap
    Clock::time_point t_submit, t_start, t_done;
};

struct Launch {
    int slot;
    std::vector<uint64_t> ids;
    int64_t walks;
};

size_t request_bytes(const tw_walk_params& p) {
    const size_t slots = (size_t)p.num_walks * (size_t)p.max_len;
    return round_up(4 * slots) + round_up(8 * slots) + round_up(4 * (size_t)p.num_walks);
}

}  // namespace

struct tw_server {
    tw_graph* g = nullptr;
    tw_server_config cfg{};
    char* arena_base = nullptr;
    Arena arena;
    void* d_tables = nullptr;  // MAX_INFLIGHT launch tables
    void* h_tables = nullptr;  // pinned staging of the tables
    unsigned long long* d_hops = nullptr;  // per slot
    unsigned long long* h_hops = nullptr;  // pinned per slot
    uint32_t* d_err = nullptr;             // per slot: two words per request of the launch
    uint32_t* h_err = nullptr;             // pinned copy
    hipEvent_t ev[MAX_INFLIGHT] = {};
    bool slot_busy[MAX_INFLIGHT] = {};
    size_t table_bytes = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> fifo;
    std::map<uint64_t, Item> items;
    uint64_t next_id = 1;
    std::deque<Launch> inflight;
    bool stop = false;
    std::thread worker;

    // counters
    int64_t requests_done = 0, walks_done = 0, hops_done = 0, launches = 0, ingests = 0;
    std::vector<double> latencies;
    Clock::time_point t0;
};

namespace {

__global__ void k_zero_u64(unsigned long long* p) { *p = 0; }

__global__ void k_zero_words(uint32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

constexpr int ERR_WORDS = 2 * MAX_REQ_PER_LAUNCH;  // per launch slot

// launches whose event has completed, in order
void retire(tw_server* S) {
    while (!S->inflight.empty()) {
        Launch& L = S->inflight.front();
        if (hipEventQuery(S->ev[L.slot]) != hipSuccess) break;
        const auto now = Clock::now();
        const uint32_t* ew = S->h_err + (size_t)L.slot * ERR_WORDS;
        for (size_t r = 0; r < L.ids.size(); ++r) {
            Item& it = S->items[L.ids[r]];
            it.state = ST_DONE;
            it.t_done = now;
            // a start node out of range fails the request (its walks read
            // length 0 there); walks ended by node2vec's trial cap are counted
            if (ew[2 * r]) it.status = TW_ERANGE;
            it.cap_hits = ew[2 * r + 1];
            S->latencies.push_back(ms_between(it.t_submit, now));
            ++S->requests_done;
            S->walks_done += it.p.num_walks;
        }
        S->hops_done += (int64_t)S->h_hops[L.slot];
        S->slot_busy[L.slot] = false;
        S->inflight.pop_front();
        S->cv_done.notify_all();
    }
}

void finish_failed(tw_server* S, const std::vector<uint64_t>& ids, tw_status st) {
    const auto now = Clock::now();
    for (uint64_t id : ids) {
        Item& it = S->items[id];
        it.state = ST_DONE;
        it.status = st;
        it.t_done = now;
    }
    S->cv_done.notify_all();
}

void worker_loop(tw_server* S) {
    (void)hipSetDevice(S->g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        retire(S);
        if (S->stop && S->fifo.empty() && S->inflight.empty()) break;
        bool progressed = false;
        if (!S->fifo.empty() && S->items[S->fifo.front()].ingest) {
            const uint64_t id = S->fifo.front();
            S->fifo.pop_front();
            Item& it = S->items[id];
            it.state = ST_RUNNING;
            it.t_start = Clock::now();
            const int32_t* src = it.src;
            const int32_t* dst = it.dst;
            const int64_t* its = it.its;
            const int64_t n = it.n;
            lk.unlock();
            tw::Error e{TW_OK, ""};
            tw_ingest_info info{};
            // the graph and its in-view (if backward walks created one)
            const tw_status st = tw::ingest_views(S->g, src, dst, its, n, &info, e);
            lk.lock();
            Item& done = S->items[id];
            done.status = st;
            done.info = info;
            done.state = ST_DONE;
            done.t_done = Clock::now();
            ++S->ingests;
            S->cv_done.notify_all();
            progressed = true;
        } else if (!S->fifo.empty() && (int)S->inflight.size() < S->cfg.max_inflight) {
            // admit the consecutive requests at the front that fit
            std::vector<uint64_t> ids;
            int64_t walks = 0;
            while (!S->fifo.empty() && (int)ids.size() < MAX_REQ_PER_LAUNCH) {
                Item& it = S->items[S->fifo.front()];
                if (it.ingest) break;
                if (!ids.empty() && walks + it.p.num_walks > S->cfg.max_walks_per_launch) break;
                const size_t off = S->arena.alloc(it.bytes);
                if (off == SIZE_MAX) break;  // wait for outputs to be released
                it.off = off;
                const size_t slots = (size_t)it.p.num_walks * (size_t)it.p.max_len;
                char* base = S->arena_base + off;
                it.nodes = reinterpret_cast<int32_t*>(base);
                it.ts = reinterpret_cast<int64_t*>(base + round_up(4 * slots));
                it.len = reinterpret_cast<int32_t*>(base + round_up(4 * slots) +
                                                    round_up(8 * slots));
                it.state = ST_RUNNING;
                it.t_start = Clock::now();
                walks += it.p.num_walks;
                ids.push_back(S->fifo.front());
                S->fifo.pop_front();
            }
            if (!ids.empty()) {
                int slot = 0;
                while (S->slot_busy[slot]) ++slot;
                S->slot_busy[slot] = true;
                std::vector<tw::ServeReq> reqs;
                for (uint64_t id : ids) {
                    const Item& it = S->items[id];
                    tw::ServeReq r;
                    r.count = it.p.num_walks;
                    r.max_len = it.p.max_len;
                    r.hop = it.p.hop_bias;
                    r.start = it.p.start_bias;
                    r.start_mode = it.p.start_mode;
                    r.start_nodes = it.p.d_start_nodes;
                    r.seed = it.p.seed;
                    r.base = it.p.walk_id_base;
                    r.nodes = it.nodes;
                    r.ts = it.ts;
                    r.len = it.len;
                    reqs.push_back(r);
                }
                lk.unlock();
                tw::Error e{TW_OK, ""};
                hipStream_t s = S->g->stream;
                char* dt = static_cast<char*>(S->d_tables) + slot * S->table_bytes;
                char* ht = static_cast<char*>(S->h_tables) + slot * S->table_bytes;
                uint32_t* de = S->d_err + (size_t)slot * ERR_WORDS;
                const int nw = 2 * (int)reqs.size();
                hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, S->d_hops + slot);
                hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, de, nw);
                tw_status st = tw::serve_launch(S->g, reqs.data(), (int)reqs.size(), dt, ht,
                                                S->d_hops + slot, de, e);
                if (st == TW_OK &&
                    (hipMemcpyAsync(S->h_hops + slot, S->d_hops + slot, sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, s) != hipSuccess ||
                     hipMemcpyAsync(S->h_err + (size_t)slot * ERR_WORDS, de, sizeof(uint32_t) * nw,
                                    hipMemcpyDeviceToHost, s) != hipSuccess ||
                     hipEventRecord(S->ev[slot], s) != hipSuccess))
                    st = TW_EDEVICE;
                lk.lock();
                if (st != TW_OK) {
                    S->slot_busy[slot] = false;
                    finish_failed(S, ids, st);
                } else {
                    S->inflight.push_back(Launch{slot, ids, walks});
                    ++S->launches;
                }
                progressed = true;
            }
        }
        if (!progressed && S->stop && S->inflight.empty() && !S->fifo.empty()) {
            // stopping with requests whose outputs cannot be placed (the
            // arena holds unreleased results): fail them instead of waiting
            std::vector<uint64_t> rest(S->fifo.begin(), S->fifo.end());
            S->fifo.clear();
            finish_failed(S, rest, TW_ENOMEM);
            continue;
        }
        if (!progressed) {
            if (!S->inflight.empty()) {
                // a launch is running: poll its event
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
                lk.lock();
            } else {
                S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
}

}  // namespace

namespace tw {

tw_status server_create(tw_graph* g, const tw_server_config* cfg, tw_server** out, Error& err) {
    if (!g || !cfg || !out || cfg->arena_bytes < (int64_t)ALIGN || cfg->max_walks_per_launch < 1 ||
        cfg->max_inflight < 1 || cfg->max_inflight > MAX_INFLIGHT) {
        err = Error{TW_EINVAL, "server_create: need arena_bytes >= 256, max_walks_per_launch >= 1, "
                               "max_inflight in 1..8"};
        return err.code;
    }
    if (!g->rec.p && init_empty(g, err) != TW_OK) return err.code;
    tw_server* S = new tw_server();
    S->g = g;
    S->cfg = *cfg;
    S->table_bytes = round_up(serve_table_bytes(MAX_REQ_PER_LAUNCH));
    auto cleanup = [&]() {
        if (S->arena_base) (void)hipFree(S->arena_base);
        if (S->d_tables) (void)hipFree(S->d_tables);
        if (S->d_hops) (void)hipFree(S->d_hops);
        if (S->d_err) (void)hipFree(S->d_err);
        if (S->h_tables) (void)hipHostFree(S->h_tables);
        if (S->h_hops) (void)hipHostFree(S->h_hops);
        if (S->h_err) (void)hipHostFree(S->h_err);
        for (hipEvent_t& e : S->ev)
            if (e) (void)hipEventDestroy(e);
        delete S;
    };
    if (hipMalloc(reinterpret_cast<void**>(&S->arena_base), (size_t)cfg->arena_bytes) != hipSuccess ||
        hipMalloc(&S->d_tables, S->table_bytes * MAX_INFLIGHT) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&S->d_hops), sizeof(unsigned long long) * MAX_INFLIGHT) !=
            hipSuccess ||
        hipHostMalloc(&S->h_tables, S->table_bytes * MAX_INFLIGHT, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&S->h_hops),
                      sizeof(unsigned long long) * MAX_INFLIGHT, hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&S->d_err),
                  sizeof(uint32_t) * ERR_WORDS * MAX_INFLIGHT) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&S->h_err),
                      sizeof(uint32_t) * ERR_WORDS * MAX_INFLIGHT, hipHostMallocDefault) !=
            hipSuccess) {
        hipGetLastError();
        cleanup();
        err = Error{TW_ENOMEM, "server_create: device or pinned allocation failed"};
        return err.code;
    }
    for (hipEvent_t& e : S->ev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            cleanup();
            err = Error{TW_EDEVICE, "server_create: event creation failed"};
            return err.code;
        }
    }
    S->arena.reset((size_t)cfg->arena_bytes / ALIGN * ALIGN);
    S->t0 = Clock::now();
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return TW_OK;
}

tw_status server_submit(tw_server* S, const tw_walk_params* p, uint64_t* id, Error& err) {
    if (check_walk_params(p, err) != TW_OK) return err.code;
    if (p->hop_bias.kind == TW_WEIGHT || p->direction != TW_FORWARD) {
        err = Error{TW_EINVAL, "server_submit: served walks are forward, without TW_WEIGHT"};
        return err.code;
    }
    if (!id) {
        err = Error{TW_EINVAL, "server_submit: null id"};
        return err.code;
    }
    const size_t bytes = request_bytes(*p);
    if (bytes > (size_t)S->cfg.arena_bytes / ALIGN * ALIGN) {
        err = Error{TW_EINVAL, "server_submit: the request's outputs exceed the arena"};
        return err.code;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t k = S->next_id++;
    Item& it = S->items[k];
    it.p = *p;
    it.bytes = bytes;
    it.t_submit = Clock::now();
    S->fifo.push_back(k);
    *id = k;
    S->cv_work.notify_one();
    return TW_OK;
}

tw_status server_ingest(tw_server* S, const int32_t* src, const int32_t* dst, const int64_t* ts,
                        int64_t n, uint64_t* id, Error& err) {
    if (n < 0 || (n > 0 && (!src || !dst || !ts)) || !id) {
        err = Error{TW_EINVAL, "server_ingest: need n >= 0, non-null arrays and id"};
        return err.code;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t k = S->next_id++;
    Item& it = S->items[k];
    it.ingest = true;
    it.src = src;
    it.dst = dst;
    it.its = ts;
    it.n = n;
    it.t_submit = Clock::now();
    S->fifo.push_back(k);
    *id = k;
    S->cv_work.notify_one();
    return TW_OK;
}

tw_status server_wait(tw_server* S, uint64_t id, int64_t timeout_us, tw_request_result* out,
                      Error& err) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto found = S->items.find(id);
    if (found == S->items.end()) {
        err = Error{TW_EINVAL, "server_wait: unknown request"};
        return err.code;
    }
    auto done = [&]() { return S->items[id].state == ST_DONE; };
    if (timeout_us < 0) S->cv_done.wait(lk, done);
    else S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
    const Item& it = S->items[id];
    if (it.state != ST_DONE) {
        err = Error{TW_ETIMEOUT, "server_wait: not finished"};
        return err.code;
    }
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->status = it.status;
        out->d_nodes = it.nodes;
        out->d_ts = it.ts;
        out->d_len = it.len;
        out->num_walks = it.ingest ? 0 : it.p.num_walks;
        out->max_len = it.ingest ? 0 : it.p.max_len;
        out->queue_ms = ms_between(it.t_submit, it.t_start);
        out->latency_ms = ms_between(it.t_submit, it.t_done);
        out->ingest = it.info;
        out->trial_cap_hits = it.cap_hits;
    }
    return TW_OK;
}

tw_status server_release(tw_server* S, uint64_t id, Error& err) {
    std::lock_guard<std::mutex> lk(S->mu);
    auto found = S->items.find(id);
    if (found == S->items.end() || found->second.state != ST_DONE) {
        err = Error{TW_EINVAL, "server_release: unknown or unfinished request"};
        return err.code;
    }
    if (found->second.off != SIZE_MAX) S->arena.release(found->second.off, found->second.bytes);
    S->items.erase(found);
    S->cv_work.notify_one();  // memory for waiting requests
    return TW_OK;
}

tw_status server_copy_out(tw_server* S, uint64_t id, int32_t* nodes, int64_t* ts, int32_t* len,
                          Error& err) {
    const int32_t* sn;
    const int64_t* st;
    const int32_t* sl;
    size_t slots, walks;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto found = S->items.find(id);
        if (found == S->items.end() || found->second.state != ST_DONE || found->second.ingest ||
            found->second.status != TW_OK) {
            err = Error{TW_EINVAL, "server_copy_out: unknown, unfinished or failed request"};
            return err.code;
        }
        const Item& it = found->second;
        sn = it.nodes;
        st = it.ts;
        sl = it.len;
        walks = (size_t)it.p.num_walks;
        slots = walks * (size_t)it.p.max_len;
    }
    // the request has finished, so its outputs are complete; it stays
    // allocated until released, which the caller does not do concurrently
    if (walks == 0) return TW_OK;
    if (nodes) TW_HIP(hipMemcpy(nodes, sn, 4 * slots, hipMemcpyDeviceToDevice));
    if (ts) TW_HIP(hipMemcpy(ts, st, 8 * slots, hipMemcpyDeviceToDevice));
    if (len) TW_HIP(hipMemcpy(len, sl, 4 * walks, hipMemcpyDeviceToDevice));
    return TW_OK;
}

tw_status server_stats(tw_server* S, tw_server_counters* out, Error& err) {
    if (!out) {
        err = Error{TW_EINVAL, "server_stats: null output"};
        return err.code;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->requests_done = S->requests_done;
    out->walks_done = S->walks_done;
    out->hops_done = S->hops_done;
    out->launches = S->launches;
    out->ingests = S->ingests;
    out->wall_s = std::chrono::duration<double>(Clock::now() - S->t0).count();
    if (!S->latencies.empty()) {
        std::vector<double> v = S->latencies;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const size_t k = (size_t)std::min<double>(v.size() - 1, q * (double)(v.size() - 1) + 0.5);
            return v[k];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        double sum = 0.0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
    }
    return TW_OK;
}

tw_status server_destroy(tw_server* S, Error& err) {
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipStreamSynchronize(S->g->stream);
    (void)hipFree(S->arena_base);
    (void)hipFree(S->d_tables);
    (void)hipFree(S->d_hops);
    (void)hipFree(S->d_err);
    (void)hipHostFree(S->h_tables);
    (void)hipHostFree(S->h_hops);
    (void)hipHostFree(S->h_err);
    for (hipEvent_t e : S->ev) (void)hipEventDestroy(e);
    delete S;
    (void)err;
    return TW_OK;
}

}  // namespace tw
