// Serving loop: continuous batching of walk requests interleaved with
// ingestion (the request loop of the C ABI's tw_server_* calls).
//
// Submissions (walk requests and ingest batches) enter one FIFO. A worker
// thread packs the consecutive requests at the front into one serving launch
// (walk.hip, k_walk_serve) on the graph's stream once their outputs are
// placed, while earlier launches may still run (continuous batching, up to
// max_inflight launches enqueued). An ingest batch at the front goes to an
// ingest thread, which plans it on a stream of its own while the walks of
// the current index still run (ingest_prepare reads the index and writes
// only ingest buffers), and changes the index after an event that marks
// every walk launch enqueued before the batch; the walk launches after it
// wait for the update. A request therefore sees exactly the batches
// submitted before it (its index epoch). Request outputs live in arena
// chunks: the first is allocated at create, more are added while the device
// keeps a reserve of free memory. Completion is observed through one HIP
// event per launch; latency runs from submission to the worker seeing that
// event.
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
    int chunk = -1;  // arena chunk of the outputs
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
    // output arena chunks (base, first-fit free list)
    std::vector<char*> chunk_base;
    std::vector<Arena> chunk;
    int64_t arena_total = 0;
    hipStream_t s_walk = nullptr;  // the graph's stream: walk launches
    hipStream_t s_ing = nullptr;   // the ingest thread's stream
    hipEvent_t ev_walks = nullptr;    // every walk launch enqueued before an ingest
    hipEvent_t ev_applied = nullptr;  // the last ingest's index update
    bool applied_pending = false;     // the next walk launch waits for ev_applied
    bool ing_busy = false;            // an ingest batch is with the ingest thread
    bool ing_taken = false;           // ... and the thread has started it
    uint64_t ing_id = 0;
    bool ing_stop = false;
    std::thread ingester;
    std::condition_variable cv_ing;
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
    int64_t chunks_added = 0;
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

// A place for `bytes` of request outputs: a free range of a chunk, else a
// new chunk when the device keeps hbm_reserve_bytes free after it (never
// when hbm_reserve_bytes < 0). Called with the lock held.
bool place_outputs(tw_server* S, size_t bytes, int* chunk, size_t* off) {
    for (size_t c = 0; c < S->chunk.size(); ++c) {
        const size_t o = S->chunk[c].alloc(bytes);
        if (o != SIZE_MAX) {
            *chunk = (int)c;
            *off = o;
            return true;
        }
    }
    if (S->cfg.hbm_reserve_bytes < 0) return false;
    const size_t want = std::max(round_up(bytes), (size_t)S->cfg.arena_bytes / ALIGN * ALIGN);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if ((int64_t)free_b < (int64_t)want + S->cfg.hbm_reserve_bytes) return false;
    char* base = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&base), want) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    S->chunk_base.push_back(base);
    S->chunk.emplace_back();
    S->chunk.back().reset(want);
    S->arena_total += (int64_t)want;
    ++S->chunks_added;
    *chunk = (int)S->chunk.size() - 1;
    *off = S->chunk.back().alloc(bytes);
    return *off != SIZE_MAX;
}

// The ingest thread: plans each batch handed to it on s_ing while the walks
// enqueued before it run, then updates the index after ev_walks.
void ingest_loop(tw_server* S) {
    (void)hipSetDevice(S->g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_ing.wait(lk, [&]() { return S->ing_stop || (S->ing_busy && !S->ing_taken); });
        if (!(S->ing_busy && !S->ing_taken)) break;  // stopping, nothing handed over
        S->ing_taken = true;
        const uint64_t id = S->ing_id;
        Item& it = S->items[id];
        const int32_t* src = it.src;
        const int32_t* dst = it.dst;
        const int64_t* its = it.its;
        const int64_t n = it.n;
        lk.unlock();
        tw_graph* g = S->g;
        tw::Error e{TW_OK, ""};
        tw_ingest_info info{};
        // the worker launches nothing while the batch is here, so the graph
        // is this thread's until it hands the batch back
        g->stream = S->s_ing;
        if (g->rev) g->rev->stream = S->s_ing;
        tw_status st = tw::ingest_views(g, src, dst, its, n, &info, e, S->ev_walks);
        if (hipEventRecord(S->ev_applied, S->s_ing) != hipSuccess && st == TW_OK) st = TW_EDEVICE;
        g->stream = S->s_walk;
        if (g->rev) g->rev->stream = S->s_walk;
        lk.lock();
        Item& done = S->items[id];
        done.status = st;
        done.info = info;
        done.state = ST_DONE;
        done.t_done = Clock::now();
        ++S->ingests;
        S->ing_busy = false;
        S->ing_taken = false;
        S->applied_pending = true;
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

void worker_loop(tw_server* S) {
    (void)hipSetDevice(S->g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        retire(S);
        if (S->stop && S->fifo.empty() && S->inflight.empty() && !S->ing_busy) break;
        bool progressed = false;
        if (!S->fifo.empty() && S->items[S->fifo.front()].ingest) {
            if (!S->ing_busy) {
                // hand the batch over; it updates the index after every
                // walk launch enqueued so far
                const uint64_t id = S->fifo.front();
                S->fifo.pop_front();
                Item& it = S->items[id];
                it.state = ST_RUNNING;
                it.t_start = Clock::now();
                if (hipEventRecord(S->ev_walks, S->s_walk) != hipSuccess) {
                    (void)hipGetLastError();
                    it.state = ST_DONE;
                    it.status = TW_EDEVICE;
                    it.t_done = Clock::now();
                    S->cv_done.notify_all();
                } else {
                    S->ing_busy = true;
                    S->ing_taken = false;
                    S->ing_id = id;
                    S->cv_ing.notify_one();
                }
                progressed = true;
            }
        } else if (!S->fifo.empty() && !S->ing_busy &&
                   (int)S->inflight.size() < S->cfg.max_inflight) {
            // admit the consecutive requests at the front that fit: one
            // direction a launch, and one time scale for its weight-based ones
            std::vector<uint64_t> ids;
            int64_t walks = 0;
            const bool rev = S->items[S->fifo.front()].p.direction == TW_BACKWARD;
            double wscale = 0.0;  // 0: no weight-based request yet
            while (!S->fifo.empty() && (int)ids.size() < MAX_REQ_PER_LAUNCH) {
                Item& it = S->items[S->fifo.front()];
                if (it.ingest) break;
                if (!ids.empty() && walks + it.p.num_walks > S->cfg.max_walks_per_launch) break;
                if ((it.p.direction == TW_BACKWARD) != rev) break;
                if (it.p.hop_bias.kind == TW_WEIGHT) {
                    const double sc = it.p.hop_bias.tau > 0.0 ? it.p.hop_bias.tau : 1.0;
                    if (wscale != 0.0 && sc != wscale) break;
                    wscale = sc;
                }
                int c = -1;
                size_t off = SIZE_MAX;
                if (!place_outputs(S, it.bytes, &c, &off)) break;  // wait for releases
                it.chunk = c;
                it.off = off;
                const size_t slots = (size_t)it.p.num_walks * (size_t)it.p.max_len;
                char* base = S->chunk_base[c] + off;
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
                const bool wait_applied = S->applied_pending;
                S->applied_pending = false;
                lk.unlock();
                tw::Error e{TW_OK, ""};
                hipStream_t s = S->s_walk;
                char* dt = static_cast<char*>(S->d_tables) + slot * S->table_bytes;
                char* ht = static_cast<char*>(S->h_tables) + slot * S->table_bytes;
                uint32_t* de = S->d_err + (size_t)slot * ERR_WORDS;
                const int nw = 2 * (int)reqs.size();
                tw_status st = TW_OK;
                // the walks of a new epoch start after its index update
                if (wait_applied && hipStreamWaitEvent(s, S->ev_applied, 0) != hipSuccess)
                    st = TW_EDEVICE;
                // an index whose update failed midway serves nothing
                if (st == TW_OK && S->g->broken) st = TW_EDEVICE;
                // backward requests walk the in-view (made from the window on
                // the first one; no batch is being ingested meanwhile)
                tw_graph* gl = S->g;
                if (st == TW_OK && rev && tw::backward_view(S->g, &gl, e) != TW_OK) st = e.code;
                if (st == TW_OK) {
                    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, S->d_hops + slot);
                    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, de, nw);
                    st = tw::serve_launch(gl, reqs.data(), (int)reqs.size(), dt, ht,
                                          S->d_hops + slot, de, rev, e);
                }
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
        if (!progressed && S->stop && S->inflight.empty() && !S->ing_busy && !S->fifo.empty() &&
            !S->items[S->fifo.front()].ingest) {
            // stopping with requests whose outputs cannot be placed (the
            // arena holds unreleased results): fail them instead of waiting
            std::vector<uint64_t> rest;
            while (!S->fifo.empty() && !S->items[S->fifo.front()].ingest) {
                rest.push_back(S->fifo.front());
                S->fifo.pop_front();
            }
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
    S->ing_stop = true;
    S->cv_ing.notify_all();
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
    S->s_walk = g->stream;
    S->table_bytes = round_up(serve_table_bytes(MAX_REQ_PER_LAUNCH));
    char* base0 = nullptr;
    auto cleanup = [&]() {
        if (base0) (void)hipFree(base0);
        if (S->d_tables) (void)hipFree(S->d_tables);
        if (S->d_hops) (void)hipFree(S->d_hops);
        if (S->d_err) (void)hipFree(S->d_err);
        if (S->h_tables) (void)hipHostFree(S->h_tables);
        if (S->h_hops) (void)hipHostFree(S->h_hops);
        if (S->h_err) (void)hipHostFree(S->h_err);
        for (hipEvent_t& e : S->ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : {S->ev_walks, S->ev_applied})
            if (e) (void)hipEventDestroy(e);
        if (S->s_ing) (void)hipStreamDestroy(S->s_ing);
        delete S;
    };
    const size_t arena = (size_t)cfg->arena_bytes / ALIGN * ALIGN;
    if (hipMalloc(reinterpret_cast<void**>(&base0), arena) != hipSuccess ||
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
    bool ok = true;
    for (hipEvent_t& e : S->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    for (hipEvent_t* e : {&S->ev_walks, &S->ev_applied})
        ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    // the ingest stream keeps the default priority, like the graph's
    ok = ok && hipStreamCreateWithFlags(&S->s_ing, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        cleanup();
        err = Error{TW_EDEVICE, "server_create: event or stream creation failed"};
        return err.code;
    }
    S->chunk_base.push_back(base0);
    S->chunk.emplace_back();
    S->chunk.back().reset(arena);
    S->arena_total = (int64_t)arena;
    S->t0 = Clock::now();
    S->worker = std::thread(worker_loop, S);
    S->ingester = std::thread(ingest_loop, S);
    *out = S;
    return TW_OK;
}

tw_status server_submit(tw_server* S, const tw_walk_params* p, uint64_t* id, Error& err) {
    if (check_walk_params(p, err) != TW_OK) return err.code;
    if (p->direction != TW_FORWARD && p->direction != TW_BACKWARD) {
        err = Error{TW_EINVAL, "server_submit: bad direction"};
        return err.code;
    }
    if (p->hop_bias.kind == TW_WEIGHT && p->direction != TW_FORWARD) {
        err = Error{TW_EINVAL, "server_submit: the weight-based picker walks forward only"};
        return err.code;
    }
    if (!id) {
        err = Error{TW_EINVAL, "server_submit: null id"};
        return err.code;
    }
    const size_t bytes = request_bytes(*p);
    if (S->cfg.hbm_reserve_bytes < 0 && bytes > (size_t)S->cfg.arena_bytes / ALIGN * ALIGN) {
        err = Error{TW_EINVAL, "server_submit: the request's outputs exceed the fixed arena"};
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
    if (found->second.off != SIZE_MAX)
        S->chunk[found->second.chunk].release(found->second.off, found->second.bytes);
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
    out->arena_bytes = S->arena_total;
    out->arena_chunks_added = S->chunks_added;
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
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->ing_stop = true;
        S->cv_ing.notify_all();
    }
    if (S->ingester.joinable()) S->ingester.join();
    (void)hipStreamSynchronize(S->s_ing);
    (void)hipStreamSynchronize(S->s_walk);
    // later calls on the graph are ordered after the last index update
    (void)hipStreamWaitEvent(S->s_walk, S->ev_applied, 0);
    for (char* b : S->chunk_base) (void)hipFree(b);
    (void)hipFree(S->d_tables);
    (void)hipFree(S->d_hops);
    (void)hipFree(S->d_err);
    (void)hipHostFree(S->h_tables);
    (void)hipHostFree(S->h_hops);
    (void)hipHostFree(S->h_err);
    for (hipEvent_t e : S->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : {S->ev_walks, S->ev_applied}) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(S->s_ing);
    delete S;
    (void)err;
    return TW_OK;
}

}  // namespace tw
