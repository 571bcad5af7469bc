/*
 * tw.h — C ABI of the MI355X streaming temporal random-walk library.
 *
 * The library keeps a sliding window of timestamped directed edges (u, v, t)
 * resident in HBM under the dual index of Tempest (arxiv 2605.16182,
 * Sec. "Dual-Index Organization"), rebuilds it on every ingested batch
 * (Sec. "Streaming Ingestion and Window Management"), and samples
 * causality-preserving temporal random walks from it with the closed-form
 * pickers of Eqs. (1)-(3) and temporal node2vec (Sec. "Temporal Bias
 * Sampling").
 *
 * Conventions shared by every call:
 *  - Every pointer named d_* is a device pointer on the graph's device.
 *    The library never frees caller memory. Input arrays are only read, and
 *    only until the call's work on the graph's stream has finished.
 *  - Work is enqueued on the graph's HIP stream (tw_config.hip_stream, or
 *    tw_set_stream). Calls that must read a count back synchronise that
 *    stream; this is stated per call.
 *  - No C++ exception crosses this boundary. A failing call returns a
 *    non-zero tw_status and tw_last_error() describes it (thread-local).
 *  - One graph handle must not be used from two host threads at once.
 *  - Timestamps are int64. Node ids are int32 in [0, num_nodes).
 *  - The active window holds at most 2^32 - 2 edges.
 */
#ifndef TW_H
#define TW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tw_graph tw_graph;

typedef enum {
    TW_OK = 0,
    TW_EINVAL = 1,  /* bad argument; nothing was changed or enqueued */
    TW_ENOMEM = 2,  /* device allocation failed; graph left unchanged */
    TW_EDEVICE = 3, /* a HIP runtime call failed */
    TW_ERANGE = 4,  /* a node id outside [0, num_nodes) */
    TW_ETIMEOUT = 5 /* tw_server_wait: the request has not finished yet */
} tw_status;

/* Pickers, Sec. "Temporal Bias Sampling".
 *  TW_UNIFORM:     Eq. (1) over the candidate edges.
 *  TW_LINEAR:      Eq. (2) over the candidate distinct-timestamp groups
 *                  (P(i) proportional to i+1, later groups heavier), then a
 *                  uniform edge inside the group (ties broken uniformly,
 *                  Sec. "Design Constraints").
 *  TW_EXPONENTIAL: Eq. (3) read as the exact inverse CDF of
 *                  P(i) ~ exp(lambda i) over the n candidate groups, with
 *                  lambda = (t_last - t_first) / ((n - 1) tau) when tau > 0
 *                  and lambda = 1 when tau <= 0; then a uniform edge in the
 *                  group.
 *  TW_NODE2VEC:    rejection on the TW_EXPONENTIAL proposal: a candidate w
 *                  is accepted when U * max(1/p, 1, 1/q) < beta, beta = 1/p
 *                  if w is the previous node, 1 if the window holds an edge
 *                  previous -> w, else 1/q. At most 4096 trials per hop; a
 *                  walk that exhausts them ends there. Hop bias only.
 *  TW_WEIGHT:      the weight-based exponential picker, the paper's default
 *                  sampler: every candidate edge weighs exp((t - t_min) /
 *                  tau) (tau <= 0: 1), and one draw u selects the first edge
 *                  whose cumulative weight reaches u times the total. The
 *                  per-node cumulative weights are built on the first walk
 *                  call after the window changes (or tau changes) and kept;
 *                  one launch of tw_sample_walks_batch (or of the server)
 *                  uses one tau for all its TW_WEIGHT biases. Hop bias
 *                  only; forward only. */
typedef enum {
    TW_UNIFORM = 0,
    TW_LINEAR = 1,
    TW_EXPONENTIAL = 2,
    TW_NODE2VEC = 3,
    TW_WEIGHT = 4
} tw_bias_kind;

/* TW_FORWARD: each hop takes an out-edge of the current node strictly after
 * the current time (Gamma_t(v), Sec. "Design Constraints").
 * TW_BACKWARD: each hop takes an in-edge (u, v, t') of the current node v
 * with t' strictly before the current time t (the backward case the paper
 * defines by analogy) and moves to u. The candidates are listed from the
 * latest to the earliest, in reverse canonical order, and every pick index
 * over n of them (edge, group, edge inside a group; the start edge or group
 * of the window) is mirrored to n - 1 - i; without equal timestamps this is
 * the forward walk on the graph with reversed edges and negated timestamps.
 * Start edge (u, v, t) of the window: the walk starts at v, then u at t.
 * A directed graph keeps an in-view (a second index fed every batch with
 * source and destination swapped) from its first backward walk on, which
 * doubles the cost of later ingests; an undirected graph is its own in-view.
 * Backward walks run on the full-walk dispatch (AUTO or FULL_WALK) or the work
 * queue (QUEUE), in tw_sample_walks and tw_sample_walks_batch, and in the
 * server (tw_server_submit); TW_WEIGHT is forward only. */
typedef enum { TW_FORWARD = 0, TW_BACKWARD = 1 } tw_direction;

/* TW_START_EDGE: the first edge is drawn from the whole window (timestamp
 * view) under start_bias. TW_START_NODE: walk i starts at d_start_nodes[i]
 * and its first edge is drawn from that node's whole run under start_bias. */
typedef enum { TW_START_EDGE = 0, TW_START_NODE = 1 } tw_start_mode;

/* Where each hop runs (Sec. "Hierarchical Cooperative Scheduling"). The
 * result never depends on it: the RNG is keyed by (seed, walk, hop, trial).
 *  TW_DISPATCH_FULL_WALK: one thread carries a walk through all its hops.
 *  TW_DISPATCH_COOP: per-step regrouping of live walks by current node and
 *    dispatch to a thread, a wavefront or a workgroup per node.
 *  TW_DISPATCH_QUEUE: one persistent launch; each lane of a wavefront runs
 *    one walk at a time and takes the next walk id from a device work queue
 *    when its walk ends, so lanes stay busy when walks end at different hops.
 *  TW_DISPATCH_AUTO: the library's choice (tw_autotune can set it). */
typedef enum {
    TW_DISPATCH_AUTO = 0,
    TW_DISPATCH_FULL_WALK = 1,
    TW_DISPATCH_COOP = 2,
    TW_DISPATCH_QUEUE = 3
} tw_dispatch;

/* Most hop biases one batched launch can mix. */
#define TW_MAX_BIASES 8

typedef struct {
    int32_t kind; /* tw_bias_kind */
    double tau;   /* exponential decay scale in timestamp units */
    double p, q;  /* node2vec return / in-out parameters, > 0 */
} tw_bias;

typedef struct {
    int32_t num_nodes; /* node ids are in [0, num_nodes), num_nodes >= 1 */
    int32_t directed;  /* 0: every edge (u,v,t) is stored as (u,v,t), (v,u,t) */
    int64_t window;    /* Delta > 0: keep t_now - Delta <= t_e; <= 0: no window */
    void* hip_stream;  /* hipStream_t; NULL is the default stream */
} tw_config;

typedef struct {
    int64_t num_walks;           /* >= 0 */
    int32_t max_len;             /* nodes per walk, >= 1 */
    tw_bias hop_bias;            /* any tw_bias_kind */
    tw_bias start_bias;          /* TW_UNIFORM, TW_LINEAR or TW_EXPONENTIAL */
    int32_t start_mode;          /* tw_start_mode */
    const int32_t* d_start_nodes;/* TW_START_NODE: num_walks ids; else ignored */
    uint64_t seed;               /* RNG key */
    uint64_t walk_id_base;       /* walk i uses RNG id walk_id_base + i */
    int32_t dispatch;            /* tw_dispatch */
    int32_t direction;           /* tw_direction (0: forward) */
} tw_walk_params;

/*
 * A batch of walks of uneven lengths and mixed hop biases, run as one
 * persistent launch with a device work queue (TW_DISPATCH_QUEUE). Walk i has
 * RNG id walk_id_base + i, length limit d_max_len[i] (or max_len), hop bias
 * hop_biases[d_bias[i]] (or hop_biases[(walk_id_base + i) mod num_biases]),
 * and writes its nodes and timestamps at d_row[i] (or i * max_len). A walk's
 * result is the one tw_sample_walks gives it with the same seed, id, start
 * and bias, cut to its length limit (the RNG is keyed by walk, hop and
 * trial, so a shorter limit only truncates).
 */
typedef struct {
    int64_t num_walks;           /* >= 0 */
    int32_t max_len;             /* row width when d_row is NULL; >= every limit, >= 1 */
    const int32_t* d_max_len;    /* num_walks limits in [1, max_len], or NULL */
    int32_t num_biases;          /* 1..TW_MAX_BIASES */
    tw_bias hop_biases[TW_MAX_BIASES];
    const uint8_t* d_bias;       /* num_walks indices < num_biases, or NULL */
    tw_bias start_bias;          /* TW_UNIFORM, TW_LINEAR or TW_EXPONENTIAL */
    int32_t start_mode;          /* tw_start_mode */
    const int32_t* d_start_nodes;/* TW_START_NODE: num_walks ids; else ignored */
    uint64_t seed;
    uint64_t walk_id_base;
    const int64_t* d_row;        /* num_walks row starts (see tw_row_offsets), or NULL */
    int64_t out_slots;           /* slots of d_nodes and d_ts, padded by the call;
                                    0 with d_row NULL: num_walks * max_len */
    int32_t dispatch;            /* TW_DISPATCH_QUEUE (AUTO means it), or
                                    TW_DISPATCH_FULL_WALK: one thread per walk, no
                                    queue (the plain form, for comparison) */
    int32_t direction;           /* tw_direction (0: forward); backward walks take
                                    no TW_WEIGHT bias */
} tw_batch_params;

typedef struct {
    int64_t accepted;     /* records merged by the last ingest (after mirroring) */
    int64_t dropped_late; /* records of the last ingest older than t_now - Delta */
    int64_t evicted;      /* records evicted by the last ingest / evict call */
    int64_t active_edges; /* records in the window now */
    int64_t t_min, t_max; /* timestamp range of the window (0, 0 when empty) */
} tw_ingest_info;

/* Create an empty graph. Allocates nothing on the device until the first
 * ingest. Returns TW_EINVAL for num_nodes < 1 or a null out. */
tw_status tw_create(const tw_config* cfg, tw_graph** out);

/* Synchronise the graph's stream and free everything the graph owns. */
tw_status tw_destroy(tw_graph* g);

/* Use another stream for all later calls. */
tw_status tw_set_stream(tw_graph* g, void* hip_stream);

/*
 * Ingest one batch of n edges (Sec. "Streaming Ingestion and Window
 * Management"): mirror (undirected graphs), advance t_now to the largest
 * timestamp seen, drop batch records older than t_now - Delta, evict window
 * records older than t_now - Delta, sort the batch by timestamp (stable) and
 * merge it after the window's records of equal timestamp, then update both
 * views of the dual index (Sec. "Dual-Index Organization"): the timestamp
 * view in place, and the node-and-timestamp view for the nodes the batch or
 * the eviction touches.
 * d_src, d_dst: int32[n]; d_ts: int64[n]; device memory, any alignment.
 * info (nullable) receives the counts and the window's timestamp range;
 * with info NULL the range is computed on the device and read back with the
 * next read-back the library makes anyway (one synchronisation fewer). The
 * call synchronises the stream (it sizes its launches from counts it reads
 * back: two read-backs, three with info); the first read-back also brings
 * the error flags of earlier walks: a pending one is reported (TW_ERANGE,
 * TW_EINVAL, see tw_sample_walks) and cleared, and the batch is not
 * ingested.
 * Returns TW_ERANGE, with the graph unchanged, if any id is outside
 * [0, num_nodes). The batch is staged, validated, sorted and its node-view
 * jobs collected before the index changes: TW_ENOMEM (device full) in that
 * part leaves the graph unchanged. A failure while the index is being
 * updated (device full while a pool or buffer grows, a HIP error) leaves it
 * partly updated: the call returns TW_ENOMEM or TW_EDEVICE and every later
 * call that reads or changes the index returns TW_EDEVICE (destroy the
 * graph). A backward in-view
 * (tw_direction) that fails to take the batch is dropped and rebuilt from
 * the window by the next backward walk.
 */
tw_status tw_ingest_batch(tw_graph* g, const int32_t* d_src, const int32_t* d_dst,
                          const int64_t* d_ts, int64_t n, tw_ingest_info* info);

/*
 * Remove every window record with timestamp < t_cutoff from both views and
 * rebuild the offsets (Sec. "Dual-Index Organization": eviction is a prefix
 * of the timestamp view). Idempotent. Does not move t_now.
 * n_evicted (nullable) receives the count. With nothing to evict (an empty
 * window, or t_cutoff <= its first timestamp) the call returns at once: no
 * device work, no synchronisation. Otherwise it synchronises the stream and
 * first reports a pending device-side error of earlier walks.
 */
tw_status tw_evict_before(tw_graph* g, int64_t t_cutoff, int64_t* n_evicted);

/*
 * Build the TW_WEIGHT picker's cumulative weights for time scale tau at
 * every later ingest and eviction (the weight stage of the paper's ingest,
 * Table 4), so the first weight-based walk after an update does not build
 * them; tau NaN: stop (the first weight-based walk after an update builds
 * them, the default). The weights also serve walks at another tau only after
 * a rebuild, which such a walk makes itself. A build that fails at ingest
 * leaves the weights to the next weight-based walk. Host-side setting, no
 * synchronisation. Returns TW_EINVAL for a null graph or an infinite tau.
 */
tw_status tw_set_ingest_weights(tw_graph* g, double tau);

/*
 * Sample params->num_walks walks (Sec. "Temporal Bias Sampling", "Hierarchical
 * Cooperative Scheduling"). Outputs are walk-major, caller-owned device
 * arrays:
 *   d_nodes: int32[num_walks * max_len], row i = walk i's nodes, padded -1;
 *   d_ts:    int64[num_walks * max_len], d_ts[i*max_len + j] = timestamp of
 *            the edge into node j; position 0 and padding hold INT64_MIN;
 *   d_len:   int32[num_walks], nodes in walk i (0 only for an empty window in
 *            TW_START_EDGE mode or a start node out of range).
 * Each hop keeps the timestamp strictly increasing (Gamma_t(v) holds edges
 * with t' > t). Asynchronous: returns after enqueue. A start node outside
 * [0, num_nodes) gives that walk length 0 and makes the next synchronising
 * call (tw_stats, tw_ingest_batch, tw_evict_before, tw_sync) return
 * TW_ERANGE. Returns TW_EINVAL for bad parameters (nothing enqueued).
 */
tw_status tw_sample_walks(tw_graph* g, const tw_walk_params* params, int32_t* d_nodes,
                          int64_t* d_ts, int32_t* d_len);

/*
 * Counts of the last ingest_batch or evict_before, host-side, no
 * synchronisation: out[0] records accepted, out[1] dropped as late, out[2]
 * evicted, out[3] records in the window now. TW_EINVAL for null arguments.
 */
tw_status tw_last_update(const tw_graph* g, int64_t out[4]);

/*
 * Where the graph's device buffers lie, as one value, with whether the
 * node2vec pair table and the weight-based picker's weights are current. A
 * walk launch (tw_sample_walks with the full-walk or queue dispatch,
 * tw_sample_walks_batch, tw_sample_walks_noalloc) recorded in a HIP graph
 * reads the window from device-side state that every update keeps current:
 * replayed after later tw_ingest_batch / tw_evict_before calls it gives the
 * walks an eager call would give, while this value equals the one read when
 * the launch was recorded. When it differs (a buffer grew or moved, the
 * window moved, the pair table or the weights were dropped), record the
 * launch again after an eager call. Host-side, no synchronisation. TW_EINVAL
 * for null arguments.
 */
tw_status tw_walk_layout(const tw_graph* g, uint64_t* out);

/*
 * Counters of the last index update (ingest_batch or evict_before), for
 * measurement: out[0] nodes whose run in the node-and-timestamp view changed
 * (appended, evicted or rewritten), out[1] node-view edges written, out[2]
 * edge slots of the node segments allocated, out[3] 1 when every active
 * node was rewritten into fresh pools (a compaction), out[4], out[5], out[6]
 * edge, group and fence pool slots handed out (live data, slack and the
 * segments of moved nodes), out[7] edge pool capacity in slots. Host-side
 * values, no synchronisation. Returns TW_EINVAL for null arguments.
 */
tw_status tw_index_stats(const tw_graph* g, int64_t out[8]);

/*
 * Walks of a tw_batch_params batch in one persistent launch (see there).
 * d_nodes: int32[out_slots], d_ts: int64[out_slots]; every slot is first set
 * to -1 / INT64_MIN, then each walk writes its nodes and timestamps from its
 * row start (position 0 of d_ts stays INT64_MIN). Rows must not overlap and
 * must fit in out_slots (the caller's layout; tw_row_offsets gives a packed
 * one). d_len: int32[num_walks] lengths. Stream-ordered, no synchronisation;
 * a limit outside [1, max_len], a bias index >= num_biases, or a row that
 * starts below 0 or ends past out_slots gives that walk length 0 (nothing
 * written) and makes the next synchronising call return TW_EINVAL. Returns TW_EINVAL for bad parameters (nothing enqueued).
 */
tw_status tw_sample_walks_batch(tw_graph* g, const tw_batch_params* params, int32_t* d_nodes,
                                int64_t* d_ts, int32_t* d_len);

/*
 * Row starts for ragged walk output: d_row[i] = sum of d_max_len[0..i), with
 * d_row[n] = the total, also returned in *total (host). d_row: int64[n + 1].
 * Synchronises. Returns TW_EINVAL for null arguments or a negative n.
 */
tw_status tw_row_offsets(tw_graph* g, const int32_t* d_max_len, int64_t n, int64_t* d_row,
                         int64_t* total);

/*
 * How TW_DISPATCH_AUTO and the cooperative dispatch run (Sec.
 * "Hierarchical Cooperative Scheduling", Sec. "Parameter Tuning"):
 *  dispatch:      what TW_DISPATCH_AUTO runs (FULL_WALK, COOP or QUEUE)
 *  queue_bpc:     queue workgroups per compute unit (0: as many as fit)
 *  coop_regroup:  per step, 0 = stable sort of the live walks by node, 1 = none
 *                 (in-order compaction only)
 *  coop_wave_min: lanes of a wavefront at its first lane's node that make it
 *                 read the node record once and stage the top of the node's
 *                 fence in LDS (the wavefront tier, 1..64); a workgroup whose
 *                 four wavefronts do so for one node stages a panel of
 *                 coop_panel words (the workgroup tier)
 *  coop_panel:    LDS fence words of a workgroup (64..8192, multiple of 64)
 *  coop_sync:     steps between read-backs of the live count (1..64); launches
 *                 in between cover the last count read
 * Defaults: FULL_WALK, 0, 0, 64, 4096, 1. The result of a walk never depends
 * on them.
 */
typedef struct {
    int32_t dispatch, queue_bpc, coop_regroup, coop_wave_min, coop_panel, coop_sync;
} tw_tuning;

/* Read the graph's tuning. Host-side. TW_EINVAL for null arguments. */
tw_status tw_get_tuning(const tw_graph* g, tw_tuning* out);

/* Set it (AUTO is not a valid dispatch here). TW_EINVAL for values outside
 * the ranges above. Host-side. */
tw_status tw_set_tuning(tw_graph* g, const tw_tuning* t);

/*
 * Time the dispatches of tw_sample_walks on the current window for these
 * parameters, with num_walks cut to at most sample_walks: full-walk, the
 * queue at 3 launch shapes, and the cooperative dispatch over its tunables
 * (sorted regroup: wave_min 64 or 16, panel 2048 or 8192 words, read-back
 * every step or every 4; no regroup, read-back every step or every 4), and
 * keep the fastest as the graph's tuning (tw_get_tuning reads it).
 * d_nodes / d_ts / d_len: scratch of the sizes tw_sample_walks needs for the
 * timed walk count. best (nullable) receives the chosen tw_dispatch and, for
 * the queue, its workgroups per compute unit in best[1]. Synchronises.
 */
tw_status tw_autotune(tw_graph* g, const tw_walk_params* params, int64_t sample_walks,
                      int32_t* d_nodes, int64_t* d_ts, int32_t* d_len, int32_t best[2]);

/* ------------------------------------------------------------------------
 * Allocation-free walks, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.
 */

/* Most walks one tw_sample_walks_noalloc call takes. */
#define TW_NOALLOC_MAX_WALKS 262144

/*
 * The walks of tw_sample_walks with TW_DISPATCH_QUEUE (the same results),
 * with no device allocation, free or memset: the call's lists (live walks
 * and their previous nodes, alive flags and their scan, the work-queue
 * counters; 44 bytes a walk, 11.5 MB in all) live in one array that the
 * library holds on every device it runs on until the process ends, set up by
 * tw_create. Every clearing is a kernel, so the call can be captured in a
 * HIP graph. Arguments and outputs as tw_sample_walks; params->dispatch is
 * ignored. Stream-ordered, no synchronisation.
 * All calls on one device share the array and each call's kernels consume
 * what its own earlier kernels wrote there: calls that overlap on one device
 * (other streams, other host threads, replays of captured graphs running
 * concurrently) race and give wrong walks. Serialise them.
 * Returns TW_EINVAL, nothing enqueued, for num_walks > TW_NOALLOC_MAX_WALKS,
 * backward walks, a TW_WEIGHT hop bias (its weights are built lazily), a
 * graph that has not ingested yet, a TW_NODE2VEC hop bias while the node2vec
 * adjacency of the current window is not built (one tw_sample_walks call
 * with a node2vec bias after the last ingest or eviction builds it), and for
 * every bad parameter tw_sample_walks rejects.
 */
tw_status tw_sample_walks_noalloc(tw_graph* g, const tw_walk_params* params, int32_t* d_nodes,
                                  int64_t* d_ts, int32_t* d_len);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of walk requests interleaved with ingestion.
 *
 * A server owns a graph (the caller must not use the graph directly while
 * the server exists), a worker thread and an ingest thread with a stream of
 * its own. Requests (tw_walk_params, dispatch ignored) and ingest batches
 * are queued in submission order. The worker packs consecutive requests
 * into one work-queue launch on the graph's stream (up to
 * max_walks_per_launch walks, 1024 requests) as soon as their outputs are
 * placed, without waiting for the launch before it (up to max_inflight
 * launches enqueued). A batch that reaches the front is planned (staged,
 * validated, sorted, its node-view jobs collected) on the ingest stream
 * while the launches before it still run, and the index is changed after
 * they finish; the launches after it wait for that update. Every request
 * sees exactly the ingest batches submitted before it (its index epoch), and
 * its walks are the ones tw_sample_walks gives on that window with the same
 * parameters: requests sharing a launch do not change each other's result.
 * Outputs are placed in the output arena; when a request fits none of its
 * chunks, a chunk is added while the device keeps hbm_reserve_bytes free
 * (admission by free device memory), else the request waits for releases.
 * Functions may be called from any host thread.
 */
typedef struct tw_server tw_server;

typedef struct {
    int64_t arena_bytes;          /* device memory for request outputs, allocated at create;
                                     also the least size of a chunk added later */
    int64_t max_walks_per_launch; /* walks of one launch (a larger request runs alone) */
    int32_t max_inflight;         /* launches enqueued at once, 1..8 */
    int64_t hbm_reserve_bytes;    /* admission by free device memory: when a request's
                                     outputs fit no arena chunk, a chunk is added if
                                     hipMemGetInfo shows this much free after it (room
                                     for the index to grow); < 0: the arena stays fixed */
} tw_server_config;

typedef struct {
    tw_status status;     /* of the request (or ingest batch) */
    int32_t* d_nodes;     /* num_walks x max_len, server memory valid until release */
    int64_t* d_ts;        /* num_walks x max_len */
    int32_t* d_len;       /* num_walks */
    int64_t num_walks;
    int32_t max_len;
    double queue_ms;      /* submission to launch */
    double latency_ms;    /* submission to completion seen by the worker */
    tw_ingest_info ingest;/* ingest batches: the counts of that ingest */
    int64_t trial_cap_hits; /* walks of the request that node2vec's trial cap ended */
} tw_request_result;

typedef struct {
    int64_t requests_done, walks_done, hops_done, launches, ingests;
    double p50_ms, p99_ms, max_ms, mean_ms; /* request latency, submission to completion */
    double wall_s;        /* seconds since create */
    int64_t arena_bytes;  /* output memory held now (every chunk) */
    int64_t arena_chunks_added; /* chunks added after create (admission by free memory) */
} tw_server_counters;

/* Start a server on g. Allocates the arena and the launch tables (TW_ENOMEM
 * if that fails). Returns TW_EINVAL for bad arguments. */
tw_status tw_server_create(tw_graph* g, const tw_server_config* cfg, tw_server** out);

/* Queue a walk request; *id names it. d_start_nodes (NODE mode) must stay
 * valid until the request finishes. Any hop bias and either direction
 * (TW_WEIGHT forward only); a launch holds requests of one direction, and
 * its TW_WEIGHT requests share one tau (a request that differs starts the
 * next launch). The first backward request builds the graph's in-view from
 * the window. Returns TW_EINVAL for bad parameters or a request whose
 * outputs can never fit in a fixed arena (hbm_reserve_bytes < 0). */
tw_status tw_server_submit(tw_server* s, const tw_walk_params* req, uint64_t* id);

/* Queue an ingest batch (as tw_ingest_batch). The arrays must already hold
 * the batch on the device when it is submitted (the ingest stream reads them
 * without ordering against the caller's streams) and stay valid until it
 * finishes. *id names it. */
tw_status tw_server_ingest(tw_server* s, const int32_t* d_src, const int32_t* d_dst,
                           const int64_t* d_ts, int64_t n, uint64_t* id);

/* Wait up to timeout_us (< 0: no limit) for request or batch id. TW_OK with
 * *out filled when it has finished (out->status is its own status),
 * TW_ETIMEOUT if it has not, TW_EINVAL for an unknown or released id. */
tw_status tw_server_wait(tw_server* s, uint64_t id, int64_t timeout_us, tw_request_result* out);

/* Return a finished request's output memory to the arena; the id is then
 * unknown. TW_EINVAL if it has not finished or is unknown. */
tw_status tw_server_release(tw_server* s, uint64_t id);

/* Copy finished request id's outputs into caller device memory: d_nodes
 * and d_ts num_walks x max_len, d_len num_walks (any pointer may be NULL).
 * Synchronous. TW_EINVAL if the request is unknown or has not finished. */
tw_status tw_server_copy_out(tw_server* s, uint64_t id, int32_t* d_nodes, int64_t* d_ts,
                             int32_t* d_len);

/* Counters and request-latency percentiles since create. */
tw_status tw_server_stats(tw_server* s, tw_server_counters* out);

/* Finish the queued work, stop the worker and free the server's memory
 * (outputs not yet released are freed too). The graph stays valid. */
tw_status tw_server_destroy(tw_server* s);

/* Synchronise the stream and report a pending device-side range error. */
tw_status tw_sync(tw_graph* g);

/* Window counts and timestamp range (active_edges, t_min, t_max; the
 * per-call fields repeat the last ingest / evict). Synchronises. */
tw_status tw_stats(tw_graph* g, tw_ingest_info* info);

/*
 * Sizes of the index: out[0] active edges m, out[1] distinct timestamps Gg,
 * out[2] distinct (node, timestamp) pairs Gn, out[3] num_nodes. Synchronises.
 */
tw_status tw_view_sizes(tw_graph* g, int64_t out[4]);

/*
 * Copy the index into caller device buffers (any pointer may be null), for
 * inspection and tests. Sizes as returned by tw_view_sizes:
 *   src, dst: int32[m], ts: int64[m]          timestamp view (the edge store)
 *   g_ts: int64[Gg], g_off: int64[Gg+1]       its timestamp-group offsets
 *   n_dst: int32[m], n_ts: int64[m]           node-and-timestamp view
 *   n_gts: int64[Gn], n_goff: int64[Gn+1]     its (node, timestamp) groups
 *   n_ebeg, n_gbeg: int64[V+1]                first edge / group of node v
 * Synchronises.
 */
tw_status tw_export_views(tw_graph* g, int32_t* src, int32_t* dst, int64_t* ts, int64_t* g_ts,
                          int64_t* g_off, int32_t* n_dst, int64_t* n_ts, int64_t* n_gts,
                          int64_t* n_goff, int64_t* n_ebeg, int64_t* n_gbeg);

/* Device bytes the graph holds now. */
int64_t tw_device_bytes(const tw_graph* g);

/* Message for the last non-OK status returned on this host thread. */
const char* tw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TW_H */
