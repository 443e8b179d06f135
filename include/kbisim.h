/*
 * kbisim.h -- C ABI of the MI355X (gfx950) k-bisimulation library.
 *
 * The library computes the k-bisimulation partition of a node- and
 * edge-labelled directed graph (Definition 1 of the paper "External memory
 * bisimulation reduction of big graphs", Section 2.1) by the signature
 * method of its construction algorithm (Algorithm 1, Build_Bisim, Section 3):
 * round i joins every edge (src, label, dst) with pId_{i-1}(dst), forms each
 * node's signature from pId_{i-1}(node) and the set of (label, pId_{i-1}(dst))
 * pairs (Definition 3, with the previous id as head -- Kaushik's equivalent
 * definition, Appendix), and maps distinct signatures to new ids
 * (S.insert, Section 2.2). All rounds run as HIP kernels on one GPU with the
 * graph resident in device memory.
 *
 * Canonical ids. pId_i(u) is the 0-based rank of u's signature among the
 * distinct signatures of round i, in lexicographic order of the int sequence
 * [pId_{i-1}(u), l1, p1, l2, p2, ...] with the pairs ascending and a proper
 * prefix ordered first; pId_0(u) is the rank of u's label among the distinct
 * node labels (Section 3.1, "k = 0"). Labels are compared as integers. The
 * ids of round i are therefore dense in [0, B_i) and fully determined by the
 * graph (the paper leaves the numbering free, Section 3.2).
 *
 * Early stop. With early stop on (default) the round loop ends after the
 * first round i with B_i == B_{i-1} (Section 3.2, "Early stopping
 * condition"); its ids equal those of every later round.
 *
 * Errors. Every call returns a kbisim_status; 0 is success. On error the
 * out-parameters are left untouched and a handle stays usable;
 * kbisim_last_error() gives a message for the calling thread. A handle is not
 * thread-safe; distinct handles may be used from distinct threads.
 *
 * Limits: 0 <= N < 2^31, 0 <= E < 2^32 - 1, labels int32 >= 0.
 */
#ifndef KBISIM_H
#define KBISIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KBISIM_OK = 0,
  KBISIM_EINVAL = -1,    /* invalid argument or input graph */
  KBISIM_ENOMEM = -2,    /* device or host allocation failed, or over budget */
  KBISIM_EDEVICE = -3,   /* a HIP call failed */
  KBISIM_ESTATE = -4,    /* call not valid in the current state */
  KBISIM_EBUSY = -5,     /* server: no capacity right now */
  KBISIM_ECANCELED = -6, /* server: request was cancelled */
  KBISIM_ETIMEDOUT = -7  /* server: wait timed out */
} kbisim_status;

typedef enum { KBISIM_MEM_HOST = 0, KBISIM_MEM_DEVICE = 1 } kbisim_mem;

typedef struct kbisim_graph kbisim_graph;

/* A graph as N node labels and E labelled edges (src, label, dst). The four
 * arrays live in host or device memory (`mem`); they are read during
 * kbisim_create only. Edges form a multiset: duplicates are allowed and
 * ignored (signatures are sets), self-loops are allowed. */
typedef struct {
  int64_t num_nodes;          /* N >= 0 */
  int64_t num_edges;          /* E >= 0 */
  const int32_t* node_label;  /* [N], values >= 0 */
  const int32_t* edge_src;    /* [E], values in [0, N) */
  const int32_t* edge_label;  /* [E], values >= 0 */
  const int32_t* edge_dst;    /* [E], values in [0, N) */
  kbisim_mem mem;             /* where the four arrays live */
  void* stream;               /* hipStream_t for all work of this handle; NULL = default stream */
} kbisim_graph_desc;

typedef struct {
  int32_t early_stop; /* 1 (default): stop at the first round with B_i == B_{i-1} */
  int32_t profile;    /* 1: time each kernel class with HIP events (kbisim_profile) and
                         count the work of the signature kernels (kbisim_work) */
  int32_t medium_cap; /* tuning: groups of 65..medium_cap members are ordered by one
                         workgroup in LDS, larger ones by global radix passes; 0..4096,
                         values <= 64 send every group above 64 members to the global
                         passes; 0 = library default (4096). Ids do not depend on it. */
  int32_t history;    /* 1: keep the partition of every computed round (the node table
                         with pId_0..pId_k of Section 4, Table 3) and the maintenance
                         state (edges also by target, the label values), about
                         8 B per node per round plus the edge table again; needed by
                         kbisim_result_round for earlier rounds and by kbisim_update.
                         0 (default): only the last round. */
  int32_t update_mode; /* how kbisim_update brings the stored rounds up to date after
                          the graph changed: 0 (default) per round by cost, level by
                          level (Algorithm 3) while that is cheaper than a full round,
                          then full rounds (Section 4, "When to switch back"); 1 level
                          by level in every round; 2 full rounds from round 1. The
                          result does not depend on it. */
  int32_t radix_tile;  /* tuning: items per tile of every radix sort pass of this handle
                          (the edge table's sort by source at create, the ordering's
                          device-wide passes, the maintenance sorts): 2048, 3072 or 4096;
                          0 = library default (3072). Ids do not depend on it. */
  int64_t edge_window_bytes; /* 0 (default): kbisim_create copies the edge table into device
                          memory. > 0: graphs whose edge table is to stay out of device
                          memory (the paper's setting of a graph larger than the fast
                          memory, Section 2.2): the table, given in host memory
                          (KBISIM_MEM_HOST), is read in chunks and kept as CSR edge words
                          in pinned host memory, cut into partitions of consecutive source
                          nodes; every round moves the partitions through two device
                          windows of at most edge_window_bytes / 2 each (copies overlap the
                          signature launch of the previous partition), or, in rounds with
                          few active nodes, reads their rows in place. Device memory then
                          holds per edge only the round's signature keys. Needs a window
                          of at least twice the longest row's edge words (4 bytes, or 8
                          when label rank and target id need more than 32 bits), edge
                          labels below 2^24 and history = 0; kbisim_create only.
                          Results are the same as without it. */
} kbisim_options;

/* Fills *opt with the defaults above. */
void kbisim_options_default(kbisim_options* opt);

/* Copies the graph into library-owned device memory, builds the CSR edge
 * table and computes pId_0 on desc->stream. The caller's arrays may be freed
 * once this returns (device arrays: once the stream has reached this point).
 * opt may be NULL. On success *out receives a new handle. */
kbisim_status kbisim_create(const kbisim_graph_desc* desc, const kbisim_options* opt,
                            kbisim_graph** out);

/* Runs refinement rounds until round k has been computed or the fixed point
 * is reached (early stop). Resumable: a later call with a larger k continues
 * from the last round; k at or below the rounds already done does nothing.
 * *rounds_done (may be NULL) receives the number of rounds executed so far.
 * k < 0 is KBISIM_EINVAL. Synchronises the handle's stream. */
kbisim_status kbisim_refine(kbisim_graph* g, int32_t k, int32_t* rounds_done);

/* For callers that cannot allocate device memory (code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * kbisim_create + kbisim_refine(k) + kbisim_result + kbisim_destroy in one
 * call that calls no hipMalloc, hipFree or allocating library routine. Every
 * intermediate buffer is carved from a static device region of
 * KBISIM_STATIC_SCRATCH_BYTES bytes (one per GPU, held until the process
 * ends; it keeps the last call's contents, which no call relies on). Work
 * runs on desc->stream only; the call returns after it has finished. Calls
 * on one GPU are serialised by the library (they share the region).
 * Inputs as for kbisim_create (host or device); pid_out[N] in out_mem;
 * num_blocks and rounds_done may be NULL. Graphs whose estimated footprint
 * (48 B per edge + 256 B per node + 1 MiB) exceeds the region are rejected
 * with KBISIM_ENOMEM before any work; the region running out anyway is
 * KBISIM_ENOMEM too. opt's profile and history fields are ignored. */
#define KBISIM_STATIC_SCRATCH_BYTES (128u << 20)
kbisim_status kbisim_refine_static(const kbisim_graph_desc* desc, int32_t k, const kbisim_options* opt,
                                   int32_t* pid_out, kbisim_mem out_mem, int64_t* num_blocks,
                                   int32_t* rounds_done);

/* Writes the ids of the last computed round (pId_k) to pid_out[N] in host or
 * device memory (device: enqueued on the handle's stream, then synchronised),
 * *num_blocks = B of that round, and counts[0..min(counts_cap, rounds+1)) =
 * B_0, B_1, ... . Any pointer may be NULL to skip that output. */
kbisim_status kbisim_result(const kbisim_graph* g, int32_t* pid_out, kbisim_mem mem,
                            int64_t* num_blocks, int64_t* counts, int32_t counts_cap);

/* Change of k (Section 4, "Change k"): the ids of round j (pId_j, canonical
 * as above) and B_j, for j <= rounds done, read from the stored history
 * without recomputing anything (a larger k is kbisim_refine). Rounds past an
 * early stop equal the last round. Earlier rounds need options.history = 1
 * (else KBISIM_ESTATE); a round not computed yet is KBISIM_ESTATE. pid_out
 * [N] in host or device memory (device: on the handle's stream, then
 * synchronised); either pointer may be NULL. */
kbisim_status kbisim_result_round(const kbisim_graph* g, int32_t round, int32_t* pid_out, kbisim_mem mem,
                                  int64_t* num_blocks);

/* One change to the graph of a handle (Section 4, maintenance), applied in
 * this order: new isolated nodes appended (Algorithm 2, Add_Nodes; ids N,
 * N+1, ...), then deletions of edge triples (every copy of each triple goes;
 * triples not in the graph are ignored), then deletions of nodes (Section 4,
 * "Deletions": with all their incoming and outgoing edges; the remaining
 * nodes keep their order and are renumbered 0, 1, ...; ids refer to the
 * numbering after the new nodes, duplicates allowed), then additions of edge
 * triples (Algorithm 3, Add_Edges; endpoints in the numbering after the node
 * deletions, may be new nodes). All arrays are in `mem` and read during the
 * call. */
typedef struct {
  int64_t num_new_nodes;          /* >= 0 */
  const int32_t* new_node_label;  /* [num_new_nodes], values >= 0 */
  int64_t num_del_edges;          /* >= 0 */
  const int32_t* del_src;         /* [num_del_edges] each */
  const int32_t* del_label;
  const int32_t* del_dst;
  int64_t num_del_nodes;          /* >= 0 */
  const int32_t* del_nodes;       /* [num_del_nodes] */
  int64_t num_add_edges;          /* >= 0 */
  const int32_t* add_src;         /* [num_add_edges] each */
  const int32_t* add_label;
  const int32_t* add_dst;
  kbisim_mem mem;
} kbisim_update_desc;

/* Applies the update and brings every stored round up to date (Algorithm 3's
 * level-by-level propagation: per round, the sources of changed edges, the
 * nodes whose class changed in the round below and their sources are
 * re-checked; classes holding none of them keep their stored split). When
 * the update moves the fixed point, rounds continue up to the largest k
 * given to kbisim_refine (or stop earlier at the new fixed point). From a
 * round whose frontier outgrows a full round, the remaining rounds run in
 * full (Section 4, "When to switch back"). Afterwards
 * the handle holds exactly what kbisim_create on the updated graph followed
 * by kbisim_refine(k) gives: every round's ids, counts and rounds done.
 * Needs options.history = 1 (else KBISIM_ESTATE). Invalid input
 * (an endpoint outside [0, N + num_new_nodes), a negative label) is
 * KBISIM_EINVAL and leaves the handle unchanged. *rounds_done may be NULL. */
kbisim_status kbisim_update(kbisim_graph* g, const kbisim_update_desc* u, int32_t* rounds_done);

/* Streamed edge table (edge_window_bytes > 0): number of partitions, bytes of
   the edge table moved host -> device by the rounds so far, and rounds that
   read their active rows in place instead. All zero for other graphs. Any
   out-parameter may be NULL. */
kbisim_status kbisim_stream_stats(const kbisim_graph* g, int64_t* partitions, int64_t* bytes_moved,
                                  int32_t* direct_rounds);

/* Work of the last kbisim_update: rounds brought up to date level by level,
 * the first round recomputed in full instead (0 if none: when a round's
 * frontier and the classes it touches hold more nodes than a full round
 * re-orders, that round and the later ones run as in kbisim_refine, the
 * switch back to Algorithm 1 that Section 4 suggests), nodes re-checked (the
 * frontiers, summed over rounds), nodes whose signature was recomputed
 * (members of the re-ordered classes) and nodes found changed. Any pointer
 * may be NULL. */
kbisim_status kbisim_update_stats(const kbisim_graph* g, int64_t* levels, int64_t* full_from, int64_t* rechecked,
                                  int64_t* recomputed, int64_t* changed);

/* Kernel classes timed when options.profile = 1. */
typedef enum {
  KBISIM_PROF_SIGNATURE = 0, /* the signature launch of a round (all out-degree buckets) */
  KBISIM_PROF_ORDER = 1,     /* ordering signatures inside classes (all kernels) */
  KBISIM_PROF_ASSIGN = 2,    /* ids of the round and the next round's active set */
  KBISIM_PROF_ROUND = 3,     /* one whole round */
  KBISIM_PROF_COUNT = 4
} kbisim_prof_class;

/* Signature work buckets (kbisim_work), by out-degree. */
typedef enum {
  KBISIM_BUCKET_THREAD = 0, /* <= 16 edges: one thread per node */
  KBISIM_BUCKET_WAVE = 1,   /* <= 64 edges: one wave per node (two per wave when both <= 32) */
  KBISIM_BUCKET_BLOCK = 2,  /* <= 4096 edges: one wave (<= 512 edges, or key-set bitmaps) or
                               one workgroup per node */
  KBISIM_BUCKET_HUB = 3,    /* more edges: all hubs of a round in one device-wide sort (or
                               in chunks of one workgroup each with key-set bitmaps) */
  KBISIM_BUCKET_COUNT = 4
} kbisim_bucket;

/* Timings collected when options.profile = 1 with HIP events recorded on the
 * handle's stream around each launch of class c: ms[c] = summed milliseconds,
 * launches[c] = number of timed launches, since create or the last reset
 * (reset != 0 clears after reading). cap = entries of ms/launches. */
kbisim_status kbisim_profile(const kbisim_graph* g, double* ms, int64_t* launches, int32_t cap,
                             int32_t reset);

/* Work done by the signature launches when options.profile = 1, summed over
 * rounds: nodes_edges[2c] = nodes of bucket c (kbisim_bucket) and
 * nodes_edges[2c+1] = their out-edges. Only active nodes (members of classes
 * with two or more members) are processed and counted. cap = entries (8). */
kbisim_status kbisim_work(const kbisim_graph* g, int64_t* nodes_edges, int32_t cap, int32_t reset);

/* One refinement round as recorded when options.profile = 1. */
typedef struct {
  double signature_ms; /* the signature launch(es) of the round (HIP events) */
  double round_ms;     /* the whole round: signatures, ordering, id assignment */
  int64_t active_nodes; /* nodes whose signature the round computed */
  int64_t active_edges; /* their out-edges */
  int64_t max_keys;     /* longest signature: unique (label, id) pairs of one node */
} kbisim_round_stat;

/* Per-round profile when options.profile = 1 (round-by-round rates of the
 * signature launch, Algorithm 1's iterations): stats[r-1] for round r of the
 * rounds computed since create or the last reset; *n (may be NULL) receives
 * their number, of which min(*n, cap) are written. Counts of rounds past the
 * 64th accumulate in the 64th entry. reset != 0 clears after reading. */
kbisim_status kbisim_round_profile(const kbisim_graph* g, kbisim_round_stat* stats, int32_t cap, int32_t* n,
                                   int32_t reset);

/* Frees everything owned by the handle. NULL is ignored. */
void kbisim_destroy(kbisim_graph* g);

/* ---- Batched form ---------------------------------------------------------
 * Many independent graphs refined together: every kernel launch of a round
 * serves all of them (a union of the graphs whose node ids and labels are
 * kept apart per graph). Results are per graph and identical to refining
 * each graph alone with kbisim_create/kbisim_refine.
 *
 * The graphs are concatenated in one kbisim_graph_desc: graph g owns nodes
 * [node_off[g], node_off[g+1]) and edges [edge_off[g], edge_off[g+1]) of the
 * arrays; edge endpoints are LOCAL node ids of their graph (0 .. N_g - 1).
 * node_off and edge_off are host arrays of num_graphs + 1 entries starting at
 * 0; desc->num_nodes / num_edges must equal their last entries. */
typedef struct kbisim_batch kbisim_batch;

kbisim_status kbisim_batch_create(int32_t num_graphs, const int64_t* node_off, const int64_t* edge_off,
                                  const kbisim_graph_desc* concat, const kbisim_options* opt,
                                  kbisim_batch** out);

/* Refines graph g for up to k_per_graph[g] rounds (host array, each >= 0),
 * stopping a graph at its own fixed point when early stop is on. One call
 * per batch (a second call is KBISIM_ESTATE). rounds_done (host, [num_graphs],
 * may be NULL) receives each graph's executed rounds. */
kbisim_status kbisim_batch_refine(kbisim_batch* b, const int32_t* k_per_graph, int32_t* rounds_done);

/* pid_out[sum N] (host or device): every graph's local ids, graph after graph;
 * num_blocks (host, [num_graphs], may be NULL): each graph's block count. */
kbisim_status kbisim_batch_result(const kbisim_batch* b, int32_t* pid_out, kbisim_mem mem,
                                  int64_t* num_blocks);

void kbisim_batch_destroy(kbisim_batch* b);

/* ---- Served form ----------------------------------------------------------
 * A request loop for many jobs of different sizes on one GPU. Requests queue
 * in FIFO order; a request is admitted when one of max_slots slots is free
 * and its estimated device footprint (about 36 B per edge + 160 B per node +
 * 64 MB) fits in what hbm_budget_bytes has left. Admitted requests run
 * concurrently, each on its own stream with its partition state resident in
 * device memory across rounds, so requests that arrive while others run
 * overlap with them on the device. Results equal those of kbisim_refine on
 * the same graph alone. Host input arrays are copied by submit. DEVICE
 * input arrays are read when the request runs, after all work enqueued on
 * desc->stream before the submit call (an event recorded there; NULL = the
 * default stream), and must stay valid until kbisim_server_wait has
 * returned for the request. opt may be NULL; its profile field is ignored. */
typedef struct kbisim_server kbisim_server;

kbisim_status kbisim_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, const kbisim_options* opt,
                                   kbisim_server** out);

/* Queues a job refining desc's graph up to k rounds. KBISIM_ENOMEM when its
 * footprint exceeds the whole budget (it could never run). */
kbisim_status kbisim_server_submit(kbisim_server* s, const kbisim_graph_desc* desc, int32_t k,
                                   uint64_t* req_id);

/* Waits up to timeout_s seconds (negative: no limit) for the request. On
 * success writes pid_out[N] (host or device), *num_blocks and *rounds_done
 * (each may be NULL). Returns KBISIM_ETIMEDOUT, KBISIM_ECANCELED, or the
 * request's own error (e.g. KBISIM_EINVAL for an invalid graph) otherwise. */
kbisim_status kbisim_server_wait(kbisim_server* s, uint64_t req_id, int32_t* pid_out, kbisim_mem mem,
                                 int64_t* num_blocks, int32_t* rounds_done, double timeout_s);

/* Cancels a queued request at once, a running one at its next round
 * boundary; KBISIM_ESTATE if it already finished. */
kbisim_status kbisim_server_cancel(kbisim_server* s, uint64_t req_id);

/* Seconds from submit to start (queued_s) and to completion (total_s) of a
 * completed request; KBISIM_ESTATE otherwise. */
kbisim_status kbisim_server_timing(kbisim_server* s, uint64_t req_id, double* queued_s, double* total_s);

/* Forgets a finished request (its results); unknown or unfinished ids are ignored. */
kbisim_status kbisim_server_release(kbisim_server* s, uint64_t req_id);

/* Device bytes currently reserved by running requests (their estimates). */
kbisim_status kbisim_server_in_use(kbisim_server* s, uint64_t* bytes);

/* Lifecycle state of a request (kbisim_request_state); KBISIM_EINVAL for an
 * unknown or released id. */
typedef enum {
  KBISIM_REQ_QUEUED = 0,
  KBISIM_REQ_RUNNING = 1,
  KBISIM_REQ_DONE = 2,
  KBISIM_REQ_FAILED = 3,
  KBISIM_REQ_CANCELLED = 4
} kbisim_request_state;
kbisim_status kbisim_server_state(kbisim_server* s, uint64_t req_id, int32_t* state);

/* Cancels queued and running requests, waits for the workers, frees all. */
void kbisim_server_destroy(kbisim_server* s);

/* The library keeps freed device memory in a process-wide cache for reuse by
 * later handles (allocation is slow). This returns every cached block to
 * the HIP runtime after the device has finished with it; *released_bytes
 * (may be NULL) receives the amount. Handles stay valid. */
kbisim_status kbisim_release_cached(int64_t* released_bytes);

/* Static text for a status code. */
const char* kbisim_status_str(kbisim_status s);

/* Message describing the last error on the calling thread ("" if none). */
const char* kbisim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KBISIM_H */
