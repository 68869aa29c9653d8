/*
 * hpm.h -- edge-centric subgraph matching on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libhpm.so.  The library finds every embedding of a small labelled
 * pattern digraph in a large labelled target digraph, for induced subgraph
 * isomorphism or for monomorphism (HiPerMotif, arXiv 2507.04130):
 *   - the pattern is reordered by degree (Sec. III-A, Alg. 1, "Structural
 *     Reordering");
 *   - every target arc is scanned as a candidate image of pattern arc (0,1)
 *     and filtered by the vertex validator (Sec. III-B, Alg. 2) and the edge
 *     validator's attribute, reverse-arc and degree checks (Sec. III-B, Alg. 3);
 *   - the survivors become depth-2 partial mappings (state injection,
 *     Sec. III-C, Alg. 4) and are extended one pattern vertex at a time under
 *     the feasibility rules of the problem definition (Sec. II-A, Eq. (1)-(3)).
 *
 * All functions return an int status: HPM_OK (0) or a negative HPM_E_* code
 * (hpm_server_poll may also return HPM_PENDING).
 * On error, hpm_last_error() returns a message for the calling thread.  No
 * C++ exception ever crosses this boundary.
 *
 * Graph and pattern conventions (Sec. II-A; storage after Sec. III-D, "double
 * index" CSR with contiguous attribute arrays):
 *   - vertices are 0..n-1; arcs are ordered pairs (u,v), u != v, no repeats;
 *   - the out-CSR lists, for each u, the heads of its out-arcs in strictly
 *     ascending order; arc id e is the position of the arc in that array;
 *   - the in-CSR is its transpose (for each v the tails of its in-arcs, strictly
 *     ascending);
 *   - attributes are int32 columns: vertex columns indexed by vertex, arc
 *     columns indexed by out-CSR arc id.
 */
#ifndef HPM_H_
#define HPM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 3: hpm_match_stats.filter_pieces appended; HPM_F_TIMING_KINDS. */
/* 4: hpm_match_batch_persistent, hpm_batch_autotune, hpm_last_batch_stats. */
/* 5: hpm_match_noalloc. */
/* 6: HPM_F_LOOKAHEAD, hpm_match_stats.lookahead_removed. */
/* 7: hpm_scan_survivors, HPM_F_COUNT_FROM_MAX. */
/* 8: HPM_F_NO_ARC_INDEX, hpm_match_stats.index_arcs. */
/* 9: HPM_K_INDEX (HPM_K_NUM = 9). */
#define HPM_ABI_VERSION 9
#define HPM_MAX_K 16   /* largest pattern, in vertices            */
#define HPM_MAX_COLS 4 /* largest number of vertex or arc columns */

enum {
  HPM_OK = 0,
  HPM_E_ARG = -1,         /* NULL or out-of-range argument                         */
  HPM_E_GRAPH = -2,       /* malformed target graph                                */
  HPM_E_PATTERN = -3,     /* malformed pattern                                     */
  HPM_E_NOMEM = -4,       /* device allocation failed or budget below one chunk    */
  HPM_E_TRUNCATED = -5,   /* more matches than the mapping buffer holds            */
  HPM_E_OVERFLOW = -6,    /* match count does not fit in uint64                    */
  HPM_E_DEVICE = -7,      /* HIP runtime error                                     */
  HPM_E_UNSUPPORTED = -8, /* valid input beyond the library's limits (n, m >= 2^31) */
  HPM_E_INTERNAL = -9,    /* unexpected internal failure                           */
  HPM_PENDING = 1         /* hpm_server_poll: the query has not finished yet       */
};

typedef enum { HPM_ISO = 0, HPM_MONO = 1 } hpm_mode;

/* Predicate on one int32 attribute.  HPM_EQ is the label equality of
 * Sec. II-A, Eq. (2)-(3); HPM_GE is a threshold (value >= val); HPM_ANY leaves
 * the column unconstrained.  A vertex or arc satisfies its predicates when
 * every column does. */
typedef enum { HPM_ANY = 0, HPM_EQ = 1, HPM_GE = 2 } hpm_op;

typedef struct hpm_graph hpm_graph; /* opaque, device-resident, immutable */

/*
 * hpm_graph_create -- copy a target graph into library-owned device memory.
 *
 * n          vertices, 0 <= n < 2^31 - 1.
 * m          arcs, 0 <= m < 2^31.
 * out_off    host int64[n+1]: out_off[0] = 0, non-decreasing, out_off[n] = m.
 * out_nbrs   host int32[m]: heads, each row strictly ascending, no u in row u.
 * in_off     host int64[n+1], in_nbrs host int32[m]: the transpose.
 * n_vcols    0..HPM_MAX_COLS vertex columns; vcols[c] is a host int32[n].
 * n_ecols    0..HPM_MAX_COLS arc columns; ecols[c] is a host int32[m] in
 *            out-CSR arc order.
 * stream     hipStream_t (NULL = default stream) used for uploads and checks;
 *            the call synchronises it before returning.
 * *out       receives the handle; destroy it with hpm_graph_destroy.
 *
 * All inputs are host pointers and are copied; the caller may free them on
 * return.  The library derives on the device the arc tail array (the paper's
 * edge-to-source index), the in-to-out arc id map and the degrees, and checks
 * on the device that rows are strictly ascending, ids are in range, there are
 * no self-loops and the in-CSR is exactly the transpose of the out-CSR.
 * Errors: HPM_E_ARG (NULL pointers, column counts out of range),
 * HPM_E_UNSUPPORTED (n or m too large), HPM_E_GRAPH (any structural check
 * fails; nothing is kept), HPM_E_NOMEM, HPM_E_DEVICE.
 */
int hpm_graph_create(hpm_graph** out, int32_t n, int64_t m, const int64_t* out_off,
                     const int32_t* out_nbrs, const int64_t* in_off, const int32_t* in_nbrs,
                     int32_t n_vcols, const int32_t* const* vcols, int32_t n_ecols,
                     const int32_t* const* ecols, void* stream);

/* Release a graph and all its device memory.  No match may be in flight on it.
 * NULL is accepted and ignored. */
int hpm_graph_destroy(hpm_graph* g);

/* Sizes of a graph and the device bytes it holds (any output may be NULL). */
int hpm_graph_info(const hpm_graph* g, int32_t* n, int64_t* m, uint64_t* device_bytes);

/*
 * A pattern (query) digraph on vertices 0..k-1 (Sec. II-A).
 * k        2..HPM_MAX_K.
 * n_arcs   1..k*(k-1); arcs src[i] -> dst[i], no self-loops, no repeats; the
 *          pattern must be weakly connected.
 * vop/vval int32[k][n_vcols] (row-major): predicate of vertex a on column c is
 *          (vop[a*n_vcols+c], vval[a*n_vcols+c]); NULL means all HPM_ANY.
 * eop/eval int32[n_arcs][n_ecols]: predicate of arc i on column c; NULL means
 *          all HPM_ANY.  A reciprocal pair (a,b),(b,a) has two arcs with their
 *          own predicates.
 * n_vcols/n_ecols must equal the graph's.  All pointers are host pointers.
 */
typedef struct {
  int32_t k, n_arcs;
  const int32_t *src, *dst;
  const int32_t *vop, *vval;
  const int32_t *eop, *eval;
} hpm_pattern;

/* Flags for hpm_match_opts.flags. */
#define HPM_F_NO_REORDER 0x1u /* keep pattern order (vertex 0 first, then the   \
                                 smallest-id vertex adjacent to those placed)   \
                                 instead of the degree-based reordering.  Same   \
                                 result, used to check that reordering does not  \
                                 change it. */
#define HPM_F_TIMING 0x2u     /* record per-phase device times (hpm_last_stats) */
/* With HPM_F_TIMING: record events only around the launches of the kernel
 * families whose bit (1 << HPM_K_*) is set in mask; mask 0 = every family.
 * Each timed launch costs two event records on the stream, so timing a few
 * families disturbs the call less than timing all of them. */
#define HPM_F_TIMING_KINDS(mask) ((((uint32_t)(mask)) & 0x1ffu) << 16)
#define HPM_F_NO_FILTER 0x4u  /* do not pre-filter long shared candidate lists \
                                 (same result; for checking and measurement) */
#define HPM_F_OVERLAP 0x8u    /* apply the edge validator's neighbour-overlap  \
                                 test (Sec. III-B, Alg. 3) to the depth-2 rows: \
                                 (u,v) is dropped when u and v share fewer      \
                                 neighbours (either direction) than pattern     \
                                 positions 0 and 1 do.  Sound, same result;     \
                                 one more pass over the depth-2 rows. */
#define HPM_F_COUNT_FROM_MAX 0x20u /* test only: the running count starts at  \
                                 2^64 - 1, so a count-only call that finds an   \
                                 embedding fails with HPM_E_OVERFLOW (exercises \
                                 the wrap check of the count reduction). */
#define HPM_F_NO_ARC_INDEX 0x40u /* do not restrict the adjacency the       \
                                 extension reads to the arcs that can match     \
                                 (monomorphism: the loosest predicate over all  \
                                 pattern arcs).  Same result. */
#define HPM_F_LOOKAHEAD 0x10u /* frontier look-ahead (VF2's frontier sets,     \
                                 Sec. II-C; Alg. 3 builds them for the         \
                                 injected state): before a depth is extended, \
                                 drop rows in which a later pattern position   \
                                 adjacent to a mapped one has no candidate     \
                                 consistent with all its mapped neighbours.    \
                                 Sound, same result; one pass per depth. */

typedef struct {
  uint32_t struct_size;      /* sizeof(hpm_match_opts); 16 = the layout without
                                max_matches (treated as 0)                     */
  uint32_t flags;            /* HPM_F_*                                        */
  uint64_t hbm_budget_bytes; /* scratch limit; 0 = 25% of the device memory
                                that is free or already held as this graph's
                                idle scratch                                  */
  uint64_t max_matches;      /* first-k: stop once this many embeddings are
                                found (0 = find all).  *count is then
                                min(total, max_matches) and the mapping rows
                                are that many valid embeddings, which ones
                                unspecified.  The search runs in pieces of
                                2^20 arcs / 2^20 candidates and stops after
                                the piece in which the limit was reached. */
} hpm_match_opts;

/*
 * hpm_match -- count (and optionally list) all embeddings of p in g.
 *
 * mode      HPM_ISO (induced: arcs and non-arcs both preserved, Eq. (1) "<=>")
 *           or HPM_MONO (arcs preserved, Eq. (1) "=>").
 * stream    hipStream_t (NULL = default) on which all work is enqueued; the call
 *           synchronises it before returning.
 * opts      NULL for defaults.
 * count     required host uint64*: number of embeddings.  Embeddings are
 *           injective maps, so automorphic images count separately.
 * mappings  NULL, or a DEVICE int32 buffer of cap rows of k entries.  Row r holds
 *           f(0), ..., f(k-1) in the caller's original pattern-vertex ids.  Row
 *           order is unspecified.
 * cap       rows available in mappings (ignored when mappings is NULL).
 *
 * The scratch space (partial-mapping frontiers) the call uses is bounded by
 * opts->hbm_budget_bytes; the frontier is expanded in chunks that fit it, so the
 * result never depends on the budget.  Scratch is kept between calls on a
 * graph for reuse; idle scratch beyond twice a call's budget is freed when
 * that call starts.  Several calls may run concurrently on
 * different streams with the same graph.
 * Errors: HPM_E_ARG, HPM_E_PATTERN (invalid pattern or column-count mismatch),
 * HPM_E_NOMEM (budget below the minimum chunk, or allocation failure),
 * HPM_E_TRUNCATED (*count > cap: *count is valid, the first cap rows written are
 * valid embeddings but which ones is unspecified), HPM_E_OVERFLOW, HPM_E_DEVICE.
 */
int hpm_match(const hpm_graph* g, const hpm_pattern* p, hpm_mode mode, void* stream,
              const hpm_match_opts* opts, uint64_t* count, int32_t* mappings, uint64_t cap);

/*
 * hpm_scan_survivors -- the injected states alone (Sec. III-C, Alg. 4): the
 * vertex validator for pattern positions 0 and 1 (Alg. 2), then every target
 * arc as a candidate image of the pattern arc between them with the edge
 * validator's checks (Alg. 3: both vertex flags, the arc's predicate, the
 * reverse arc required with its predicate for a reciprocal pattern pair and,
 * under induced isomorphism, forbidden otherwise).  Positions are those of
 * hpm_plan_order (flags as for hpm_match).  *count receives the number of
 * surviving arcs; rows (NULL, or a DEVICE int32 buffer of cap rows of 2)
 * receives them as (image of position 0, image of position 1), in an order
 * that is the same on every call but otherwise unspecified (tiles of arcs in
 * arc order, rows within a tile interleaved).  Nothing is extended.  Errors:
 * as hpm_match; HPM_E_TRUNCATED when *count > cap (the first cap rows are
 * written).
 */
int hpm_scan_survivors(const hpm_graph* g, const hpm_pattern* p, hpm_mode mode, void* stream,
                       const hpm_match_opts* opts, uint64_t* count, int32_t* rows,
                       uint64_t cap);

/*
 * hpm_match_noalloc -- hpm_match for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as hpm_match; the
 * call itself calls no hipMalloc, hipFree or other allocating routine.  Its
 * scratch is a fixed 128 MiB device array that the library holds on every GPU
 * it runs on until the process ends (resolved once per device, on that
 * device's first call).  A call may use a quarter of it as its budget
 * (opts->hbm_budget_bytes is capped there; frontiers are expanded in chunks
 * that fit, so results never depend on it); a pattern whose minimum chunk
 * does not fit fails with HPM_E_NOMEM.  Calls on one GPU share that GPU's
 * array: the library runs them one at a time (a later call waits for an
 * earlier one to return), and each call clears what it needs.  Calls from
 * other code that write the same array would race with it.  HPM_F_TIMING is
 * ignored (timing events are created on demand).
 */
int hpm_match_noalloc(const hpm_graph* g, const hpm_pattern* p, hpm_mode mode, void* stream,
                      const hpm_match_opts* opts, uint64_t* count, int32_t* mappings,
                      uint64_t cap);

/*
 * hpm_match_batch -- count the embeddings of n patterns in one resident graph.
 *
 * patterns[i] is matched in mode modes[i] (HPM_ISO or HPM_MONO) exactly as
 * hpm_match would, counts only: counts[i] and status[i] (HPM_OK or an error
 * code of hpm_match) are written for every i.  The patterns are spread over
 * `workers` host threads (0 = 4), each driving its own non-blocking HIP stream
 * with its own scratch (opts->hbm_budget_bytes, or its default, is divided
 * among them), so the device works on several patterns at once.  Work already
 * queued on `stream` completes first; the call returns when all patterns are
 * done.  Returns HPM_OK, or the status of the first failed pattern (the
 * others are still matched).  This is the batched form of the edge-centric
 * search: many small queries sharing one graph (Sec. IV-B uses patterns of
 * 3 to 20 vertices).
 */
int hpm_match_batch(const hpm_graph* g, int32_t n, const hpm_pattern* patterns,
                    const int32_t* modes, void* stream, const hpm_match_opts* opts,
                    int32_t workers, uint64_t* counts, int32_t* status);

/*
 * hpm_batch_tune -- pick the worker count for hpm_match_batch on this batch.
 *
 * Runs the batch once to warm every worker's scratch, then once with each of
 * 1, 2, 4, 8, 16 and 32 workers (each run checked to give the same counts),
 * and returns in *best_workers the fastest count (host wall time; in *best_ms
 * that time when best_ms is not NULL).  The batched form runs independent
 * queries on concurrent streams, so its best width depends on the query mix
 * and the graph.  Errors: as for hpm_match_batch; HPM_E_ARG for an empty
 * batch.
 */
int hpm_batch_tune(const hpm_graph* g, int32_t n, const hpm_pattern* patterns,
                   const int32_t* modes, void* stream, const hpm_match_opts* opts,
                   int32_t* best_workers, double* best_ms);

/*
 * The batched form as ONE persistent launch (Sec. IV-B: random patterns of
 * many sizes against one graph).  One launch computes the vertex-validator
 * bitmaps of every pattern; then the arc scan with state injection and the
 * extension position by position run as tasks of a device work queue that
 * one kernel of resident blocks drains: (pattern, arc range) scan tasks and
 * (pattern, depth, chunk of partial mappings, candidate range) extension
 * tasks, each pushing the tasks it creates.  No host round trip happens
 * between depths or patterns.
 *
 * STATUS: switched off.  On the device the launch did not return (twice, on a
 * batch of small patterns) and no cause has been shown, so both entry points
 * below return HPM_E_UNSUPPORTED without launching anything; the batched form
 * runs through hpm_match_batch.
 *
 * hpm_batch_config selects how the extension runs (hpm_batch_autotune picks
 * it by timing the batch):
 *   items_per_lane  candidates a lane holds per tile, 1, 2 or 4: the states a
 *                   wavefront extends at once are 64 x items_per_lane
 *   chunk_rows      partial mappings per task, 16..1024
 *   task_work       candidates per task before its chunk is split into more
 *                   tasks (>= 256; long hub lists spread over many blocks)
 *   strategy        arc lookups: HPM_X_MAPPED binary-searches the mapped
 *                   vertex's list (shared by a row's candidates);
 *                   HPM_X_SHORTER searches the shorter of that list and the
 *                   candidate's own list in the other direction
 *   blocks_per_cu   resident blocks per compute unit (0 = as many as fit)
 */
#define HPM_X_MAPPED 0
#define HPM_X_SHORTER 1

typedef struct {
  uint32_t struct_size;    /* sizeof(hpm_batch_config)                         */
  int32_t items_per_lane;  /* 1, 2 or 4 (0 = 2)                                 */
  int32_t chunk_rows;      /* 16..1024 (0 = 256)                                */
  int32_t strategy;        /* HPM_X_MAPPED or HPM_X_SHORTER                     */
  int64_t task_work;       /* >= 256 (0 = 16384)                                */
  int32_t blocks_per_cu;   /* 0 = occupancy limit                              */
  int32_t idle_us;         /* microseconds a block waits for a task before it  */
                           /* leaves (0 = 1000); work left when all blocks have */
                           /* left is drained by launching again               */
} hpm_batch_config;

/* Statistics of the calling thread's last hpm_match_batch_persistent. */
typedef struct {
  uint32_t struct_size;      /* sizeof(hpm_batch_stats)                         */
  uint32_t error_bits;       /* 1 queue full, 2 a block left after waiting idle,   */
                             /* 4 arena full, 8 a descriptor out of bounds      */
  uint64_t tasks[4];         /* tasks run: [2] scan, [3] extension              */
  int32_t launches;          /* persistent launches (1 unless blocks left idle)  */
  int32_t reserved;
  uint64_t queue_slots;      /* queue slots used                                 */
  uint64_t arena_bytes;      /* partial-mapping bytes written                    */
  uint64_t scratch_bytes;    /* device bytes the call held                       */
  uint64_t fixed_bytes;      /* of the budget: queue, bitmaps, plans, results;   */
                             /* the rest is the arena                           */
  uint64_t arena_capacity;   /* arena bytes the launch could hand out            */
  int32_t grid;              /* resident blocks of the launch                    */
  int32_t fallback_patterns; /* patterns rerun with hpm_match (arena or queue full) */
  double kernel_ms;          /* device time of the launch (HIP events)           */
  double ms_total;           /* host wall time of the call                       */
} hpm_batch_stats;

/*
 * hpm_match_batch_persistent -- counts of n patterns in one persistent launch.
 * Arguments and results as hpm_match_batch (counts[i], status[i] for every
 * i; counts only); cfg NULL = defaults.  opts->hbm_budget_bytes (0 = 25% of
 * free device memory) bounds the call's scratch: the queue, the validator
 * bitmaps and an arena that holds every partial mapping of the batch.  A
 * pattern whose rows do not fit the arena (or tasks the queue) is finished
 * with hpm_match on the same stream afterwards, so results never depend on
 * the budget; hpm_batch_stats.fallback_patterns counts them.  opts with a
 * max_matches limit or HPM_F_OVERLAP run every pattern through hpm_match.
 * Returns HPM_OK or the status of the first failed pattern.  Errors:
 * HPM_E_ARG, HPM_E_NOMEM (budget below queue + bitmaps), HPM_E_DEVICE, and
 * per pattern the codes of hpm_match.
 */
int hpm_match_batch_persistent(const hpm_graph* g, int32_t n, const hpm_pattern* patterns,
                               const int32_t* modes, void* stream, const hpm_match_opts* opts,
                               const hpm_batch_config* cfg, uint64_t* counts, int32_t* status);

/*
 * hpm_batch_autotune -- pick the hpm_batch_config for this batch on this
 * graph: runs the batch once to warm up, then once per candidate
 * configuration (items_per_lane x chunk_rows x task_work x strategy, 24
 * settings), checks that every run gives the same counts, and returns the
 * fastest (device time of the launch) in *best and its time in *best_ms
 * (may be NULL).  Errors: as hpm_match_batch_persistent; HPM_E_ARG for an
 * empty batch; HPM_E_INTERNAL if two settings disagree.
 */
int hpm_batch_autotune(const hpm_graph* g, int32_t n, const hpm_pattern* patterns,
                       const int32_t* modes, void* stream, const hpm_match_opts* opts,
                       hpm_batch_config* best, double* best_ms);

int hpm_last_batch_stats(hpm_batch_stats* out);

/*
 * Serving: a resident graph answering a stream of queries.
 *
 * A server owns `workers` host threads, each driving its own non-blocking HIP
 * stream, and a device scratch budget.  Queries are submitted at any time and
 * run as soon as a worker is free and the query is admitted: each query's
 * scratch need is estimated on submission from the pattern and host-side
 * statistics of the graph (attribute-column samples, size-biased mean degree),
 * and it is granted twice that many bytes (at least min(256 MiB, budget / 2),
 * at most budget / 2; the estimate of deep frontiers is rough, and a query
 * granted less than its frontiers need runs in more pieces) out of a pool of
 * budget / 2; the query then runs exactly as
 * hpm_match with the grant as its scratch limit, so its result does not depend
 * on the grant or on the other queries in flight.  Workspaces (device
 * allocations reused between queries) are shared by the workers, a query
 * taking the one returned last; those not in use keep at most budget / 2 in
 * all (the least recently used give theirs back first), so device scratch
 * stays within the budget.  Admission is in arrival order, except that a query
 * that does not fit may be overtaken by later ones that do, at most 32 times.
 * Queries submitted while others run join them on the device (continuous
 * batching).  While some workers are idle, one of them polls for arrivals
 * instead of sleeping (one host core), so a query submitted to an idle server
 * starts without a thread wake-up.  This is the served form of the
 * edge-centric search on a large
 * resident graph (Sec. I and Sec. IV-D: whole-brain connectomes held in
 * memory and queried repeatedly).
 */
typedef struct hpm_server hpm_server; /* opaque */

typedef struct {
  uint32_t struct_size;      /* sizeof(hpm_server_opts)                              */
  int32_t workers;           /* queries in flight at most (0 = 4, at most 64)        */
  uint64_t hbm_budget_bytes; /* scratch of all queries together; 0 = 25% of free HBM */
  uint32_t flags;            /* HPM_F_NO_REORDER / HPM_F_NO_FILTER for every query   */
} hpm_server_opts;

typedef struct {
  uint32_t struct_size;   /* sizeof(hpm_query_result)                              */
  int32_t status;         /* the query's hpm_match status                          */
  uint64_t count;         /* embeddings (valid for HPM_OK and HPM_E_TRUNCATED)     */
  uint64_t est_bytes;     /* estimated scratch need used for admission             */
  uint64_t granted_bytes; /* scratch limit the query ran with                      */
  double queue_ms;        /* submission -> start on a worker (host clock)          */
  double run_ms;          /* start -> result                                       */
} hpm_query_result;

typedef struct {
  uint32_t struct_size;        /* sizeof(hpm_server_stats)                       */
  int32_t workers, running, queued, peak_running;
  uint64_t budget_bytes, grant_pool_bytes, granted_bytes, peak_granted_bytes;
  uint64_t admitted;           /* queries started so far                         */
} hpm_server_stats;

/* Start a server on g (which must outlive it).
 * opts NULL = defaults.  Errors: HPM_E_ARG, HPM_E_NOMEM (budget too small for
 * one query), HPM_E_DEVICE. */
int hpm_server_create(hpm_server** out, const hpm_graph* g, const hpm_server_opts* opts);

/* Queue one query; the pattern is validated and copied (the caller may free
 * it on return).  mappings/cap: as for hpm_match (a DEVICE buffer that must
 * stay valid until the result is polled), or NULL.  *ticket identifies the
 * query for hpm_server_poll.  Errors: HPM_E_ARG, HPM_E_PATTERN (the query is
 * then not queued). */
int hpm_server_submit(hpm_server* s, const hpm_pattern* p, hpm_mode mode, int32_t* mappings,
                      uint64_t cap, uint64_t* ticket);

/* Collect a query's result.  Returns HPM_PENDING if it has not finished and
 * wait == 0; otherwise blocks until it has, fills *out (out->status is the
 * query's own status; on a query error hpm_last_error() describes it) and
 * forgets the ticket (poll each ticket to completion exactly once, from one
 * thread).  Errors: HPM_E_ARG (NULL, unknown or already collected ticket). */
int hpm_server_poll(hpm_server* s, uint64_t ticket, int32_t wait, hpm_query_result* out);

/* Current load and admission counters. */
int hpm_server_read_stats(hpm_server* s, hpm_server_stats* out);

/* Run every query already submitted to completion, stop the workers and free
 * the server.  Results not yet polled are discarded.  NULL is ignored. */
int hpm_server_destroy(hpm_server* s);

/*
 * hpm_plan_order -- the matching order hpm_match would use (host only, no device).
 *
 * order[pos] receives the original pattern vertex placed at position pos
 * (int32[k]).  Positions 0 and 1 are the arc the target scan starts from.
 * Implements the structural reordering of Sec. III-A (Alg. 1): rank
 * sigma(v) = (in+out degree, out degree), first the best-ranked vertex, then
 * repeatedly the best-ranked unplaced out-neighbour of the last placed vertex;
 * when there is none, the best-ranked unplaced vertex adjacent to any placed
 * vertex (the paper takes any unplaced vertex; restricting to adjacent ones
 * keeps every position after the first connected to an earlier one).  Ties
 * go to the smaller original id.  flags: 0 or HPM_F_NO_REORDER.
 * n_vcols/n_ecols: the column counts the predicates are laid out for.
 * Errors: HPM_E_ARG, HPM_E_PATTERN.
 */
int hpm_plan_order(const hpm_pattern* p, int32_t n_vcols, int32_t n_ecols, uint32_t flags,
                   int32_t* order);

/* Kernel families, indexing hpm_match_stats.kernel_ms / kernel_launches. */
enum {
  HPM_K_VERTEX_VALIDATOR = 0, /* flags for positions 0 and 1 (Alg. 2)               */
  HPM_K_EDGE_SCAN = 1,        /* every arc vs pattern arc (0,1), compaction (Alg. 3) */
  HPM_K_ROW_PIVOT = 2,        /* candidate source and list length per partial map    */
  HPM_K_PREFIX_SUM = 3,       /* exclusive sums of the list lengths                  */
  HPM_K_EXPAND = 4,           /* extend partial mappings by one vertex               */
  HPM_K_LAST_LEVEL = 5,       /* final vertex: count (and write mappings)            */
  HPM_K_REDUCE = 6,           /* per-block counts -> total                           */
  HPM_K_FILTER = 7,           /* pre-filtering of long shared candidate lists,       */
                              /* look-ahead and overlap passes                       */
  HPM_K_INDEX = 8,            /* arc-predicate index (restricted adjacency)          */
  HPM_K_NUM = 9
};

/* Per-call statistics of the calling thread's most recent successful hpm_match.
 * kernel_ms is filled only when HPM_F_TIMING was set (device time from HIP
 * events recorded around every launch on the caller's stream, or around the
 * launches of the families HPM_F_TIMING_KINDS selects), else 0;
 * kernel_launches counts every launch either way. */
typedef struct {
  uint64_t struct_size;          /* sizeof(hpm_match_stats)                           */
  uint64_t count;                /* embeddings                                        */
  uint64_t arcs_scanned;         /* target arcs tested as images of pattern arc (0,1)  */
  uint64_t survivors;            /* depth-2 partial mappings after the validators     */
  uint64_t rows[HPM_MAX_K + 1];  /* partial mappings materialised per depth           */
  uint64_t work[HPM_MAX_K + 1];  /* candidates examined to fill position d            */
  uint64_t chunks;               /* frontier chunks processed                         */
  uint64_t scratch_bytes;        /* device scratch held by the call                   */
  uint64_t kernel_launches[HPM_K_NUM];
  double kernel_ms[HPM_K_NUM];
  double ms_total;               /* host wall time of the call                        */
  uint64_t filtered_lists;       /* distinct candidate lists pre-filtered             */
  uint64_t raw_work[HPM_MAX_K + 1]; /* candidates per depth before pre-filtering      */
  uint64_t overlap_removed;      /* depth-2 rows dropped by HPM_F_OVERLAP             */
  uint64_t counted_rows;         /* last-level rows counted from their filtered list's */
  uint64_t counted_work;         /* length (and the candidates those lists hold)       */
  uint64_t filter_rows;          /* rows of the depths whose lists were pre-filtered   */
  uint64_t filter_entries;       /* list entries the pre-filter read (all its groups)  */
  uint64_t filter_pieces;        /* blocks its list pass ran: one per group, more for  */
                                 /* lists longer than one piece of 1024 entries         */
  uint64_t lookahead_removed;    /* rows dropped by HPM_F_LOOKAHEAD (all depths)       */
  uint64_t index_arcs;           /* arcs of the arc-predicate index (0: not built)     */
} hpm_match_stats;

int hpm_last_stats(hpm_match_stats* out);

/* Static description of a status code, and the calling thread's last error
 * message ("" if none).  The returned strings stay valid until the thread's
 * next hpm_* call. */
const char* hpm_status_string(int status);
const char* hpm_last_error(void);

/* ABI version this library was built with (HPM_ABI_VERSION). */
int hpm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HPM_H_ */
