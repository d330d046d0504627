/*
 * lv.h - C ABI of the MI355X (gfx950) Louvain local-moving library.
 *
 * Method: F. Li, Z. Du, D. A. Bader, "Designing Parallel Algorithms for
 * Community Detection using Arachne" (arXiv 2507.06471): Louvain = local
 * moving (Algorithm 2, gain of Equation 1) alternating with aggregation
 * (Algorithm 3), and label propagation (Algorithm 1) as a second mode of the
 * same neighbour-aggregation step.  Modularity as in Section II-C.
 *
 * Deterministic semantics implemented by every entry point:
 *   - integer edge weights >= 1; a loop (v, v, w) counts twice in the weighted
 *     degree (Section II-A), so it enters the method as A_vv = 2w;
 *   - synchronous sweeps: every vertex decides against the previous sweep's
 *     labels and community volumes;
 *   - each vertex takes the best neighbouring community (ties to the smallest
 *     id) by the exact integer score  M*W_i(C) - k_i*Sigma_tot(C)  (Louvain; the
 *     gain of Equation 1 is 2*(score - stay)/M^2) or W_i(C) (LPA), and moves
 *     only if it beats staying and lies in the sweep's direction: odd sweeps
 *     allow only moves to smaller community ids, even sweeps only to larger;
 *   - a level ends after two consecutive sweeps with no move (LPA: with at
 *     most lpa_threshold moves) or after max_sweeps sweeps;
 *   - communities are renumbered by their smallest member vertex id;
 *   - a Louvain level is kept only if it raises modularity (Section III-B;
 *     Algorithm 3 stops once a level brings no gain), at most max_levels
 *     levels.
 * Every decision is integer arithmetic (int64 products of values < 2^31), so
 * results do not depend on tuning, scheduling or batching.
 *
 * Conventions for all calls:
 *   - every call returns an lv_status; out-parameters are written only on
 *     LV_OK; the library never aborts or prints; lv_last_error() gives a
 *     thread-local detail string for the last failure on the calling thread;
 *   - the caller owns every buffer it passes; inputs need to live only for the
 *     duration of the call; handles are library-owned until *_destroy;
 *   - LV_MEM_HOST / LV_MEM_DEVICE says where a caller buffer lives; device
 *     buffers must be hipMalloc'd memory of the current device;
 *   - a graph handle is bound to one HIP stream and must be used by one host
 *     thread at a time; calls are synchronous unless stated otherwise.
 */
#ifndef LV_H
#define LV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lv_status {
    LV_OK = 0,
    LV_E_ARG = 1,        /* null pointer, negative size, bad parameter value          */
    LV_E_CSR = 2,        /* offsets not monotone / not ending at nnz, index out of
                            range, or a row not strictly increasing                   */
    LV_E_ASYMMETRIC = 3, /* entry (i,j,w) without a matching (j,i,w)                  */
    LV_E_WEIGHT = 4,     /* a weight < 1                                              */
    LV_E_OVERFLOW = 5,   /* total volume M = sum_i k_i >= 2^31, or more than
                            LV_MAX_NNZ CSR entries (one graph or a packed set)        */
    LV_E_NOMEM = 6,      /* device allocation failed; the handle stays usable         */
    LV_E_HIP = 7,        /* a HIP runtime call failed                                 */
    LV_E_BUSY = 8,       /* server queue full                                         */
    LV_E_TOO_LARGE = 9,  /* job exceeds the server's device-memory budget             */
    LV_E_CANCELLED = 10, /* job cancelled before it ran                               */
    LV_E_STATE = 11,     /* call not valid in the object's current state              */
    LV_E_NOT_FOUND = 12  /* unknown ticket or level                                   */
} lv_status;

typedef enum lv_memkind { LV_MEM_HOST = 0, LV_MEM_DEVICE = 1 } lv_memkind;

/* Largest number of CSR entries a handle (one graph, or all graphs packed in
 * one handle or one server step) may hold: 2^31 - 1 - 2^16.  Row loops step
 * 32-bit entry counters by up to 2^13 past a row's end; the margin keeps every
 * such counter below 2^31. */
#define LV_MAX_NNZ (2147483647 - 65536)

/* lv_graph_create_csr flags */
#define LV_VALIDATE 1u /* check CSR shape, sortedness, symmetry and weights on the device */
#define LV_KEEP_ORDER 2u  /* create: store the vertices in input order (default: by descending    */
                          /* degree within each graph, for cache locality; results are the same)  */
#define LV_EDGES_NO_LOOPS 4u /* lv_graph_create_edges: drop loops (u, u)                          */
#define LV_EDGES_SIMPLE 8u   /* lv_graph_create_edges: a pair listed several times keeps weight 1 */
                             /* (no weights may be given)                                        */
#define LV_NO_ENTRY_CACHE 16u /* create: skip the reverse-entry map (int32 per CSR entry); calls on  */
                              /* the handle then never use the entry cache (see LV_NO_CACHE)         */

/* lv_params.flags */
#define LV_TIMING 1u      /* record per-kernel HIP event times (see lv_level_info); sweeps */
                          /* are then launched one by one instead of from a HIP graph     */
#define LV_KEEP_GRAPHS 2u /* lv_louvain keeps every coarse graph for lv_result_level_graph */
#define LV_NO_HIPGRAPH 4u /* launch sweeps one by one even without LV_TIMING              */
#define LV_AUTOTUNE 8u    /* with tuning == NULL: use the handle's autotuned setting (lv_autotune), */
                           /* chosen on the handle's first such call                               */
#define LV_PRUNE 16u      /* active-vertex pruning (Alg. 1's V_active, Alg. 2's needCheck), read   */
                          /* for synchronous sweeps: sweep s evaluates every vertex while s <= 2,   */
                          /* afterwards only a vertex that, or one of whose neighbours, changed     */
                          /* community in sweep s-1 or s-2; the others keep their community.        */
                          /* Changes results (for Louvain; LPA's are provably the same).           */
#define LV_ASYNC 32u      /* asynchronous sweeps, as Alg. 1 and 2 are written: every vertex reads */
                          /* the labels and community volumes as they stand, and a mover updates  */
                          /* both in place at once (atomics); no direction gate; a level ends     */
                          /* after one sweep with at most threshold moves.  Results depend on     */
                          /* scheduling and are not reproducible; every invariant (Sigma_tot sums */
                          /* to M, exact Q_int of the returned labels, level acceptance) holds.  */
                          /* With LV_PRUNE the active set looks one sweep back (Alg. 2).          */
#define LV_NO_CACHE 64u   /* do not use the entry cache.  By default the sweeps of a handle's input */
                          /* graph (Louvain's first level, LPA) keep each CSR entry's neighbour     */
                          /* (community, volume) pair in an int2[nnz] device array once few pairs   */
                          /* change between sweeps, rewriting after each commit only the entries    */
                          /* whose pair changed; a sweep then streams the array instead of gathering */
                          /* one pair per entry at random.  Results are identical either way.       */
                          /* Needs the handle's reverse-entry map (not LV_NO_ENTRY_CACHE); off with */
                          /* LV_PRUNE and LV_ASYNC.                                                  */

typedef struct lv_graph lv_graph;   /* device-resident CSR + workspace, library-owned */
typedef struct lv_result lv_result; /* per-level labels and statistics, library-owned */

/*
 * Scheduling knobs.  They choose which kernel handles a vertex (by its number
 * of CSR entries L) and the LDS table sizes; they never change results.
 * Zero fields take the built-in defaults.
 */
typedef struct lv_tuning {
    int32_t sub_max;   /* rows up to sub_max entries: groups of 1..32 lanes (<= 128)      */
    int32_t wave_max;  /* rows up to wave_max entries: one wavefront (<= 256)              */
    int32_t block_max; /* rows up to block_max entries: 128..1024-thread groups (<= 8192)  */
                       /* L >  block_max: ceil(L / part_keys) workgroups per vertex, each  */
                       /* aggregating one hash partition of the communities in LDS         */
    int32_t part_keys;  /* expected communities per partition workgroup (clamped to       */
                        /* [32, 3/4 of part_slots])                                       */
    int32_t part_slots; /* LDS table slots of a partition workgroup, power of two,       */
                        /* 64..16384 (mode 1) or 64..2048 (mode 2); a partition whose     */
                        /* communities do not fit is redone with a global-memory table    */
    int32_t hub_mode;   /* partition workgroups: 1 = compact tables, each workgroup       */
                        /* re-reading the vertex's entries; 0/2 = one scatter pass sums   */
                        /* the entries per community within chunks and appends them to    */
                        /* per-partition buckets that the partition workgroups read       */
    int32_t hub_chunk;  /* mode 2: entries per scatter workgroup, 1024, 2048 (default) or */
                        /* 4096, summed in passes of 1024 with one bucket allocation      */
    int32_t order_min;  /* coarse levels with at least this many entries are stored by    */
                        /* descending degree, like level 0 (0 = 2^22)                      */
    int32_t agg_sort;   /* aggregation: 1 = always sort and reduce the keys               */
                        /* (label(i), label(j)) of the entries; 0 = by community after a   */
                        /* level with at most 20 vertices per community (members' rows    */
                        /* laid out by label, each community's entries summed in LDS, the */
                        /* longest sorted), sorting otherwise.  Same coarse graphs.       */
    int32_t cache_pct;  /* entry cache: the next sweep reads the cache when at most this  */
                        /* percentage of the level's entries saw their pair change in the */
                        /* last commit (0 = 10, at most 100); a sweep fills it when at    */
                        /* most min(100, 2 cache_pct + 5) percent changed                  */
    int32_t fused;      /* later sweeps: 1 = every class below block_max in one persistent */
                        /* launch (1024-thread workgroups taking blocks of rows of any    */
                        /* class from a device counter); 0 = one launch per class          */
    int32_t table_pct;  /* LDS table slots per row of L entries in later sweeps: about    */
                        /* L * table_pct / 100 + 1, at least L + 1 and at most the        */
                        /* class's table (0 = 300)                                         */
} lv_tuning;

typedef struct lv_params {
    int32_t max_sweeps;    /* sweeps per level, default 20 (Alg. 2 maxIteration)          */
    int32_t max_levels;    /* accepted Louvain levels, default 32                         */
    int64_t lpa_threshold; /* LPA stops after two sweeps with <= this many moves (Alg. 1) */
    uint32_t flags;        /* LV_TIMING | LV_KEEP_GRAPHS | LV_NO_HIPGRAPH | LV_AUTOTUNE |  */
                           /* LV_PRUNE | LV_ASYNC                                          */
    const lv_tuning* tuning; /* NULL = built-in defaults                                   */
} lv_params;

#define LV_KERNEL_SLOTS 26

/* Per-level statistics; times are milliseconds from HIP events.  sweep_ms,
   renumber_ms and aggregate_ms are always measured (events around each
   phase); move_ms and the per-kernel arrays need LV_TIMING, which also
   launches the sweeps one kernel at a time. */
typedef struct lv_level_info {
    int32_t n;          /* vertices of this level's graph                        */
    int32_t n_next;     /* communities after renumbering                          */
    int64_t nnz;        /* CSR entries of this level's graph                      */
    int32_t sweeps;     /* sweeps run                                             */
    int32_t accepted;   /* 1 if the level raised modularity and was kept          */
    int64_t q_start;    /* Q_int of the singleton partition of this level         */
    int64_t q_end;      /* Q_int of the level's partition (= singletons of next)  */
    double move_ms;     /* summed duration of the move kernels (all sweeps)       */
    double sweep_ms;    /* whole local-moving phase (moves + commits)             */
    double renumber_ms;
    double aggregate_ms;
    int64_t move_launches; /* number of move-kernel launches                       */
    int64_t move_bytes;    /* compulsory bytes of the sweeps: (8 nnz + 36 n) each  */
    /* Per move kernel (LV_TIMING): slot 2*(class-1) + (1 for the first sweep
       of a level, where every community is a single vertex); classes 1..10 =
       rows of at most 4, 8, 32, 128, 256, 512, 1024, 2048, 3072 and 8192
       entries (from one lane a row up to 1024-thread workgroups), 11 =
       partition workgroups (with their merge and fallback kernels); slot 22
       = the bucketed mode's scatter pass, which then carries class 11's
       bytes; slot 23 = the commit (labels, volumes, pairs, sweep control);
       slot 24 = the entry cache's refresh; slot 25 = the fused persistent
       kernel of the classes below the hub class (lv_tuning.fused), which
       then carries their bytes.  Bytes are the compulsory bytes
       of the kernel's rows: 8 per CSR entry (index and weight) and 36 per
       vertex (offsets, label, degree and volume read; label and volume
       written), as for a whole sweep. */
    double kern_ms[LV_KERNEL_SLOTS];
    int64_t kern_launches[LV_KERNEL_SLOTS];
    int64_t kern_bytes[LV_KERNEL_SLOTS];
    int32_t cached_sweeps;      /* sweeps that read the entry cache (0 without it)        */
    int32_t reserved;
    int64_t refreshed_entries;  /* cache entries rewritten after commits, all sweeps      */
} lv_level_info;

void lv_params_default(lv_params* p);
const char* lv_status_str(lv_status s);
const char* lv_last_error(void);

/*
 * Create a device-resident graph from a symmetric CSR (Section II-A graph
 * model).  offsets int32[n+1] (offsets[0] = 0, non-decreasing, offsets[n] =
 * nnz); indices int32[nnz] in [0,n), strictly increasing within each row;
 * weights int32[nnz] >= 1, or NULL for unit weights; a diagonal entry is a
 * loop.  All three arrays live in `kind` memory.  The library copies them;
 * `stream` (a hipStream_t, NULL = a library-created stream) is used for all
 * work on this graph.  With LV_VALIDATE the layout, symmetry and weights are
 * checked (LV_E_CSR, LV_E_ASYMMETRIC, LV_E_WEIGHT); the volume bound is
 * always checked (LV_E_OVERFLOW).
 */
lv_status lv_graph_create_csr(int32_t n, const int32_t* offsets, const int32_t* indices,
                              const int32_t* weights, lv_memkind kind, uint32_t flags, void* stream,
                              lv_graph** out);
/*
 * Create a device-resident graph from an undirected edge list (Section II-A:
 * G(V, E, w) with E a set of unordered pairs, loops allowed).  Edge t joins
 * src[t] and dst[t] (both in [0, n)) with weight weights[t] >= 1 (NULL =
 * unit); m edges, each array int32[m] in `kind` memory.  A pair listed
 * several times, in either orientation, becomes one edge whose weight is the
 * sum of its listings (as the aggregation phase of Section III-B sums the
 * weights of edges whose endpoints coincide); with LV_EDGES_SIMPLE its weight
 * is 1 instead.  A loop (v, v, w) is one edge of weight w at v (its weighted
 * degree counts 2w), unless LV_EDGES_NO_LOOPS drops it.  The graph is built
 * on the device (keys sorted, equal pairs merged) and stored exactly as
 * lv_graph_create_csr would store its symmetric CSR with sorted rows;
 * LV_KEEP_ORDER applies as there.  Errors: LV_E_CSR (endpoint out of
 * range), LV_E_WEIGHT (weight < 1), LV_E_OVERFLOW (2m >= 2^31 or total
 * volume >= 2^31), LV_E_ARG (bad arguments, or weights with
 * LV_EDGES_SIMPLE).
 */
lv_status lv_graph_create_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                const int32_t* weights, lv_memkind kind, uint32_t flags, void* stream,
                                lv_graph** out);
/*
 * The graph held by a handle as a symmetric CSR in vertex-id order with
 * sorted rows, in the caller's convention (a loop's diagonal entry carries
 * its weight w, not 2w): offsets int32[n+1], indices and weights int32[nnz]
 * in `kind` memory (weights may be NULL).  *nnz_out (if not NULL) receives
 * nnz; with all three buffers NULL only nnz is returned.  For a packed handle
 * the packed CSR is returned (graph g's vertices after graph g-1's).
 */
lv_status lv_graph_csr(lv_graph* g, int32_t* offsets, int32_t* indices, int32_t* weights, int64_t* nnz_out,
                       lv_memkind kind);
/*
 * Create one device-resident handle holding `count` independent graphs,
 * packed one after another into a single CSR (vertex segment offsets), so
 * that every sweep of every graph runs in the same kernel launches.  Graph g
 * is given like lv_graph_create_csr's arguments: n[g], offsets[g],
 * indices[g], weights[g] (weights may be NULL, or weights[g] NULL for unit
 * weights), all in `kind` memory.  Each graph keeps its own total volume,
 * sweep counts, stopping rule and levels: lv_louvain / lv_lpa on the handle
 * give every graph exactly the result it gets alone.  Total vertices and
 * entries must each stay below 2^31.
 */
lv_status lv_graph_create_batch(int32_t count, const int32_t* n, const int32_t* const* offsets,
                                const int32_t* const* indices, const int32_t* const* weights,
                                lv_memkind kind, uint32_t flags, void* stream, lv_graph** out);
/*
 * Autotuner: picks the degree-class bounds (sub_max, wave_max, block_max)
 * and the partition settings (hub_mode, part_keys, hub_chunk) for this
 * handle by coordinate descent, timing each candidate on the handle's
 * level-0 graph (one first sweep and two later sweeps, HIP events) and
 * scoring it as a whole level of params->max_sweeps sweeps.  Writes the
 * fastest setting to *out (zero fields = defaults) and, if est_ms is not
 * NULL, its estimated level time in milliseconds; the handle keeps it for
 * LV_AUTOTUNE calls.  Tuning never changes results.  About 11 timed trials;
 * the handle's state is otherwise unchanged.
 */
lv_status lv_autotune(lv_graph* g, const lv_params* params, lv_tuning* out, double* est_ms);

lv_status lv_graph_destroy(lv_graph* g);
/* number of graphs packed in the handle (1 for lv_graph_create_csr) */
lv_status lv_graph_count(const lv_graph* g, int32_t* count);
/* n, nnz and total volume M = sum of weighted degrees (loops counted twice). */
lv_status lv_graph_info(const lv_graph* g, int32_t* n, int64_t* nnz, int64_t* volume);

/*
 * Multi-level Louvain (Algorithm 3 driving Algorithm 2).  params NULL =
 * defaults.  The result keeps every attempted level's statistics and every
 * accepted level's labels on the device.
 */
lv_status lv_louvain(lv_graph* g, const lv_params* params, lv_result** out);
/* accepted levels, attempted levels (attempted = accepted + 1 unless max_levels hit) */
lv_status lv_result_num_levels(const lv_result* r, int32_t* accepted, int32_t* attempted);
lv_status lv_result_level_info(const lv_result* r, int32_t level, lv_level_info* out);
/* per-sweep mover counts of an attempted level; writes min(cap, sweeps) values */
lv_status lv_result_level_moves(const lv_result* r, int32_t level, int64_t* moves, int32_t cap);
/* labels int32[n_level] of an accepted level: vertex of level l -> vertex of level l+1 */
lv_status lv_result_level_labels(const lv_result* r, int32_t level, int32_t* labels, lv_memkind kind);
/*
 * Coarse graph produced by accepted level `level` (the Aggregation of
 * Algorithm 3: A' = S^T A S with merged parallel edges and the community's
 * internal weight on the diagonal, already counted twice like a loop), as a
 * CSR with sorted columns: offsets int32[n_next+1], indices/weights int32[nnz].
 * Needs LV_KEEP_GRAPHS (else LV_E_STATE).  Any of the three buffers may be
 * NULL; *nnz is always written.
 */
lv_status lv_result_level_graph(const lv_result* r, int32_t level, int32_t* offsets, int32_t* indices,
                                int32_t* weights, int64_t* nnz, lv_memkind kind);
/* labels int32[n] of the input vertices after all accepted levels (singletons if none) */
lv_status lv_result_final_labels(const lv_result* r, int32_t* labels, lv_memkind kind);
/* Q_int, M and Q = (double)Q_int / ((double)M * (double)M) of the final partition */
lv_status lv_result_modularity(const lv_result* r, int64_t* q_int, int64_t* m, double* q);
lv_status lv_result_destroy(lv_result* r);

/*
 * Per-graph accessors for handles holding several graphs (graph index g in
 * [0, count)); the accessors above address graph 0.  Level statistics hold
 * the timings of the shared launches of that level.
 */
lv_status lv_result_graph_num_levels(const lv_result* r, int32_t g, int32_t* accepted, int32_t* attempted);
lv_status lv_result_graph_level_info(const lv_result* r, int32_t g, int32_t level, lv_level_info* out);
lv_status lv_result_graph_level_moves(const lv_result* r, int32_t g, int32_t level, int64_t* moves, int32_t cap);
lv_status lv_result_graph_level_labels(const lv_result* r, int32_t g, int32_t level, int32_t* labels,
                                       lv_memkind kind);
lv_status lv_result_graph_final_labels(const lv_result* r, int32_t g, int32_t* labels, lv_memkind kind);
lv_status lv_result_graph_modularity(const lv_result* r, int32_t g, int64_t* q_int, int64_t* m, double* q);
/* Every graph at once: final labels int32[total vertices] packed like the
   handle (graph g at its vertex offset, numbered within graph g), and
   per-graph q_int, m, q arrays of length count (any may be NULL). */
lv_status lv_result_final_labels_all(const lv_result* r, int32_t* labels, lv_memkind kind);
lv_status lv_result_modularity_all(const lv_result* r, int64_t* q_int, int64_t* m, double* q);

/*
 * Label propagation (Algorithm 1) as one level of synchronous sweeps with the
 * LPA score, then renumbering.  labels int32[n] in `kind` memory; info may be
 * NULL (then only labels are written); moves_out (may be NULL) receives up to
 * moves_cap per-sweep mover counts.
 */
lv_status lv_lpa(lv_graph* g, const lv_params* params, int32_t* labels, lv_memkind kind,
                 lv_level_info* info, int64_t* moves_out, int32_t moves_cap);
/*
 * LPA on every graph of a handle: labels int32[sum of n] (graph g's labels at
 * its packed vertex offset, numbered from 0 within the graph); per graph
 * (arrays of `count`, each may be NULL): sweeps, Q_int, M; moves int64
 * [count * moves_stride] (per-sweep mover counts, may be NULL).
 */
lv_status lv_lpa_batch(lv_graph* g, const lv_params* params, int32_t* labels, lv_memkind kind,
                       int32_t* sweeps, int64_t* q_int, int64_t* m, int64_t* moves, int32_t moves_stride);

/*
 * Diagnostic: the gather ceiling of the local-moving kernels on this handle.
 * Streams the handle's stored column indices (all packed graphs, in storage
 * order) and gathers one 8-byte (label, volume) pair per entry from a
 * scratch table of n pairs, with no other work, `reps` times (HIP events on
 * the handle's stream).  *entries_per_s receives entries per second.  A sweep
 * of the move kernels does this and more, so its entry rate cannot exceed
 * it; bandwidth figures, which count each entry's bytes once, miss that the
 * pairs arrive one cache line at a time.  Allocates and frees the table.
 */
lv_status lv_probe_gather(lv_graph* g, int32_t reps, double* entries_per_s);
/*
 * Diagnostic: a STREAM-style copy on the handle's device, the measured
 * bandwidth the HBM roofline is set against.  Copies the handle's stored
 * column indices (nnz int32) into a scratch buffer of the same size with
 * 16-byte loads and stores, `reps` times (HIP events on the handle's
 * stream); *bytes_per_s receives bytes read plus written per second (0 for
 * a handle without entries).  Allocates and frees the scratch buffer.
 */
lv_status lv_probe_copy(lv_graph* g, int32_t reps, double* bytes_per_s);

/* Modularity (Section II-C) of any labels int32[n] with values in [0, n). */
lv_status lv_modularity(lv_graph* g, const int32_t* labels, lv_memkind kind, int64_t* q_int,
                        int64_t* m, double* q);

/*
 * lv_modularity for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * (Q_int, M, Q) for labels int32[n] in DEVICE memory, computed without any
 * allocation.  Its scratch memory (12 bytes per vertex + 256) is a fixed
 * device array of LV_NOALLOC_SCRATCH_BYTES that every GPU the library runs
 * on holds until the process ends, so n is limited to
 * (LV_NOALLOC_SCRATCH_BYTES - 256) / 12 vertices (LV_E_TOO_LARGE beyond).
 * Calls on one GPU share that array: calls that overlap on one GPU race (run
 * them one at a time per device).  The handle's device must be current
 * (LV_E_STATE otherwise); labels outside [0, n) give LV_E_ARG.  Reads the
 * three results back with one synchronous copy.
 */
#define LV_NOALLOC_SCRATCH_BYTES (64u << 20)
lv_status lv_modularity_noalloc(lv_graph* g, const int32_t* labels, int64_t* q_int, int64_t* m, double* q);

/* ---------------------------------------------------------------------------
 * Serving loop (continuous batching).  A server owns two threads, each with
 * a stream of its own on the current device (default priority).  Jobs (CSR
 * graphs, same conventions as lv_graph_create_csr) are submitted at any time
 * and copied (host input to host memory, device input to device memory).
 * The staging thread admits queued jobs in arrival order while their
 * working-set estimates (72 B per entry + 96 B per vertex + 1 MiB) fit the
 * memory budget and the in-flight count fits max_jobs, and sets up each
 * admitted job's graph on the device while the worker runs the current
 * level.  At every level boundary the worker packs the coarse graphs of the
 * jobs that continue together with the graphs staged since, and runs one
 * Louvain level (Algorithm 3) for all of them in the same launches.  Each job
 * keeps its own M, stopping rule and acceptance, so its partition equals
 * lv_louvain's on its graph alone.  A device-resident submission's copy is
 * not counted in the budget.  Every server call is thread-safe; results are
 * kept until lv_server_result.
 * ------------------------------------------------------------------------- */
typedef struct lv_server lv_server;

typedef struct lv_server_config {
    int64_t mem_budget;  /* bytes for the in-flight jobs' estimates; 0 = half the free device memory */
    int32_t max_jobs;    /* in-flight jobs at most; 0 = 256                                           */
    int32_t max_sweeps;  /* 0 = 20                                                                    */
    int32_t max_levels;  /* 0 = 32                                                                    */
    uint32_t flags;      /* LV_VALIDATE: check each job's CSR (symmetry included) at admission         */
    const lv_tuning* tuning; /* NULL = defaults                                                      */
} lv_server_config;

#define LV_JOB_QUEUED 0
#define LV_JOB_RUNNING 1
#define LV_JOB_DONE 2

typedef struct lv_job_info {
    int32_t status;     /* lv_status of the job                                   */
    int32_t n;          /* vertices                                               */
    int32_t levels;     /* accepted levels                                        */
    int32_t steps;      /* levels attempted (batch steps the job took part in)    */
    int64_t q_int;      /* Q_int of the final partition                           */
    int64_t m;          /* total volume M                                         */
    double q;           /* Q_int / M^2                                            */
    int64_t entries;    /* sum over its levels of CSR entries x sweeps            */
    double queue_ms;    /* submit -> admission                                    */
    double total_ms;    /* submit -> result ready                                 */
} lv_job_info;

typedef struct lv_server_stats {
    int64_t submitted, completed;
    int64_t steps;      /* packed levels run                                      */
    int64_t max_batch;  /* most jobs in one packed level                          */
    int64_t entries;    /* packed entries x sweeps executed                       */
    int64_t queued, in_flight;
    int64_t mem_in_use, mem_budget;
} lv_server_stats;

/* cfg may be NULL (defaults).  LV_E_STATE if the worker thread cannot start. */
lv_status lv_server_create(const lv_server_config* cfg, lv_server** out);
/* Copies the CSR (host input to host memory, device input to device memory)
   and queues the job; *ticket names it.  LV_E_TOO_LARGE if its estimate
   alone exceeds the budget, LV_E_OVERFLOW above LV_MAX_NNZ entries.
   Malformed input is reported by the job's result (validation happens at
   admission). */
lv_status lv_server_submit(lv_server* s, int32_t n, const int32_t* offsets, const int32_t* indices,
                           const int32_t* weights, lv_memkind kind, uint64_t* ticket);
/* *state = LV_JOB_QUEUED / RUNNING / DONE; LV_E_NOT_FOUND for an unknown ticket. */
lv_status lv_server_poll(lv_server* s, uint64_t ticket, int32_t* state);
/* Blocks until the job is done (timeout_ms < 0: no limit); LV_E_BUSY on timeout. */
lv_status lv_server_wait(lv_server* s, uint64_t ticket, int64_t timeout_ms);
/* For a done job: labels int32[n] (final partition, renumbered by smallest
   member; may be NULL) and *info (may be NULL); then forgets the ticket.
   Returns the job's status (its error text through lv_last_error). */
lv_status lv_server_result(lv_server* s, uint64_t ticket, int32_t* labels, lv_memkind kind, lv_job_info* info);
/* A queued job is dropped; a running one leaves at its next level boundary
   with LV_E_CANCELLED (unless it finished there). */
lv_status lv_server_cancel(lv_server* s, uint64_t ticket);
lv_status lv_server_stats_get(lv_server* s, lv_server_stats* out);
/* Cancels what is queued or running, joins the worker, frees everything. */
lv_status lv_server_destroy(lv_server* s);

#ifdef __cplusplus
}
#endif
#endif /* LV_H */
