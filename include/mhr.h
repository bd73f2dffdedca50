/*
 * mhr.h - exact three-hop top-K path search over a typed knowledge graph,
 * on AMD Instinct MI355X (gfx950).
 *
 * The problem (paper section 3.1 and the generic algorithm of section 5):
 * given an edge list of typed directed edges (h, r, t), a relation
 * embedding table and an entity embedding table, and queries (s, t, K),
 * return the K best paths from s to t.  This library fixes the three-hop
 * case: a path is a walk s -r1-> a -r2-> b -r3-> t of exactly three edges
 * (a and b may repeat s, t or each other).  Edge weights come from the
 * learned embeddings (section 1 leaves the function open).  Two scorers:
 *
 *   DistMult + log-sigmoid (the default):
 *     x(u,r,v) = sum_i X[u][i] * Y[r][i] * X[v][i]
 *     w(u,r,v) = logsigmoid(x) = min(x,0) - log1p(exp(-|x|))
 *   TransE-L1, the paper's own score (section 3.3; gamma = 1.0 there):
 *     w(u,r,v) = gamma - sum_i |(X[u][i] + Y[r][i]) - X[v][i]|
 *
 *     S        = w(s,r1,a) + w(a,r2,b) + w(b,r3,t)
 *
 * Results are ranked by S descending, then a, b, r1, r2, r3 ascending (a
 * total order; the paper returns a ranked heap, section 5), and are exact:
 * the set and order equal those of an FP64 evaluation, up to pairs whose
 * scores differ by less than the reported error bound (flagged).
 *
 * Conventions.
 *  - Every function returns mhr_status.  No exception or abort crosses the
 *    ABI.  Argument errors are detected on the host before anything is
 *    enqueued; out-parameters are untouched on error.  The message of the
 *    last error on the calling thread is available from mhr_last_error().
 *  - Pointers documented as "device" point to device memory of the current
 *    HIP device; the library never frees them.  Host pointers are read
 *    before the call returns.
 *  - "stream" is a hipStream_t (NULL = the null stream).  Query calls are
 *    asynchronous on it; results are valid once the stream is synchronised.
 *  - A graph handle may be queried concurrently from several streams, each
 *    with its own workspace.
 *  - Limits: num_relations <= 32; embedding dimension a power of two in
 *    [8, 512]; K <= MHR_MAX_K.
 */
#ifndef MHR_H
#define MHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mhr_status {
    MHR_OK = 0,
    MHR_ERR_INVALID_ARGUMENT = 1,
    MHR_ERR_WORKSPACE_TOO_SMALL = 2,
    MHR_ERR_UNSUPPORTED = 3,
    MHR_ERR_OUT_OF_MEMORY = 4,
    MHR_ERR_DEVICE = 5,
    MHR_ERR_NO_EMBEDDINGS = 6,
    MHR_ERR_BAD_EDGE = 7,
    MHR_ERR_INTERNAL = 8,         /* an internal consistency check failed */
    MHR_ERR_IO = 9,               /* a file could not be read or written */
    MHR_ERR_CORRUPT = 10,         /* a file failed its format or checksum checks */
    MHR_ERR_NOT_FOUND = 11        /* no matching record (tuning cache) */
} mhr_status;

typedef enum mhr_dtype {
    MHR_DTYPE_F32 = 0,   /* IEEE binary32 */
    MHR_DTYPE_BF16 = 1   /* bfloat16 bit patterns (uint16) */
} mhr_dtype;

/* Edge scorer (the weight of an edge from the embeddings). */
typedef enum mhr_scorer {
    MHR_SCORER_DISTMULT = 0,   /* logsigmoid(sum_i X[u][i] Y[r][i] X[v][i]); matrix-core scoring */
    MHR_SCORER_TRANSE_L1 = 1   /* gamma - sum_i |X[u][i] + Y[r][i] - X[v][i]|; vector-unit scoring */
} mhr_scorer;

#define MHR_MAX_K 224u
#define MHR_MAX_RELATIONS 32u

/* Per-query status word (out_status[q]); bits may combine. */
#define MHR_Q_OK          0u
#define MHR_Q_BAD_ID      1u   /* s or t >= num_vertices: count 0 */
#define MHR_Q_BAD_K       2u   /* k == 0 or k > k_max: count 0 */
#define MHR_Q_EXACT_PASS  4u   /* informational: the FP32 candidate band overflowed and
                                  the exhaustive compensated pass produced the result */
/* No capacity can truncate a result: a query whose candidates overflow the
 * tile lists is answered by the exhaustive pass (MHR_Q_EXACT_PASS). */

/* Per-path flags. */
#define MHR_PATH_RESCORED       1u  /* score evaluated in compensated FP32 (float-float) */
#define MHR_PATH_PRECISION_TIE  2u  /* the next path's score differs from this one by less
                                       than the error bounds (their relative order is not
                                       certified) */

/* One ranked path s -r1-> a -r2-> b -r3-> t (24 bytes).  Unused slots of an
 * output row hold a = b = 0xFFFFFFFF, score = -inf. */
typedef struct mhr_path {
    uint32_t a, b;
    uint16_t r1, r2, r3, flags;
    float score;      /* S rounded to FP32 */
    float err_bound;  /* rigorous bound on |score - S| with S the exact real score
                         (includes the final rounding to FP32) */
} mhr_path;

typedef struct mhr_graph mhr_graph;

/* Edge list of the problem statement (section 3.1): triples (h, r, t).
 * head/rel/tail: device arrays of num_edges uint32, read during
 * mhr_graph_create only.  Identical triples are merged; h == t is allowed. */
typedef struct mhr_graph_desc {
    uint32_t num_vertices;
    uint32_t num_relations;     /* 1 .. 32 */
    uint64_t num_edges;         /* < 2^32 */
    const uint32_t *head;
    const uint32_t *rel;
    const uint32_t *tail;
} mhr_graph_desc;

typedef struct mhr_graph_stats {
    uint32_t num_vertices, num_relations;
    uint64_t num_triples;        /* distinct (h, r, t) */
    uint64_t num_pairs;          /* distinct (h, t); the length of each CSR */
    uint32_t max_out_degree;     /* in distinct pairs */
    uint32_t max_in_degree;
    uint32_t dim;                /* 0 until embeddings are set */
    uint32_t dtype;              /* mhr_dtype */
    uint64_t device_bytes;       /* device memory held by the handle */
    uint32_t heavy_rows_out, heavy_rows_in;  /* rows with a probe directory */
} mhr_graph_stats;

/* Builds the graph G of the problem (section 3.1: the multi-relational
 * graph searched for paths) on the device (one-time ingest): forward CSR (rows =
 * heads, entries = distinct tails ascending) and reverse CSR (rows = tails,
 * entries = distinct heads ascending), each entry carrying the bitmask of
 * relations joining the pair; plus bucket directories of long rows.  The
 * handle owns the device memory it allocates (hipMalloc, here only).
 * Synchronises `stream` before returning.  Errors: INVALID_ARGUMENT (null
 * pointers, zero vertices, num_relations outside 1..32), BAD_EDGE (an id out
 * of range), OUT_OF_MEMORY, DEVICE. */
mhr_status mhr_graph_create(const mhr_graph_desc *desc, void *stream, mhr_graph **out);

/* Device bytes the caller provides to mhr_graph_create_in for a graph of
 * num_vertices vertices and num_edges triples (section 3.1: the graph G the
 * paths are searched in):
 *   csr_buffer_bytes  storage of both CSRs and their directories, kept by the
 *                     handle until mhr_graph_destroy; sized for the worst
 *                     case (every triple a distinct pair, every row long);
 *   tmp_buffer_bytes  scratch of the build (sort keys, scans), free again
 *                     when mhr_graph_create_in returns.
 * Host only; enqueues nothing.  Errors: INVALID_ARGUMENT (the shape checks
 * of mhr_graph_create). */
mhr_status mhr_graph_buffer_sizes(uint32_t num_vertices, uint32_t num_relations, uint64_t num_edges,
                                  size_t *csr_buffer_bytes, size_t *tmp_buffer_bytes);

/* mhr_graph_create with every device byte supplied by the caller: the
 * library calls no hipMalloc.  csr_buffer (device, 256-byte aligned, at least
 * csr_buffer_bytes of mhr_graph_buffer_sizes) is BORROWED for the handle's
 * lifetime and must not be written while the handle lives; tmp_buffer
 * (device, 256-byte aligned, at least tmp_buffer_bytes) is used during the
 * call only.  Results and synchronisation as mhr_graph_create; the stats'
 * device_bytes is the part of csr_buffer the CSRs occupy.  Errors: as
 * mhr_graph_create, plus WORKSPACE_TOO_SMALL when a buffer is smaller than
 * its size (nothing enqueued). */
mhr_status mhr_graph_create_in(const mhr_graph_desc *desc, void *csr_buffer, size_t csr_buffer_bytes,
                               void *tmp_buffer, size_t tmp_buffer_bytes, void *stream, mhr_graph **out);

/* Attaches the embeddings that define the edge weights (section 3.1: the
 * weight of an edge is computed from its head, relation and tail vectors):
 * entity[num_vertices][dim] and relation[num_relations][dim],
 * row-major device arrays of `dtype`, BORROWED (they must stay valid and
 * unchanged while the graph is queried), 16-byte aligned.  dim: power of two
 * in [8, 512].  Enqueues nothing (`stream` is unused). */
mhr_status mhr_graph_set_embeddings(mhr_graph *g, mhr_dtype dtype, uint32_t dim,
                                    const void *entity, const void *relation, void *stream);

/* Selects the edge scorer for every later query on g (default: DistMult).
 * TransE-L1 is the score of the paper's experiments (section 3.3, the person
 * and affiliation scoring algorithms): the L1 distance between head plus
 * relation and tail, subtracted from gamma (1.0 in the paper).  The weight
 * is directed (w(u,r,v) != w(v,r,u) in general).  gamma must be finite.
 * Enqueues nothing.  Errors: INVALID_ARGUMENT. */
mhr_status mhr_graph_set_scorer(mhr_graph *g, mhr_scorer scorer, float gamma);

mhr_status mhr_graph_get_stats(const mhr_graph *g, mhr_graph_stats *out);

/* Copies one CSR into caller device buffers: row_ptr[num_vertices+1],
 * col[num_pairs], rmask[num_pairs].  reverse = 0: forward, 1: reverse. */
mhr_status mhr_graph_export_csr(const mhr_graph *g, int reverse, uint32_t *row_ptr,
                                uint32_t *col, uint32_t *rmask, void *stream);

mhr_status mhr_graph_destroy(mhr_graph *g);

/* Query options.  Zero-initialise, then set what is needed. */
typedef struct mhr_query_opts {
    uint32_t k;            /* K for every query when the per-query array is NULL */
    uint32_t tile_edges;   /* scan entries per work tile (0 = default) */
    uint32_t grid_blocks;  /* persistent gather workgroups (0 = default) */
    uint32_t hash_log2;    /* log2 of the LDS probe-table slots, 10..12 (0 = the largest of
                              10..12 whose workgroup fits in LDS) */
    float band_abs;        /* minimum width of the rescoring band below the K-th score:
                              every candidate with fast-pass score >= S_K - max(2 eps, band_abs)
                              that the tile lists hold is rescored in float-float (0 = the
                              rigorous band 2 eps alone, which already makes the result exact).
                              A candidate below S_K - 2 eps cannot be returned, so one that a
                              tile list dropped is never looked for again: the exhaustive pass
                              runs only when a dropped candidate could still be returned, and
                              that does not depend on band_abs.  A wider band costs only the
                              extra rescoring.  The result does not depend on band_abs.
                              Finite, >= 0. */
    uint32_t reserved[7];  /* must be zero */
} mhr_query_opts;

/* Device workspace bytes needed by mhr_topk_paths for nq queries with
 * K <= k_max.  Errors: INVALID_ARGUMENT, NO_EMBEDDINGS. */
mhr_status mhr_workspace_size(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                              uint32_t k_max, size_t *bytes);

/* Exact top-K three-hop paths for nq queries (src[q], dst[q], k[q]): the K
 * highest-scoring paths s -> a -> b -> t of section 3.1, a path's score the
 * sum of its three edge weights (the generic search of section 5 with three
 * levels and no frontier bound).
 *   src, dst   device uint32[nq]
 *   k          device uint32[nq], or NULL to use opts->k for every query
 *   k_max      1..MHR_MAX_K; every k[q] must be <= k_max (else MHR_Q_BAD_K)
 *   out        device mhr_path[nq][k_max]; row q holds out_count[q] paths, best first
 *   out_count  device uint32[nq]: min(k[q], |P(s,t)|)
 *   out_total  device uint64[nq] or NULL: |P(s,t)|, the number of paths scored
 *   out_status device uint32[nq] or NULL: MHR_Q_* bits
 *   workspace  device buffer of ws_bytes >= mhr_workspace_size(...)
 * Asynchronous on `stream`; allocates nothing.  Errors: INVALID_ARGUMENT,
 * WORKSPACE_TOO_SMALL, NO_EMBEDDINGS, DEVICE (launch failure). */
mhr_status mhr_topk_paths(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                          const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                          uint32_t k_max, mhr_path *out, uint32_t *out_count,
                          uint64_t *out_total, uint32_t *out_status,
                          void *workspace, size_t ws_bytes, void *stream);

/* Allocation-free form of mhr_topk_paths, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments and results as mhr_topk_paths
 * without the workspace: the workspace is a fixed array of
 * MHR_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends.  The call allocates nothing (no hipMalloc / hipFree).
 *  - Limit: the batch's workspace, mhr_workspace_size(g, opts, nq, k_max),
 *    must not exceed MHR_NOALLOC_SCRATCH_BYTES (e.g. up to 4,096 queries at
 *    k_max <= 96); larger batches return MHR_ERR_WORKSPACE_TOO_SMALL before
 *    anything is enqueued.
 *  - Every call on one GPU shares that GPU's array: calls that overlap in
 *    time on one GPU (other streams, other threads) race and must not be
 *    issued.  Calls on one stream are ordered and safe.
 *  - The current device must be the graph's device. */
#define MHR_NOALLOC_SCRATCH_BYTES (64u << 20)
mhr_status mhr_topk_paths_noalloc(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                                  const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                  uint32_t k_max, mhr_path *out, uint32_t *out_count,
                                  uint64_t *out_total, uint32_t *out_status, void *stream);

/* Events recorded on `stream` around the phases of one mhr_topk_paths call,
 * for timing the kernels on the stream they run on.  Each member is a
 * hipEvent_t created by the caller, or NULL to skip it. */
typedef struct mhr_phase_events {
    void *begin;          /* before the planning kernel */
    void *gather_begin;   /* before the gather kernel (after planning and scheduling) */
    void *gather_end;     /* after the gather kernel */
    void *end;            /* after the last kernel of the call */
} mhr_phase_events;

/* mhr_topk_paths with phase events (same arguments and semantics; ev may be
 * NULL).  For benchmarks and profilers. */
mhr_status mhr_topk_paths_profiled(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                                   const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                   uint32_t k_max, mhr_path *out, uint32_t *out_count,
                                   uint64_t *out_total, uint32_t *out_status,
                                   void *workspace, size_t ws_bytes, void *stream,
                                   const mhr_phase_events *ev);

/* Pruned search: mhr_topk_paths restricted by keep flags, as a frontier
 * pruner decides them (the learned pruner below, or any other rule; section
 * 5 bounds each level's frontier, here the first and last levels).
 *   keep      device uint8 flags; for query q, keep[keep_off[q] + i] is the
 *             flag of entry i of s's out-row (i < deg+(s), forward CSR order)
 *             and keep[keep_off[q] + deg+(s) + j] that of entry j of t's
 *             in-row (reverse CSR order); nonzero = kept
 *   keep_off  device uint64[nq]
 * The result is the exact top-K over the paths s -> a -> b -> t whose pair
 * (s, a) and pair (b, t) are kept: the search of the full graph with the
 * pruned-away first and last edges removed.  out_total counts those paths.
 * Other arguments and errors as mhr_topk_paths. */
mhr_status mhr_topk_paths_pruned(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                                 const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                 uint32_t k_max, const uint8_t *keep, const uint64_t *keep_off,
                                 mhr_path *out, uint32_t *out_count, uint64_t *out_total,
                                 uint32_t *out_status, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batched form: one captured launch for a fixed batch shape.
 *
 * Many queries with uneven frontiers already run as one persistent gather
 * launch inside mhr_topk_paths (tiles of bounded work pulled from a device
 * counter).  A plan additionally captures the whole call (planning,
 * scheduling, gather, merge, and the exhaustive pass) into a HIP graph once,
 * so that a serving loop replays it with a single launch.
 * ------------------------------------------------------------------------- */
typedef struct mhr_plan mhr_plan;

/* Captures mhr_topk_paths(g, opts, nq, src, dst, k, k_max, out, out_count,
 * out_total, out_status, workspace, ws_bytes) into a HIP graph.  The
 * pointers are fixed in the plan; their contents are read at each launch, so
 * the caller may write a new batch of nq queries into src/dst/k between
 * launches.  stream: the stream captured on (NULL = a private stream the call
 * creates and destroys); nothing runs during the call.  The plan holds
 * references to g and the buffers: they must outlive it.  Errors: those of
 * mhr_topk_paths (checked before capture), DEVICE (capture/instantiation). */
mhr_status mhr_plan_create(const mhr_graph *g, const mhr_query_opts *opts, uint32_t nq,
                           const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                           uint32_t k_max, mhr_path *out, uint32_t *out_count,
                           uint64_t *out_total, uint32_t *out_status,
                           void *workspace, size_t ws_bytes, void *stream, mhr_plan **plan);

/* Launches the captured call on `stream` (asynchronous; one graph launch).
 * Launches of one plan must not overlap (they share the workspace). */
mhr_status mhr_plan_launch(mhr_plan *plan, void *stream);

mhr_status mhr_plan_destroy(mhr_plan *plan);

/* Autotuner (an engineering addition; the paper tunes nothing).  Times
 * mhr_topk_paths on the given batch for candidate values of
 * tile_edges and hash_log2 (the other fields of *base are kept), `reps` timed
 * runs each after one untimed run, and writes the fastest setting to *tuned
 * and its mean time per call (ms) to *best_ms (may be NULL).  Tuning never
 * changes results: every candidate's outputs (out, out_count, out_total,
 * out_status) are compared byte for byte with the first candidate's, and a
 * difference returns MHR_ERR_INTERNAL.  Blocks the calling thread (it
 * synchronises `stream` and copies outputs to host memory); not for the
 * query path.  The output buffers hold the last candidate's results on
 * return.  Errors: those of mhr_topk_paths, INTERNAL. */
mhr_status mhr_autotune(const mhr_graph *g, const mhr_query_opts *base, uint32_t nq,
                        const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                        uint32_t k_max, mhr_path *out, uint32_t *out_count,
                        uint64_t *out_total, uint32_t *out_status,
                        void *workspace, size_t ws_bytes, void *stream, uint32_t reps,
                        mhr_query_opts *tuned, float *best_ms);

/* Tuning cache: the autotuner's chosen settings (tile_edges, hash_log2,
 * grid_blocks) and time per call, keyed by the device architecture name,
 * the graph's vertices, relations and distinct pairs, the embedding
 * dimension and dtype, the scorer, the batch size nq and k_max.  The file is
 * a sequence of 96-byte records, each with its own CRC-32; save replaces the
 * record of the same key (or appends one) and rewrites the file atomically,
 * refusing to touch a damaged file (CORRUPT).  load fills *tuned (other
 * fields zero) and *ms (may be NULL), or returns NOT_FOUND.  Errors:
 * INVALID_ARGUMENT, IO, CORRUPT, NOT_FOUND, DEVICE. */
mhr_status mhr_tuning_save(const char *path, const mhr_graph *g, uint32_t nq, uint32_t k_max,
                           const mhr_query_opts *tuned, float ms);
mhr_status mhr_tuning_load(const char *path, const mhr_graph *g, uint32_t nq, uint32_t k_max,
                           mhr_query_opts *tuned, float *ms);

/* Checks a tuning cache on the host alone and counts its records.  Errors:
 * IO, CORRUPT. */
mhr_status mhr_tuning_file_records(const char *path, uint32_t *count);

/* ---------------------------------------------------------------------------
 * Wide-relation graphs (up to 65,535 relations).
 *
 * The paper's experiments search a knowledge graph of 91.23M entities, 1,387
 * relations and 601.06M triples with 8-dimensional TransE embeddings
 * (section 4.1).  mhr_graph keeps one 32-bit relation mask per vertex pair,
 * which caps it at 32 relations.  A wide graph stores every distinct triple
 * as its own CSR entry (neighbour id and 16-bit relation; rows sorted by
 * (neighbour, relation), so the relations of one pair are consecutive) and
 * scores edges with TransE-L1 (section 3.3) in FP64:
 *     w(u, r, v) = gamma - sum_i |(X[u,i] + Y[r,i]) - X[v,i]|,
 * every operation in FP64 in ascending i, and a path's score is
 * S = w1 + w2 + w3 rounded once (the correctly rounded sum).  Scores are
 * therefore exact functions of the inputs; paths are ranked by S
 * descending, then a, b, r1, r2, r3 ascending (the problem of section 3.1).
 * ------------------------------------------------------------------------- */
#define MHR_WIDE_MAX_RELATIONS 65535u
#define MHR_WIDE_MAX_K 256u

typedef struct mhr_wide_graph mhr_wide_graph;

/* Builds a wide graph from the triples in desc (num_relations in
 * 1..65535, num_edges < 2^32; head/rel/tail device arrays read during the
 * call only).  Identical triples are merged.  The handle owns the device
 * memory it allocates: per direction (n + 1) * 4 + 6 bytes per distinct
 * triple, plus 8 bytes per vertex (the scan cost of its row as a query's
 * frontier and its count of distinct neighbours with a nonempty row, which
 * make query planning a constant-time lookup).  Synchronises `stream`.  Errors: INVALID_ARGUMENT, BAD_EDGE,
 * OUT_OF_MEMORY, DEVICE. */
mhr_status mhr_wide_graph_create(const mhr_graph_desc *desc, void *stream, mhr_wide_graph **out);
mhr_status mhr_wide_graph_destroy(mhr_wide_graph *g);

/* Attaches the TransE embeddings (section 3.3): entity[num_vertices][dim]
 * and relation[num_relations][dim] row-major device arrays of dtype
 * (FP32 or bfloat16 bits), BORROWED; dim in 1..1024; gamma finite (1.0 in
 * the paper).  Enqueues nothing.  Errors: INVALID_ARGUMENT. */
mhr_status mhr_wide_graph_set_embeddings(mhr_wide_graph *g, mhr_dtype dtype, uint32_t dim, const void *entity,
                                         const void *relation, double gamma);

typedef struct mhr_wide_stats {
    uint32_t num_vertices, num_relations;
    uint64_t num_triples;        /* distinct (h, r, t) */
    uint32_t max_out_degree, max_in_degree;   /* in entries (triples) */
    uint32_t dim, dtype;
    uint64_t device_bytes;
} mhr_wide_stats;

mhr_status mhr_wide_graph_get_stats(const mhr_wide_graph *g, mhr_wide_stats *out);

/* Copies one CSR into caller device buffers: row_ptr[num_vertices + 1],
 * col[num_triples], rel[num_triples] (uint16).  reverse = 0: rows are heads;
 * 1: rows are tails. */
mhr_status mhr_wide_graph_export_csr(const mhr_wide_graph *g, int reverse, uint32_t *row_ptr, uint32_t *col,
                                     uint16_t *rel, void *stream);

/* One ranked path s -r1-> a -r2-> b -r3-> t (24 bytes).  Unused slots of an
 * output row hold a = b = 0xFFFFFFFF, score = -inf. */
typedef struct mhr_wide_path {
    double score;   /* S, exact as defined above */
    uint32_t a, b;
    uint16_t r1, r2, r3, reserved;
} mhr_wide_path;

/* Work of one query (diagnostics and the benchmark's byte counts). */
typedef struct mhr_wide_work {
    uint64_t scanned;    /* adjacency entries scanned in the middle hop */
    uint64_t matches;    /* of those, entries whose neighbour lies in the probe row */
    uint64_t paths;      /* |P(s,t)| */
    uint64_t frontier;   /* |out(s)| + |in(t)| entries (weighted once each) */
    uint64_t distinct;   /* distinct list-side vertices whose rows were scanned */
    uint64_t probe_len;  /* entries of the probe row */
    uint64_t tiles;      /* work tiles of the query */
    uint64_t forward;    /* 1: scanned out-rows of out(s); 0: in-rows of in(t) */
} mhr_wide_work;

/* Device workspace bytes for mhr_wide_topk_paths on this batch (the same
 * src, dst, k and k_max).  The size depends on the queries' frontiers, so
 * the call plans the batch on the device and synchronises `stream`.
 * Errors: as mhr_wide_topk_paths. */
mhr_status mhr_wide_workspace_size(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                   const uint32_t *k, uint32_t k_max, size_t *bytes, void *stream);

/* Exact top-K three-hop paths for nq queries (the problem of section 3.1 on
 * a wide graph).
 *   src, dst   device uint32[nq]
 *   k          device uint32[nq], or NULL for k_max on every query
 *   k_max      1..MHR_WIDE_MAX_K
 *   out        device mhr_wide_path[nq][k_max], best first
 *   out_count  device uint32[nq]: min(k[q], |P(s,t)|)
 *   out_total  device uint64[nq] or NULL: |P(s,t)|
 *   out_status device uint32[nq] or NULL: MHR_Q_BAD_ID, MHR_Q_BAD_K
 *   out_work   device mhr_wide_work[nq] or NULL
 *   workspace  device buffer of ws_bytes >= mhr_wide_workspace_size(...)
 *   ev         phase events or NULL: begin before planning, gather_begin and
 *              gather_end around the tile kernel (after the frontier
 *              kernel), end after the merge
 * The call plans the batch, synchronises `stream` once to read the plan's
 * totals, then enqueues the search and returns.  Allocates nothing.
 * Errors: INVALID_ARGUMENT, NO_EMBEDDINGS, WORKSPACE_TOO_SMALL (nothing of
 * the search enqueued), UNSUPPORTED, DEVICE. */
mhr_status mhr_wide_topk_paths(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                               const uint32_t *k, uint32_t k_max, mhr_wide_path *out, uint32_t *out_count,
                               uint64_t *out_total, uint32_t *out_status, mhr_wide_work *out_work,
                               void *workspace, size_t ws_bytes, void *stream, const mhr_phase_events *ev);

/* ---------------------------------------------------------------------------
 * Learned frontier pruner.
 *
 * The generic search of section 5 bounds each level's frontier by a per-
 * parent top-K; here a small network ranks a query's frontier candidates
 * instead, so that cold ones are skipped, and the exact search stays as the
 * fallback and as the reference for its recall.  Candidates of a query (s, t):
 *   first hop   one per relation r1 of each entry a of s's out-row (edge s -r1-> a)
 *   second hop  one per relation r3 of each entry b of t's in-row  (edge b -r3-> t)
 * Network input f = [X[u], X[w], X[v], Y[r]]: v the candidate vertex (a or
 * b), r its edge's relation (r1 or r3), u the query endpoint that edge
 * touches (s for the first hop, t for the second) and w the other endpoint
 * (the same functional form for both hops: the DistMult weight is
 * symmetric).  A sample's query word carries the hop in bit 31
 * (MHR_PRUNER_HOP2).  Network:
 *   h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), z = w3 . h2 + b3, p = sigmoid(z)
 * with W1 [hidden][4 dim], W2 [hidden][hidden], w3 [hidden].  Parameters are
 * one flat FP32 vector: W1 (row-major), b1, W2 (row-major), b2, w3, b3.
 * Products use bfloat16 operands (features, W1, W2, w3, h1, h2 and the back-
 * propagated gradients rounded to nearest even) with FP32 accumulation; the
 * master weights and Adam state are FP32.
 * ------------------------------------------------------------------------- */
typedef struct mhr_pruner mhr_pruner;

#define MHR_PRUNER_HOP2 0x80000000u   /* second-hop flag in a sample's or candidate's query word */

/* Checkpoint of a pruner: parameters, Adam moments and step count, to
 * resume training or reuse a trained network.  Little-endian file: a 40-byte
 * header ("MHRPRUN1", format version, dim, hidden, step, parameter count,
 * CRC-32 of the payload, CRC-32 of the header) and the payload (FP32
 * parameters, first moments, second moments).  save synchronises `stream`
 * and writes the file atomically (temporary name, then rename).  load
 * checks the magic, version, sizes and both checksums before anything is
 * copied, requires the pruner's dim and hidden, restores the step count and
 * synchronises.  Errors: INVALID_ARGUMENT, IO, CORRUPT, UNSUPPORTED (another
 * format version), DEVICE. */
mhr_status mhr_pruner_save(const mhr_pruner *p, const char *path, void *stream);
mhr_status mhr_pruner_load(mhr_pruner *p, const char *path, void *stream);

/* Checks a pruner checkpoint on the host alone (no device needed) and
 * reports its dimensions and step count (each output may be NULL).
 * Errors: IO, CORRUPT, UNSUPPORTED. */
mhr_status mhr_pruner_file_info(const char *path, uint32_t *dim, uint32_t *hidden, uint32_t *step);

/* CRC-32 (IEEE 802.3 polynomial, reflected 0xEDB88320, the zlib / PNG
 * checksum) of n bytes, continuing from crc (0 to start). */
uint32_t mhr_crc32(uint32_t crc, const void *data, size_t n);

/* Number of parameters for embedding dimension dim and hidden width hidden. */
size_t mhr_pruner_param_count(uint32_t dim, uint32_t hidden);

/* dim: multiple of 8 in [8, 512] (the graph's embedding dimension);
 * hidden: multiple of 16 in [16, 4096].  Parameters start at zero (set them
 * with mhr_pruner_set_params).  Allocates device memory (hipMalloc). */
mhr_status mhr_pruner_create(uint32_t dim, uint32_t hidden, mhr_pruner **out);
mhr_status mhr_pruner_destroy(mhr_pruner *p);

/* Device bytes of a pruner's state for mhr_pruner_create_in: FP32 master
 * weights, gradient and both Adam moments (param_count each), and the
 * bfloat16 copies of the three weight matrices.  Host only.  Errors:
 * INVALID_ARGUMENT (dim or hidden outside the ranges of mhr_pruner_create). */
mhr_status mhr_pruner_buffer_bytes(uint32_t dim, uint32_t hidden, size_t *bytes);

/* mhr_pruner_create with its state in the caller's device buffer (256-byte
 * aligned, at least mhr_pruner_buffer_bytes): the library calls no
 * hipMalloc.  The buffer is BORROWED until mhr_pruner_destroy.  Zeroes the
 * state on `stream` and synchronises it.  Errors: INVALID_ARGUMENT,
 * WORKSPACE_TOO_SMALL (nothing enqueued), DEVICE. */
mhr_status mhr_pruner_create_in(uint32_t dim, uint32_t hidden, void *buffer, size_t bytes, void *stream,
                                mhr_pruner **out);

/* Copies params (device FP32 [param_count]) in and resets the Adam state. */
mhr_status mhr_pruner_set_params(mhr_pruner *p, const float *params, void *stream);

/* Copies the parameters and/or the gradient of the last training step out
 * (device FP32 [param_count] each; either may be NULL). */
mhr_status mhr_pruner_get_params(const mhr_pruner *p, float *params, float *grad, void *stream);

/* Device workspace bytes for forward or training calls on n samples. */
mhr_status mhr_pruner_workspace_size(const mhr_pruner *p, uint32_t n, size_t *bytes);

/* Logits z for n samples: sample i is the candidate (v[i], r[i]) of query
 * q[i] & ~MHR_PRUNER_HOP2 (a second-hop candidate when bit 31 is set), whose
 * endpoints are src[...], dst[...].  All device arrays; the
 * embeddings are the graph's (dimension must equal the pruner's). */
mhr_status mhr_pruner_forward(mhr_pruner *p, const mhr_graph *g, uint32_t n, const uint32_t *q,
                              const uint32_t *src, const uint32_t *dst, const uint32_t *v,
                              const uint32_t *r, float *logits, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes of mhr_pruner_score for nq queries of graph g, scoring
 * `chunk` candidates per pass (chunk >= 1, at most 8,388,480). */
mhr_status mhr_pruner_score_workspace_size(const mhr_pruner *p, const mhr_graph *g, uint32_t nq, uint32_t chunk,
                                           size_t *bytes);

/* Logits of ncand frontier candidates of a batch of nq queries (the network
 * that ranks the frontier in place of the per-parent top-K of the generic
 * search, section 5): candidate i is (v[i], r[i]) of query q[i] &
 * ~MHR_PRUNER_HOP2 (second hop when bit 31 is set), endpoints src[...],
 * dst[...].  The same network as mhr_pruner_forward, with the first layer
 * split by input block: the endpoints' part once per (query, hop), the
 * relation's part once per relation, the candidate's part per candidate,
 * then the second layer and the output fused into one product per chunk of
 * `chunk` candidates.  Requires q[i] & ~MHR_PRUNER_HOP2 < nq, v[i] <
 * num_vertices and r[i] < num_relations (the candidates of
 * mhr_pruner_enumerate do); an out-of-range v reads as a zero row and an
 * out-of-range q or r gives a NaN logit.  Asynchronous on `stream`.
 * Errors: INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, DEVICE. */
mhr_status mhr_pruner_score(mhr_pruner *p, const mhr_graph *g, uint32_t nq, const uint32_t *src,
                            const uint32_t *dst, uint64_t ncand, const uint32_t *q, const uint32_t *v,
                            const uint32_t *r, float *logits, uint32_t chunk, void *ws, size_t ws_bytes,
                            void *stream);

/* One training step on n labelled samples (label: device FP32 0/1 [n]):
 * forward, the mean binary cross-entropy with positive-class weight
 * pos_weight (written to *loss, device, if not NULL), the gradient (kept in
 * the pruner, see get_params), and, if update != 0, one Adam step with
 * learning rate lr (bias-corrected, step count kept in the pruner). */
mhr_status mhr_pruner_train_step(mhr_pruner *p, const mhr_graph *g, uint32_t n, const uint32_t *q,
                                 const uint32_t *src, const uint32_t *dst, const uint32_t *v,
                                 const uint32_t *r, const float *label, float pos_weight, float lr,
                                 float beta1, float beta2, float eps, int update, float *loss,
                                 void *ws, size_t ws_bytes, void *stream);

/* A whole training run on nq training queries (src, dst: device uint32[nq]),
 * the sequence of the calls above:
 *   per epoch, the queries in a shuffled order (SplitMix64-driven
 *   Fisher-Yates from seed), in batches of batch_queries; per batch the
 *   exact top-k labels the candidates (mhr_topk_paths, mhr_pruner_count /
 *   enumerate / label), every positive and about neg_per_hop negatives per
 *   hop and query are sampled (mhr_pruner_sample), and the network takes
 *   Adam steps of step_samples samples each with a positive weight of
 *   negatives / positives (mhr_pruner_train_step).
 * The loss of each step is written to losses[0 .. min(steps, max_losses))
 * (host), the step count to *nsteps (host).  Allocates its device buffers
 * (hipMalloc) and frees them before returning; synchronises `stream` once or
 * twice per batch to size them.  Zero option fields take the defaults in
 * the comments; reserved fields must be zero.  Errors: those of the calls
 * above, INVALID_ARGUMENT, DEVICE. */
typedef struct mhr_train_opts {
    uint32_t k;              /* K of the labelling search (1 .. MHR_MAX_K), e.g. 32 */
    uint32_t batch_queries;  /* 0 = 4096 */
    uint32_t step_samples;   /* 0 = 65536 */
    uint32_t epochs;         /* 0 = 1 */
    uint32_t neg_per_hop;    /* 0 = 64 */
    float lr, beta1, beta2, eps;   /* 0 = 1e-3, 0.9, 0.999, 1e-8 */
    uint32_t pad;
    uint64_t seed;
    uint32_t reserved[8];
} mhr_train_opts;

mhr_status mhr_pruner_train(mhr_pruner *p, const mhr_graph *g, const mhr_train_opts *opts, uint32_t nq,
                            const uint32_t *src, const uint32_t *dst, float *losses, uint32_t max_losses,
                            uint32_t *nsteps, void *stream);

/* Candidate bookkeeping for nq queries (device arrays).  entry_off and
 * cand_off receive [nq + 1] exclusive offsets: entries are the keep-flag
 * layout of mhr_topk_paths_pruned (deg+(s) then deg-(t) per query), cand_off
 * the candidates (relations summed over those entries); [nq] holds the
 * totals.  A query with an id out of range has none. */
mhr_status mhr_pruner_count(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                            uint64_t *entry_off, uint64_t *cand_off, void *stream);

/* Writes the candidates: query word (the query index, | MHR_PRUNER_HOP2 for
 * second-hop candidates), vertex, relation and keep-flag index of each
 * (first-hop ones of a query first, in CSR order and ascending relation),
 * and cand_split[q], the index of the query's first second-hop candidate.
 * Output arrays hold cand_off[nq] elements. */
mhr_status mhr_pruner_enumerate(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                const uint64_t *entry_off, const uint64_t *cand_off, uint64_t *cand_split,
                                uint32_t *cand_q, uint32_t *cand_v, uint32_t *cand_r, uint64_t *cand_e,
                                void *stream);

/* Per query and hop, keeps the ceil(n * keep_permille / 1000) of the hop's
 * n entries (vertices) with the best entry score, an entry's score being
 * the highest score of its candidates (and every entry tied with the lowest
 * kept one).  Writes the keep flags (all entries of the query, see
 * mhr_topk_paths_pruned) and, if mass is not NULL, mass[2q + hop] = the
 * share of sum(sigmoid(score)) held by the candidates of kept entries (1
 * when the hop has none).  Scores may be logits or any other ranking (NaN
 * ranks lowest).  ncand = cand_off[nq], nentries = entry_off[nq] (host
 * values); entry_key: device workspace of nentries uint32. */
mhr_status mhr_pruner_select(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                             const uint64_t *entry_off, const uint64_t *cand_off,
                             const uint64_t *cand_split, const float *score, const uint64_t *cand_e,
                             uint64_t ncand, uint64_t nentries, uint32_t keep_permille, uint8_t *keep,
                             float *mass, uint32_t *entry_key, void *stream);

/* Training labels: pos[e] = 1 for the entries e (keep-flag layout) whose
 * vertex is the a (first-hop entry) or the b (second-hop entry) of one of the
 * query's paths paths[q][0 .. count[q]) (e.g. the exact top-K), else 0. */
mhr_status mhr_pruner_label(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                            const uint64_t *entry_off, const mhr_path *paths, const uint32_t *count,
                            uint32_t kmax, uint8_t *pos, void *stream);

/* Device workspace bytes of mhr_pruner_sample. */
size_t mhr_pruner_sample_workspace(uint32_t nq, uint64_t ncand);

/* Training samples from the candidates: every positive candidate (pos of
 * its entry) and each negative with probability min(1, neg_per_hop / the
 * negatives of its query and hop), drawn from a counter-based generator
 * (SplitMix64 of seed and the candidate index).  Writes, in candidate order,
 * the samples' query, vertex, relation and label (0/1) into arrays of
 * capacity ncand, and their number to *nsamples (device). */
mhr_status mhr_pruner_sample(uint32_t nq, const uint64_t *cand_off, const uint64_t *cand_split,
                             uint64_t ncand, const uint32_t *cand_q, const uint32_t *cand_v,
                             const uint32_t *cand_r, const uint64_t *cand_e, const uint8_t *pos,
                             uint32_t neg_per_hop, uint64_t seed, uint32_t *sq, uint32_t *sv,
                             uint32_t *sr, float *slabel, uint64_t *nsamples, void *ws, size_t ws_bytes,
                             void *stream);

/* Confidence test of a pruned search: the queries (status 0) whose pruned
 * result has fewer than k paths, or whose kept share of the predicted mass
 * (mass[2q], mass[2q + 1] from mhr_pruner_select) is below tau at either
 * hop, are compacted in order into fb_src / fb_dst / fb_k / fb_idx (the
 * original index), their number in *nfb (device).  k may be NULL (kdef). */
mhr_status mhr_pruner_fallback(uint32_t nq, const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                               uint32_t kdef, const uint32_t *count, const uint32_t *status,
                               const float *mass, float tau, uint32_t *fb_src, uint32_t *fb_dst,
                               uint32_t *fb_k, uint32_t *fb_idx, uint32_t *nfb, void *stream);

/* The weight of each candidate's own edge under the graph's scorer, in FP32
 * as the search's fast pass evaluates it: s -r-> v for a first-hop
 * candidate of query q, v -r-> t for a second-hop one (query words with
 * MHR_PRUNER_HOP2, as mhr_pruner_enumerate writes them).  This is the
 * ranking a per-level score beam keeps (the paper's generic search bounds
 * each level by the best partial scores, section 5): the pruner's
 * no-network baseline.  Device arrays of ncand entries. */
mhr_status mhr_pruner_candidate_weights(const mhr_graph *g, uint64_t ncand, const uint32_t *src,
                                        const uint32_t *dst, const uint32_t *cand_q, const uint32_t *cand_v,
                                        const uint32_t *cand_r, float *w, void *stream);

/* Copies result row i of a compact batch (paths[i][0..kmax), count, total,
 * status) to row idx[i] of a full batch, for i < n (host count). */
mhr_status mhr_scatter_results(uint32_t n, const uint32_t *idx, uint32_t kmax, const mhr_path *src_paths,
                               const uint32_t *src_count, const uint64_t *src_total,
                               const uint32_t *src_status, mhr_path *paths, uint32_t *count,
                               uint64_t *total, uint32_t *status, void *stream);

/* Edge-weight kernel on its own (for checking the scorer):
 * for each i < ne, the edge (u[i], r[i], v[i]) (it need not exist in the
 * graph): w_f32[i] = the graph's scorer evaluated in FP32 as the fast pass
 * does it and err_f32[i] a rigorous bound on its error; w_hi[i] + w_lo[i] =
 * the compensated (float-float) value.  Any output pointer may be NULL.
 * Device arrays. */
mhr_status mhr_edge_weights(const mhr_graph *g, uint64_t ne, const uint32_t *u,
                            const uint32_t *r, const uint32_t *v, float *w_f32,
                            float *err_f32, float *w_hi, float *w_lo, void *stream);

/* ---------------------------------------------------------------------------
 * Generic multi-hop search (section 5, the generic algorithm and its path
 * expansion): a beam search of up to `hops` edges, the per-parent top-K of
 * the paper's level-by-level frontier.  Unlike mhr_topk_paths it is not
 * exact over all paths: it keeps K children per path and level.
 * ------------------------------------------------------------------------- */
#define MHR_BEAM_MAX_HOPS 4

/* One recorded path s -r[0]-> v[0] -r[1]-> ... -> v[len-1] = t (40 bytes);
 * unused slots hold len 0, vertices 0xFFFFFFFF and score -inf. */
typedef struct mhr_beam_path {
    double score;                     /* the edge weights summed along the path, FP64 */
    uint32_t len;                     /* edges, 1 .. hops */
    uint32_t v[MHR_BEAM_MAX_HOPS];
    uint16_t r[MHR_BEAM_MAX_HOPS];
} mhr_beam_path;

/* Workspace bytes of mhr_beam_search (it grows as nq * k^(hops-1)). */
mhr_status mhr_beam_workspace_size(const mhr_graph *g, uint32_t nq, uint32_t hops, uint32_t k, size_t *bytes);

/* For each query (src[q], dst[q]): start from the path holding s alone; at
 * each of `hops` levels every current path grows by each typed out-edge
 * (h, r, nb) of its last vertex h whose head nb is not on the path yet, its
 * score plus w(h, r, nb) (the graph's scorer, FP64); an extension reaching t
 * is recorded and not grown further; of the others each parent passes its
 * best k (score descending, then nb, then r ascending) to the next level.
 * out[q][0 .. out_count[q]) holds the best k recorded paths (score
 * descending, then the vertex sequence lexicographically with a proper
 * prefix first, then the relation sequence); out_recorded[q] (may be NULL)
 * the number recorded.  hops 1..MHR_BEAM_MAX_HOPS, k 1..64, k^(hops-1) <=
 * 2^20.  Asynchronous on `stream` (one launch per level); allocates
 * nothing.  Errors: INVALID_ARGUMENT, NO_EMBEDDINGS, WORKSPACE_TOO_SMALL,
 * DEVICE. */
mhr_status mhr_beam_search(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                           uint32_t hops, uint32_t k, mhr_beam_path *out, uint32_t *out_count,
                           uint64_t *out_recorded, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Candidate scan: the workload of the paper's three-hop award pipeline
 * (section 3.2, the simple algorithm's three scoring steps; section 3.3,
 * the person, field and affiliation scoring with the TransE-L1 score).
 * These calls take the embedding tables directly (no graph handle): the
 * pipeline scores lists of candidate entities, not graph paths.
 * ------------------------------------------------------------------------- */

/* Device workspace bytes of mhr_scan_topk for nq queries over lists of ncand
 * candidates with K = k. */
mhr_status mhr_scan_workspace_size(uint32_t nq, uint32_t ncand, uint32_t k, size_t *bytes);

/* For each query q, the TransE-L1 score of every candidate c of its list,
 *     score = gamma - sum_i |(X[head[q], i] + Y[rel[q], i]) - X[c, i]|
 * (c as the tail), evaluated in FP64 (head plus relation, minus the
 * candidate, summed in ascending i), and the best min(k, list length)
 * candidates under (score descending, id ascending).
 *   entity, relation  device tables [num_entities][dim], [num_relations][dim]
 *                     of dtype, 16-byte aligned; dim a multiple of 8 <= 512
 *   head              device uint32[nq]
 *   rel               device uint32[nq], or NULL: rel_default for every query
 *   cand              device uint32 lists: query q's list is cand + q *
 *                     cand_stride, ncand entries (cand_stride = 0: one list
 *                     shared by all queries).  0xFFFFFFFF entries are absent
 *                     and skipped; other ids >= num_entities are skipped and
 *                     flagged.
 *   k                 1..256
 *   out_id, out_score device [nq][k]: best first; unused slots 0xFFFFFFFF / -inf
 *   out_status        device uint32[nq] or NULL: MHR_Q_BAD_ID when head or rel
 *                     is out of range (no result) or a candidate id was
 * Asynchronous on `stream`; allocates nothing.  Errors: INVALID_ARGUMENT,
 * WORKSPACE_TOO_SMALL, DEVICE. */
mhr_status mhr_scan_topk(mhr_dtype dtype, uint32_t dim, const void *entity, const void *relation,
                         uint32_t num_entities, uint32_t num_relations, uint32_t nq, const uint32_t *head,
                         const uint32_t *rel, uint32_t rel_default, const uint32_t *cand, uint32_t ncand,
                         uint32_t cand_stride, uint32_t k, float gamma, uint32_t *out_id, double *out_score,
                         uint32_t *out_status, void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes of mhr_scan_pipeline. */
mhr_status mhr_scan_pipeline_workspace_size(uint32_t npipe, uint32_t npersons, uint32_t nuniv, uint32_t k,
                                            size_t *bytes);

/* npipe independent runs of the three-hop pipeline, all on `stream` with no
 * host synchronisation (each hop's device output feeds the next):
 *   hop 1  every person p of `persons` scored against award[j] + r_award;
 *          the best k -> hop1_id/score[j][k];
 *   hop 2  those k persons scored against field[j] + r_works and ranked by
 *          it -> hop2_id/score[j][k];
 *   hop 3  for each ranked person p (in rank order) every university of
 *          `universities` scored against p + r_affil; the best k ->
 *          hop3_id/score[j][rank][k].
 * award, field: device uint32[npipe]; persons, universities: device lists.
 * Errors as mhr_scan_topk. */
mhr_status mhr_scan_pipeline(mhr_dtype dtype, uint32_t dim, const void *entity, const void *relation,
                             uint32_t num_entities, uint32_t num_relations, uint32_t npipe, const uint32_t *award,
                             const uint32_t *field, uint32_t r_award, uint32_t r_works, uint32_t r_affil,
                             const uint32_t *persons, uint32_t npersons, const uint32_t *universities,
                             uint32_t nuniv, uint32_t k, float gamma, uint32_t *hop1_id, double *hop1_score,
                             uint32_t *hop2_id, double *hop2_score, uint32_t *hop3_id, double *hop3_score,
                             void *workspace, size_t ws_bytes, void *stream);

/* Profiling aid: the gather kernel's per-phase wall-clock ticks, summed over
 * its workgroups since the last reset, and its work counts, for each of two
 * tile kinds (probe side in the LDS table; probing through the row
 * directory).  out (host, n >= 42) receives per kind 11 phase sums (tile
 * fetch, setup, list rows, probe, sub-batch formation, scoring,
 * log-sigmoids, bounds, enumeration, stage merges, tile end) then 10 counts
 * (tiles, row batches, chunks, scanned entries, sub-batches, matches, edge
 * values, enumeration items, staged candidates, stage merges).  *rate_hz:
 * the clock rate.  Recorded only by the library's phase-clock build
 * (paper_2406_07727_amd/build.py --phase-clocks); the regular build returns
 * MHR_ERR_UNSUPPORTED.  Synchronises the device. */
mhr_status mhr_debug_phase_ticks(uint64_t *out, uint32_t n, double *rate_hz, int reset);

const char *mhr_status_string(mhr_status s);
const char *mhr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MHR_H */
