/*
 * steiner.h -- C ABI of the MI355X (gfx950) Voronoi-cell 2-approximation
 * Steiner tree library.
 *
 * The method is the one of Reza, Sanders and Pearce, "Towards Distributed
 * 2-Approximation Steiner Minimal Trees in Billion-edge Graphs"
 * (arXiv:2205.14503), Alg. 2: Voronoi cells of the seeds (Step 1), the
 * distance graph G'1 of minimum cross-cell edges (Step 2, Mehlhorn's
 * construction, Section II), its MST (Step 3), pruning to the MST's cross-cell
 * edges (Step 4), predecessor walks to the seeds (Steps 5-6) and the total
 * distance D (Step 7).
 *
 * Conventions shared by every entry point
 *  - Every call returns an int: STEINER_OK (0) or a negative STEINER_E* code.
 *    Output parameters are written only on success.  steiner_last_error()
 *    returns a thread-local string describing the most recent failure.
 *  - Graphs are undirected, given as a symmetric CSR: row_ptr[n+1] (uint64),
 *    col[nnz] and w[nnz] (uint32).  Rows must be sorted by column.  Weights
 *    must be >= 1 (Table II: distances are positive integers).  Self-loops are
 *    accepted and never used; parallel edges are accepted.  nnz must be below
 *    2^32 because an edge is identified by its CSR offset.
 *  - Seeds are vertex ids < n; duplicates are ignored.  Seed index i is the
 *    rank of a seed in the sorted, deduplicated seed list.  A query holds at
 *    most STEINER_MAX_SEEDS distinct seeds, so that the k(k-1)/2 cell pairs
 *    of G'1 have 32-bit indices.
 *  - Results are exact and unique under these tie rules (the paper leaves
 *    ties open): a vertex joins the cell minimising (distance, seed index);
 *    pred(v) is the smallest in-cell neighbour on a shortest path (then the
 *    smallest CSR offset); each cell pair keeps the cross-cell edge minimising
 *    (d1(s,u)+d(u,v)+d1(v,t), edge id), the edge id being the CSR offset of the
 *    half edge leaving the smaller endpoint; the MST of G'1 is the unique one
 *    under the order (d'1, i, j).  No option changes any result.
 *  - EOVERFLOW: some finite distance is >= 2^32-1, or some cross-cell sum
 *    d1+d+d1 is >= 2^32.  EDISCONNECTED: the seeds do not lie in one
 *    connected component.  k == 1 after deduplication gives an empty tree,
 *    D = 0, without running any kernel.
 *  - All device work of a graph runs on the HIP stream given at upload and
 *    on the device given at upload.  Calls on one graph are serialised by the
 *    library; distinct graphs are independent.
 */
#ifndef STEINER_H
#define STEINER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    STEINER_OK = 0,
    STEINER_EINVAL = -1,        /* malformed graph, seeds, sizes or options */
    STEINER_ENOMEM = -2,        /* device or host allocation failed, or a caller buffer is too small */
    STEINER_EDISCONNECTED = -3, /* seeds span more than one connected component */
    STEINER_EOVERFLOW = -4,     /* a distance or cross-cell sum does not fit (see above) */
    STEINER_EDEVICE = -5,       /* a HIP call failed */
    STEINER_ETIMEDOUT = -6,     /* steiner_server_wait ran out of time */
    STEINER_ECANCELED = -7      /* the server was destroyed before the request finished */
};

#define STEINER_MAX_SEEDS 92682u

typedef struct steiner_graph steiner_graph;   /* device-resident CSR; owned by the library */
typedef struct steiner_result steiner_result; /* host arrays of one tree; freed by steiner_result_free */
typedef struct steiner_server steiner_server; /* continuous-batching query server over one graph */

/* Execution knobs.  Pass NULL for defaults.  None of them changes any result. */
typedef struct steiner_options {
    uint32_t delta;       /* bucket width of the distance-ordered relaxation; 0 = default for the graph,
                             0xFFFFFFFF = one unbounded bucket (plain label correcting) */
    uint32_t driver;      /* 0 = default, 1 = host-stepped rounds, 2 = one persistent cooperative kernel,
                             3 = cluster-local relaxation in LDS (single queries; batches use 1),
                             4 = host-stepped rounds replayed as HIP graphs of 8 launches (built once per
                             graph and pass shape; the server replays its 4-round chunks) */
    uint32_t block;       /* threads per workgroup (multiple of 64, <= 1024); 0 = default */
    uint32_t grid;        /* workgroups of the relaxation pass; 0 = default */
    uint32_t small_max;   /* rows up to this degree are expanded wave-cooperatively; 0 = default */
    uint32_t chunk;       /* larger rows are split into chunks of this many edges; 0 = default */
    uint32_t flags;       /* STEINER_FLAG_* */
    uint32_t local_iters; /* batches of 64 improved vertices a wave expands itself before deferring the rest
                             to the next round; 0 = default, 0xFFFFFFFF = none */
} steiner_options;

#define STEINER_FLAG_TIMING 1u   /* record per-phase device times (adds synchronisation) */
#define STEINER_FLAG_COUNTERS 2u /* count relaxation events on the device (the analogue of the
                                    paper's per-phase message counts, Fig. 6) */
#define STEINER_FLAG_SPLIT 4u    /* within a bucket relax edges of weight <= delta first and the
                                    heavier ones once per settled vertex (Delta-stepping's
                                    light/heavy split); no effect with an unbounded bucket */
#define STEINER_FLAG_LAZY_PRED 8u  /* the boundary scan gathers each edge's far key once and the tree
                                      walks find the preds of ordinary rows (dense graphs) */
#define STEINER_FLAG_EAGER_PRED 16u /* the boundary scan also finds every pred (sparse, high-diameter
                                       graphs); without either flag the graph's default applies */
#define STEINER_FLAG_DEFER 32u    /* a row of more than small_max entries whose distance improves inside the
                                     open bucket is expanded once, when the bucket advances, instead of in the
                                     next round (fewer re-expansions of hubs); ignored with the split */
#define STEINER_FLAG_NO_DEFER 64u /* expand such rows in the next round; without either flag the graph's
                                     default applies (deferral on degree-renumbered graphs) */

/* Per-solve statistics (filled for steiner_solve / steiner_solve_batch results). */
typedef struct steiner_stats {
    uint32_t rounds;          /* relaxation rounds executed */
    uint32_t advances;        /* bucket advances (summed over queries) */
    uint32_t pairs;           /* entries of G'1 (cell pairs joined by a cross-cell edge) */
    uint32_t tree_edges;      /* |E_S| */
    uint32_t relax_launches;  /* kernel launches of the relaxation pass */
    uint32_t reserved;
    /* Phase times in ms.  With STEINER_FLAG_TIMING the device phases come from
     * HIP events on the graph's stream and ms_relax_kernels is the summed
     * duration of the relaxation kernels alone (event pair per launch);
     * otherwise only ms_total (host wall clock) is set. */
    double ms_init, ms_voronoi, ms_scan, ms_compact, ms_mst, ms_expand, ms_total, ms_relax_kernels;
    /* With STEINER_FLAG_COUNTERS, summed over the pass (all queries of a
     * batch): edges relaxed, atomicMins issued after the stale-value filter,
     * keys improved, improved vertices expanded by the same wave, vertices
     * moved to the next round's list, vertices parked beyond their bucket,
     * frontier items expanded. */
    uint64_t relax_attempts, relax_atomics, relax_improved, pushes_local, pushes_next, parked, items;
    /* With STEINER_FLAG_COUNTERS, the boundary scan (Step 2): CSR entries
     * read, neighbour keys gathered, cross-cell candidates (each reads its
     * pair's current entry), atomicMins issued on the pair table. */
    uint64_t scan_entries, scan_gathers, scan_candidates, scan_atomics;
    /* With STEINER_FLAG_COUNTERS: the relaxation attempts made from chunks of
     * rows above small_max (part of relax_attempts). */
    uint64_t relax_attempts_large;
} steiner_stats;

/* Upload flags. */
#define STEINER_UPLOAD_SYMMETRY 1u   /* also verify that the CSR is symmetric (O(nnz)) */
#define STEINER_UPLOAD_REORDER 2u    /* renumber the vertices internally (see below) */
#define STEINER_UPLOAD_KEEP_ORDER 4u /* never renumber */

/* Upload a graph from HOST arrays (copied; the caller keeps ownership).
 * device: HIP device ordinal.  hip_stream: a hipStream_t on that device, or
 * NULL for the null stream.  flags: STEINER_UPLOAD_*.
 * Internal order: on a skewed graph (maximum degree at least 32 times the
 * mean) or with STEINER_UPLOAD_REORDER, and never with
 * STEINER_UPLOAD_KEEP_ORDER, the library renumbers the vertices by descending
 * degree and sorts each row by the new ids, which puts the keys that most
 * gathers read on few cache lines.  Every input and output stays in the
 * caller's ids and every result is unchanged: the tie rules are evaluated on
 * the caller's ids and CSR offsets.  Cost: 8 more device bytes per entry and
 * per vertex, and host work at upload (a sort per row).
 * Device memory held: 4 B per vertex and 8 B per entry (the CSR), and, when
 * every row has at most 4 entries (a grid), 32 B more per vertex for a
 * fixed-stride copy of the rows that the Voronoi pass reads instead.
 * EINVAL for n == 0, non-monotone row_ptr, row_ptr[0] != 0, row_ptr[n] != nnz,
 * nnz >= 2^32, col >= n, w == 0, unsorted rows, (STEINER_UPLOAD_SYMMETRY)
 * asymmetry, or both order flags. */
int steiner_graph_upload(uint32_t n, uint64_t nnz, const uint64_t *row_ptr, const uint32_t *col,
                         const uint32_t *w, int device, void *hip_stream, uint32_t flags, steiner_graph **out);

/* Same, from DEVICE arrays on `device` (e.g. torch tensors); the library copies
 * them into its own layout and validates them on the device. */
int steiner_graph_upload_device(uint32_t n, uint64_t nnz, const void *d_row_ptr, const void *d_col,
                                const void *d_w, int device, void *hip_stream, uint32_t flags,
                                steiner_graph **out);

int steiner_graph_free(steiner_graph *g);

/* Autotuner: times a small set of relaxation settings (bucket width with and
 * without the deferred expansion of large rows, depth of the wave-local queue,
 * the light/heavy split, the pred placement, workgroups of a host-stepped pass)
 * on the given sample seed set and keeps the fastest as this graph's defaults
 * for every later call that passes NULL options or zero fields.  Results never
 * depend on the choice.  out (optional) receives the chosen settings (the
 * split, pred and deferral choices as STEINER_FLAG_* bits).  EINVAL for fewer
 * than 2 distinct seeds. */
int steiner_graph_tune(steiner_graph *g, const uint32_t *seeds, uint32_t k, steiner_options *out);

/* Alg. 2 end to end for one seed set (host array of k vertex ids). */
int steiner_solve(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                  steiner_result **out);

/* q seed sets solved in one multi-query pass over the shared graph.
 * seeds[i] points to ks[i] host vertex ids.  outs[i] receives a result when
 * status[i] == STEINER_OK.  Returns STEINER_OK if the pass itself ran (check
 * status[] per query), or an error for the whole call. */
int steiner_solve_batch(steiner_graph *g, uint32_t q, const uint32_t *const *seeds, const uint32_t *ks,
                        const steiner_options *opt, steiner_result **outs, int *status);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): steiner_solve
 * without any device or pinned-host allocation and without creating streams
 * or events.  Same kernels and the same result as steiner_solve with the same
 * options (the relaxation is always host-stepped).  Every device buffer comes
 * from one library-wide array of STEINER_NOALLOC_SCRATCH_BYTES on each device,
 * which the library sets aside when it is loaded on that device and holds
 * until the process ends; a solve that needs more (vertex state, frontier
 * lists, pair table, tree scratch: about 80 B per vertex plus 8 B per seed
 * pair) returns ENOMEM, and so do more than 8192 seeds (duplicates
 * included).  The tree goes to the caller's HOST arrays a, b, w of capacity
 * cap (sorted by (a, b, w)), its size to *m and D to *total; ENOMEM with *m
 * set if cap is too small.  Calls in one process run one at a time (the array
 * keeps the last call's contents; each call re-initialises what it reads);
 * calls that overlapped on one GPU would race on the array.  The host thread
 * waits for the solve to finish. */
#define STEINER_NOALLOC_SCRATCH_BYTES (256ull << 20)
int steiner_solve_noalloc(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                          uint64_t cap, uint64_t *m, uint32_t *a, uint32_t *b, uint32_t *w, uint64_t *total);

/* Tree edges (a < b, sorted by (a, b, w)); pointers stay valid until
 * steiner_result_free. */
int steiner_result_edges(const steiner_result *r, uint64_t *m, const uint32_t **a, const uint32_t **b,
                         const uint32_t **w);
uint64_t steiner_result_total(const steiner_result *r); /* D(G_S) */
int steiner_result_stats(const steiner_result *r, steiner_stats *out);
void steiner_result_free(steiner_result *r);

/* Step 1 only: key_out[v] = (d1(src(v), v) << 32) | seed index, all ones when
 * unreached; pred_out[v] = canonical predecessor (seed: itself; unreached:
 * 0xFFFFFFFF).  Host arrays of n entries.  k must be >= 2 after deduplication. */
int steiner_voronoi(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                    uint64_t *key_out, uint32_t *pred_out);

/* Steps 1-2: the entries of G'1 sorted by (i, j): pi < pj are seed indices,
 * packed = (d'1 << 32) | edge id.  cap is the capacity of the host arrays;
 * *npairs receives the count (ENOMEM if cap is too small, with *npairs set). */
int steiner_boundary(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                     uint64_t *npairs, uint32_t *pi, uint32_t *pj, uint64_t *packed, uint64_t cap);

/* Serving: a request loop over a resident graph.  Requests are admitted
 * first come first served while a slot is free and their pool region fits
 * the free pool, are spliced into the running multi-query pass between
 * relaxation rounds, and their tails run as soon as their own cells converge.
 * Everything the server allocates on the device fits mem_budget_bytes (see
 * steiner_server_memory); EINVAL if the budget cannot hold one slot and one
 * smallest request. */
int steiner_server_create(steiner_graph *g, uint64_t mem_budget_bytes, uint32_t max_slots,
                          const steiner_options *opt, steiner_server **out);
int steiner_server_submit(steiner_server *s, const uint32_t *seeds, uint32_t k, uint64_t *ticket);
/* timeout_us < 0 waits forever.  ETIMEDOUT leaves the request pending (wait
 * again later).  ECANCELED if the server is destroyed first.  Each ticket is
 * consumed by the wait that returns its result or its error. */
int steiner_server_wait(steiner_server *s, uint64_t ticket, int64_t timeout_us, steiner_result **out);
/* Device memory of a request with k seeds: its slot's share (vertex state and
 * frontier lists) plus its pool region (pair table, G'1 indices, MST scratch,
 * seeds).  Submit refuses (ENOMEM) a request whose pool region exceeds the
 * whole pool. */
uint64_t steiner_server_query_bytes(const steiner_server *s, uint32_t k);
/* How the budget is split (any pointer may be NULL): fixed_bytes (control
 * region, tree output, vertex marks) + slots * slot_bytes + pool_bytes equals
 * mem_budget_bytes, and is everything the server holds on the device.  slots
 * is max_slots, or fewer if the budget cannot hold that many slots and one
 * smallest request each. */
int steiner_server_memory(const steiner_server *s, uint64_t *fixed_bytes, uint64_t *slot_bytes, uint32_t *slots,
                          uint64_t *pool_bytes);
/* Stops the server; requests not yet finished are canceled.  A thread blocked
 * in steiner_server_wait at that moment returns STEINER_ECANCELED, and destroy
 * returns after it has left.  No call on this server may start once destroy
 * has begun. */
int steiner_server_destroy(steiner_server *s);

const char *steiner_strerror(int code);
const char *steiner_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STEINER_H */
