// Host-side engine internals (not part of the public ABI).
#pragma once
#include <memory>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/steiner.h"
#include "kernels.h"

namespace stn {

int fail(int code, const char *fmt, ...);
int dev_alloc(void **p, size_t bytes);
// Error-path testing: every device or pinned-host allocation after the next n
// fails with STEINER_ENOMEM (n < 0: off); resets the allocation count.
void set_fault_alloc_after(long n);
long alloc_calls();
void dev_free(void *p);
int hip_check(hipError_t e, const char *what);

// Grow-only device buffer.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want, bool exact = false);  // exact: no growth headroom
    void release();
    template <typename T>
    T *as() const { return (T *)ptr; }
};

// Grow-only pinned host buffer.
struct HostPinned {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
    void release();
    template <typename T>
    T *as() const { return (T *)ptr; }
};

struct Options {
    uint32_t delta, driver, block, grid, small_max, chunk, local_iters, lq_mode;
    uint32_t defer_min;   // improved rows above this many entries are expanded at the bucket's advance (0: never)
    uint32_t grid_tuned;  // relaxation workgroups of a host-stepped pass (the tuned count unless given)
    bool timing, counting, split;
    bool lazy_pred;  // pred of ordinary rows found by the tree walks instead of the scan
};

// Device buffers of Alg. 2 Steps 3-7 for one query at a time: the MST's
// lists and per-seed arrays, the expansion's vertex marks (kept all zero
// between calls) and its output edges.
struct TailScratch {
    DevBuf mst, mark, out;
    HostPinned host;
    uint32_t mark_n = 0;  // mark holds this many zero bytes
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    // own_mst: the MST scratch lives in `mst` (else the caller passes a region of mst_scratch_bytes)
    int prepare(uint32_t n, uint32_t k, uint64_t m, bool own_mst, hipStream_t st);
    void release();
};

// An instantiated graph of consecutive round-kernel launches (the graph-captured driver), rebuilt when the
// pass parameters, launch shape or length change.
struct RoundGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> key;  // VorParams bytes, grid, block, rounds
    int get(const VorParams &P, uint32_t grid, uint32_t block, uint32_t rounds, hipGraphExec_t *out);
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key.clear();
    }
};

// Device workspace of a multi-query pass, reused across solves of a graph.
struct Workspace {
    DevBuf key, aux, dirty, settled, items_s[2], items_b[2], ctl, heavy_pe, seeds, pt, cidx, cval, ptrs, xkey;
    HostPinned host;
    TailScratch tail;
    RoundGraph rgraph;
    std::vector<hipEvent_t> events;  // timing mode: reused event pool
    void release() {
        DevBuf *all[] = {&key, &aux, &dirty, &settled, &items_s[0], &items_s[1], &items_b[0], &items_b[1], &ctl, &heavy_pe,
                         &seeds, &pt, &cidx, &cval, &ptrs, &xkey};
        for (DevBuf *b : all) b->release();
        host.release();
        tail.release();
        rgraph.release();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        events.clear();
    }
};
// Rounds per launch of the graph-captured driver.
constexpr uint32_t GRAPH_ROUNDS = 8;

enum StopAfter { STOP_NEVER = 0, STOP_AFTER_SCAN = 1, STOP_AFTER_COMPACT = 2 };

// Offsets of the per-pass control region (counters, pass control, per-slot
// arrays) for Q slots; every array starts on a 256-byte boundary.
struct Layout {
    size_t counters, pass, thr, thr_prev, pt_ptr, pt_len, oidx_ptr, oval_ptr, ocap, tr_ptr, ts_ptr, far_min, near_mark,
        settle_mark,
        carry, active,
        adv, done, advances, slot_err, out_cnt, slot_ids, total;
    explicit Layout(uint32_t Q) {
        size_t o = 0;
        auto take = [&](size_t bytes) {
            size_t at = o;
            o += (bytes + 255) & ~(size_t)255;
            return at;
        };
        counters = take(sizeof(Counters));
        pass = take(sizeof(PassCtl));
        thr = take(8ull * Q);
        thr_prev = take(8ull * Q);
        pt_ptr = take(8ull * Q);
        pt_len = take(8ull * Q);
        oidx_ptr = take(8ull * Q);
        oval_ptr = take(8ull * Q);
        ocap = take(8ull * Q);
        tr_ptr = take(8ull * Q);
        ts_ptr = take(8ull * Q);
        far_min = take(12ull * Q);
        near_mark = take(12ull * Q);
        settle_mark = take(12ull * Q);
        carry = take(4ull * Q);
        active = take(4ull * Q);
        adv = take(4ull * Q);
        done = take(4ull * Q);
        advances = take(4ull * Q);
        slot_err = take(4ull * Q);
        out_cnt = take(4ull * Q);
        slot_ids = take(4ull * Q);
        total = o;
    }
};


// VorParams of a pass whose control region starts at `ctl` (layout L).
void bind_pass(VorParams &P, const DevGraph &dg, uint8_t *ctl, const Layout &L, uint32_t Q);


}  // namespace stn

struct steiner_result {
    std::vector<uint32_t> a, b, w;
    uint64_t total = 0;
    steiner_stats stats{};
};

namespace stn {
// Chunk numbering of the rows above small_max for the relaxation's chunk memory (VorParams::xkey): built
// when those rows are the vertices below nxrow (a degree-renumbered graph).
struct ChunkTable {
    DevBuf start;  // [nxrow + 1] first chunk number of each row
    uint32_t nxrow = 0, xchunks = 0;
};
// BFS-grown vertex clusters of the cluster-local driver (built on first use).
struct ClusterSet {
    bool built = false;
    uint32_t nclusters = 0;
    DevBuf members, cstart, cl_of, irp, erp, ie, ee, expanded, lists, stamp, ctl;
    int build(steiner_graph *g);
    void release() {
        DevBuf *all[] = {&members, &cstart, &cl_of, &irp, &erp, &ie, &ee, &expanded, &lists, &stamp, &ctl};
        for (DevBuf *b : all) b->release();
        built = false;
    }
};
}  // namespace stn

struct steiner_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t n = 0;
    uint64_t nnz = 0;
    uint32_t *d_rp = nullptr;
    uint2 *d_adj = nullptr;
    uint4 *d_ell = nullptr;  // fixed-stride rows when every row has at most ELL_W entries
    uint32_t *d_heavy_rows = nullptr, *d_heavy_off = nullptr;
    uint32_t nheavy = 0;
    uint64_t max_deg = 0;
    // Internal vertex order (steiner_graph_upload flags): when renumbered, d_perm / h_perm give the
    // caller's id of each internal vertex and d_inv / h_inv the inverse; d_eo maps each entry that
    // leaves its smaller caller-id endpoint to the caller's CSR offset (NONE on the twin entry) and
    // d_onew maps those offsets back.  All null / empty when the caller's order is kept.
    bool reordered = false;
    uint32_t *d_perm = nullptr, *d_inv = nullptr, *d_eo = nullptr, *d_onew = nullptr;
    std::vector<uint32_t> h_perm, h_inv;
    stn::DevGraph dg{};
    std::vector<uint64_t> h_rp;  // host copy of the (internal) row offsets
    uint32_t default_delta = 0xFFFFFFFFu;
    uint32_t classic_delta = 1;
    uint32_t tuned_delta = 0;    // set by steiner_graph_tune
    uint32_t tuned_local = 0;
    uint32_t tuned_split = 0;
    uint32_t tuned_pred = 0;     // 0: untuned, 1: eager, 2: lazy
    uint32_t tuned_defer = 0;    // 0: untuned, 1: large rows expanded in the next round, 2: at the bucket's advance
    uint32_t tuned_grid = 0;     // relaxation workgroups of a host-stepped pass (0: as many as are resident)
    uint32_t last_rounds = 0;    // relaxation rounds of the previous pass (sizes the first launch chunk)
    double avg_w = 1.0;
    int cu_count = 256;
    std::mutex mu;               // serialises solves on this graph
    mutable std::mutex memo_mu;  // guards chunk_memo
    mutable std::map<uint64_t, uint64_t> chunk_memo;  // (small_max << 32 | chunk) -> chunks of rows above small_max
    std::map<uint64_t, std::unique_ptr<stn::ChunkTable>> chunk_tables;  // (small_max << 32 | chunk), guarded by mu
    stn::Workspace ws;
    stn::ClusterSet clusters;
};

namespace stn {

// One query of a pass.
struct Query {
    std::vector<uint32_t> S;   // distinct seeds as internal ids, in ascending caller-id order (seed index = position)
    int status = STEINER_OK;
    std::unique_ptr<steiner_result> result;
    // debug outputs
    uint64_t *want_key = nullptr;
    uint32_t *want_pred = nullptr;
    int stop_after = STOP_NEVER;
    std::vector<uint32_t> pidx;  // G'1 entries (lower-triangular pair index), STOP_AFTER_COMPACT only
    std::vector<uint64_t> pval;  // (d'1 << 32) | edge id
};

Options resolve_options(const steiner_graph *g, const steiner_options *o);
int run_pass(steiner_graph *g, const Options &o, std::vector<Query> &qs);
// Steps 3-7 of one query, on the device: MST of its G'1 (m compacted pair
// indices g1_idx into its pair table pt), the kept cross-cell edges, the pred
// walks and D.  key / pred are the query's slot arrays.  The tree's edges come
// back sorted by (a, b, w); EDISCONNECTED if the MST has fewer than k-1 edges.
// mst_buf: a device region of mst_scratch_bytes(k, m) for the MST, or null
// for ts.mst.
int tree_from_g1(steiner_graph *g, hipStream_t st, const uint64_t *key, uint32_t *pred, uint32_t k,
                 const uint64_t *pt, const uint32_t *tr, const uint32_t *g1_idx, uint32_t m, bool pred_ready,
                 TailScratch &ts, uint8_t *mst_buf, std::unique_ptr<steiner_result> &out, double *ms_mst,
                 double *ms_expand, uint32_t mst_block = 0);
// Bytes of the MST's scratch for k seeds and a G'1 of m entries.
size_t mst_scratch_bytes(uint32_t k, uint64_t m);
// Device buffers of Steps 3-6 for one query: the MST's scratch (mst_scratch_bytes; its first 16 bytes
// receive the chosen cross-cell edges' count at [2] and the tree's edge count at [3]), the vertex marks
// (all zero on entry and again on exit) and the output edges (a, b, w at out, out + n, out + 2n).
struct TreeBufs {
    uint8_t *mst;
    uint32_t *mark, *out;
    uint32_t mst_block = 0;  // threads of the MST's single-workgroup kernels (0: 1024)
};
// Launches Steps 3-6 of one query on st (see tree_from_g1); ev_mid (optional) is recorded between the MST and
// the expansion.
int launch_tree(const steiner_graph *g, hipStream_t st, const uint64_t *key, uint32_t *pred, uint32_t k,
                const uint64_t *pt, const uint32_t *tr, const uint32_t *g1_idx, uint32_t m, bool pred_ready,
                const TreeBufs &tb, hipEvent_t ev_mid);
// Pair-table ranks of a query's seeds (see pair_slot): rk[i] is the rank of
// seed index i among the seeds ordered by internal id and rk[k + r] the seed
// index of rank r.  Empty when the graph keeps the caller's order (identity).
void seed_ranks(const steiner_graph *g, const std::vector<uint32_t> &S, std::vector<uint32_t> &rk);
void pair_from_index(uint64_t p, uint32_t *i, uint32_t *j);
int canon_seeds(const steiner_graph *g, const uint32_t *seeds, uint32_t k, std::vector<uint32_t> &S);
uint64_t big_row_chunks(const steiner_graph *g, uint32_t small_max, uint32_t chunk, bool remember = true);
// The chunk numbering for (small_max, chunk), built once per graph; null when the rows above small_max are
// not a prefix of the vertex ids (then the relaxation runs without chunk memory).  Caller holds g->mu.
const ChunkTable *chunk_table(steiner_graph *g, uint32_t small_max, uint32_t chunk, int *rc);
// Looks up the allocation-free solve's device scratch on `device` (the current device) once per device.
void noalloc_setup(int device);
// Fills the pass parameters shared by every driver for Q slots.
void bind_state(VorParams &P, const Options &o, uint64_t cap_s, uint64_t cap_b);
// After bind_state: the large rows' chunk memory for Q slots in `xkey` (allocated here; a DevBuf with enough
// room already is reused), where the graph allows it.  Caller holds g->mu.
int bind_chunk_memory(VorParams &P, steiner_graph *g, const Options &o, uint32_t Q, DevBuf &xkey);

}  // namespace stn
