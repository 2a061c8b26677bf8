// Launch wrappers for the gfx950 kernels (defined in kernels.hip).
#pragma once
#include "common.h"

namespace stn {

struct ScanParams {
    DevGraph g;
    const uint64_t *key;   // [slots * n]
    uint32_t *aux;         // [slots * n] -> pred
    uint32_t *heavy_pe;    // [slots * nheavy] smallest caller id of a qualifying neighbour of each heavy row
    uint64_t *const *pt;   // device array of per-slot pair-table pointers
    const uint32_t *const *tr; // device array of per-slot table ranks (null: identity), see pair_slot
    const uint32_t *slot_ids; // slots to scan
    uint32_t nscan;        // number of slots in slot_ids
    uint32_t *slot_err;    // [slots] ERR_DIST_OVERFLOW / ERR_SUM_OVERFLOW per query
    uint32_t with_pred;    // 1: pred of every vertex; 0: pred of rows above scan_heavy only (the tree
                           // expansion finds the others), and each edge's key gathered from one side only
    unsigned long long *ev; // null, or SCAN_EV_N event counts (summed over the scanned slots)
};
// Boundary-scan event counters: CSR entries read, neighbour keys gathered, cross-cell candidates (each reads
// its pair-table entry), atomicMins issued on the pair table.
enum { SCAN_EV_ENTRIES = 0, SCAN_EV_GATHERS, SCAN_EV_CANDIDATES, SCAN_EV_ATOMICS, SCAN_EV_N };

struct CompactParams {
    uint64_t *const *pt;        // per-slot pair tables
    const uint32_t *const *ts;  // per-slot seed index of each table rank (null: identity)
    const uint64_t *pt_len;     // per-slot pair-table lengths
    uint32_t *const *out_idx;   // per-slot pair index output
    uint64_t *const *out_val;   // per-slot packed value output (a null entry: indices only)
    const uint64_t *out_cap;    // per-slot capacities
    uint32_t *out_cnt;          // per-slot counts; the output indices are in seed-index order (i < j: j(j-1)/2 + i)
    const uint32_t *slot_ids;
    uint32_t nscan;
    PassCtl *pass;
};

struct ExpandParams {
    DevGraph g;
    const uint64_t *key;     // slot base
    uint32_t *pred;          // slot base: pred of rows above scan_heavy on entry; the walks add the others
    const uint32_t *sel_e;   // chosen cross-cell edge ids (caller CSR offsets, see DevGraph::onew)
    const uint32_t *nsel;    // their number (device)
    uint32_t nsel_max;       // upper bound of *nsel, sizes the launch
    uint32_t *mark;          // n bytes (rounded up to 4), all zero on entry and again on exit
    uint32_t *oa, *ob, *ow;  // output edges, capacity n
    uint32_t *ocnt;          // output count, zero on entry
    uint32_t pred_ready;     // 1: pred holds every vertex's pred (the scan ran with pred)
};

hipError_t launch_fill_u64(uint64_t *p, uint64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint64_t count, uint8_t value, hipStream_t s);

// Reset pass-wide control (round 0, counters, far minima) for a fresh pass.
hipError_t launch_pass_reset(const VorParams &P, hipStream_t s);
// Initialise slot `slot` (keys, stamps, marks, control) and push its seeds
// (device array of k sorted seeds) into the list of the pass's current round.
hipError_t launch_slot_start(const VorParams &P, uint32_t slot, const uint32_t *d_seeds, uint32_t k,
                             uint32_t *heavy_pe_slot, uint32_t nheavy, hipStream_t s);
// One round of the host-stepped driver: relax + control + advance scan.
hipError_t launch_round(const VorParams &P, uint32_t grid, uint32_t block, hipStream_t s);
// A HIP graph of `rounds` consecutive round-kernel launches with parameters P
// (the graph-captured driver): launched as one unit, it replaces a chunk of
// host launches; rounds after convergence exit at once.
hipError_t build_round_graph(const VorParams &P, uint32_t grid, uint32_t block, uint32_t rounds, hipGraphExec_t *exec);
// The persistent driver: rounds until convergence or `max_rounds` rounds.
hipError_t launch_persistent(const VorParams &P, uint32_t grid, uint32_t block, uint32_t max_rounds,
                             hipStream_t s);
int persistent_max_grid(uint32_t block);
// Workgroups of the round kernel that fit on the device at once (0 if unknown).
int round_max_grid(uint32_t block);

hipError_t launch_scan(const ScanParams &S, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_compact(const CompactParams &C, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_expand(const ExpandParams &E, uint32_t emit_grid, hipStream_t s);

// Borůvka MST of one query's G'1 on the device (Alg. 2 Step 3).  The edge
// order is the strict (d'1, i, j): key = (d'1 << 32) | rank(i, j) with the
// row-major rank of the pair among all i < j, which fits in 32 bits while
// k(k-1)/2 does; so the tree is the one Kruskal or Prim under that order
// returns.  Scratch for m G'1 entries and k seeds, see MstParams.
struct MstParams {
    const uint64_t *pt;       // the query's pair table: (d'1 << 32) | edge id at pair_slot(i, j)
    const uint32_t *tr;       // the query's table ranks (null: identity)
    uint32_t k;
    uint32_t *edges[2];       // [m] each: ping-pong lists of pair indices that still join two components
    uint32_t *hdr;            // [4]: edge counts of the two lists, chosen-edge count, expansion output count
    uint32_t *par;            // [k] component root of each seed
    uint32_t *hook;           // [k] parent of each root after the current round's hooking
    unsigned long long *best; // [k] lightest key leaving each root
    uint32_t *sel;            // [k] chosen cross-cell edge ids (caller CSR offsets), hdr[2] of them
    uint32_t block;           // threads of the single-workgroup steps (1024; 256 fits beside a running pass)
};
hipError_t launch_mst(const MstParams &M, const uint32_t *g1_idx, uint32_t m, hipStream_t s);

// Pair-table layout.  The entry of seed pair (i, j) lives at slot
// r(r-1)/2 + q with q < r the table ranks of i and j: a seed's rank among the
// query's seeds by internal vertex id.  On a renumbered graph that puts the
// pairs of the high-degree seeds, whose large cells take most candidates,
// into the first lines of the table; in the caller's order the rank is the
// seed index.  Values and ties do not depend on the layout.
__host__ __device__ inline uint64_t pair_slot(const uint32_t *tr, uint32_t i, uint32_t j) {
    const uint32_t a = tr ? tr[i] : i, b = tr ? tr[j] : j;
    const uint64_t q = a < b ? a : b, r = a < b ? b : a;
    return r * (r - 1) / 2 + q;
}

// Cluster-local relaxation of one query (Alg. 2 Step 1; driver 3): the
// vertices form BFS-grown clusters of at most CLUSTER_MAX vertices; a
// workgroup relaxes an active cluster's internal edges in LDS to local
// convergence, then its external edges with global atomics.
constexpr uint32_t CLUSTER_MAX = 1024;    // vertices per cluster
constexpr uint32_t CLUSTER_EDGES = 4096;  // edge entries of a cluster's members (staged in LDS)
struct ClusterCtl {
    uint32_t cnt[3];       // list lengths, rotating by round mod 3
    uint32_t round;
    uint32_t done;
    uint32_t blocks_done;
    uint32_t err;
    uint32_t pad;
};
struct ClusterParams {
    uint32_t n, nclusters;
    const uint32_t *members;  // [n] vertices grouped by cluster
    const uint32_t *cstart;   // [nclusters + 1] cluster c = members[cstart[c], cstart[c+1])
    const uint32_t *cl_of;    // [n] cluster of each vertex
    const uint32_t *irp;      // [n + 1] internal edges of member position p: ie[irp[p], irp[p+1])
    const uint2 *ie;          // (local index of the target, w)
    const uint32_t *erp;      // [n + 1] external edges of member position p: ee[erp[p], erp[p+1])
    const uint2 *ee;          // (target vertex, w)
    uint64_t *key;            // the query's keys
    uint64_t *expanded;       // [n] key with which each vertex's edges were last relaxed
    uint32_t *list[2];        // [nclusters] each: clusters active in the current / next round
    uint32_t *stamp;          // [nclusters] last round a cluster was listed for, plus one
    ClusterCtl *ctl;
};
hipError_t launch_cluster_start(const ClusterParams &C, const uint32_t *seeds, uint32_t k, hipStream_t s);
hipError_t launch_cluster_round(const ClusterParams &C, uint32_t grid, hipStream_t s);
int cluster_max_grid();

}  // namespace stn
