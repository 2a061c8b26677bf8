// Internal types shared by the gfx950 kernels (kernels.hip) and the host
// engine (engine.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stn {

constexpr uint64_t KEY_INF = ~0ull;          // unreached vertex key
constexpr uint32_t DIST_INF = 0xFFFFFFFFu;   // unreached distance (also the saturation limit)
constexpr uint32_t NONE = 0xFFFFFFFFu;       // no vertex / no predecessor
constexpr uint32_t MAX_SLOTS = 4096;         // queries resident in one pass (12-bit slot field)

// Frontier item encodings.  A light item relaxes the row's light edges
// (w <= delta) of a vertex inside its bucket; a heavy item (flag set) relaxes
// the heavy edges (w > delta) of a vertex whose bucket has closed.
//  S item: (heavy << 63) | (slot << 32) | v                  -- row of degree <= small_max
//  B item: (slot << 52) | (heavy << 51) | (chunk << 32) | v  -- chunk < 2^19 of a larger row
constexpr uint32_t CHUNK_BITS = 19;
__host__ __device__ inline uint64_t s_item(uint32_t slot, uint32_t v, bool heavy = false) {
    return ((uint64_t)heavy << 63) | ((uint64_t)slot << 32) | v;
}
__host__ __device__ inline uint32_t s_slot(uint64_t it) { return (uint32_t)(it >> 32) & 0xFFFu; }
__host__ __device__ inline bool s_heavy(uint64_t it) { return (it >> 63) != 0; }
__host__ __device__ inline uint64_t b_item(uint32_t slot, uint32_t chunk, uint32_t v, bool heavy = false) {
    return ((uint64_t)slot << 52) | ((uint64_t)heavy << 51) | ((uint64_t)chunk << 32) | v;
}

// Per-query control, stored structure-of-arrays so the persistent kernel can
// mirror it in LDS.  thr is the exclusive upper end of the query's current
// distance bucket: a relaxed vertex with dist < thr is processed in the next
// round, otherwise it is parked (dirty) until its bucket comes up.
struct SlotArrays {
    uint64_t *thr;       // current bucket end
    uint64_t *thr_prev;  // bucket end before the latest advance
    uint32_t *carry;     // lower bound on dist of parked vertices (DIST_INF = none)
    uint32_t *active;    // 1 while resident and unconverged
    uint32_t *adv;       // 1 if the query advances its bucket this round
    uint32_t *done;      // 1 once its cells have converged
    uint32_t *advances;  // bucket advances so far
};

// Pass-wide control block (one per multi-query pass).
// Round numbers wrap at a multiple of 6, so that the list parity (r & 1) and the rotating counters (r % 3)
// continue across the wrap in a pass that lives for ever (the server's), and the round fits the 30 bits it has
// in PassCtl::word.
constexpr uint32_t ROUND_WRAP = 3u << 28;
__host__ __device__ inline uint32_t next_round(uint32_t r) { return r + 1 == ROUND_WRAP ? 0u : r + 1; }

struct PassCtl {
    uint32_t round;     // current round r
    uint32_t all_done;  // 1 when no resident query has work left
    uint32_t any_adv;   // 1 if some query advances this round
    uint32_t nslots;    // slots in use (upper bound of active slot ids)
    uint32_t err;       // device-side error bits
    uint32_t pad;
    // The round kernel's view of round, any_adv and all_done, with the identity of the launch that last took a
    // round decision, in one atomic word (bits 0-31 that launch's dispatch-packet address, 32-61 the round,
    // 62 any_adv, 63 all_done); written with the fields above wherever they change.
    uint64_t word;
};
constexpr uint32_t NO_LAUNCH = 0xFFFFFFFFu;
__host__ __device__ inline uint64_t pass_word(uint32_t round, uint32_t any_adv, uint32_t all_done, uint32_t launch) {
    return (uint64_t)launch | ((uint64_t)(round & 0x3FFFFFFFu) << 32) | ((uint64_t)(any_adv != 0) << 62) |
           ((uint64_t)(all_done != 0) << 63);
}

// Rotating counters: index (r % 3) holds the S and B item counts of the list
// that round r processes; (r + 1) % 3 is filled during round r; (r + 2) % 3 is
// cleared during round r.
struct Counters {
    uint32_t s[3];
    uint32_t b[3];
    uint32_t bar_count;  // persistent-kernel grid barrier
    uint32_t bar_gen;
    uint32_t abort;      // set when a barrier wait gives up
    uint32_t blocks_done; // workgroup groups finished in the current round (the last one decides)
    uint32_t pad[6];
    // workgroups finished per group (blockIdx mod ROUND_GROUPS), one counter per 128-byte line: the round's
    // completion count takes ROUND_GROUPS short chains of device-scope atomics instead of one long one
    uint32_t grp_done[8 * 32];
    // event counters (only with counting enabled): relaxation attempts,
    // atomicMins issued, improvements, local-queue pushes, next-round pushes,
    // parked vertices, items expanded, attempts from chunks of large rows
    unsigned long long ev[8];
    unsigned long long scan_ev[4];  // boundary-scan events (counting mode), see ScanParams::ev
};
constexpr uint32_t ROUND_GROUPS = 8;
enum { EV_ATTEMPT = 0, EV_ATOMIC, EV_IMPROVED, EV_LOCAL, EV_GLOBAL, EV_PARK, EV_ITEMS, EV_LARGE, EV_N };

constexpr uint32_t ELL_W = 4;
constexpr uint32_t ELL_NONE = 0xFFFFFFFFu;

struct DevGraph {
    uint32_t n;
    uint32_t nnz;
    uint32_t max_deg;     // largest row (clamped to 2^32 - 1)
    // Graphs whose rows have at most ELL_W entries also hold them at a fixed
    // stride: row v is ell[2v], ell[2v + 1], each the (col, w) pairs of two
    // entries in CSR order, col = ELL_NONE past the row's end.  Null otherwise.
    const uint4 *ell;
    const uint32_t *rp;   // row offsets, n+1 (32-bit: nnz < 2^32)
    const uint2 *adj;     // (col, w) per CSR entry
    // Rows of degree > scan_heavy are split into chunks of scan_chunk edges
    // for the boundary scan; heavy_rows lists them (ascending) and
    // heavy_chunk_off[h] is the index of row h's first chunk (nheavy+1 entries).
    // Every other row is scanned by the wave owning its group of 64 rows.
    uint32_t nheavy;
    uint32_t nheavy_chunks;
    const uint32_t *heavy_rows;
    const uint32_t *heavy_chunk_off;
    uint32_t scan_heavy;
    uint32_t scan_chunk;
    // 1 when the boundary scan may read each edge from its larger internal id: the graph was renumbered by
    // degree (the heavy rows are the vertices below nheavy, hub keys sit on few lines) and every entry
    // carries its edge id (eo)
    uint32_t reverse_scan;
    // Internal vertex order.  Null when the ids are the caller's; otherwise
    // the graph was renumbered at upload and results are stated in the
    // caller's ids and CSR offsets: perm[v] is the caller's id of internal
    // vertex v and inv its inverse; eo[e] is the edge id of entry e, the
    // caller's CSR offset of the edge's entry leaving its smaller caller id
    // (NONE for self-loops), and onew[f] is, for such an offset f, the
    // edge's entry leaving its smaller internal id.
    const uint32_t *perm;
    const uint32_t *inv;
    const uint32_t *eo;
    const uint32_t *onew;
};

struct VorParams {
    DevGraph g;
    uint64_t *key;       // [slots * n]
    uint32_t *aux;       // [slots * n]: near-push stamp during the pass, pred after the scan
    uint8_t *dirty;      // [slots * n]: parked (far) marks
    uint64_t *items_s[2];
    uint64_t *items_b[2];
    uint32_t cap_s, cap_b;
    Counters *cnt;
    uint32_t *far_min;   // [3][slots]: min dist parked in round r (rotating)
    uint32_t *near_mark; // [3][slots]: 1 if the query pushed near items in round r (rotating)
    uint32_t *settle_mark; // [3][slots]: 1 if the query expanded a vertex in round r whose heavy edges wait
    uint8_t *settled;    // [slots * n]: vertex expanded in its query's open bucket, heavy edges pending
    SlotArrays slot;     // [slots] each
    PassCtl *pass;
    uint32_t nslots;     // allocated slots
    uint32_t delta;
    uint32_t small_max;
    uint32_t chunk;
    uint32_t local_iters; // batches of the wave-local queue expanded per unit (0 = no local queue)
    uint32_t counting;    // 1: accumulate Counters::ev
    uint32_t split;       // 1: light/heavy edge split (finite delta)
    uint32_t lq_mode;     // bit 0: drain the local queue smallest distance first; bit 1: skip superseded entries
    uint32_t defer_min;   // improved rows above this many entries wait for the bucket's advance (0: never)
    // Chunk memory (null when off): the rows above small_max are the vertices below nxrow (a degree-renumbered
    // graph) and chunk c of row v is chunk number xchunk[v] + c of xchunks per query; xkey[slot * xchunks + i]
    // is the key chunk i was last expanded with (all ones: never).  A chunk whose row still holds that key
    // has nothing new to push and is skipped.
    uint64_t *xkey;
    const uint32_t *xchunk;
    uint32_t nxrow, xchunks;
};

enum : uint32_t {
    ERR_DIST_OVERFLOW = 1u,   // some reached vertex has an unreached neighbour after convergence
    ERR_SUM_OVERFLOW = 2u,    // some cross-cell sum >= 2^32
    ERR_LIST_OVERFLOW = 4u,   // frontier capacity exceeded (internal bug guard)
    ERR_ROUND_LIMIT = 8u,     // round safety cap reached
    ERR_BARRIER_TIMEOUT = 16u // persistent kernel barrier spin cap reached
};

}  // namespace stn
