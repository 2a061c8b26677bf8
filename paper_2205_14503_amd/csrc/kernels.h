// Launch wrappers for the gfx950 kernels (defined in kernels.hip).
#pragma once
#include "common.h"

namespace stn {

struct ScanParams {
    DevGraph g;
    const uint64_t *key;   // [slots * n]
    uint32_t *aux;         // [slots * n] -> pred
    uint32_t *heavy_pe;    // [slots * nheavy] first qualifying CSR offset of each heavy row
    uint64_t *const *pt;   // device array of per-slot pair-table pointers
    const uint32_t *slot_ids; // slots to scan
    uint32_t nscan;        // number of slots in slot_ids
    uint32_t *slot_err;    // [slots] ERR_DIST_OVERFLOW / ERR_SUM_OVERFLOW per query
};

struct CompactParams {
    uint64_t *const *pt;        // per-slot pair tables
    const uint64_t *pt_len;     // per-slot pair-table lengths
    uint32_t *const *out_idx;   // per-slot pair index output
    uint64_t *const *out_val;   // per-slot packed value output
    const uint64_t *out_cap;    // per-slot capacities
    uint32_t *out_cnt;          // per-slot counts
    const uint32_t *slot_ids;
    uint32_t nscan;
    PassCtl *pass;
};

struct ExpandParams {
    DevGraph g;
    const uint64_t *key;     // slot base
    const uint32_t *pred;    // slot base
    const uint32_t *sel_e;   // chosen cross-cell edge ids
    uint32_t nsel;
    uint32_t *visited;       // bitmap, n bits, zeroed
    uint32_t *oa, *ob, *ow;  // outputs, capacity n
    uint32_t *ocnt;
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
// The persistent driver: rounds until convergence or `max_rounds` rounds.
hipError_t launch_persistent(const VorParams &P, uint32_t grid, uint32_t block, uint32_t max_rounds,
                             hipStream_t s);
int persistent_max_grid(uint32_t block);

hipError_t launch_scan(const ScanParams &S, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_compact(const CompactParams &C, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_expand(const ExpandParams &E, hipStream_t s);

}  // namespace stn
