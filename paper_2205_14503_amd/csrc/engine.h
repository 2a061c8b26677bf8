// Host-side engine internals (not part of the public ABI).
#pragma once
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/steiner.h"
#include "kernels.h"

namespace stn {

int fail(int code, const char *fmt, ...);
int dev_alloc(void **p, size_t bytes);
void dev_free(void *p);
int hip_check(hipError_t e, const char *what);

// Grow-only device buffer.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want);
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
    uint32_t delta, driver, block, grid, small_max, chunk, local_iters;
    bool timing;
};

// Device workspace of a multi-query pass, reused across solves of a graph.
struct Workspace {
    DevBuf key, aux, dirty, items_s[2], items_b[2], ctl, heavy_pe, seeds, pt, cidx, cval, ptrs, visited, oedges,
        sel;
    HostPinned host;
    void release() {
        DevBuf *all[] = {&key, &aux, &dirty, &items_s[0], &items_s[1], &items_b[0], &items_b[1], &ctl, &heavy_pe,
                         &seeds, &pt, &cidx, &cval, &ptrs, &visited, &oedges, &sel};
        for (DevBuf *b : all) b->release();
        host.release();
    }
};

enum StopAfter { STOP_NEVER = 0, STOP_AFTER_SCAN = 1, STOP_AFTER_COMPACT = 2 };

}  // namespace stn

struct steiner_result {
    std::vector<uint32_t> a, b, w;
    uint64_t total = 0;
    steiner_stats stats{};
};

struct steiner_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t n = 0;
    uint64_t nnz = 0;
    uint32_t *d_rp = nullptr;
    uint2 *d_adj = nullptr;
    uint32_t *d_heavy_rows = nullptr, *d_heavy_off = nullptr;
    uint32_t nheavy = 0;
    stn::DevGraph dg{};
    std::vector<uint64_t> h_rp;  // host copy of the row offsets
    uint32_t default_delta = 1;
    int cu_count = 256;
    std::mutex mu;               // serialises solves on this graph
    stn::Workspace ws;
};

namespace stn {

// One query of a pass.
struct Query {
    std::vector<uint32_t> S;   // sorted distinct seeds
    int status = STEINER_OK;
    std::unique_ptr<steiner_result> result;
    // debug outputs
    uint64_t *want_key = nullptr;
    uint32_t *want_pred = nullptr;
    int stop_after = STOP_NEVER;
    std::vector<uint32_t> pidx;  // G'1 entries (lower-triangular pair index)
    std::vector<uint64_t> pval;  // (d'1 << 32) | edge id
};

Options resolve_options(const steiner_graph *g, const steiner_options *o);
int run_pass(steiner_graph *g, const Options &o, std::vector<Query> &qs);
int prim_mst(uint32_t k, const std::vector<uint32_t> &pidx, const std::vector<uint64_t> &pval,
             std::vector<uint32_t> &chosen);
void pair_from_index(uint64_t p, uint32_t *i, uint32_t *j);
int canon_seeds(const steiner_graph *g, const uint32_t *seeds, uint32_t k, std::vector<uint32_t> &S);
uint64_t big_row_chunks(const steiner_graph *g, uint32_t small_max, uint32_t chunk);

}  // namespace stn
