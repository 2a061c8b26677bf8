// Host engine and C ABI of the MI355X Steiner tree library (include/steiner.h).
//
// A graph lives on one device as a 32-bit row-offset array plus interleaved
// (col, w) pairs.  A solve runs a multi-query pass (a single query is a pass
// with one slot): slot start -> relaxation rounds to convergence -> fused
// pred/boundary scan -> G'1 compaction -> MST of G'1 on the host (Prim under
// the strict order (d'1, i, j); Alg. 2 Step 3 keeps this step sequential) ->
// predecessor-walk expansion on the device -> sorted edge list and D.
#include "engine.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <queue>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

namespace stn {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// Allocation fault injection for error-path tests: STEINER_FAULT_ALLOC_AFTER=N
// (read at the first allocation) or set_fault_alloc_after(N) makes every
// device or pinned-host allocation after the first N of the process fail.
static std::atomic<long> g_alloc_calls{0};
static std::atomic<long> g_fault_after{-2};  // -2: not yet read from the environment, -1: off
static bool fault_injected(size_t bytes) {
    long lim = g_fault_after.load(std::memory_order_relaxed);
    if (lim == -2) {
        const char *s = getenv("STEINER_FAULT_ALLOC_AFTER");
        long want = s ? atol(s) : -1;
        g_fault_after.compare_exchange_strong(lim, want);
        lim = g_fault_after.load(std::memory_order_relaxed);
    }
    const long c = g_alloc_calls.fetch_add(1, std::memory_order_relaxed);
    if (lim >= 0 && c >= lim) {
        fail(STEINER_ENOMEM, "injected allocation failure (%zu bytes)", bytes);
        return true;
    }
    return false;
}

void set_fault_alloc_after(long n) {
    g_alloc_calls.store(0);
    g_fault_after.store(n < 0 ? -1 : n);
}

long alloc_calls() { return g_alloc_calls.load(); }

int dev_alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (fault_injected(bytes)) return STEINER_ENOMEM;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(STEINER_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return STEINER_OK;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return STEINER_OK;
    (void)hipGetLastError();
    return fail(STEINER_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------- buffers

void DevBuf::release() {
    dev_free(ptr);
    ptr = nullptr;
    bytes = 0;
}

int DevBuf::ensure(size_t want, bool exact) {
    if (want <= bytes && ptr) return STEINER_OK;
    release();
    size_t cap = exact ? want : want + want / 8 + 256;
    int rc = dev_alloc(&ptr, cap);
    if (rc) return rc;
    bytes = cap;
    return STEINER_OK;
}

void HostPinned::release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int HostPinned::ensure(size_t want) {
    if (want <= bytes && ptr) return STEINER_OK;
    release();
    size_t cap = want + want / 8 + 256;
    if (fault_injected(cap)) return STEINER_ENOMEM;
    if (hipHostMalloc(&ptr, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        return fail(STEINER_ENOMEM, "hipHostMalloc(%zu) failed", cap);
    }
    bytes = cap;
    return STEINER_OK;
}

// ------------------------------------------------------------- options

Options resolve_options(const steiner_graph *g, const steiner_options *o) {
    Options r;
    r.delta = g->tuned_delta ? g->tuned_delta : g->default_delta;
    r.driver = 1;
    r.block = 256;
    r.grid = 0;
    r.small_max = 64;
    r.chunk = 512;
    r.local_iters = g->tuned_local ? (g->tuned_local == 0xFFFFFFFFu ? 0 : g->tuned_local) : 8;
    r.timing = false;
    r.counting = false;
    r.split = g->tuned_split != 0;
    r.lq_mode = 3;  // local queue drained smallest distance first, superseded entries skipped
    // deferring the expansion of improved large rows to the bucket's advance pays on skewed graphs (the ones
    // renumbered by degree), whose hubs are otherwise expanded about twice per solve
    bool defer = g->tuned_defer ? g->tuned_defer == 2 : g->reordered;
    // lazy preds pay one row scan per tree vertex to save half the scan's gathers: a win on
    // dense graphs, a loss on sparse high-diameter ones (long walks, cheap scan)
    r.lazy_pred = g->tuned_pred ? g->tuned_pred == 2 : (g->n && (double)g->nnz / g->n >= 8.0);
    if (const char *s = getenv("STEINER_LAZY_PRED")) r.lazy_pred = atoi(s) != 0;
    if (const char *s = getenv("STEINER_LQ_MODE")) r.lq_mode = (uint32_t)atoi(s);

    if (const char *s = getenv("STEINER_DRIVER")) r.driver = (uint32_t)atoi(s);
    if (const char *s = getenv("STEINER_LOCAL")) r.local_iters = (uint32_t)strtoul(s, nullptr, 10);
    if (const char *s = getenv("STEINER_DELTA")) r.delta = (uint32_t)strtoul(s, nullptr, 10);
    if (o) {
        if (o->delta) r.delta = o->delta;
        if (o->driver) r.driver = o->driver;
        if (o->block) r.block = o->block;
        if (o->grid) r.grid = o->grid;
        if (o->small_max) r.small_max = o->small_max;
        if (o->chunk) r.chunk = o->chunk;
        if (o->local_iters) r.local_iters = o->local_iters == 0xFFFFFFFFu ? 0 : o->local_iters;
        r.timing = (o->flags & STEINER_FLAG_TIMING) != 0;
        r.counting = (o->flags & STEINER_FLAG_COUNTERS) != 0;
        if (o->flags & STEINER_FLAG_SPLIT) r.split = true;
        if (o->flags & STEINER_FLAG_LAZY_PRED) r.lazy_pred = true;
        if (o->flags & STEINER_FLAG_EAGER_PRED) r.lazy_pred = false;
        if (o->flags & STEINER_FLAG_DEFER) defer = true;
        if (o->flags & STEINER_FLAG_NO_DEFER) defer = false;
    }
    r.defer_min = defer ? std::max<uint32_t>(r.small_max, 1) : 0;
    if (const char *s = getenv("STEINER_DEFER")) r.defer_min = (uint32_t)strtoul(s, nullptr, 10);
    if (r.delta == 0) r.delta = 1;
    if (r.block < 64 || r.block > 1024 || r.block % 64) r.block = 256;
    if (r.block > 256) r.block = 256;  // per-wave LDS scratch of the relaxation kernels (~10 KB per wave)
    if (r.chunk < 64) r.chunk = 64;
    while ((g->max_deg + r.chunk - 1) / r.chunk >= (1ull << CHUNK_BITS)) r.chunk *= 2;  // chunk index field
    // host-stepped: as many workgroups as are resident at once (the round kernel's occupancy);
    // persistent: one per CU on fixed-stride graphs and two elsewhere (co-resident, as its grid barrier needs;
    // measured: grid2048 5.2 / 7.8 ms and RMAT-22 18.7 / 14.0 ms at one / two per CU)
    // passes of the host-stepped driver use the tuned count (a latency-bound graph often runs faster on
    // fewer workgroups), batches at least half the resident count (their frontier is larger); the server
    // keeps every resident one
    const bool given = r.grid != 0;
    if (!given) {
        if (r.driver == 2) {
            r.grid = (uint32_t)std::max(1, g->cu_count) * (g->d_ell ? 1u : 2u);
        } else {
            const int resident = round_max_grid(r.block);
            r.grid = resident > 0 ? (uint32_t)resident : (uint32_t)std::max(1, g->cu_count) * 4u;
        }
    }
    r.grid_tuned = r.grid;
    if (!given && r.driver != 2 && g->tuned_grid && g->tuned_grid <= r.grid && r.block == 256) r.grid_tuned = g->tuned_grid;
    return r;
}

// ------------------------------------------------------------- pair index

// (i, j), i < j, of lower-triangular index p = j(j-1)/2 + i.
void pair_from_index(uint64_t p, uint32_t *i, uint32_t *j) {
    uint64_t jj = (uint64_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)p)) / 2.0);
    while (jj * (jj - 1) / 2 > p) jj--;
    while ((jj + 1) * jj / 2 <= p) jj++;
    *j = (uint32_t)jj;
    *i = (uint32_t)(p - jj * (jj - 1) / 2);
}

}  // namespace stn

using namespace stn;

// ===================================================================== graph

static __global__ void k_validate_rows(const uint64_t *rp, uint32_t n, uint64_t nnz, uint8_t *is_start,
                                       uint32_t *bad) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        uint64_t a = rp[v], b = rp[v + 1];
        if (b < a || b > nnz) atomicOr(bad, 1u);
        else if (a < b) is_start[a] = 1;
    }
}

static __global__ void k_validate_entries(const uint32_t *col, const uint32_t *w, uint64_t nnz, uint32_t n,
                                          const uint8_t *is_start, uint32_t *bad) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t c = col[e];
        if (c >= n || w[e] == 0) atomicOr(bad, 2u);
        if (e + 1 < nnz && !is_start[e + 1] && col[e + 1] < c) atomicOr(bad, 4u);
    }
}

static __global__ void k_convert(const uint64_t *rp64, uint32_t n, const uint32_t *col, const uint32_t *w,
                                 uint64_t nnz, uint32_t *rp32, uint2 *adj) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) rp32[v] = (uint32_t)rp64[v];
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) adj[e] = make_uint2(col[e], w[e]);
}

// Fixed-stride copy of a CSR whose rows have at most ELL_W = 4 entries.
static __global__ void k_build_ell(const uint32_t *rp, const uint2 *adj, uint32_t n, uint4 *ell) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint32_t beg = rp[v], deg = rp[v + 1] - beg;
        uint32_t c[ELL_W], w[ELL_W];
        for (uint32_t i = 0; i < ELL_W; i++) {
            c[i] = i < deg ? adj[beg + i].x : ELL_NONE;
            w[i] = i < deg ? adj[beg + i].y : 0u;
        }
        ell[2 * v] = make_uint4(c[0], w[0], c[1], w[1]);
        ell[2 * v + 1] = make_uint4(c[2], w[2], c[3], w[3]);
    }
}

static __global__ void k_weight_sum(const uint32_t *w, uint64_t nnz, unsigned long long *sum) {
    unsigned long long s = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x) s += w[e];
    atomicAdd(sum, s);
}

// Twin matching for the renumbering: one wave per row, a lane per entry.  An
// entry u -> v, u < v, without a parallel entry finds its twin v -> u by
// binary search in row v (rows are sorted by column) and both get the edge id
// f, the entry's own offset; self-loops get NONE.  Runs of parallel entries
// are listed as (row, first offset) for the host.  A twin that is missing,
// repeated or of another weight sets ctr[1] bit 0, a full list bit 1.
static __global__ void k_twins(const uint32_t *rp, const uint2 *adj, uint32_t n, uint32_t *canon, uint2 *multi,
                               uint32_t multi_cap, uint32_t *ctr) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t uu = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; uu < n; uu += nwaves) {
        const uint32_t u = (uint32_t)uu, b = rp[u], end = rp[u + 1];
        for (uint32_t f = b + lane; f < end; f += 64) {
            const uint2 a = adj[f];
            const uint32_t v = a.x;
            if (f > b && adj[f - 1].x == v) continue;  // inside a run: its first entry's lane handles it
            if (v == u) {
                for (uint32_t t = f; t < end && adj[t].x == v; t++) canon[t] = NONE;
                continue;
            }
            if (v < u) continue;  // the row of the smaller endpoint handles the edge
            if (f + 1 < end && adj[f + 1].x == v) {
                const uint32_t pos = atomicAdd(ctr, 1u);
                if (pos < multi_cap) multi[pos] = make_uint2(u, f);
                else atomicOr(ctr + 1, 2u);
                continue;
            }
            const uint32_t rv = rp[v + 1];
            uint32_t lo = rp[v], hi = rv;
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (adj[mid].x < u) lo = mid + 1; else hi = mid;
            }
            if (lo >= rv || adj[lo].x != u || (lo + 1 < rv && adj[lo + 1].x == u) || adj[lo].y != a.y) {
                atomicOr(ctr + 1, 1u);
                continue;
            }
            canon[f] = f;
            canon[lo] = f;
        }
    }
}

// Symmetry: every entry (a, b, w) has a partner (b, a, w); checked by binary
// search for (a, w) in row b among equal columns.
static __global__ void k_validate_symmetry(const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t n,
                                           uint32_t *bad) {
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
        for (uint64_t e = rp[a]; e < rp[a + 1]; e++) {
            uint32_t b = col[e], wt = w[e];
            uint64_t lo = rp[b], hi = rp[b + 1];
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                if (col[mid] < a) lo = mid + 1; else hi = mid;
            }
            bool ok = false;
            for (uint64_t f = lo; f < rp[b + 1] && col[f] == a; f++)
                if (w[f] == wt) { ok = true; break; }
            if (!ok) { atomicOr(bad, 8u); return; }
        }
    }
}

// Host array left uninitialised (every element is written before it is read).
template <typename T>
struct HostArray {
    T *p;
    explicit HostArray(size_t count) : p(static_cast<T *>(::operator new(std::max<size_t>(count, 1) * sizeof(T)))) {}
    ~HostArray() { ::operator delete(p); }
    HostArray(const HostArray &) = delete;
    HostArray &operator=(const HostArray &) = delete;
    T &operator[](size_t i) { return p[i]; }
    const T &operator[](size_t i) const { return p[i]; }
    T *data() { return p; }
};

// Renumbers the vertices by descending degree (ties by id), so that the
// high-degree vertices, whose keys most gathers read, share few cache lines,
// and sorts every row by the new ids (entries to one neighbour keep their
// order).  Builds the maps that let the kernels evaluate every tie rule on
// the caller's ids and offsets (DevGraph::perm, inv, eo, onew), so no result
// changes.  Each entry's eo is the caller offset of its edge's entry leaving
// the smaller caller id; a parallel group's entries are paired with their
// twins in (weight, offset) order on both sides.  Returns 1 without touching
// the graph if the CSR is not symmetric (some entry has no twin).
static int reorder_graph(steiner_graph *g) {
    const uint32_t n = g->n;
    const uint64_t nnz = g->nnz;
    hipStream_t s = g->stream;
    const std::vector<uint64_t> rp = g->h_rp;  // caller's offsets
    HostArray<uint2> adj(nnz);
    int rc;
    if (nnz && (rc = hip_check(hipMemcpyAsync(adj.data(), g->d_adj, nnz * 8, hipMemcpyDeviceToHost, s), "D2H adjacency")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(s), "D2H adjacency"))) return rc;
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    struct Scratch {
        std::vector<uint64_t> row;
        std::vector<std::pair<uint32_t, uint32_t>> mine, theirs;  // (w, offset)
    };
    // body(v, scratch) for every v, in blocks of 1024 claimed in order; one scratch per worker
    auto parallel_rows = [&](auto &&body) {
        std::atomic<uint32_t> next{0};
        auto work = [&]() {
            Scratch sc;
            for (;;) {
                const uint32_t v0 = next.fetch_add(1024);
                if (v0 >= n) return;
                for (uint32_t v = v0; v < std::min<uint64_t>((uint64_t)v0 + 1024, n); v++) body(v, sc);
            }
        };
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; t++) pool.emplace_back(work);
        work();
        for (std::thread &t : pool) t.join();
    };
    // canon[f]: caller offset of the entry of f's edge that leaves the smaller caller id (NONE for
    // self-loops).  The device pairs the runs of one entry; a run of parallel entries u -> v, u < v, is
    // paired here with the run v -> u in (weight, offset) order.  False if the twins do not match.
    HostArray<uint32_t> canon(nnz);
    auto match_run = [&](uint32_t u, uint64_t f, Scratch &sc) -> bool {
        const uint32_t v = adj[f].x;
        uint64_t f1 = f;
        while (f1 < rp[u + 1] && adj[f1].x == v) f1++;
        uint64_t lo = rp[v], hi = rp[v + 1];
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            if (adj[mid].x < u) lo = mid + 1; else hi = mid;
        }
        uint64_t g1 = lo;
        while (g1 < rp[v + 1] && adj[g1].x == u) g1++;
        if (g1 - lo != f1 - f) return false;
        std::vector<std::pair<uint32_t, uint32_t>> &mine = sc.mine, &theirs = sc.theirs;
        mine.clear();
        theirs.clear();
        for (uint64_t t = f; t < f1; t++) mine.emplace_back(adj[t].y, (uint32_t)t);
        for (uint64_t t = lo; t < g1; t++) theirs.emplace_back(adj[t].y, (uint32_t)t);
        std::sort(mine.begin(), mine.end());
        std::sort(theirs.begin(), theirs.end());
        for (size_t t = 0; t < mine.size(); t++) {
            if (mine[t].first != theirs[t].first) return false;
            canon[mine[t].second] = mine[t].second;
            canon[theirs[t].second] = mine[t].second;
        }
        return true;
    };
    std::atomic<bool> asym{false};
    {
        const uint32_t multi_cap = 1u << 20;
        struct DevTemp {  // freed on every exit, allocation failures included
            void *p = nullptr;
            ~DevTemp() { dev_free(p); }
        } t_canon, t_multi, t_ctr;
        uint32_t hctr[2] = {0, 0};
        rc = dev_alloc(&t_canon.p, nnz * 4);
        if (!rc) rc = dev_alloc(&t_multi.p, (size_t)multi_cap * 8);
        if (!rc) rc = dev_alloc(&t_ctr.p, 8);
        void *d_canon = t_canon.p, *d_multi = t_multi.p, *d_ctr = t_ctr.p;
        if (!rc) rc = hip_check(hipMemsetAsync(d_ctr, 0, 8, s), "twins");
        if (!rc) {
            hipLaunchKernelGGL(k_twins, dim3(4096), dim3(256), 0, s, g->d_rp, g->d_adj, n, (uint32_t *)d_canon,
                               (uint2 *)d_multi, multi_cap, (uint32_t *)d_ctr);
            rc = hip_check(hipGetLastError(), "twins");
        }
        if (!rc) rc = hip_check(hipMemcpyAsync(hctr, d_ctr, 8, hipMemcpyDeviceToHost, s), "twins");
        if (!rc && nnz) rc = hip_check(hipMemcpyAsync(canon.data(), d_canon, nnz * 4, hipMemcpyDeviceToHost, s), "twins");
        std::vector<uint2> multi;
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "twins");
        if (!rc && !(hctr[1] & 3u) && hctr[0]) {
            multi.resize(hctr[0]);
            rc = hip_check(hipMemcpyAsync(multi.data(), d_multi, (size_t)hctr[0] * 8, hipMemcpyDeviceToHost, s), "twins");
            if (!rc) rc = hip_check(hipStreamSynchronize(s), "twins");
        }
        if (rc) return rc;
        if (hctr[1] & 1u) return 1;
        if (hctr[1] & 2u) {  // more parallel runs than the list holds: pair every run here
            parallel_rows([&](uint32_t u, Scratch &sc) {
                for (uint64_t f = rp[u]; f < rp[u + 1];) {
                    const uint32_t v = adj[f].x;
                    uint64_t f1 = f;
                    while (f1 < rp[u + 1] && adj[f1].x == v) f1++;
                    if (v == u) {
                        for (uint64_t t = f; t < f1; t++) canon[t] = NONE;
                    } else if (v > u && !match_run(u, f, sc)) {
                        asym = true;
                        return;
                    }
                    f = f1;
                }
            });
        } else {
            Scratch sc;
            for (const uint2 &m : multi)
                if (!match_run(m.x, m.y, sc)) {
                    asym = true;
                    break;
                }
        }
    }
    if (asym) return 1;
    // perm: stable LSD radix sort of the vertices by ~degree, two 16-bit digits
    std::vector<uint32_t> perm(n), tmp(n), key(n);
    for (uint32_t v = 0; v < n; v++) {
        perm[v] = v;
        key[v] = ~(uint32_t)std::min<uint64_t>(rp[v + 1] - rp[v], 0xFFFFFFFFu);
    }
    std::vector<uint32_t> cnt(65536);
    for (int pass = 0; pass < 2; pass++) {
        const int shift = 16 * pass;
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (uint32_t v = 0; v < n; v++) cnt[(key[v] >> shift) & 0xFFFFu]++;
        uint32_t sum = 0;
        for (uint32_t &c : cnt) {
            const uint32_t x = c;
            c = sum;
            sum += x;
        }
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t v = perm[i];
            tmp[cnt[(key[v] >> shift) & 0xFFFFu]++] = v;
        }
        perm.swap(tmp);
    }
    std::vector<uint32_t> inv(n);
    for (uint32_t i = 0; i < n; i++) inv[perm[i]] = i;
    std::vector<uint64_t> nrp((size_t)n + 1, 0);
    for (uint32_t i = 0; i < n; i++) nrp[i + 1] = nrp[i] + (rp[perm[i] + 1] - rp[perm[i]]);
    // rows in the new order, each sorted by new column id; onew points at the entry that leaves the
    // smaller new id, the one the boundary scan reads
    // (onew is read only at canonical offsets, each written below)
    HostArray<uint2> nadj(nnz);
    HostArray<uint32_t> eo(nnz), onew(nnz);
    parallel_rows([&](uint32_t i, Scratch &sc) {
        std::vector<uint64_t> &row = sc.row;
        const uint32_t v = perm[i];
        const uint64_t b = rp[v], d = rp[v + 1] - b;
        row.resize(d);
        for (uint64_t j = 0; j < d; j++) row[j] = ((uint64_t)inv[adj[b + j].x] << 32) | j;
        std::sort(row.begin(), row.end());
        for (uint64_t t = 0; t < d; t++) {
            const uint64_t f = b + (uint32_t)row[t], e = nrp[i] + t;
            const uint32_t nu = (uint32_t)(row[t] >> 32);
            nadj[e] = make_uint2(nu, adj[f].y);
            eo[e] = canon[f];
            if (i < nu) onew[canon[f]] = (uint32_t)e;
        }
    });
    std::vector<uint32_t> nrp32((size_t)n + 1);
    for (size_t i = 0; i <= n; i++) nrp32[i] = (uint32_t)nrp[i];
    if ((rc = dev_alloc((void **)&g->d_perm, (size_t)n * 4)) || (rc = dev_alloc((void **)&g->d_inv, (size_t)n * 4)) ||
        (rc = dev_alloc((void **)&g->d_eo, nnz * 4)) || (rc = dev_alloc((void **)&g->d_onew, nnz * 4)))
        return rc;
    rc = hip_check(hipMemcpyAsync(g->d_rp, nrp32.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice, s), "H2D row_ptr");
    if (!rc && nnz) rc = hip_check(hipMemcpyAsync(g->d_adj, nadj.data(), nnz * 8, hipMemcpyHostToDevice, s), "H2D adjacency");
    if (!rc && nnz) rc = hip_check(hipMemcpyAsync(g->d_eo, eo.data(), nnz * 4, hipMemcpyHostToDevice, s), "H2D offsets");
    if (!rc && nnz) rc = hip_check(hipMemcpyAsync(g->d_onew, onew.data(), nnz * 4, hipMemcpyHostToDevice, s), "H2D offsets");
    if (!rc) rc = hip_check(hipMemcpyAsync(g->d_perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "H2D perm");
    if (!rc) rc = hip_check(hipMemcpyAsync(g->d_inv, inv.data(), (size_t)n * 4, hipMemcpyHostToDevice, s), "H2D perm");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "reorder upload");
    if (rc) return rc;
    g->h_rp.swap(nrp);
    g->h_perm.swap(perm);
    g->h_inv.swap(inv);
    g->reordered = true;
    return STEINER_OK;
}

static int finish_graph(steiner_graph *g, const uint64_t *d_rp64, const uint32_t *d_col, const uint32_t *d_w,
                        uint32_t flags) {
    const uint32_t n = g->n;
    const uint64_t nnz = g->nnz;
    hipStream_t s = g->stream;
    int rc;
    uint64_t ends[2];
    if ((rc = hip_check(hipMemcpyAsync(&ends[0], d_rp64, 8, hipMemcpyDeviceToHost, s), "row_ptr[0]"))) return rc;
    if ((rc = hip_check(hipMemcpyAsync(&ends[1], d_rp64 + n, 8, hipMemcpyDeviceToHost, s), "row_ptr[n]"))) return rc;
    if ((rc = hip_check(hipStreamSynchronize(s), "sync"))) return rc;
    if (ends[0] != 0 || ends[1] != nnz) return fail(STEINER_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
    void *is_start = nullptr, *bad = nullptr;
    if ((rc = dev_alloc(&is_start, nnz + 1))) return rc;
    if ((rc = dev_alloc(&bad, 16))) { dev_free(is_start); return rc; }
    (void)hipMemsetAsync(is_start, 0, nnz + 1, s);
    (void)hipMemsetAsync(bad, 0, 16, s);
    hipLaunchKernelGGL(k_validate_rows, dim3(2048), dim3(256), 0, s, d_rp64, n, nnz, (uint8_t *)is_start, (uint32_t *)bad);
    hipLaunchKernelGGL(k_validate_entries, dim3(4096), dim3(256), 0, s, d_col, d_w, nnz, n, (const uint8_t *)is_start,
                       (uint32_t *)bad);
    uint32_t hbad = 0;
    rc = hip_check(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "validate");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "validate sync");
    if (!rc && !hbad && (flags & STEINER_UPLOAD_SYMMETRY)) {
        hipLaunchKernelGGL(k_validate_symmetry, dim3(2048), dim3(256), 0, s, d_rp64, d_col, d_w, n, (uint32_t *)bad);
        rc = hip_check(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "symmetry");
        if (!rc) rc = hip_check(hipStreamSynchronize(s), "symmetry sync");
    }
    dev_free(is_start);
    if (rc) { dev_free(bad); return rc; }
    if (hbad) {
        dev_free(bad);
        return fail(STEINER_EINVAL, "invalid graph:%s%s%s%s", (hbad & 1) ? " non-monotone row_ptr" : "",
                    (hbad & 2) ? " column out of range or zero weight" : "", (hbad & 4) ? " unsorted row" : "",
                    (hbad & 8) ? " asymmetric" : "");
    }
    if ((rc = dev_alloc((void **)&g->d_rp, ((size_t)n + 1) * 4))) { dev_free(bad); return rc; }
    if ((rc = dev_alloc((void **)&g->d_adj, nnz * 8))) { dev_free(bad); return rc; }
    hipLaunchKernelGGL(k_convert, dim3(4096), dim3(256), 0, s, d_rp64, n, d_col, d_w, nnz, g->d_rp, g->d_adj);
    (void)hipMemsetAsync(bad, 0, 16, s);
    hipLaunchKernelGGL(k_weight_sum, dim3(1024), dim3(256), 0, s, d_w, nnz, (unsigned long long *)bad);
    unsigned long long wsum = 0;
    g->h_rp.resize((size_t)n + 1);
    rc = hip_check(hipMemcpyAsync(&wsum, bad, 8, hipMemcpyDeviceToHost, s), "weights");
    if (!rc) rc = hip_check(hipMemcpyAsync(g->h_rp.data(), d_rp64, ((size_t)n + 1) * 8, hipMemcpyDeviceToHost, s), "row_ptr");
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "convert");
    dev_free(bad);
    if (rc) return rc;
    // Internal order: renumber skewed graphs (maximum degree at least 32 times the mean) unless the
    // flags say otherwise.
    bool reorder = (flags & STEINER_UPLOAD_REORDER) != 0;
    if (!(flags & (STEINER_UPLOAD_REORDER | STEINER_UPLOAD_KEEP_ORDER)) && nnz) {
        uint64_t mx = 0;
        for (uint32_t v = 0; v < n; v++) mx = std::max(mx, g->h_rp[v + 1] - g->h_rp[v]);
        reorder = (double)mx >= 32.0 * (double)nnz / (double)n;
    }
    if (reorder) {
        try {
            rc = reorder_graph(g);
        } catch (const std::bad_alloc &) {
            rc = fail(STEINER_ENOMEM, "host memory for the renumbering is exhausted");
        }
    }
    if (reorder && rc) {
        if (rc != 1) return rc;
        // an asymmetric CSR has no twin for some entry: keep the caller's order
        if (flags & STEINER_UPLOAD_REORDER) return fail(STEINER_EINVAL, "renumbering needs a symmetric CSR");
    }
    // Heavy rows of the boundary scan and the default bucket width.
    const uint32_t scan_heavy = 1024, scan_chunk = 1024;
    std::vector<uint32_t> hrows, hoff;
    hoff.push_back(0);
    for (uint32_t v = 0; v < n; v++) {
        uint64_t d = g->h_rp[v + 1] - g->h_rp[v];
        g->max_deg = std::max(g->max_deg, d);
        if (d > scan_heavy) {
            hrows.push_back(v);
            hoff.push_back(hoff.back() + (uint32_t)((d + scan_chunk - 1) / scan_chunk));
        }
    }
    g->nheavy = (uint32_t)hrows.size();
    if ((rc = dev_alloc((void **)&g->d_heavy_rows, hrows.size() * 4 + 4))) return rc;
    if ((rc = dev_alloc((void **)&g->d_heavy_off, hoff.size() * 4))) return rc;
    if (!hrows.empty())
        (void)hipMemcpyAsync(g->d_heavy_rows, hrows.data(), hrows.size() * 4, hipMemcpyHostToDevice, s);
    (void)hipMemcpyAsync(g->d_heavy_off, hoff.data(), hoff.size() * 4, hipMemcpyHostToDevice, s);
    if ((rc = hip_check(hipStreamSynchronize(s), "heavy rows"))) return rc;
    if (n && g->max_deg <= ELL_W) {
        if ((rc = dev_alloc((void **)&g->d_ell, (size_t)n * 2 * sizeof(uint4)))) return rc;
        hipLaunchKernelGGL(k_build_ell, dim3(4096), dim3(256), 0, s, g->d_rp, g->d_adj, n, g->d_ell);
        if ((rc = hip_check(hipGetLastError(), "fixed-stride rows"))) return rc;
        if ((rc = hip_check(hipStreamSynchronize(s), "fixed-stride rows"))) return rc;
    }
    DevGraph &dg = g->dg;
    dg.n = n;
    dg.nnz = (uint32_t)nnz;
    dg.max_deg = (uint32_t)std::min<uint64_t>(g->max_deg, 0xFFFFFFFFull);
    dg.rp = g->d_rp;
    dg.adj = g->d_adj;
    dg.ell = g->d_ell;
    dg.nheavy = g->nheavy;
    dg.nheavy_chunks = hoff.back();
    dg.heavy_rows = g->d_heavy_rows;
    dg.heavy_chunk_off = g->d_heavy_off;
    dg.scan_heavy = scan_heavy;
    dg.scan_chunk = scan_chunk;
    dg.perm = g->d_perm;
    dg.inv = g->d_inv;
    dg.eo = g->d_eo;
    dg.onew = g->d_onew;
    bool prefix = true;
    for (uint32_t h = 0; h < hrows.size() && prefix; h++) prefix = hrows[h] == h;
    dg.reverse_scan = (g->reordered && g->d_eo && prefix && !std::getenv("STEINER_FORWARD_SCAN")) ? 1u : 0u;
    const double avg_w = nnz ? (double)wsum / (double)nnz : 1.0;
    const double avg_deg = n ? (double)nnz / (double)n : 1.0;
    // the classic bucket width (about the mean weight over the mean degree) is one of the tuner's
    // candidates; untuned solves use one unbounded bucket, which is never far from the best here
    const double d = 2.0 * avg_w / std::max(1.0, avg_deg);
    g->classic_delta = (uint32_t)std::max(1.0, std::min(d, 4.0e9));
    g->default_delta = 0xFFFFFFFFu;
    g->avg_w = avg_w;
    return STEINER_OK;
}

static int graph_create(uint32_t n, uint64_t nnz, int device, void *stream, steiner_graph **out) {
    if (!out) return fail(STEINER_EINVAL, "out is NULL");
    if (n == 0) return fail(STEINER_EINVAL, "n must be > 0");
    if (n == 0xFFFFFFFFu) return fail(STEINER_EINVAL, "n must be < 2^32-1");
    if (nnz >= (1ull << 32)) return fail(STEINER_EINVAL, "nnz must be < 2^32 (edge ids are 32-bit)");
    int rc = hip_check(hipSetDevice(device), "hipSetDevice");
    if (rc) return rc;
    steiner_graph *g = new steiner_graph();
    g->device = device;
    g->stream = (hipStream_t)stream;
    g->n = n;
    g->nnz = nnz;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) g->cu_count = prop.multiProcessorCount;
    noalloc_setup(device);
    *out = g;
    return STEINER_OK;
}

extern "C" int steiner_graph_upload(uint32_t n, uint64_t nnz, const uint64_t *row_ptr, const uint32_t *col,
                                    const uint32_t *w, int device, void *hip_stream, uint32_t flags,
                                    steiner_graph **out) {
    if (!row_ptr || (nnz && (!col || !w))) return fail(STEINER_EINVAL, "NULL array");
    if ((flags & STEINER_UPLOAD_REORDER) && (flags & STEINER_UPLOAD_KEEP_ORDER))
        return fail(STEINER_EINVAL, "STEINER_UPLOAD_REORDER and STEINER_UPLOAD_KEEP_ORDER exclude each other");
    steiner_graph *g = nullptr;
    int rc = graph_create(n, nnz, device, hip_stream, &g);
    if (rc) return rc;
    void *rp = nullptr, *c = nullptr, *ww = nullptr;
    rc = dev_alloc(&rp, ((size_t)n + 1) * 8);
    if (!rc) rc = dev_alloc(&c, nnz * 4);
    if (!rc) rc = dev_alloc(&ww, nnz * 4);
    if (!rc) rc = hip_check(hipMemcpyAsync(rp, row_ptr, ((size_t)n + 1) * 8, hipMemcpyHostToDevice, g->stream), "H2D row_ptr");
    if (!rc && nnz) rc = hip_check(hipMemcpyAsync(c, col, nnz * 4, hipMemcpyHostToDevice, g->stream), "H2D col");
    if (!rc && nnz) rc = hip_check(hipMemcpyAsync(ww, w, nnz * 4, hipMemcpyHostToDevice, g->stream), "H2D w");
    if (!rc) rc = finish_graph(g, (const uint64_t *)rp, (const uint32_t *)c, (const uint32_t *)ww, flags);
    (void)hipStreamSynchronize(g->stream);
    dev_free(rp);
    dev_free(c);
    dev_free(ww);
    if (rc) {
        std::string keep = g_last_error;
        steiner_graph_free(g);
        g_last_error = keep;
        return rc;
    }
    *out = g;
    return STEINER_OK;
}

extern "C" int steiner_graph_upload_device(uint32_t n, uint64_t nnz, const void *d_row_ptr, const void *d_col,
                                           const void *d_w, int device, void *hip_stream, uint32_t flags,
                                           steiner_graph **out) {
    if (!d_row_ptr || (nnz && (!d_col || !d_w))) return fail(STEINER_EINVAL, "NULL array");
    if ((flags & STEINER_UPLOAD_REORDER) && (flags & STEINER_UPLOAD_KEEP_ORDER))
        return fail(STEINER_EINVAL, "STEINER_UPLOAD_REORDER and STEINER_UPLOAD_KEEP_ORDER exclude each other");
    steiner_graph *g = nullptr;
    int rc = graph_create(n, nnz, device, hip_stream, &g);
    if (rc) return rc;
    rc = finish_graph(g, (const uint64_t *)d_row_ptr, (const uint32_t *)d_col, (const uint32_t *)d_w, flags);
    if (rc) {
        std::string keep = g_last_error;
        steiner_graph_free(g);
        g_last_error = keep;
        return rc;
    }
    *out = g;
    return STEINER_OK;
}

extern "C" int steiner_graph_free(steiner_graph *g) {
    if (!g) return STEINER_OK;
    (void)hipSetDevice(g->device);
    (void)hipStreamSynchronize(g->stream);
    g->ws.release();
    g->clusters.release();
    for (auto &kv : g->chunk_tables)
        if (kv.second) kv.second->start.release();
    dev_free(g->d_rp);
    dev_free(g->d_adj);
    dev_free(g->d_ell);
    dev_free(g->d_heavy_rows);
    dev_free(g->d_heavy_off);
    dev_free(g->d_perm);
    dev_free(g->d_inv);
    dev_free(g->d_eo);
    dev_free(g->d_onew);
    delete g;
    return STEINER_OK;
}

// ==================================================================== results

extern "C" int steiner_result_edges(const steiner_result *r, uint64_t *m, const uint32_t **a, const uint32_t **b,
                                    const uint32_t **w) {
    if (!r || !m) return fail(STEINER_EINVAL, "NULL argument");
    *m = r->a.size();
    if (a) *a = r->a.data();
    if (b) *b = r->b.data();
    if (w) *w = r->w.data();
    return STEINER_OK;
}

extern "C" uint64_t steiner_result_total(const steiner_result *r) { return r ? r->total : 0; }

extern "C" int steiner_result_stats(const steiner_result *r, steiner_stats *out) {
    if (!r || !out) return fail(STEINER_EINVAL, "NULL argument");
    *out = r->stats;
    return STEINER_OK;
}

extern "C" void steiner_result_free(steiner_result *r) { delete r; }

extern "C" const char *steiner_strerror(int code) {
    switch (code) {
    case STEINER_OK: return "ok";
    case STEINER_EINVAL: return "invalid argument";
    case STEINER_ENOMEM: return "out of memory";
    case STEINER_EDISCONNECTED: return "seeds are not connected";
    case STEINER_EOVERFLOW: return "distance overflow";
    case STEINER_EDEVICE: return "device error";
    case STEINER_ETIMEDOUT: return "timed out";
    case STEINER_ECANCELED: return "canceled";
    default: return "unknown error";
    }
}

extern "C" const char *steiner_last_error(void) { return g_last_error.c_str(); }

// ===================================================================== solves

// Distinct seeds in ascending caller-id order (seed index = position), as
// internal ids; EINVAL for k == 0 or a seed >= n.
int stn::canon_seeds(const steiner_graph *g, const uint32_t *seeds, uint32_t k, std::vector<uint32_t> &S) {
    if (k == 0) return fail(STEINER_EINVAL, "k must be > 0");
    if (!seeds) return fail(STEINER_EINVAL, "seeds is NULL");
    S.assign(seeds, seeds + k);
    for (uint32_t s : S)
        if (s >= g->n) return fail(STEINER_EINVAL, "seed %u >= n", s);
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
    if (S.size() > STEINER_MAX_SEEDS)
        return fail(STEINER_EINVAL, "%zu distinct seeds; at most %u", S.size(), (unsigned)STEINER_MAX_SEEDS);
    if (g->reordered)
        for (uint32_t &s : S) s = g->h_inv[s];
    return STEINER_OK;
}

void stn::seed_ranks(const steiner_graph *g, const std::vector<uint32_t> &S, std::vector<uint32_t> &rk) {
    rk.clear();
    if (!g->reordered) return;
    const uint32_t k = (uint32_t)S.size();
    rk.resize(2ull * k);
    uint32_t *tr = rk.data(), *ts = rk.data() + k;
    for (uint32_t i = 0; i < k; i++) ts[i] = i;
    std::sort(ts, ts + k, [&](uint32_t a, uint32_t b) { return S[a] < S[b]; });
    for (uint32_t r = 0; r < k; r++) tr[ts[r]] = r;
}

extern "C" int steiner_solve(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                             steiner_result **out) {
    if (!g || !out) return fail(STEINER_EINVAL, "NULL argument");
    const uint32_t *ps[1] = {seeds};
    uint32_t ks[1] = {k};
    steiner_result *res[1] = {nullptr};
    int st[1] = {0};
    int rc = steiner_solve_batch(g, 1, ps, ks, opt, res, st);
    if (rc) return rc;
    if (st[0]) return st[0];
    *out = res[0];
    return STEINER_OK;
}

extern "C" int steiner_solve_batch(steiner_graph *g, uint32_t q, const uint32_t *const *seeds, const uint32_t *ks,
                                   const steiner_options *opt, steiner_result **outs, int *status) {
    if (!g || !outs || !status || (q && (!seeds || !ks))) return fail(STEINER_EINVAL, "NULL argument");
    if (q == 0) return STEINER_OK;
    if (q > MAX_SLOTS) return fail(STEINER_EINVAL, "at most %u queries per batch", MAX_SLOTS);
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    Options o = resolve_options(g, opt);
    std::vector<Query> qs(q);
    for (uint32_t i = 0; i < q; i++) {
        outs[i] = nullptr;
        status[i] = canon_seeds(g, seeds[i], ks[i], qs[i].S);
        qs[i].status = status[i];
    }
    rc = run_pass(g, o, qs);
    if (rc) return rc;
    for (uint32_t i = 0; i < q; i++) {
        status[i] = qs[i].status;
        if (qs[i].status == STEINER_OK) outs[i] = qs[i].result.release();
    }
    return STEINER_OK;
}

extern "C" int steiner_graph_tune(steiner_graph *g, const uint32_t *seeds, uint32_t k, steiner_options *out) {
    if (!g) return fail(STEINER_EINVAL, "NULL graph");
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    std::vector<uint32_t> S;
    if ((rc = canon_seeds(g, seeds, k, S))) return rc;
    if (S.size() < 2) return fail(STEINER_EINVAL, "tuning needs at least 2 distinct seeds");
    const double w = std::max(1.0, g->avg_w);
    std::vector<uint32_t> deltas = {g->classic_delta, (uint32_t)std::max(1.0, w / 4), (uint32_t)std::max(1.0, w / 2),
                                    (uint32_t)std::max(1.0, w),
                                    (uint32_t)std::max(1.0, 4 * w), (uint32_t)std::max(1.0, 16 * w), 0xFFFFFFFFu};
    std::sort(deltas.begin(), deltas.end());
    deltas.erase(std::unique(deltas.begin(), deltas.end()), deltas.end());
    // coarse to fine: the bucket width at the default queue depth, then the depth, then the split
    const bool lazy_default = resolve_options(g, nullptr).lazy_pred;
    g->tuned_grid = 0;
    auto measure = [&](uint32_t d, uint32_t l, uint32_t split, double *t_out, bool lazy, uint32_t grid = 0,
                       int defer = -1) -> int {
        Options o = resolve_options(g, nullptr);
        o.delta = d;
        o.local_iters = l;
        o.split = split != 0 && d != 0xFFFFFFFFu;
        o.lazy_pred = lazy;
        if (defer >= 0) o.defer_min = defer ? std::max<uint32_t>(o.small_max, 1) : 0;
        if (grid) o.grid = o.grid_tuned = grid;
        double t_min = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            std::vector<Query> qs(1);
            qs[0].S = S;
            const auto t0 = std::chrono::steady_clock::now();
            int e = run_pass(g, o, qs);
            if (e) return e;
            const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (qs[0].status && qs[0].status != STEINER_EDISCONNECTED && qs[0].status != STEINER_EOVERFLOW)
                return qs[0].status;
            t_min = std::min(t_min, t);
        }
        *t_out = t_min;
        return STEINER_OK;
    };
    double best = 1e300, t;
    uint32_t best_d = g->default_delta, best_l = 8, best_split = 0;
    // deferral is tried beside each bucket width wherever some row exceeds the small-row bound
    const bool can_defer = g->max_deg > resolve_options(g, nullptr).small_max;
    int best_defer = 0;
    // after the bucket width, a candidate replaces the default it competes with (depth 8, no split, the
    // graph's pred placement, every resident workgroup) only when it is clearly faster (3%), so repeated
    // tunings of one graph settle on the same settings despite timing noise
    auto better = [&](double tt) { return tt < best * 0.97; };
    for (uint32_t d : deltas)
        for (int df = 0; df <= (can_defer ? 1 : 0); df++) {
            if ((rc = measure(d, 8, 0, &t, lazy_default, 0, df))) return rc;
            if (t < best) { best = t; best_d = d; best_defer = df; }
        }
    for (uint32_t l : {2u, 4u, 16u, 32u}) {
        if ((rc = measure(best_d, l, 0, &t, lazy_default, 0, best_defer))) return rc;
        if (better(t)) { best = t; best_l = l; }
    }
    if (best_d != 0xFFFFFFFFu) {  // the split expands every settled row's heavy edges at the advance: no deferral
        if ((rc = measure(best_d, best_l, 1, &t, lazy_default, 0, 0))) return rc;
        if (better(t)) { best = t; best_split = 1; best_defer = 0; }
    }
    bool best_lazy = lazy_default;
    if ((rc = measure(best_d, best_l, best_split, &t, !lazy_default, 0, best_defer))) return rc;
    if (better(t)) { best = t; best_lazy = !lazy_default; }
    // then fewer relaxation workgroups (a quarter to three quarters of the resident count), at the chosen depth
    // and at 8
    uint32_t best_grid = 0;
    const int resident = round_max_grid(256);
    if (resident >= 8) {
        std::vector<uint32_t> ls = {best_l};
        if (best_l != 8) ls.push_back(8);
        for (uint32_t l : ls)
            for (uint32_t gsz : {(uint32_t)resident / 4, (uint32_t)resident * 3 / 8, (uint32_t)resident / 2,
                                 (uint32_t)resident * 3 / 4}) {
                if ((rc = measure(best_d, l, best_split, &t, best_lazy, gsz, best_defer))) return rc;
                if (better(t)) { best = t; best_l = l; best_grid = gsz; }
            }
    }
    g->tuned_grid = best_grid;
    g->tuned_delta = best_d;
    g->tuned_local = best_l;
    g->tuned_split = best_split;
    g->tuned_pred = best_lazy ? 2 : 1;
    g->tuned_defer = best_defer ? 2 : 1;
    if (out) {
        memset(out, 0, sizeof(*out));
        out->delta = best_d;
        out->local_iters = best_l;
        out->grid = best_grid;
        out->flags = (best_split ? STEINER_FLAG_SPLIT : 0u) | (best_lazy ? STEINER_FLAG_LAZY_PRED : STEINER_FLAG_EAGER_PRED) |
                     (best_defer ? STEINER_FLAG_DEFER : STEINER_FLAG_NO_DEFER);
    }
    return STEINER_OK;
}

extern "C" int steiner_voronoi(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                               uint64_t *key_out, uint32_t *pred_out) {
    if (!g || !key_out || !pred_out) return fail(STEINER_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    std::vector<Query> qs(1);
    if ((rc = canon_seeds(g, seeds, k, qs[0].S))) return rc;
    if (qs[0].S.size() < 2) return fail(STEINER_EINVAL, "steiner_voronoi needs at least 2 distinct seeds");
    qs[0].want_key = key_out;
    qs[0].want_pred = pred_out;
    qs[0].stop_after = STOP_AFTER_SCAN;
    Options o = resolve_options(g, opt);
    rc = run_pass(g, o, qs);
    if (rc) return rc;
    return qs[0].status;
}

extern "C" int steiner_boundary(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                                uint64_t *npairs, uint32_t *pi, uint32_t *pj, uint64_t *packed, uint64_t cap) {
    if (!g || !npairs || (cap && (!pi || !pj || !packed))) return fail(STEINER_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    std::vector<Query> qs(1);
    if ((rc = canon_seeds(g, seeds, k, qs[0].S))) return rc;
    if (qs[0].S.size() < 2) return fail(STEINER_EINVAL, "steiner_boundary needs at least 2 distinct seeds");
    qs[0].stop_after = STOP_AFTER_COMPACT;
    Options o = resolve_options(g, opt);
    rc = run_pass(g, o, qs);
    if (rc) return rc;
    if (qs[0].status) return qs[0].status;
    const size_t m = qs[0].pidx.size();
    std::vector<size_t> ord(m);
    for (size_t t = 0; t < m; t++) ord[t] = t;
    std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return qs[0].pidx[x] < qs[0].pidx[y]; });
    *npairs = m;
    if (m > cap) return fail(STEINER_ENOMEM, "G'1 has %zu entries, capacity %llu", m, (unsigned long long)cap);
    // lower-triangular index order is (j, i) order; report sorted by (i, j)
    std::vector<std::tuple<uint32_t, uint32_t, uint64_t>> rows(m);
    for (size_t t = 0; t < m; t++) {
        uint32_t i, j;
        pair_from_index(qs[0].pidx[ord[t]], &i, &j);
        rows[t] = std::make_tuple(i, j, qs[0].pval[ord[t]]);
    }
    std::sort(rows.begin(), rows.end());
    for (size_t t = 0; t < m; t++) {
        pi[t] = std::get<0>(rows[t]);
        pj[t] = std::get<1>(rows[t]);
        packed[t] = std::get<2>(rows[t]);
    }
    return STEINER_OK;
}
